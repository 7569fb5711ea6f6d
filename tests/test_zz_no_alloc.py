"""rsa_decrypt_noalloc (the decryption entry point that allocates nothing)
against rsa_decrypt on the same inputs, bit for bit, through the C ABI: two
calls in a row, the second smaller, for CRT and plain decryption, plus the
size limit."""
import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rsa2048():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the GPU tests need an MI355X")
    from paper_1305_3699_amd import RsaKey, rnsrsa
    rnsrsa.lib()
    key = gen.rsa_key(2048, seed=gen.config_seed(2, 1))
    rk = RsaKey(key.n, key.e, key.d, key.p, key.q, key.dp, key.dq, key.qinv, window=6)
    return key, rk


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("use_crt,sizes", [(True, (1500, 333)), (False, (700, 97))])
def test_noalloc_matches_rsa_decrypt(rsa2048, use_crt, sizes):
    key, rk = rsa2048
    for i, B in enumerate(sizes):
        c = gen.uniform_below(key.n, B, seed=7000 + 10 * i + int(use_crt))
        c[:3] = [0, 1, key.n - 1]
        dc = _dev(gen.to_limbs(c, 64))
        want = _host(rk.decrypt(dc, use_crt=use_crt))
        out = torch.full((B, 64), -1, dtype=torch.int32, device="cuda")
        got = _host(rk.decrypt_noalloc(dc, out, use_crt=use_crt))
        assert np.array_equal(got, want), "call %d (batch %d) differs from rsa_decrypt" % (i + 1, B)


def test_noalloc_rejects_batches_beyond_its_scratch(rsa2048):
    from paper_1305_3699_amd import rnsrsa
    key, rk = rsa2048
    B = 4096                    # about 177 MB of window tables at window 6: above the 64 MiB array
    dc = torch.zeros((B, 64), dtype=torch.int32, device="cuda")
    out = torch.full((B, 64), -1, dtype=torch.int32, device="cuda")
    with pytest.raises(rnsrsa.RnsError) as ei:
        rk.decrypt_noalloc(dc, out, use_crt=True)
    assert rnsrsa.STATUS_NAMES[ei.value.status] == "RNS_EINVAL"
    assert "bytes of scratch" in str(ei.value)
    assert bool((out == -1).all())          # nothing was enqueued
