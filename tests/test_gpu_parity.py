"""GPU parity: every output of the HIP path equals the CPU oracle, bit for bit.

All calls go through the C ABI (ctypes binding) on torch-allocated device
buffers.  Inputs are seeded and synthetic (gen); expected values come from
the oracle only.
"""
import json
import math
import os
import random

import numpy as np
import pytest

import gen
import oracle
from oracle import primality, rns_ref

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the GPU tests need an MI355X")
    from paper_1305_3699_amd import rnsrsa
    rnsrsa.lib()          # fails loudly if the HIP library is missing
    yield


def _threads() -> int:
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(n, 16))


def _dev(a: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


def _host(t) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint32)


def _ctx(N, L, **kw):
    from paper_1305_3699_amd import RnsContext
    return RnsContext(N, L, **kw)


def _run_modexp(ctx, bases, exp):
    b = _dev(bases)
    e = _dev(exp)
    out = ctx.modexp(b, e)
    return _host(out)


def _oracle_pow(bases, e, N):
    """b^e mod N for each base, from the oracle: e an int shared by every
    base, or a list with one exponent per base."""
    bases = [int(b) for b in bases]
    nl = lambda v: max(1, (int(v).bit_length() + 31) // 32)
    bl = oracle.int_to_limbs(0, 1)[None, :] if not bases else np.stack(
        [oracle.int_to_limbs(b, max(nl(v) for v in bases)) for b in bases])
    if isinstance(e, (list, tuple)):
        le = max([nl(v) for v in e] + [1])
        el = np.stack([oracle.int_to_limbs(int(v), le) for v in e])
    else:
        el = oracle.int_to_limbs(int(e), nl(e))
    out = oracle.modexp_batch(bl, el, oracle.int_to_limbs(N, nl(N)), nthreads=_threads())
    return oracle.rows_to_ints(out)[:len(bases)]


def test_toy_key_all_messages():
    """Encrypt and decrypt every m < 3233 with the textbook key (51 groups of
    64 plus a ragged tail of 33)."""
    N, e, d = 3233, 17, 2753
    ctx = _ctx(N, 1)
    msgs = np.arange(N, dtype=np.uint32)[:, None]
    c = _run_modexp(ctx, msgs, np.array([e], np.uint32))
    assert np.array_equal(c, oracle.modexp_batch(msgs, np.array([e], np.uint32), np.array([N], np.uint32)))
    m = _run_modexp(ctx, c, np.array([d], np.uint32))
    assert np.array_equal(m, msgs)
    assert c[65, 0] == 2790


@pytest.mark.parametrize("bits", [20, 64, 100, 500, 1024, 1500, 2048, 3072, 4096])
def test_modexp_sizes(bits):
    rng = random.Random(bits)
    N = rng.getrandbits(bits) | (1 << (bits - 1)) | rng.getrandbits(1)
    L = (bits + 31) // 32
    ctx = _ctx(N, L)
    B = 130                                   # two full groups of 64 and a tail of 2
    bases = [rng.getrandbits(32 * L) for _ in range(B - 4)] + [0, 1, N - 1, (1 << (32 * L)) - 1]
    ebits = 96 if bits > 1024 else 257
    e = rng.getrandbits(ebits) | (1 << (ebits - 1))
    el = gen.to_limbs(e, (ebits + 31) // 32)[0]
    got = _run_modexp(ctx, gen.to_limbs(bases, L), el)
    want = oracle.modexp_batch(gen.to_limbs(bases, L), el, gen.to_limbs(N, L)[0])
    assert np.array_equal(got, want)


def test_edge_exponents():
    rng = random.Random(5)
    N = rng.getrandbits(777) | (1 << 776) | 1
    L = 25
    ctx = _ctx(N, L, window=3)
    bases = [0, 1, 2, N - 1, N, N + 1, (1 << (32 * L)) - 1] + [rng.getrandbits(32 * L) for _ in range(9)]
    for e in (0, 1, 2, 3, 8, 65537, (1 << 64) - 1, (1 << 33) | (1 << 31) | 1, (1 << 63) | (1 << 32) | (1 << 30)):
        el = gen.to_limbs(e, 2)[0]
        got = _run_modexp(ctx, gen.to_limbs(bases, L), el)
        assert oracle.rows_to_ints(got) == _oracle_pow(bases, e, N), e


@pytest.mark.parametrize("window", [2, 5, 6])
def test_windows_across_limbs(window):
    """Sliding windows that straddle two exponent limbs, the lower one with
    its top bit set (read back as a signed value it would corrupt the
    window)."""
    rng = random.Random(window)
    N = rng.getrandbits(512) | (1 << 511) | 1
    ctx = _ctx(N, 16, window=window)
    bases = [rng.getrandbits(512) for _ in range(40)]
    limbs = [rng.getrandbits(32) | (1 << 31) for _ in range(6)]
    e = sum(v << (32 * i) for i, v in enumerate(limbs))
    got = _run_modexp(ctx, gen.to_limbs(bases, 16), gen.to_limbs(e, 6)[0])
    assert oracle.rows_to_ints(got) == _oracle_pow(bases, e, N)


def test_per_element_exponents():
    rng = random.Random(8)
    N = rng.getrandbits(1024) | (1 << 1023) | 1
    ctx = _ctx(N, 32)
    B = 100
    bases = [rng.getrandbits(1024) for _ in range(B)]
    exps = [rng.getrandbits(rng.choice([0, 1, 7, 64, 130])) for _ in range(B)]
    got = _run_modexp(ctx, gen.to_limbs(bases, 32), gen.to_limbs(exps, 5))
    assert oracle.rows_to_ints(got) == _oracle_pow(bases, exps, N)


@pytest.mark.parametrize("window", [1, 2, 3, 4, 5, 6])
def test_window_invariance(window):
    rng = random.Random(77)
    N = rng.getrandbits(1024) | (1 << 1023) | 1
    ctx = _ctx(N, 32, window=window)
    bases = [rng.getrandbits(1024) for _ in range(70)]
    e = rng.getrandbits(1024)
    el = gen.to_limbs(e, 32)[0]
    got = _run_modexp(ctx, gen.to_limbs(bases, 32), el)
    assert oracle.rows_to_ints(got) == _oracle_pow(bases, e, N)


@pytest.mark.parametrize("k,waves", [(17, 1), (17, 2), (33, 1), (33, 2), (33, 3), (33, 4), (49, 7), (65, 5)])
def test_shape_invariance(k, waves):
    """Every wave shape of the channel engine gives the oracle's results."""
    from paper_1305_3699_amd import ENGINE_CHANNEL
    rng = random.Random(k * 10 + waves)
    bits = 32 * (k - 1)
    N = rng.getrandbits(bits) | (1 << (bits - 1)) | 1
    L = k - 1
    ctx = _ctx(N, L, k=k, waves=waves, engine=ENGINE_CHANNEL)
    info = ctx.info
    assert info["k"] == k and info["waves"] == waves
    bases = [rng.getrandbits(32 * L) for _ in range(66)]
    e = rng.getrandbits(80)
    el = gen.to_limbs(e, 3)[0]
    got = _run_modexp(ctx, gen.to_limbs(bases, L), el)
    assert oracle.rows_to_ints(got) == _oracle_pow(bases, e, N)


@pytest.mark.parametrize("bits,k", [(512, 33), (512, 65), (1024, 49), (1024, 65), (1024, 97), (1536, 65), (2048, 129)])
def test_base_size_invariance(bits, k):
    """A base larger than the smallest one the modulus fits (the matrix
    engine's kernels for k channels) gives the oracle's results."""
    rng = random.Random(bits * 1000 + k)
    N = rng.getrandbits(bits) | (1 << (bits - 1)) | 1
    L = bits // 32
    ctx = _ctx(N, L, k=k)
    assert ctx.info["k"] == k
    bases = [rng.getrandbits(bits) for _ in range(40)] + [0, 1, N - 1]
    e = rng.getrandbits(bits) | (1 << (bits - 1))
    got = _run_modexp(ctx, gen.to_limbs(bases, L), gen.to_limbs(e, L)[0])
    assert oracle.rows_to_ints(got) == _oracle_pow(bases, e, N)


@pytest.mark.parametrize("bits", [20, 64, 130, 500, 1024, 1500, 2048, 3072, 4096])
def test_engines_agree(bits):
    """Channel and matrix-core engines give identical bytes, equal to the oracle."""
    from paper_1305_3699_amd import ENGINE_CHANNEL, ENGINE_MATRIX
    rng = random.Random(bits + 5)
    N = rng.getrandbits(bits) | (1 << (bits - 1)) | rng.getrandbits(1)
    L = (bits + 31) // 32
    bases = gen.to_limbs([rng.getrandbits(32 * L) for _ in range(97)] + [0, 1, N - 1], L)
    e = gen.to_limbs(rng.getrandbits(70) | (1 << 69), 3)[0]
    outs = []
    for eng in (ENGINE_CHANNEL, ENGINE_MATRIX):
        ctx = _ctx(N, L, engine=eng, window=4)
        assert ctx.info["engine"] == eng
        outs.append(_run_modexp(ctx, bases, e))
    assert np.array_equal(outs[0], outs[1])
    assert np.array_equal(outs[1], oracle.modexp_batch(bases, e, gen.to_limbs(N, L)[0]))


@pytest.mark.parametrize("engine,group", [(1, 0), (2, 16), (2, 32)])
def test_rsa2048_crt_both_engines(engine, group):
    from paper_1305_3699_amd import RsaKey
    key = gen.rsa_key(2048, seed=gen.config_seed(2, 1))
    rk = RsaKey(key.n, key.e, key.d, key.p, key.q, key.dp, key.dq, key.qinv, engine=engine, group=group)
    assert rk.info(1)["engine"] == engine
    assert rk.info(1)["group"] == (group or 64)
    c = gen.uniform_below(key.n, 70, seed=12) + [0, 1, key.n - 1, key.p, key.q]
    cl = gen.to_limbs(c, 64)
    got = _host(rk.decrypt(_dev(cl), use_crt=True))
    assert np.array_equal(got, oracle.rsa_crt_batch(cl, key.p, key.q, key.dp, key.dq, key.qinv))
    got2 = _host(rk.decrypt(_dev(cl), use_crt=False))
    assert np.array_equal(got2, got)


@pytest.mark.parametrize("bits", [512, 1024, 2048])
def test_scaled_and_unscaled_b_residues(bits):
    """Both forms of the matrix engine's B residues (scaled x R s_i, the
    default on these bases, and the plain x R on request) on the same
    inputs: a shared exponent over two groups and a ragged tail,
    per-element exponents, and one grouped launch that holds a job of each
    form (it runs the unscaled form on both keys); every output equals the
    oracle's pow."""
    from paper_1305_3699_amd import modexp_jobs
    rng = random.Random(bits + 11)
    N = rng.getrandbits(bits) | (1 << (bits - 1)) | 1
    L = bits // 32
    cs, cu = _ctx(N, L), _ctx(N, L, unscaled=True)
    assert cs.info["scaled"] == 1 and cu.info["scaled"] == 0
    bases = gen.to_limbs([rng.getrandbits(bits) for _ in range(37)] + [0, 1, N - 1], L)
    e = gen.to_limbs(rng.getrandbits(bits) | 1, L)[0]
    want = oracle.modexp_batch(bases, e, gen.to_limbs(N, L)[0])
    for c in (cs, cu):
        assert np.array_equal(_run_modexp(c, bases, e), want)
    pe = gen.to_limbs([rng.getrandbits(100) for _ in range(40)], 4)
    want_pe = oracle.modexp_batch(bases, pe, gen.to_limbs(N, L)[0])
    for c in (cs, cu):
        assert np.array_equal(_run_modexp(c, bases, pe), want_pe)
    outs = modexp_jobs([(cs, _dev(bases), _dev(e)), (cu, _dev(bases), _dev(e))])
    for o in outs:
        assert np.array_equal(_host(o), want)


@pytest.mark.parametrize("bits,k", [(64, 3), (128, 5)])
def test_scaled_b_residues_primes_1_mod_4(bits, k):
    """The kernel's scaled form on an explicit base whose B primes are all
    1 mod 4 (roots from the general square-root path; the first seeded draw
    on which every channel has one): outputs equal the oracle's pow."""
    from paper_1305_3699_amd import Plan
    rng = random.Random(bits + 3)
    N = rng.getrandbits(bits) | (1 << (bits - 1)) | 1
    L = bits // 32
    primes = None
    for seed in range(400):
        pr = gen.rns_primes(8 * k, seed=seed, lo=(1 << 32) - (1 << 24), hi=(1 << 32) - (1 << 19))
        B, Bp = [m for m in pr if m % 4 == 1][:k], [m for m in pr if m % 4 == 3][:k]
        if len(B) == k and len(Bp) == k and Plan(N, L, primes=B + Bp).info["scaled"]:
            primes = B + Bp
            break
    assert primes is not None
    ctx = _ctx(N, L, primes=primes)
    assert ctx.info["scaled"] == 1
    bases = gen.to_limbs([rng.getrandbits(bits) for _ in range(37)] + [0, 1, N - 1, N, (1 << bits) - 1], L)
    e = gen.to_limbs(rng.getrandbits(bits) | 1, L)[0]
    assert np.array_equal(_run_modexp(ctx, bases, e), oracle.modexp_batch(bases, e, gen.to_limbs(N, L)[0]))


def test_rsa2048_crt_unscaled():
    """RSA-2048 CRT and plain decryption with the B residues unscaled
    (opts.unscaled) equal the oracle and the default (scaled) key."""
    from paper_1305_3699_amd import RsaKey
    key = gen.rsa_key(2048, seed=gen.config_seed(2, 1))
    c = gen.uniform_below(key.n, 40, seed=13) + [0, 1, key.n - 1]
    cl = gen.to_limbs(c, 64)
    want = oracle.rsa_crt_batch(cl, key.p, key.q, key.dp, key.dq, key.qinv)
    for unscaled in (True, False):
        rk = RsaKey(key.n, key.e, key.d, key.p, key.q, key.dp, key.dq, key.qinv, unscaled=unscaled)
        assert rk.info(1)["scaled"] == (0 if unscaled else 1)
        assert np.array_equal(_host(rk.decrypt(_dev(cl), use_crt=True)), want)
        assert np.array_equal(_host(rk.decrypt(_dev(cl), use_crt=False)), want)


def _indep_base(k: int, seed: int) -> list:
    """2k seeded channel primes from [2^32 - 2^24, 2^32 - 2^19) drawn here (B
    first, then B'), handed to the library through opts.primes, so the
    expected residues do not depend on the library's own choice of base (the
    upper end keeps B' primes inside the matrix engine's one-step reduction
    bound up to k = 513; both engines take such a base)."""
    return gen.rns_primes(2 * k, seed=seed, lo=(1 << 32) - (1 << 24), hi=(1 << 32) - (1 << 19))


@pytest.mark.parametrize("engine", [1, 2])
def test_mont_mul_matches_definition(engine):
    """The standalone product on both engines (channel kernels, matrix cores)
    against its definition, 200 elements (12 tiles and a ragged tail)."""
    rng = random.Random(3)
    N = rng.getrandbits(1024) | (1 << 1023) | 1
    k = 33
    pr = _indep_base(k, seed=gen.config_seed(6, 4))
    ctx = _ctx(N, 32, primes=pr, engine=engine)
    assert ctx.info["k"] == k and ctx.primes == pr and ctx.info["engine"] == engine
    B, Bp = pr[:k], pr[k:]
    n = 200
    X = [rng.randrange((k + 1) * N) for _ in range(n - 2)] + [0, (k + 1) * N - 1]
    Y = [rng.randrange((k + 1) * N) for _ in range(n - 2)] + [(k + 1) * N - 1, (k + 1) * N - 1]

    def res(vals):
        return np.array([[v % m for v in vals] for m in B] + [[v % m for v in vals] for m in Bp]
                        + [[v % (1 << 32) for v in vals]], dtype=np.uint32)

    out = _host(ctx.mont_mul(_dev(res(X)), _dev(res(Y))))
    want = res([rns_ref.mont_mul(x, y, N, B) for x, y in zip(X, Y)])
    assert np.array_equal(out, want)


@pytest.mark.parametrize("k,engine", [(97, 1), (97, 2), (129, 1), (129, 2)])
def test_mont_mul_3072_bit(k, engine):
    """The standalone product at the modulus size of the modular
    multiplication benchmark (3072 bits), with 97 and 129 channels, on both
    engines."""
    rng = random.Random(k)
    N = rng.getrandbits(3072) | (1 << 3071) | 1
    pr = _indep_base(k, seed=gen.config_seed(6, 4) + k)
    ctx = _ctx(N, 96, primes=pr, engine=engine)
    assert ctx.info["k"] == k and ctx.primes == pr and ctx.info["engine"] == engine
    B, Bp = pr[:k], pr[k:]
    n = 70
    X = [rng.randrange((k + 1) * N) for _ in range(n - 1)] + [(k + 1) * N - 1]
    Y = [rng.randrange((k + 1) * N) for _ in range(n - 1)] + [0]

    def res(vals):
        return np.array([[v % m for v in vals] for m in B] + [[v % m for v in vals] for m in Bp]
                        + [[v % (1 << 32) for v in vals]], dtype=np.uint32)

    out = _host(ctx.mont_mul(_dev(res(X)), _dev(res(Y))))
    assert np.array_equal(out, res([rns_ref.mont_mul(x, y, N, B) for x, y in zip(X, Y)]))


@pytest.mark.parametrize("bits,group", [(3072, 16), (3072, 32), (4096, 16), (4096, 32)])
def test_modexp_large_k_both_tiles(bits, group):
    """Full-length exponents modulo 3072- and 4096-bit moduli (k = 97 and
    129, whose matrix kernels read their constant tiles from global memory)
    with both workgroup tiles: 70 bases = several tiles and a ragged tail."""
    rng = random.Random(bits + group)
    N = rng.getrandbits(bits) | (1 << (bits - 1)) | 1
    L = bits // 32
    ctx = _ctx(N, L, group=group)
    assert ctx.info["k"] == {3072: 97, 4096: 129}[bits] and ctx.info["group"] == group
    bases = [rng.getrandbits(32 * L) for _ in range(66)] + [0, 1, N - 1, (1 << (32 * L)) - 1]
    e = rng.getrandbits(bits) | (1 << (bits - 1))
    el = gen.to_limbs(e, L)[0]
    got = _run_modexp(ctx, gen.to_limbs(bases, L), el)
    want = oracle.modexp_batch(gen.to_limbs(bases, L), el, gen.to_limbs(N, L)[0])
    assert np.array_equal(got, want)


@pytest.mark.parametrize("engine", [1, 2])
def test_modexp_8192_bit(engine):
    """8192-bit moduli on bases of 256 + 1 channels (k = 257): 20 bases (a
    full 16-element tile and a ragged one) including 0, 1, N - 1 and
    2^8192 - 1, a 64-bit exponent; the matrix engine also takes a full-length
    exponent on 17 bases."""
    rng = random.Random(8192 + engine)
    N = rng.getrandbits(8192) | (1 << 8191) | 1
    ctx = _ctx(N, 256, engine=engine)
    assert ctx.info["k"] == 257 and ctx.info["engine"] == engine
    bases = gen.to_limbs([rng.getrandbits(8192) for _ in range(16)] + [0, 1, N - 1, (1 << 8192) - 1], 256)
    nl = gen.to_limbs(N, 256)[0]
    e = gen.to_limbs(rng.getrandbits(64) | (1 << 63), 2)[0]
    assert np.array_equal(_run_modexp(ctx, bases, e), oracle.modexp_batch(bases, e, nl))
    if engine == 2:
        e = gen.to_limbs(rng.getrandbits(8192) | (1 << 8191), 256)[0]
        assert np.array_equal(_run_modexp(ctx, bases[:17], e), oracle.modexp_batch(bases[:17], e, nl))


def test_modexp_16384_bit():
    """16384-bit moduli on bases of 512 + 1 channels (k = 513, the matrix
    engine alone): 20 bases (a full 16-element tile and a ragged one)
    including 0, 1, N - 1 and 2^16384 - 1 with a 64-bit exponent, and with
    per-element 40-bit exponents; the channel engine refuses this base."""
    from paper_1305_3699_amd import ENGINE_CHANNEL, ENGINE_MATRIX, RnsError
    rng = random.Random(16384)
    N = rng.getrandbits(16384) | (1 << 16383) | 1
    ctx = _ctx(N, 512)
    assert ctx.info["k"] == 513 and ctx.info["engine"] == ENGINE_MATRIX and ctx.info["group"] == 16
    bases = gen.to_limbs([rng.getrandbits(16384) for _ in range(16)] + [0, 1, N - 1, (1 << 16384) - 1], 512)
    nl = gen.to_limbs(N, 512)[0]
    e = gen.to_limbs(rng.getrandbits(64) | (1 << 63), 2)[0]
    assert np.array_equal(_run_modexp(ctx, bases, e), oracle.modexp_batch(bases, e, nl))
    ex = gen.to_limbs([rng.getrandbits(40) for _ in range(19)] + [0], 2)
    assert np.array_equal(_run_modexp(ctx, bases, ex), oracle.modexp_batch(bases, ex, nl))
    with pytest.raises(RnsError) as err:
        _ctx(N, 512, engine=ENGINE_CHANNEL)
    assert err.value.status == -8


def test_modexp_jobs_mixed_moduli():
    """rns_modexp_jobs: three 1024-bit moduli (one grouped launch), a 2048-bit
    one with per-element exponents, a channel-engine context, a job of
    count 0 and a job whose out aliases its base, in one call; every output
    equals the oracle's and the job's own rns_modexp_batch."""
    from paper_1305_3699_amd import ENGINE_CHANNEL, modexp_jobs
    rng = random.Random(77)
    specs = [(1024, {}), (1024, {}), (1024, {"window": 3}), (2048, {}), (1536, {"engine": ENGINE_CHANNEL})]
    jobs, want = [], []
    for i, (bits, opts) in enumerate(specs):
        N = rng.getrandbits(bits) | (1 << (bits - 1)) | 1
        L = bits // 32
        ctx = _ctx(N, L, **opts)
        B = [17, 40, 3, 33, 20][i]
        bases = gen.to_limbs([rng.getrandbits(bits) for _ in range(B - 2)] + [0, N - 1], L)
        if i == 3:
            e = gen.to_limbs([rng.getrandbits(200) for _ in range(B)], 7)
        else:
            e = gen.to_limbs(rng.getrandbits(bits) | 1, L)[0]
        jobs.append((ctx, _dev(bases), _dev(e)))
        want.append(oracle.modexp_batch(bases, e, gen.to_limbs(N, L)[0]))
    alias = jobs[1][1].clone()
    jobs.append((jobs[1][0], alias, jobs[1][2], alias))
    want.append(want[1])
    empty = torch.zeros((0, 32), dtype=torch.int32, device="cuda")
    jobs.append((jobs[0][0], empty, jobs[0][2]))
    outs = modexp_jobs(jobs)
    torch.cuda.synchronize()
    for i, w in enumerate(want):
        assert np.array_equal(_host(outs[i]), w), i
        assert np.array_equal(_host(jobs[i][0].modexp(jobs[i][1] if i != 5 else jobs[1][1], jobs[i][2])), w), i
    assert outs[6].shape == (0, 32)


def test_crt_verify_detects_faulty_half():
    """rsa_crt_verify, the check against faults in CRT decryption: 40
    RSA-2048 ciphertexts through rsa_crt_halves and rsa_crt_combine all pass;
    with a bit of m_p flipped in row 5 and a bit of m_q in row 17 between the
    two launches (faults planted in the data from the host), exactly those
    two rows fail and are zeroed, and the others equal the oracle's."""
    from paper_1305_3699_amd import RsaKey
    k = gen.rsa_key(2048, seed=gen.config_seed(3, 12))
    rk = RsaKey(k.n, k.e, k.d, k.p, k.q, k.dp, k.dq, k.qinv)
    c = gen.to_limbs(gen.uniform_below(k.n, 40, seed=gen.config_seed(8, 26)), 64)
    want = oracle.rsa_crt_batch(c, k.p, k.q, k.dp, k.dq, k.qinv)
    dc = _dev(c)
    mpq = rk.crt_halves(dc)
    m = rk.crt_combine(mpq)
    assert rk.verify_crt(dc, m) == 0
    assert np.array_equal(_host(m), want)
    bad = mpq.clone()
    bad[5, 3] ^= 1 << 9
    bad[17, rk.half_limbs + 7] ^= 1
    m2 = rk.crt_combine(bad)
    assert rk.verify_crt(dc, m2) == 2
    got = _host(m2)
    assert not got[[5, 17]].any()
    keep = [i for i in range(40) if i not in (5, 17)]
    assert np.array_equal(got[keep], want[keep])


def test_probe_alu_rates():
    """rns_probe_alu measures both wide multiply forms at a plausible rate:
    above a quarter of the full per-lane issue rate (256 CUs x 64 lanes x
    2.4 GHz = 39.3 T lane-ops/s) and not above it."""
    import ctypes
    from paper_1305_3699_amd import rnsrsa
    for op in (0, 1):
        v = ctypes.c_double(0.0)
        assert rnsrsa.lib().rns_probe_alu(op, ctypes.byref(v), None) == 0
        assert 0.25 * 39.3e12 < v.value <= 1.02 * 39.3e12, (op, v.value)


@pytest.mark.parametrize("engine", [1, 2])
def test_mont_mul_8192_bit(engine):
    """The standalone product at 8192 bits (k = 257) on both engines."""
    rng = random.Random(257)
    N = rng.getrandbits(8192) | (1 << 8191) | 1
    k = 257
    pr = _indep_base(k, seed=gen.config_seed(6, 4) + k)
    ctx = _ctx(N, 256, primes=pr, engine=engine)
    assert ctx.info["k"] == k and ctx.primes == pr and ctx.info["engine"] == engine
    B, Bp = pr[:k], pr[k:]
    n = 70
    X = [rng.randrange((k + 1) * N) for _ in range(n - 1)] + [(k + 1) * N - 1]
    Y = [rng.randrange((k + 1) * N) for _ in range(n - 1)] + [0]

    def res(vals):
        return np.array([[v % m for v in vals] for m in B] + [[v % m for v in vals] for m in Bp]
                        + [[v % (1 << 32) for v in vals]], dtype=np.uint32)

    out = _host(ctx.mont_mul(_dev(res(X)), _dev(res(Y))))
    assert np.array_equal(out, res([rns_ref.mont_mul(x, y, N, B) for x, y in zip(X, Y)]))


def test_mont_mul_16384_bit():
    """The standalone product at 16384 bits (k = 513, matrix cores only),
    20 elements: a full 16-element tile and a ragged one."""
    rng = random.Random(513)
    N = rng.getrandbits(16384) | (1 << 16383) | 1
    k = 513
    pr = _indep_base(k, seed=gen.config_seed(6, 4) + k)
    ctx = _ctx(N, 512, primes=pr)
    assert ctx.info["k"] == k and ctx.primes == pr and ctx.info["engine"] == 2
    B, Bp = pr[:k], pr[k:]
    n = 20
    X = [rng.randrange((k + 1) * N) for _ in range(n - 1)] + [(k + 1) * N - 1]
    Y = [rng.randrange((k + 1) * N) for _ in range(n - 2)] + [0, (k + 1) * N - 1]

    def res(vals):
        return np.array([[v % m for v in vals] for m in B] + [[v % m for v in vals] for m in Bp]
                        + [[v % (1 << 32) for v in vals]], dtype=np.uint32)

    out = _host(ctx.mont_mul(_dev(res(X)), _dev(res(Y))))
    assert np.array_equal(out, res([rns_ref.mont_mul(x, y, N, B) for x, y in zip(X, Y)]))


def test_rsa16384_crt_only_key():
    """RSA-16384 CRT decryption: 8192-bit halves on bases of 257 channels.
    With the channel engine requested, which has no kernel for the
    513-channel base of the full modulus, the key loads CRT-only: decryption
    through the halves works, encryption is refused.  20 ciphertexts (a full
    16-element tile and a ragged one) against the oracle's CRT path, two of
    them also by m^e = c.  The key is the stored seeded fixture."""
    from paper_1305_3699_amd import ENGINE_CHANNEL, RnsError
    rk, parts = _rsa16384_key(engine=ENGINE_CHANNEL)
    n, e, p, q, dp, dq, qinv = (parts[k] for k in ("n", "e", "p", "q", "dp", "dq", "qinv"))
    assert n.bit_length() == 16384
    assert rk.info(1)["k"] == 257 and rk.info(2)["k"] == 257
    with pytest.raises(RnsError) as err:
        rk.info(0)
    assert err.value.status == -8
    B = 20
    c = gen.uniform_below(n, B, seed=gen.config_seed(8, 17))
    cl = gen.to_limbs(c, 512)
    m = _host(rk.decrypt(_dev(cl), use_crt=True))
    assert np.array_equal(m, oracle.rsa_crt_batch(cl, p, q, dp, dq, qinv))
    mi = oracle.rows_to_ints(m)
    for i in (0, B - 1):
        assert pow(mi[i], e, n) == c[i]
    with pytest.raises(RnsError) as err:
        rk.encrypt(_dev(cl))
    assert err.value.status == -8


def _rsa16384_key(**opts):
    from paper_1305_3699_amd import RsaKey
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rsa16384_key.json")) as fh:
        fx = json.load(fh)
    p, q, e = int(fx["p"], 16), int(fx["q"], 16), int(fx["e"])
    d = pow(e, -1, (p - 1) * (q - 1))
    parts = dict(n=p * q, e=e, d=d, p=p, q=q, dp=d % (p - 1), dq=d % (q - 1), qinv=pow(q, -1, p))
    return RsaKey(**parts, **opts), parts


def test_rsa16384_full_modulus():
    """RSA-16384 with the full modulus on bases of 512 + 1 channels (k = 513,
    matrix engine only): 20 encryptions (a full tile and a ragged one) against
    the oracle; non-CRT decryption with the full-length d of 3 of them gives
    the messages back and agrees with the CRT path (257-channel halves),
    whose results pass the re-encryption check."""
    from paper_1305_3699_amd import ENGINE_MATRIX
    rk, parts = _rsa16384_key()
    n, e = parts["n"], parts["e"]
    assert rk.info(0)["k"] == 513 and rk.info(0)["engine"] == ENGINE_MATRIX
    assert rk.info(1)["k"] == 257
    msgs = gen.uniform_below(n, 18, seed=gen.config_seed(8, 22)) + [0, n - 1]
    ml = gen.to_limbs(msgs, 512)
    c = _host(rk.encrypt(_dev(ml)))
    assert np.array_equal(c, oracle.modexp_batch(ml, gen.to_limbs(e, 1)[0], gen.to_limbs(n, 512)[0]))
    sel = c[[0, 1, 19]]
    full = _host(rk.decrypt(_dev(sel), use_crt=False))
    assert np.array_equal(full, ml[[0, 1, 19]])
    dsel = _dev(sel)
    crt = rk.decrypt(dsel, use_crt=True)
    assert np.array_equal(full, _host(crt))
    assert rk.verify_crt(dsel, crt) == 0          # re-encryption on the 513-channel base


def test_batched_with_rsa16384_crt_only_key():
    """A batch mixing RSA-16384 CRT decryptions (halves on 257-channel bases,
    a CRT-only key) with RSA-2048 encryptions and decryptions: every output
    equals the oracle's; an encryption with the CRT-only key is refused at
    creation."""
    from paper_1305_3699_amd import ENGINE_CHANNEL, OP_DECRYPT, OP_ENCRYPT, RnsError, RsaBatch, RsaKey
    big, bp = _rsa16384_key(engine=ENGINE_CHANNEL)
    k2 = gen.rsa_key(2048, seed=gen.config_seed(3, 12))
    small = RsaKey(k2.n, k2.e, k2.d, k2.p, k2.q, k2.dp, k2.dq, k2.qinv)
    c_big = gen.to_limbs(gen.uniform_below(bp["n"], 18, seed=gen.config_seed(8, 18)), 512)
    x2 = gen.to_limbs(gen.uniform_below(k2.n, 40, seed=gen.config_seed(8, 19)), 64)
    ins = [_dev(c_big), _dev(x2), _dev(x2)]
    outs = [torch.zeros_like(t) for t in ins]
    ops = [(big, OP_DECRYPT, ins[0], outs[0]), (small, OP_ENCRYPT, ins[1], outs[1]),
           (small, OP_DECRYPT, ins[2], outs[2])]
    b = RsaBatch(ops)
    b.run()
    torch.cuda.synchronize()
    assert np.array_equal(_host(outs[0]), oracle.rsa_crt_batch(c_big, bp["p"], bp["q"], bp["dp"], bp["dq"], bp["qinv"]))
    assert np.array_equal(_host(outs[1]), oracle.modexp_batch(x2, gen.to_limbs(k2.e, 1)[0], gen.to_limbs(k2.n, 64)[0]))
    assert np.array_equal(_host(outs[2]), oracle.rsa_crt_batch(x2, k2.p, k2.q, k2.dp, k2.dq, k2.qinv))
    b.close()
    with pytest.raises(RnsError) as err:
        RsaBatch([(big, OP_ENCRYPT, ins[0], outs[0])])
    assert err.value.status == -8


def test_rsa1024_config_bit_exact():
    """One seeded RSA-1024 key, 64 messages, 64 encryptions and 64 plain
    decryptions with bases of 2 x 33 random 32-bit primes."""
    from paper_1305_3699_amd import PRIMES_FULL, RsaKey
    key = gen.rsa_key(1024, seed=gen.config_seed(1, 1))
    rk = RsaKey(key.n, key.e, key.d, prime_range=PRIMES_FULL, prime_seed=gen.config_seed(1, 4))
    assert rk.info(0)["k"] == 33
    ms = gen.uniform_below(key.n, 64, seed=gen.config_seed(1, 2))
    c = _host(rk.encrypt(_dev(gen.to_limbs(ms, 32))))
    want_c = oracle.modexp_batch(gen.to_limbs(ms, 32), gen.to_limbs(key.e, 1)[0], gen.to_limbs(key.n, 32)[0])
    assert np.array_equal(c, want_c)
    m = _host(rk.decrypt(_dev(c), use_crt=False))
    want_m = oracle.modexp_batch(c, gen.to_limbs(key.d, 32)[0], gen.to_limbs(key.n, 32)[0])
    assert np.array_equal(m, want_m)
    assert oracle.rows_to_ints(m) == ms


def _rsa2048(**opts):
    from paper_1305_3699_amd import RsaKey
    key = gen.rsa_key(2048, seed=gen.config_seed(2, 1))
    return key, RsaKey(key.n, key.e, key.d, key.p, key.q, key.dp, key.dq, key.qinv, **opts)


def test_rsa2048_crt_decrypt_small():
    key, rk = _rsa2048()
    c = gen.uniform_below(key.n, 120, seed=11) + [0, 1, key.n - 1, key.p, 2 * key.q, key.q, key.p * 3, key.n - key.p]
    cl = gen.to_limbs(c, 64)
    got = _host(rk.decrypt(_dev(cl), use_crt=True))
    want = oracle.rsa_crt_batch(cl, key.p, key.q, key.dp, key.dq, key.qinv)
    assert np.array_equal(got, want)
    # the definition: c^d mod n
    assert oracle.rows_to_ints(got[:8]) == _oracle_pow(c[:8], key.d, key.n)


@pytest.mark.parametrize("window", [1, 2, 3, 4, 5, 6])
def test_rsa2048_crt_full_batch_sampled(window):
    """The benchmark's launch at each window width of the per-width sweep:
    16384 ciphertexts in one CRT decryption.  The oracle checks 48 sampled
    rows; every row is checked by re-encryption."""
    key, rk = _rsa2048(window=window)
    B = 16384
    c = gen.uniform_below(key.n, B, seed=gen.config_seed(2, 2))
    cl = gen.to_limbs(c, 64)
    dc = _dev(cl)
    m = rk.decrypt(dc, use_crt=True)
    back = _host(rk.encrypt(m))
    assert np.array_equal(back, cl)
    mh = _host(m)
    idx = sorted(random.Random(1).sample(range(B), 46)) + [0, B - 1]
    want = oracle.rsa_crt_batch(cl[idx], key.p, key.q, key.dp, key.dq, key.qinv)
    assert np.array_equal(mh[idx], want)


def test_determinism_and_aliasing():
    rng = random.Random(12)
    N = rng.getrandbits(2048) | (1 << 2047) | 1
    ctx = _ctx(N, 64)
    bases = gen.to_limbs([rng.getrandbits(2048) for _ in range(64)], 64)
    el = gen.to_limbs(rng.getrandbits(300), 10)[0]
    b = _dev(bases)
    e = _dev(el)
    r1 = _host(ctx.modexp(b, e))
    r2 = _host(ctx.modexp(b, e))
    assert np.array_equal(r1, r2)
    ctx.modexp(b, e, out=b)                   # out aliases base
    assert np.array_equal(_host(b), r1)


def test_zero_batch_is_a_no_op():
    ctx = _ctx(3233, 1)
    empty = torch.zeros((0, 1), dtype=torch.int32, device="cuda")
    out = ctx.modexp(empty, torch.tensor([5], dtype=torch.int32, device="cuda"))
    assert out.shape == (0, 1)


@pytest.mark.parametrize("ebits", [4096, 8192, 16128])
def test_long_exponents_2048_bit_modulus(ebits):
    """2048-bit modulus (a seeded RSA-2048 n), 1024 bases uniform in [0, n),
    one seeded exponent of 4096 / 8192 / 16128 bits with the top bit set; the
    oracle checks every row on all host threads."""
    key = gen.rsa_key(2048, seed=gen.config_seed(3, 1))
    ctx = _ctx(key.n, 64, window=6)
    B = 1024
    bases = gen.uniform_below(key.n, B, seed=gen.config_seed(3, 2))
    e = gen.random_exponent(ebits, seed=gen.config_seed(3, 3) + ebits)
    el = gen.to_limbs(e, ebits // 32 + (ebits % 32 != 0))[0]
    bl = gen.to_limbs(bases, 64)
    got = _run_modexp(ctx, bl, el)
    want = oracle.modexp_batch(bl, el, gen.to_limbs(key.n, 64)[0], nthreads=_threads())
    assert np.array_equal(got, want)


@pytest.mark.parametrize("bits,group", [(3072, 16), (3072, 32), (4096, 16), (4096, 32)])
def test_rsa_crt_3072_4096_batch_4096(bits, group):
    """RSA-3072 and RSA-4096 CRT decryption, 4096 ciphertexts each, with both
    workgroup tiles: sampled rows against the oracle's CRT path, every row by
    re-encryption."""
    from paper_1305_3699_amd import RsaKey
    key = gen.rsa_key(bits, seed=gen.config_seed(3, 10 + bits // 1024))
    rk = RsaKey(key.n, key.e, key.d, key.p, key.q, key.dp, key.dq, key.qinv, group=group)
    assert rk.info(1)["group"] == group
    L = bits // 32
    B = 4096
    c = gen.uniform_below(key.n, B, seed=gen.config_seed(3, 20 + bits // 1024))
    cl = gen.to_limbs(c, L)
    m = rk.decrypt(_dev(cl), use_crt=True)
    assert np.array_equal(_host(rk.encrypt(m)), cl)
    mh = _host(m)
    idx = sorted(random.Random(bits).sample(range(1, B - 1), 14)) + [0, B - 1]
    want = oracle.rsa_crt_batch(cl[idx], key.p, key.q, key.dp, key.dq, key.qinv)
    assert np.array_equal(mh[idx], want)


def _mixed_setup(n_keys, median, cap):
    from paper_1305_3699_amd import OP_DECRYPT, OP_ENCRYPT, RsaKey
    specs, ops = gen.mixed_batch_spec(n_keys=n_keys, median=median, cap=cap)
    keys = gen.rsa_keys(specs, processes=1)
    rks = [RsaKey(k.n, k.e, k.d, k.p, k.q, k.dp, k.dq, k.qinv) for k in keys]
    items = []
    for o in ops:
        k = keys[o.key_index]
        L = o.bits // 32
        vals = gen.uniform_below(k.n, o.count, seed=o.msg_seed)
        inp = _dev(gen.to_limbs(vals, L))
        out = torch.zeros_like(inp)
        items.append((o, k, rks[o.key_index], OP_ENCRYPT if o.kind == "encrypt" else OP_DECRYPT, inp, out))
    return items


@pytest.mark.parametrize("use_graph,autotune", [(True, False), (False, True)])
def test_batched_mixed_sizes(use_graph, autotune):
    """Mixed-size batch (keys of 1024-4096 bits, lognormal per-key counts,
    encryptions and CRT decryptions) in one batched run: every output equals
    the oracle's, and equals the same operation run alone."""
    from paper_1305_3699_amd import RsaBatch
    items = _mixed_setup(8, 24, 96)
    b = RsaBatch([(rk, kind, inp, out) for (o, k, rk, kind, inp, out) in items], autotune=autotune,
                 use_graph=use_graph)
    info = b.info
    assert info["jobs"] == sum(2 if o.kind == "decrypt" else 1 for o, *_ in items)
    classes = b.classes
    assert sum(c["jobs"] for c in classes) == info["jobs"]
    for c in classes:
        assert c["tuned"] == autotune and c["group"] in (16, 32) and 1 <= c["window"] <= 6
        assert c["window_offset"] in ((-1, 0, 1) if autotune else (0,))
        assert c["exp_bits"] in (32, 512, 1024, 1536, 2048)
    for rep in range(2):                      # a graph is replayed; results must not change
        for *_, out in items:
            out.zero_()
        b.run()
        torch.cuda.synchronize()
        for o, k, rk, kind, inp, out in items:
            x = _host(inp)
            got = _host(out)
            if o.kind == "encrypt":
                want = oracle.modexp_batch(x, gen.to_limbs(k.e, 1)[0], gen.to_limbs(k.n, o.bits // 32)[0])
                alone = _host(rk.encrypt(inp))
            else:
                want = oracle.rsa_crt_batch(x, k.p, k.q, k.dp, k.dq, k.qinv)
                alone = _host(rk.decrypt(inp, use_crt=True))
            assert np.array_equal(got, want), (rep, o)
            assert np.array_equal(alone, got)
    b.close()


def test_served_continuous_batching():
    """Request server: a Poisson trace over resident keys of 1024-4096 bits
    (70% CRT decryptions) with continuous batching; every result equals the
    oracle's and, for a sample, the same request run alone."""
    from paper_1305_3699_amd import RnsError, RsaKey, RsaServer
    per = 2
    specs = gen.served_keys(per_size=per)
    keys = gen.rsa_keys(specs, processes=1)
    rks = [RsaKey(k.n, k.e, k.d, k.p, k.q, k.dp, k.dq, k.qinv) for k in keys]
    arrival, kidx, kind, seeds = gen.served_trace(20000.0, 0.08, per_size=per)
    n = arrival.size
    W = 128
    msgs = np.zeros((n, W), np.uint32)
    for i in range(n):
        k = keys[kidx[i]]
        msgs[i, :k.n.bit_length() // 32] = gen.to_limbs(gen.uniform_below_fast(k.n, int(seeds[i])), k.n.bit_length() // 32)[0]
    srv = RsaServer(rks, max_inflight=4)
    outs, lat, stats = srv.replay(kidx, kind, arrival, msgs)
    assert stats["completed"] == n and stats["dispatches"] >= 1
    assert np.all(lat > 0) and stats["p99_latency"] >= stats["p50_latency"] > 0
    for j, k in enumerate(keys):
        L = k.n.bit_length() // 32
        for kd in (0, 1):
            sel = np.nonzero((kidx == j) & (kind == kd))[0]
            if sel.size == 0:
                continue
            x = np.ascontiguousarray(msgs[sel, :L])
            want = (oracle.modexp_batch(x, gen.to_limbs(k.e, 1)[0], gen.to_limbs(k.n, L)[0]) if kd == 0
                    else oracle.rsa_crt_batch(x, k.p, k.q, k.dp, k.dq, k.qinv))
            assert np.array_equal(outs[sel, :L], want), (j, kd)
            assert not outs[sel, L:].any()
    for i in random.Random(3).sample(range(n), 24):
        k, rk = keys[kidx[i]], rks[kidx[i]]
        L = k.n.bit_length() // 32
        one = _dev(msgs[i:i + 1, :L])
        alone = _host(rk.encrypt(one) if kind[i] == 0 else rk.decrypt(one, use_crt=True))
        assert np.array_equal(alone[0], outs[i, :L])
    # admission: a budget below one request is refused (RNS_EBUSY); a small one still completes
    with pytest.raises(RnsError) as err:
        RsaServer(rks, hbm_budget=1024).replay(kidx[:4], kind[:4], arrival[:4], msgs[:4])
    assert err.value.status == -7
    small = RsaServer(rks, hbm_budget=64 << 20, max_inflight=2)
    outs2, _, st2 = small.replay(kidx[:300], kind[:300], arrival[:300], msgs[:300])
    assert np.array_equal(outs2, outs[:300]) and st2["peak_inflight_bytes"] <= 64 << 20


@pytest.mark.parametrize("group", [16, 32])
def test_rsa1024_crt_both_tiles(group):
    """RSA-1024 CRT decryption (k = 17 halves) with both workgroup tiles."""
    from paper_1305_3699_amd import RsaKey
    key = gen.rsa_key(1024, seed=gen.config_seed(1, 1))
    rk = RsaKey(key.n, key.e, key.d, key.p, key.q, key.dp, key.dq, key.qinv, group=group)
    assert rk.info(1)["group"] == group and rk.info(1)["k"] == 17
    c = gen.uniform_below(key.n, 300, seed=21) + [0, 1, key.n - 1]
    cl = gen.to_limbs(c, 32)
    got = _host(rk.decrypt(_dev(cl), use_crt=True))
    assert np.array_equal(got, oracle.rsa_crt_batch(cl, key.p, key.q, key.dp, key.dq, key.qinv))


# ---------------------------------------------------------------------------
# Primality steps of key generation

def _flags(t) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_trial_division_flags():
    """Flags of the small-primes step against the oracle: every integer in
    [2, 3000) (one-limb rows, including the listed primes themselves),
    seeded 1024-bit candidates with crafted multiples of listed primes and
    of primes just past the list, with the first 10,000 and the first 100
    primes, and ragged 4096-bit rows."""
    from paper_1305_3699_amd import trial_division
    pr = primality.small_primes(10000)
    small = list(range(2, 3000))
    got = _flags(trial_division(_dev(gen.to_limbs(small, 1))))
    assert [int(v) for v in got] == [int(primality.trial_division(n, primes=pr)) for n in small]
    rng = random.Random(1024)
    vals = [rng.getrandbits(1024) | (1 << 1023) | 1 for _ in range(500)]
    vals += [104729 * (rng.getrandbits(1000) | 1), 3 * (rng.getrandbits(1020) | 1),
             104743 * 104759 * (rng.getrandbits(900) | 1), 541 * 547 * (rng.getrandbits(1000) | 1)]
    cl = _dev(gen.to_limbs(vals, 32))
    for n_primes in (10000, 100):
        got = _flags(trial_division(cl, n_primes=n_primes))
        assert [int(v) for v in got] == [int(primality.trial_division(n, primes=pr[:n_primes])) for n in vals]
    big = [rng.getrandbits(4096) | 1 for _ in range(21)]
    got = _flags(trial_division(_dev(gen.to_limbs(big, 128))))
    assert [int(v) for v in got] == [int(primality.trial_division(n, primes=pr)) for n in big]


def _mr_case(cands, rounds, limbs, seed):
    from paper_1305_3699_amd import miller_rabin
    rng = random.Random(seed)
    bases = [[rng.randrange(2, n - 1) for _ in range(rounds)] for n in cands]
    got = miller_rabin(gen.to_limbs(cands, limbs), np.stack([gen.to_limbs(b, limbs) for b in bases]))
    want = [int(primality.miller_rabin(n, b)) for n, b in zip(cands, bases)]
    assert [int(v) for v in got] == want
    return want


@pytest.mark.parametrize("bits", [512, 1024])
def test_miller_rabin_verdicts(bits):
    """Verdicts of the Miller-Rabin step (exponentiations in RNS, one
    context per candidate) against the oracle: seeded primes, products of
    two seeded primes and seeded random odd numbers, 5 random bases each."""
    rng = random.Random(bits)
    primes = [gen.random_prime(bits, rng) for _ in range(6)]
    semis = [gen.random_prime(bits // 2, rng) * gen.random_prime(bits // 2, rng) for _ in range(4)]
    semis = [n for n in semis if n.bit_length() == bits]
    odd = [rng.getrandbits(bits) | (1 << (bits - 1)) | 1 for _ in range(6)]
    want = _mr_case(primes + semis + odd, 5, bits // 32, bits + 1)
    assert want[:6] == [1] * 6 and want[6:6 + len(semis)] == [0] * len(semis)


def test_miller_rabin_small_cases():
    """Strong pseudoprimes, a Carmichael number, and primes and composites
    whose N - 1 has many factors of two (the squaring loop)."""
    from paper_1305_3699_amd import miller_rabin

    def mr(n, bases, limbs):
        return int(miller_rabin(gen.to_limbs([n], limbs), np.stack([gen.to_limbs(bases, limbs)]))[0])

    assert mr(2047, [2], 1) == 1 and mr(2047, [3], 1) == 0
    assert mr(3215031751, [2, 3, 5, 7], 1) == 1 and mr(3215031751, [2, 3, 5, 7, 11], 1) == 0
    assert mr(41041, [2], 1) == 0
    assert mr(65537, [3, 5, 65535], 1) == 1                  # s = 16
    gold = (1 << 64) - (1 << 32) + 1                          # prime, s = 32
    assert mr(gold, [2, 3, 12345678901, gold - 2], 2) == 1
    f6 = (1 << 64) + 1                                        # 274177 * 67280421310721, s = 64
    assert mr(f6, [3, 5], 3) == 0
    for n, bases, limbs in ((gold, [7, 11], 2), (f6, [2], 3), (2047, [2, 3], 1)):
        assert mr(n, bases, limbs) == int(primality.miller_rabin(n, bases))


def test_miller_rabin_channel_primes():
    """Candidates that share a factor with the RNS base the Miller-Rabin
    step runs on (the default base for candidates of their length, taken
    here from a context on the largest such value): a channel prime itself
    (prime), and products with channel primes (composite); mixed into one
    call with ordinary candidates."""
    from paper_1305_3699_amd import RnsContext, miller_rabin
    for limbs in (1, 2):
        ctx = RnsContext((1 << (32 * limbs)) - 1, limbs)
        pr = ctx.primes
        k = len(pr) // 2
        ctx.close()
        if limbs == 1:
            cands = [pr[0], pr[k - 1], pr[k], pr[-1], 4294967291, 4294967279]
        else:
            cands = [pr[0] * pr[1], pr[k] * pr[-1], 3 * pr[0], pr[1] * 4294967291,
                     (1 << 61) - 1, (1 << 64) - 59]
        rng = random.Random(limbs)
        bases = [[rng.randrange(2, n - 1) for _ in range(3)] for n in cands]
        got = miller_rabin(gen.to_limbs(cands, limbs), np.stack([gen.to_limbs(b, limbs) for b in bases]))
        want = [int(primality.miller_rabin(n, b)) for n, b in zip(cands, bases)]
        assert [int(v) for v in got] == want
        assert want[:4] == ([1] * 4 if limbs == 1 else [0] * 4)


@pytest.mark.parametrize("bits,count", [(1024, 1500), (2048, 2500)])
def test_keygen_agrees_with_oracle(bits, count):
    """RSA key generation from two seeded candidate streams: the primes the
    library picks (trial division and Miller-Rabin on the GPU) are the
    oracle's first primes of each stream; n matches, and the key works:
    encryption against the oracle, decryption with and without CRT back to
    the messages."""
    from paper_1305_3699_amd import keygen
    half = bits // 64
    rng = random.Random(bits * 7 + count)
    cp = [rng.getrandbits(32 * half) | (3 << (32 * half - 2)) | 1 for _ in range(count)]
    cq = [rng.getrandbits(32 * half) | (3 << (32 * half - 2)) | 1 for _ in range(count)]
    bp = [[rng.randrange(2, c - 1) for _ in range(5)] for c in cp]
    bq = [[rng.randrange(2, c - 1) for _ in range(5)] for c in cq]
    stack = lambda bs: np.stack([gen.to_limbs(b, half) for b in bs])
    key = keygen(gen.to_limbs(cp, half), stack(bp), gen.to_limbs(cq, half), stack(bq), e=65537)
    p = primality.first_prime(cp, bp, 65537)
    q = primality.first_prime(cq, bq, 65537, exclude=p)
    assert p and q and key.n == p * q
    ref = primality.rsa_key_from_primes(p, q, 65537)
    L = bits // 32
    msgs = gen.uniform_below(key.n, 40, seed=bits + 3)
    ml = gen.to_limbs(msgs, L)
    c = key.encrypt(_dev(ml))
    ch = _host(c)
    assert np.array_equal(ch, oracle.modexp_batch(ml, gen.to_limbs(65537, 1)[0], gen.to_limbs(key.n, L)[0]))
    assert np.array_equal(_host(key.decrypt(c, use_crt=True)), ml)
    assert np.array_equal(_host(key.decrypt(c, use_crt=False)), ml)
    assert oracle.rows_to_ints(ch[:2]) == _oracle_pow(msgs[:2], 65537, key.n)
    assert pow(pow(msgs[0], 65537, key.n), ref["d"], key.n) == msgs[0]


def test_keygen_and_primality_edges():
    """Edges of the key generation entry points: a stream without a prime
    (RNS_ERANGE), trial division at the 4096-limb maximum, Miller-Rabin with
    the maximum of 64 rounds."""
    from paper_1305_3699_amd import RnsError, keygen, miller_rabin, trial_division
    half = 16
    base = (3 << 510) + 1
    base += (3 - base % 3) % 3
    base += 3 if base % 2 == 0 else 0
    comp = [base + 6 * i for i in range(32)]                          # odd multiples of 3: no prime
    assert all(c % 3 == 0 and c % 2 == 1 and c.bit_length() == 512 for c in comp)
    b = np.stack([gen.to_limbs([2, 3, 5, 7, 11], half) for _ in comp])
    cl = gen.to_limbs(comp, half)
    with pytest.raises(RnsError) as err:
        keygen(cl, b, cl, b)
    assert err.value.status == -2
    rng = random.Random(4096)
    big = [rng.getrandbits(4096 * 32) | 1 for _ in range(3)] + [3 * ((1 << (4096 * 32 - 3)) + 1)]
    got = _flags(trial_division(_dev(gen.to_limbs(big, 4096))))
    pr = primality.small_primes(10000)
    assert [int(v) for v in got] == [int(primality.trial_division(n, primes=pr)) for n in big]
    p = (1 << 127) - 1
    bases = [rng.randrange(2, p - 1) for _ in range(64)]
    assert int(miller_rabin(gen.to_limbs([p], 4), np.stack([gen.to_limbs(bases, 4)]))[0]) == 1


def test_batched_and_served_with_rsa16384_full_modulus():
    """A batch and a served trace mixing RSA-16384 encryptions (full modulus,
    513-channel group) and CRT decryptions (257-channel halves) with RSA-2048
    work: every output equals the oracle's."""
    from paper_1305_3699_amd import OP_DECRYPT, OP_ENCRYPT, RsaBatch, RsaKey, RsaServer
    big, bp = _rsa16384_key()
    k2 = gen.rsa_key(2048, seed=gen.config_seed(3, 12))
    small = RsaKey(k2.n, k2.e, k2.d, k2.p, k2.q, k2.dp, k2.dq, k2.qinv)
    n, e = bp["n"], bp["e"]
    m_big = gen.to_limbs(gen.uniform_below(n, 21, seed=gen.config_seed(8, 23)), 512)
    c_big = gen.to_limbs(gen.uniform_below(n, 5, seed=gen.config_seed(8, 24)), 512)
    x2 = gen.to_limbs(gen.uniform_below(k2.n, 33, seed=gen.config_seed(8, 25)), 64)
    ins = [_dev(m_big), _dev(c_big), _dev(x2)]
    outs = [torch.zeros_like(t) for t in ins]
    b = RsaBatch([(big, OP_ENCRYPT, ins[0], outs[0]), (big, OP_DECRYPT, ins[1], outs[1]),
                  (small, OP_DECRYPT, ins[2], outs[2])])
    b.run()
    torch.cuda.synchronize()
    nl = gen.to_limbs(n, 512)[0]
    assert np.array_equal(_host(outs[0]), oracle.modexp_batch(m_big, gen.to_limbs(e, 1)[0], nl))
    assert np.array_equal(_host(outs[1]), oracle.rsa_crt_batch(c_big, bp["p"], bp["q"], bp["dp"], bp["dq"], bp["qinv"]))
    assert np.array_equal(_host(outs[2]), oracle.rsa_crt_batch(x2, k2.p, k2.q, k2.dp, k2.dq, k2.qinv))
    b.close()
    srv = RsaServer([big], max_inflight=2)
    msgs = np.concatenate([m_big[:3], c_big[:3]])
    ops = np.array([OP_ENCRYPT] * 3 + [OP_DECRYPT] * 3, np.int32)
    got, lat, stats = srv.replay(np.zeros(6, np.int32), ops, np.linspace(0.0, 0.001, 6), msgs)
    assert np.array_equal(got[:3], oracle.modexp_batch(m_big[:3], gen.to_limbs(e, 1)[0], nl))
    assert np.array_equal(got[3:], oracle.rsa_crt_batch(c_big[:3], bp["p"], bp["q"], bp["dp"], bp["dq"], bp["qinv"]))
    srv.close()


def test_served_refuses_encryption_with_crt_only_key():
    """A served trace that asks a CRT-only key (RSA-16384 loaded for the
    channel engine) to encrypt is refused before any work
    (RNS_EUNSUPPORTED); its CRT decryptions are served and match the
    oracle."""
    from paper_1305_3699_amd import ENGINE_CHANNEL, OP_DECRYPT, OP_ENCRYPT, RnsError, RsaServer
    big, bp = _rsa16384_key(engine=ENGINE_CHANNEL)
    srv = RsaServer([big], max_inflight=2)
    msgs = gen.to_limbs(gen.uniform_below(bp["n"], 4, seed=gen.config_seed(8, 21)), 512)
    kidx = np.zeros(4, np.int32)
    arrival = np.linspace(0.0, 0.001, 4)
    with pytest.raises(RnsError) as err:
        srv.replay(kidx, np.array([OP_DECRYPT, OP_ENCRYPT, OP_DECRYPT, OP_DECRYPT], np.int32), arrival, msgs)
    assert err.value.status == -8
    outs, lat, stats = srv.replay(kidx, np.full(4, OP_DECRYPT, np.int32), arrival, msgs)
    assert np.array_equal(outs, oracle.rsa_crt_batch(msgs, bp["p"], bp["q"], bp["dp"], bp["dq"], bp["qinv"]))
    srv.close()


def test_rsa_input_range_status():
    """Raw RSA works on integers below n (Sec. 3.3).  Inputs >= n are still
    reduced and exponentiated; each is counted in the key's device status
    word, which rsa_key_status reads (RNS_ERANGE) and clears: for
    encryption, both decryptions, the CRT halves launch and the batched form.
    The server checks its host inputs before it starts (RNS_ERANGE)."""
    from paper_1305_3699_amd import OP_DECRYPT, OP_ENCRYPT, RnsError, RsaBatch, RsaKey, RsaServer
    key = gen.rsa_key(1024, seed=gen.config_seed(1, 1))
    rk = RsaKey(key.n, key.e, key.d, key.p, key.q, key.dp, key.dq, key.qinv)
    L = 32
    vals = [0, 1, key.n - 1, key.n, key.n + 1, (1 << 1024) - 1] + gen.uniform_below(key.n, 14, seed=77)
    xl = gen.to_limbs(vals, L)
    x = _dev(xl)
    assert rk.status() == 0
    c = rk.encrypt(x)
    assert rk.status() == 3 and rk.status() == 0
    assert oracle.rows_to_ints(_host(c)) == _oracle_pow(vals, key.e, key.n)
    want_d = _oracle_pow(vals, key.d, key.n)
    for use_crt in (True, False):
        m = rk.decrypt(x, use_crt=use_crt)
        assert rk.status() == 3
        assert oracle.rows_to_ints(_host(m)) == want_d
    rk.crt_halves(x)
    assert rk.status() == 3
    outs = [torch.zeros_like(x), torch.zeros_like(x)]
    b = RsaBatch([(rk, OP_ENCRYPT, x, outs[0]), (rk, OP_DECRYPT, x, outs[1])])
    b.run()
    assert rk.status() == 6
    b.run()
    b.run()
    assert rk.status() == 12 and rk.status() == 0
    assert oracle.rows_to_ints(_host(outs[0])) == _oracle_pow(vals, key.e, key.n)
    assert oracle.rows_to_ints(_host(outs[1])) == want_d
    b.close()
    ok = _dev(gen.to_limbs(vals[6:], L))
    rk.encrypt(ok)
    rk.decrypt(ok)
    assert rk.status() == 0
    srv = RsaServer([rk])
    with pytest.raises(RnsError) as err:
        srv.replay([0, 0], [0, 1], [0.0, 0.0], gen.to_limbs([5, key.n], L))
    assert err.value.status == -2
    srv.close()


def test_served_queue_limit_refuses_requests():
    """Load shedding: with max_pending requests waiting, later arrivals are
    refused (latency -1, output untouched, RNS_EBUSY after the others
    complete); every admitted request still matches the oracle."""
    from paper_1305_3699_amd import RnsError, RsaKey, RsaServer
    key = gen.rsa_key(1024, seed=gen.config_seed(1, 1))
    rk = RsaKey(key.n, key.e, key.d, key.p, key.q, key.dp, key.dq, key.qinv)
    n = 40
    vals = gen.uniform_below(key.n, n, seed=78)
    msgs = gen.to_limbs(vals, 32)
    kind = [i % 2 for i in range(n)]
    arrival = np.zeros(n)
    srv = RsaServer([rk], max_inflight=1, max_pending=8)
    with pytest.raises(RnsError) as err:
        srv.replay([0] * n, kind, arrival, msgs)
    assert err.value.status == -7
    outs, lat, st = srv.replay([0] * n, kind, arrival, msgs, allow_refused=True)
    assert st["rejected"] == n - 8 and st["completed"] == 8
    took = np.nonzero(lat >= 0)[0]
    assert took.size == 8 and np.all(lat[lat < 0] == -1.0)
    want = _oracle_pow(vals, [key.e if kd == 0 else key.d for kd in kind], key.n)
    for i in range(n):
        got = int.from_bytes(outs[i].astype("<u4").tobytes(), "little")
        if lat[i] < 0:
            assert got == 0
        else:
            assert got == want[i]
    srv.close()


def test_batched_mix_full_shape():
    """The mixed-size workload at its real shape: 64 keys (16 each of 1024,
    2048, 3072 and 4096 bits), lognormal per-key counts (median 128, cap
    8192), encryptions and CRT decryptions, one batched run (hipGraph,
    autotuned tiles).  Every output of the first and the last four rows of
    each (key, op) and of a seeded sample of 8 more is compared with the
    oracle, and every output equals the same operations run one call each."""
    from paper_1305_3699_amd import OP_DECRYPT, OP_ENCRYPT, RsaBatch, RsaKey
    specs, ops = gen.mixed_batch_spec()
    keys = gen.rsa_keys(specs, processes=1)
    rks = [RsaKey(k.n, k.e, k.d, k.p, k.q, k.dp, k.dq, k.qinv) for k in keys]
    items = []
    for o in ops:
        k = keys[o.key_index]
        xl = gen.to_limbs(gen.uniform_below(k.n, o.count, seed=o.msg_seed), o.bits // 32)
        inp = _dev(xl)
        items.append((o, k, rks[o.key_index], xl, inp, torch.zeros_like(inp)))
    assert sum(o.count for o in ops) > 10000
    b = RsaBatch([(rk, OP_ENCRYPT if o.kind == "encrypt" else OP_DECRYPT, inp, out)
                  for o, k, rk, xl, inp, out in items], autotune=True, use_graph=True)
    b.run()
    torch.cuda.synchronize()
    rng = random.Random(4)
    for o, k, rk, xl, inp, out in items:
        got = _host(out)
        idx = sorted(set(list(range(min(4, o.count))) + list(range(max(0, o.count - 4), o.count))
                         + rng.sample(range(o.count), min(8, o.count))))
        if o.kind == "encrypt":
            want = oracle.modexp_batch(xl[idx], gen.to_limbs(k.e, 1)[0], gen.to_limbs(k.n, o.bits // 32)[0])
            alone = _host(rk.encrypt(inp))
        else:
            want = oracle.rsa_crt_batch(xl[idx], k.p, k.q, k.dp, k.dq, k.qinv, nthreads=_threads())
            alone = _host(rk.decrypt(inp, use_crt=True))
        assert np.array_equal(got[idx], want), o
        assert np.array_equal(alone, got), o
    b.close()
