"""Host-side tests of librnsrsa (no GPU): the library loads and exports every
declared symbol, base planning obeys its bounds, error paths return the
documented status codes, and the host model of the kernels agrees with the
oracle (which pins the constant tables and the algorithm before any GPU run).
"""
import math
import os
import random
import re

import ctypes

import numpy as np
import pytest

import gen
import oracle
from oracle import rns_ref
from paper_1305_3699_amd import rnsrsa
from paper_1305_3699_amd.rnsrsa import Plan, RnsError

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in ("rnsrsa.h", "rnsrsa_host.h"):
        txt = open(os.path.join(ROOT, "include", h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"\b(?:int|void|const char \*)\s*\*?\s*((?:rns|rsa)_\w+)\s*\(", txt):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    lib = rnsrsa.lib()
    declared = _declared_functions()
    assert len(declared) >= 18
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(rnsrsa.exported_symbols())
    assert lib.rns_abi_version() == rnsrsa.ABI_VERSION == 6


def _check_bounds(plan, N, L):
    info = plan.info
    k = info["k"]
    pr = plan.primes
    B, Bp = pr[:k], pr[k:]
    assert len(set(pr)) == 2 * k
    assert all((1 << 31) < p < (1 << 32) and pow(2, p - 1, p) == 1 for p in pr)
    M, Mp = math.prod(B), math.prod(Bp)
    assert M >= (k + 1) ** 2 * N and M >= 2 ** (32 * L + 1) and Mp >= (k + 1) * N
    assert math.gcd(M, N) == 1


@pytest.mark.parametrize("bits", [2, 12, 64, 512, 1024, 2048, 3072, 4096])
def test_plan_bounds(bits):
    N = (1 << bits) - 1 if bits > 2 else 3
    L = (bits + 31) // 32
    p = Plan(N, L)
    _check_bounds(p, N, L)
    assert p.info["k"] >= L + 1


def test_plan_full_range_primes_rsa1024():
    key = gen.rsa_key(1024, seed=gen.config_seed(1, 1))
    p = Plan(key.n, 32, prime_range=rnsrsa.PRIMES_FULL, prime_seed=gen.config_seed(1, 4))
    assert p.info["k"] == 33
    _check_bounds(p, key.n, 32)


def test_plan_errors():
    with pytest.raises(RnsError) as e:
        Plan(1)
    assert e.value.status == -2                      # RNS_ERANGE
    with pytest.raises(RnsError) as e:
        Plan(3233, window=9)
    assert e.value.status == -1                      # RNS_EINVAL
    with pytest.raises(RnsError) as e:
        Plan(3233, k=7)                              # no kernel for k = 7
    assert e.value.status == -8
    with pytest.raises(RnsError) as e:
        Plan(3233, primes=[5, 7, 11, 13])            # not 32-bit primes
    assert e.value.status == -1
    pr = gen.rns_primes(4, seed=1)
    with pytest.raises(RnsError) as e:
        Plan(pr[0] * 3, primes=pr)                   # a channel prime divides N
    assert e.value.status == -3
    with pytest.raises(RnsError) as e:
        Plan((1 << 200) + 1, 7, primes=pr)           # base too small
    assert e.value.status == -2


def _res(vals, B, Bp):
    return np.array([[v % m for v in vals] for m in B] + [[v % m for v in vals] for m in Bp]
                    + [[v % (1 << 32) for v in vals]], dtype=np.uint32)


@pytest.mark.parametrize("bits", [12, 300, 1024, 2048])
def test_emul_mont_mul_matches_definition(bits):
    rng = random.Random(bits)
    N = rng.getrandbits(bits) | (1 << (bits - 1)) | 1
    L = (bits + 31) // 32
    p = Plan(N, L)
    k = p.info["k"]
    B, Bp = p.primes[:k], p.primes[k:]
    X = [rng.randrange((k + 1) * N) for _ in range(20)] + [0, (k + 1) * N - 1]
    Y = [rng.randrange((k + 1) * N) for _ in range(20)] + [(k + 1) * N - 1, (k + 1) * N - 1]
    out = p.emul_mont_mul(_res(X, B, Bp), _res(Y, B, Bp))
    want = [rns_ref.mont_mul(x, y, N, B) for x, y in zip(X, Y)]
    assert np.array_equal(out, _res(want, B, Bp))


ENGINES = [rnsrsa.ENGINE_CHANNEL, rnsrsa.ENGINE_MATRIX]


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("bits,window", [(12, 5), (64, 1), (250, 3), (1024, 5), (1024, 6), (2048, 4)])
def test_emul_modexp_matches_oracle(bits, window, engine):
    rng = random.Random(bits * 7 + window)
    N = rng.getrandbits(bits) | (1 << (bits - 1)) | rng.getrandbits(1)
    L = (bits + 31) // 32
    p = Plan(N, L, window=window, engine=engine)
    assert p.info["engine"] == engine
    bases = [rng.getrandbits(32 * L) for _ in range(5)] + [0, 1, N - 1, N, (1 << (32 * L)) - 1]
    e = rng.getrandbits(min(bits, 200)) | 1
    out = p.emul_modexp(gen.to_limbs(bases, L), gen.to_limbs(e, (e.bit_length() + 31) // 32)[0])
    want = oracle.modexp_batch(gen.to_limbs(bases, L), gen.to_limbs(e, (e.bit_length() + 31) // 32)[0],
                               gen.to_limbs(N, L)[0])
    assert np.array_equal(out, want)


@pytest.mark.parametrize("engine", ENGINES)
def test_emul_edge_exponents_and_per_element(engine):
    N = 3233
    p = Plan(N, 1, window=2, engine=engine)
    bases = list(range(0, 40)) + [N - 1, N, 2 ** 32 - 1]
    for e in (0, 1, 2, 3, 17, 2753):
        out = p.emul_modexp(gen.to_limbs(bases, 1), np.array([e], np.uint32))
        assert out[:, 0].tolist() == [pow(b, e, N) for b in bases]
    rng = random.Random(3)
    exps = [rng.getrandbits(40) for _ in bases]
    out = p.emul_modexp(gen.to_limbs(bases, 1), gen.to_limbs(exps, 2))
    assert out[:, 0].tolist() == [pow(b, e, N) for b, e in zip(bases, exps)]


@pytest.mark.parametrize("engine", ENGINES)
def test_emul_rsa1024_config_round_trip(engine):
    key = gen.rsa_key(1024, seed=gen.config_seed(1, 1))
    p = Plan(key.n, 32, prime_range=rnsrsa.PRIMES_FULL, prime_seed=gen.config_seed(1, 4), engine=engine)
    ms = gen.uniform_below(key.n, 4, seed=gen.config_seed(1, 2))
    c = p.emul_modexp(gen.to_limbs(ms, 32), gen.to_limbs(key.e, 1)[0])
    assert oracle.rows_to_ints(c) == [pow(m, key.e, key.n) for m in ms]
    m = p.emul_modexp(c, gen.to_limbs(key.d, 32)[0])
    assert oracle.rows_to_ints(m) == ms


def test_scaled_b_residues_selection():
    """The matrix engine keeps a key's B residues scaled (x R s_i, s_i^2 =
    +-c_i R^-1 mod m_i) on bases of at most 5 k-steps (k <= 66) when every B
    prime has such a root: always for the drawn bases (primes = 3 mod 4);
    never on request (unscaled), on wider bases or on the channel engine."""
    for bits, want in ((12, 1), (512, 1), (1024, 1), (2048, 1), (3072, 0), (4096, 0)):
        N = (1 << bits) - 1 if bits > 12 else 3233
        L = (bits + 31) // 32
        p = Plan(N, L)
        assert p.info["scaled"] == want, bits
        assert all(m % 4 == 3 for m in p.primes)
        assert Plan(N, L, unscaled=True).info["scaled"] == 0
        assert Plan(N, L, engine=rnsrsa.ENGINE_CHANNEL).info["scaled"] == 0
    key = gen.rsa_key(1024, seed=gen.config_seed(1, 1))
    assert Plan(key.n, 32, prime_range=rnsrsa.PRIMES_FULL, prime_seed=gen.config_seed(1, 4)).info["scaled"] == 1


@pytest.mark.parametrize("bits,window,unscaled", [(64, 3, True), (1024, 5, True), (2048, 4, True),
                                                  (1024, 6, False), (2048, 5, False)])
def test_emul_modexp_scaled_and_unscaled(bits, window, unscaled):
    """The matrix engine's model in both forms of the B residues, on the
    drawn base and on explicit bases with primes = 1 mod 4 among B (which
    may lack the square roots, then the key keeps the unscaled form), equals
    the oracle's pow."""
    rng = random.Random(bits * 3 + window)
    N = rng.getrandbits(bits) | (1 << (bits - 1)) | 1
    L = (bits + 31) // 32
    bases = [rng.getrandbits(32 * L) for _ in range(6)] + [0, 1, N - 1]
    e = rng.getrandbits(min(bits, 160)) | 1
    el = gen.to_limbs(e, (e.bit_length() + 31) // 32)[0]
    want = oracle.modexp_batch(gen.to_limbs(bases, L), el, gen.to_limbs(N, L)[0])
    p = Plan(N, L, window=window, unscaled=unscaled)
    assert p.info["engine"] == rnsrsa.ENGINE_MATRIX and p.info["scaled"] == (0 if unscaled else 1)
    assert np.array_equal(p.emul_modexp(gen.to_limbs(bases, L), el), want)
    k = p.info["k"]
    pr = gen.rns_primes(2 * k, seed=bits + window, lo=(1 << 32) - (1 << 24), hi=(1 << 32) - (1 << 19))
    assert k < 9 or any(m % 4 == 1 for m in pr[:k])
    q = Plan(N, L, window=window, primes=pr, unscaled=unscaled)
    assert q.info["engine"] == rnsrsa.ENGINE_MATRIX
    assert np.array_equal(q.emul_modexp(gen.to_limbs(bases, L), el), want)


def _scaled_base_1mod4(N: int, L: int, k: int):
    """An explicit base whose B primes are all 1 mod 4 (square roots by
    Tonelli-Shanks) and on which the key still takes the scaled form: the
    first seeded draw where every c_i 2^-32 is a square (probability 2^-k)."""
    for seed in range(400):
        pr = gen.rns_primes(8 * k, seed=seed, lo=(1 << 32) - (1 << 24), hi=(1 << 32) - (1 << 19))
        B = [m for m in pr if m % 4 == 1][:k]
        Bp = [m for m in pr if m % 4 == 3][:k]
        if len(B) < k or len(Bp) < k:
            continue
        p = Plan(N, L, primes=B + Bp)
        if p.info["scaled"]:
            return p
    raise AssertionError("no scaled base found")


@pytest.mark.parametrize("bits,k", [(64, 3), (128, 5)])
def test_emul_modexp_scaled_primes_1_mod_4(bits, k):
    """Scaled B residues on primes = 1 mod 4, whose roots come from the
    general square-root path: the host model equals the oracle's pow."""
    rng = random.Random(bits + 3)
    N = rng.getrandbits(bits) | (1 << (bits - 1)) | 1
    L = bits // 32
    p = _scaled_base_1mod4(N, L, k)
    assert p.info["k"] == k and all(m % 4 == 1 for m in p.primes[:k])
    bases = [rng.getrandbits(bits) for _ in range(20)] + [0, 1, N - 1, N, (1 << bits) - 1]
    e = rng.getrandbits(bits) | 1
    el = gen.to_limbs(e, L)[0]
    want = oracle.modexp_batch(gen.to_limbs(bases, L), el, gen.to_limbs(N, L)[0])
    assert np.array_equal(p.emul_modexp(gen.to_limbs(bases, L), el), want)


def test_engine_selection():
    assert Plan(3233).info["engine"] == rnsrsa.ENGINE_MATRIX          # auto: matrix cores when built
    assert Plan(3233, engine=rnsrsa.ENGINE_CHANNEL).info["engine"] == rnsrsa.ENGINE_CHANNEL
    assert Plan(3233, engine=rnsrsa.ENGINE_CHANNEL).info["group"] == 64
    with pytest.raises(RnsError) as e:
        Plan(3233, engine=7)
    assert e.value.status == -1
    with pytest.raises(RnsError) as e:
        Plan(3233, group=24)
    assert e.value.status == -1


def test_group_selection():
    N = (1 << 1023) + 1155
    for g in (16, 32):
        p = Plan(N, 32, group=g)
        assert p.info["engine"] == rnsrsa.ENGINE_MATRIX and p.info["group"] == g
    assert Plan(N, 32).info["group"] == 32                           # default tile for k = 33
    assert Plan((1 << 4095) + 4095, 128).info["group"] == 32         # default tile for k = 129
    small = (1 << 255) + 4095
    assert Plan(small, 8, group=16).info["group"] == 32              # no 16-element kernel for k = 9


def test_matrix_engine_prime_limit():
    """The matrix engine reduces x' y' + S in one step, which needs every B'
    prime <= 2^32 - 2^18; a base with a larger B' prime takes the channel
    engine (auto) or is refused (matrix engine requested)."""
    B = [4293918689, 4293918683]
    ok = Plan(3233, 1, primes=B + [4293918589, 4293918583])
    assert ok.info["engine"] == rnsrsa.ENGINE_MATRIX
    big = B + [4293918589, 4294967291]                   # 2^32 - 5 in B'
    assert Plan(3233, 1, primes=big).info["engine"] == rnsrsa.ENGINE_CHANNEL
    with pytest.raises(RnsError) as e:
        Plan(3233, 1, primes=big, engine=rnsrsa.ENGINE_MATRIX)
    assert e.value.status == -8
    # the limit concerns B' only
    assert Plan(3233, 1, primes=[4294967291, 4294967279, 4293918589, 4293918583]).info["engine"] == rnsrsa.ENGINE_MATRIX
    edge = Plan(3233, 1, primes=B + [4293918589, 4294705139])    # largest prime <= the limit
    assert edge.info["engine"] == rnsrsa.ENGINE_MATRIX
    msgs = np.arange(3233, dtype=np.uint32)[:, None]
    assert [int(v) for v in edge.emul_modexp(msgs, np.array([17], np.uint32))[:, 0]] == [pow(m, 17, 3233) for m in range(3233)]


@pytest.mark.parametrize("group", [16, 32])
def test_emul_group_sizes_agree(group):
    rng = random.Random(group)
    N = rng.getrandbits(1024) | (1 << 1023) | 1
    bases = gen.to_limbs([rng.getrandbits(1024) for _ in range(37)] + [0, N - 1], 32)
    e = gen.to_limbs(rng.getrandbits(100), 4)[0]
    out = Plan(N, 32, window=3, group=group).emul_modexp(bases, e)
    assert np.array_equal(out, oracle.modexp_batch(bases, e, gen.to_limbs(N, 32)[0]))


@pytest.mark.parametrize("bits", [96, 1536, 3000])
def test_emul_engines_agree_per_element_exponents(bits):
    rng = random.Random(bits)
    N = rng.getrandbits(bits) | (1 << (bits - 1)) | 1
    L = (bits + 31) // 32
    bases = gen.to_limbs([rng.getrandbits(32 * L) for _ in range(33)], L)
    exps = gen.to_limbs([rng.getrandbits(rng.choice([1, 9, 40])) for _ in range(33)], 2)
    outs = [Plan(N, L, window=3, engine=e).emul_modexp(bases, exps) for e in ENGINES]
    assert np.array_equal(outs[0], outs[1])
    assert oracle.rows_to_ints(outs[1]) == [pow(b, e, N) for b, e in zip(oracle.rows_to_ints(bases),
                                                                         oracle.rows_to_ints(exps))]


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("bits", [64, 100, 128, 1000])
def test_emul_zero_residue_bases(bits, engine):
    """Bases that are multiples of N (all-zero quotient digits) on moduli
    including the 100-bit one whose exit once mis-decoded such a state."""
    rng = random.Random(bits)
    N = rng.getrandbits(bits) | (1 << (bits - 1)) | rng.getrandbits(1)
    L = (bits + 31) // 32
    p = Plan(N, L, window=2, engine=engine)
    bases = [b for b in (0, N, 2 * N, 3 * N, 1, N - 1) if b < 1 << (32 * L)]
    for e in (1, 2, 65537):
        out = p.emul_modexp(gen.to_limbs(bases, L), gen.to_limbs(e, 1)[0])
        assert oracle.rows_to_ints(out) == [pow(b, e, N) for b in bases]


@pytest.mark.parametrize("engine", ENGINES)
def test_emul_8192_bit_modulus(engine):
    """256 + 1 channels per base (k = 257): an 8192-bit modulus, the doubled
    base the paper names for 8192-bit modular multiplication."""
    rng = random.Random(8192)
    N = rng.getrandbits(8192) | (1 << 8191) | 1
    p = Plan(N, 256, window=3, engine=engine)
    assert p.info["k"] == 257 and p.info["engine"] == engine
    bases = [rng.getrandbits(8192) for _ in range(3)] + [0, 1, N - 1]
    e = rng.getrandbits(40) | (1 << 39)
    out = p.emul_modexp(gen.to_limbs(bases, 256), gen.to_limbs(e, 2)[0])
    assert oracle.rows_to_ints(out) == [pow(b, e, N) for b in bases]


def test_emul_16384_bit_modulus():
    """512 + 1 channels per base (k = 513): a 16384-bit modulus, the base
    doubled once more instead of 64-bit channels; the matrix engine alone
    serves it (its REDC offset grows to m 2^18).  The host model checks that
    every one-step reduction input stays in [0, m 2^32) (else RNS_EVERIFY)."""
    rng = random.Random(16384)
    N = rng.getrandbits(16384) | (1 << 16383) | 1
    p = Plan(N, 512, window=2)
    assert p.info["k"] == 513 and p.info["engine"] == rnsrsa.ENGINE_MATRIX
    bases = [rng.getrandbits(16384) for _ in range(3)] + [0, 1, N - 1]
    e = 65537
    out = p.emul_modexp(gen.to_limbs(bases, 512), gen.to_limbs(e, 1)[0])
    assert oracle.rows_to_ints(out) == [pow(b, e, N) for b in bases]
    with pytest.raises(RnsError) as err:
        Plan(N, 512, engine=rnsrsa.ENGINE_CHANNEL)      # no channel-engine kernel for k = 513
    assert err.value.status == -8


def test_matrix_engine_sum_bound():
    """The one-REDC steps (iii)/(iv) add m 2^s to the extension's signed sum
    S, |S| <= 4k 0x80808080 128 + 0x80808080, and need m 2^s > |S|: at
    k = 257 (s = 17) every prime must exceed about 2^31.011, so bases drawn
    from the full 32-bit range (with primes just above 2^31) take the channel
    engine; requesting the matrix engine for them is refused.  The default
    high-range bases of k = 257 and 513 satisfy the bound."""
    def smax(k):
        return 4 * k * 0x80808080 * 128 + 0x80808080

    rng = random.Random(6000)
    N = rng.getrandbits(6000) | (1 << 5999) | 1
    full = Plan(N, 188, prime_range=rnsrsa.PRIMES_FULL, prime_seed=0)
    assert full.info["k"] == 257 and full.info["engine"] == rnsrsa.ENGINE_CHANNEL
    assert min(full.primes) << 17 <= smax(257)
    with pytest.raises(RnsError) as err:
        Plan(N, 188, prime_range=rnsrsa.PRIMES_FULL, prime_seed=0, engine=rnsrsa.ENGINE_MATRIX)
    assert err.value.status == -8
    for bits, k, s in ((6000, 257, 17), (16384, 513, 18)):
        M = rng.getrandbits(bits) | (1 << (bits - 1)) | 1
        pl = Plan(M, (bits + 31) // 32)
        assert pl.info["k"] == k and pl.info["engine"] == rnsrsa.ENGINE_MATRIX
        pr = pl.primes
        assert all(m << s > smax(k) for m in pr)
        # B' (second half): x'y' + S + m 2^s < m 2^32 with x', y' <= m - 1
        assert all((m - 1) ** 2 + (m << s) + smax(k) < m << 32 for m in pr[k:])


def _aligned_digits(a_row: np.ndarray) -> np.ndarray:
    """Digit words whose signed digit bytes take the sign of a_row (one A
    row's bytes over the 4k digit positions): +127 where the constant byte is
    positive, -128 elsewhere, the largest |sum| any digits reach."""
    d = np.where(a_row > 0, 127, -128).astype(np.int64)
    by = ((d & 0xFF) ^ 0x80).astype(np.uint32).reshape(-1, 4)
    return by[:, 0] | (by[:, 1] << 8) | (by[:, 2] << 16) | (by[:, 3] << 24)


@pytest.mark.parametrize("bits", [2048, 4096, 8192, 16384])
def test_matrix_extension_extreme_digits(bits):
    """Byte partials of the matrix cores' extensions under digits aligned to
    the signs of a constant row (the largest sums any digits give).  Each
    partial P_b is an int32 sum; the kernel pairs P_0 + 2^8 P_1 in int32 only
    up to 127 channels, where the extreme still fits, and combines every
    partial in 64 bits for the wider bases (k = 129, 257, 513), where the
    pairing would wrap.  S as the model forms it must equal the exact
    sum_b 2^(8b) P_b computed here from the constant bytes."""
    rng = random.Random(bits + 7)
    N = rng.getrandbits(bits) | (1 << (bits - 1)) | 1
    pl = Plan(N, bits // 32)
    k = pl.info["k"]
    assert pl.info["engine"] == rnsrsa.ENGINE_MATRIX
    for which in (1, 2):
        A = pl.emul_mfma_matrix(which).astype(np.int64)        # [rows, 4, kdim]
        rows = A.shape[0]
        # the row with the largest possible pair P_0 + 2^8 P_1
        r = int(np.argmax(np.abs(A[:, 0, :4 * k]).sum(1) + 256 * np.abs(A[:, 1, :4 * k]).sum(1)))
        dig = _aligned_digits(A[r, 1, :4 * k])[None, :]          # aligned to byte 1, the pair's heavy term
        rc, parts, value = pl.emul_mfma_extension(which, dig)
        db = ((np.frombuffer(dig.astype("<u4").tobytes(), dtype=np.uint8).astype(np.int64) ^ 0x80) + 128) % 256 - 128
        dvec = np.concatenate([db, [1], np.zeros(A.shape[2] - 4 * k - 1, np.int64)])
        exact_p = A @ dvec                                       # [rows, 4]
        assert np.array_equal(parts[0], exact_p)
        assert np.all(np.abs(exact_p) < 2 ** 31)
        exact_s = exact_p @ np.array([1, 1 << 8, 1 << 16, 1 << 24], np.int64)
        assert rc == 0 and np.array_equal(value[0], exact_s)
        pair = exact_p[r, 0] + 256 * exact_p[r, 1]
        if k <= 127:
            assert abs(pair) < 2 ** 31
        elif k >= 257:
            assert abs(pair) >= 2 ** 31, "the crafted digits reach the int32 limit of the pairing"
        assert rows == pl.info["waves"] * 4 * ((rows // pl.info["waves"]) // 4)


def test_modexp_jobs_argument_errors():
    """rns_modexp_jobs validates every job before touching the device: no
    jobs is a no-op, a null job array or a job without a context is
    RNS_EINVAL and names the job."""
    lib = rnsrsa.lib()
    assert lib.rns_modexp_jobs(None, 0, None) == 0
    assert lib.rns_modexp_jobs(None, 1, None) == -1
    arr = (rnsrsa.RnsJob * 2)()
    arr[1] = rnsrsa.RnsJob(None, None, None, 1, 0, None, 4)
    assert lib.rns_modexp_jobs(arr, 2, None) == -1
    assert b"job 0" in lib.rns_last_error()


def test_crt_verify_argument_errors():
    """rsa_crt_verify refuses a null key or buffer before any device work and
    reports no failing element."""
    lib = rnsrsa.lib()
    nb = ctypes.c_size_t(7)
    assert lib.rsa_crt_verify(None, None, None, 1, ctypes.byref(nb), None) == -1
    assert nb.value == 0


def test_probe_alu_argument_errors():
    """rns_probe_alu refuses an unknown instruction form or a null output
    before any device work."""
    lib = rnsrsa.lib()
    v = ctypes.c_double(1.0)
    assert lib.rns_probe_alu(7, ctypes.byref(v), None) == -1
    assert v.value == 0.0
    assert lib.rns_probe_alu(0, None, None) == -1


def test_keygen_argument_errors():
    """Argument checks of the primality entry points that fail before any
    device work (a nonzero count with null buffers, an even candidate, a
    base outside [2, N - 2], rounds out of range)."""
    lib = rnsrsa.lib()
    assert lib.rsa_trial_division(None, 0, 1, 10000, None, None) == 0         # nothing to do
    assert lib.rsa_trial_division(None, 1, 1, 10000, None, None) == -1
    cand = np.array([[101]], np.uint32)
    flags = np.zeros(1, np.uint8)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    assert lib.rsa_trial_division(ptr(cand), 1, 1, 10001, ptr(flags), None) == -1
    assert lib.rsa_trial_division(ptr(cand), 1, 0, 10000, ptr(flags), None) == -1
    bases = np.array([[[2]]], np.uint32)
    assert lib.rsa_miller_rabin(ptr(np.array([[100]], np.uint32)), 1, 1, ptr(bases), 1, ptr(flags), None) == -1
    assert lib.rsa_miller_rabin(ptr(cand), 1, 1, ptr(np.array([[[100]]], np.uint32)), 1, ptr(flags), None) == -1
    assert lib.rsa_miller_rabin(ptr(cand), 1, 1, ptr(np.array([[[1]]], np.uint32)), 1, ptr(flags), None) == -1
    assert lib.rsa_miller_rabin(ptr(cand), 1, 1, ptr(bases), 0, ptr(flags), None) == -1
    assert lib.rsa_miller_rabin(ptr(cand), 1, 1, ptr(bases), 65, ptr(flags), None) == -1


def test_batch_and_server_argument_errors():
    import ctypes
    lib = rnsrsa.lib()
    h = ctypes.c_void_p()
    assert lib.rsa_server_create(None, 0, None, ctypes.byref(h)) == -1          # no keys
    assert lib.rsa_batch_create(None, 0, None, None, None) == -1                # null handle
    n = ctypes.c_size_t(7)
    assert lib.rsa_batch_classes(None, None, 0, ctypes.byref(n)) == -1           # null batch
    op = rnsrsa.RsaOp(None, 0, None, None, 1)
    assert lib.rsa_batch_create(ctypes.byref(op), 1, None, None, ctypes.byref(h)) == -1   # null key
    assert rnsrsa.REQUEST_DTYPE.itemsize == 32
    assert lib.rsa_key_status(None, None, None) == -1                            # null key
    # the server options and statistics keep the header's layout
    assert ctypes.sizeof(rnsrsa.ServerOpts) == 32 and ctypes.sizeof(rnsrsa.ServerStats) == 80


class _FakeKey:
    def __init__(self, L):
        self.L = L


def _fake_server(limbs):
    srv = rnsrsa.RsaServer.__new__(rnsrsa.RsaServer)
    srv._keys = [_FakeKey(L) for L in limbs]
    srv._h = None
    return srv


def test_server_replay_shape_checks():
    """RsaServer.replay checks its arrays before the library reads them: one
    message row per request, rows as wide as the widest key used, matching
    sequence lengths, key indices in range."""
    srv = _fake_server([32, 64])
    arr = np.zeros(3)
    with pytest.raises(ValueError):
        srv.replay([0, 1, 0], [0, 0], arr, np.zeros((3, 64), np.uint32))      # kind too short
    with pytest.raises(ValueError):
        srv.replay([0, 1, 0], [0, 0, 0], arr[:2], np.zeros((3, 64), np.uint32))   # arrival too short
    with pytest.raises(ValueError):
        srv.replay([0, 1, 0], [0, 0, 0], arr, np.zeros((2, 64), np.uint32))   # too few rows
    with pytest.raises(ValueError):
        srv.replay([0, 1, 0], [0, 0, 0], arr, np.zeros((3, 32), np.uint32))   # rows narrower than key 1
    with pytest.raises(ValueError):
        srv.replay([0, 2, 0], [0, 0, 0], arr, np.zeros((3, 64), np.uint32))   # no key 2
    with pytest.raises(ValueError):
        srv.replay([0, 1, 0], [0, 0, 0], arr, np.zeros(64, np.uint32))        # not 2-D
