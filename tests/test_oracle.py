"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test checks the oracle's b^e mod N (and its Algorithm D division) against
the textbook RSA example, exhaustive small cases computed by iterated uint64
multiplication, number-theoretic identities (Fermat, Euler, RSA round trip,
multiplicativity) and CPython's independent ``pow``.
"""
import math
import os
import random

import numpy as np
import pytest

import gen
import oracle
from oracle import rns_ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                vals[k] = int(v)
    return vals


def test_toy_key_textbook_values():
    g = _golden("toy_rsa.txt")
    assert g["n"] == g["p"] * g["q"]
    assert g["e"] * g["d"] % g["phi"] == 1
    assert oracle.modexp_int(g["m"], g["e"], g["n"]) == g["c"]
    assert oracle.modexp_int(g["c"], g["d"], g["n"]) == g["m"]


def test_toy_key_round_trip_all_messages():
    g = _golden("toy_rsa.txt")
    n = g["n"]
    msgs = np.arange(n, dtype=np.uint32)[:, None]
    c = oracle.modexp_batch(msgs, np.array([g["e"]], np.uint32), np.array([n], np.uint32))
    m = oracle.modexp_batch(c, np.array([g["d"]], np.uint32), np.array([n], np.uint32))
    assert np.array_equal(m[:, 0], msgs[:, 0])
    # encryption is a permutation of Z_n (n squarefree, gcd(e, phi) = 1)
    assert len(set(c[:, 0].tolist())) == n


def test_brute_force_small_moduli():
    """Every N in [2, 512], every b < N, every e in [0, 64], against powers
    built by iterated uint64 multiplication."""
    for N in range(2, 513):
        b = np.arange(N, dtype=np.uint64)
        bases = b.astype(np.uint32).repeat(65)[:, None]
        exps = np.tile(np.arange(65, dtype=np.uint32), N)[:, None]
        got = oracle.modexp_batch(bases, exps, np.array([N], np.uint32))[:, 0].reshape(N, 65)
        want = np.empty((N, 65), dtype=np.uint64)
        acc = np.ones(N, dtype=np.uint64) % N
        for e in range(65):
            want[:, e] = acc
            acc = acc * b % N
        assert np.array_equal(got.astype(np.uint64), want), N


def test_zero_exponent_and_unreduced_base():
    n = (1 << 127) - 1
    assert oracle.modexp_int(0, 0, n) == 1
    assert oracle.modexp_int(12345, 0, n) == 1
    assert oracle.modexp_int(0, 5, n) == 0
    big = (1 << 200) + 987654321          # base >= N is reduced first
    assert oracle.modexp_int(big, 3, n) == pow(big, 3, n)
    assert oracle.modexp_int(5, 7, 1) == 0


def test_division_identity_random():
    rng = random.Random(7)
    for _ in range(3000):
        lu = rng.randint(1, 40)
        lv = rng.randint(1, lu)
        u = rng.getrandbits(32 * lu)
        v = rng.getrandbits(32 * lv) | 1
        # force long runs of 0xffffffff / 0 limbs now and then
        if rng.random() < 0.3:
            v |= ((1 << (32 * lv)) - 1) ^ ((1 << (32 * (lv - 1))) - 1)
        if rng.random() < 0.3:
            u = (1 << (32 * lu)) - 1 - rng.getrandbits(20)
        q, r = oracle.divmod_limbs(oracle.int_to_limbs(u, lu), oracle.int_to_limbs(v, lv))
        qi, ri = oracle.limbs_to_int(q), oracle.limbs_to_int(r)
        assert qi * v + ri == u and 0 <= ri < v


def test_division_add_back_path_8bit_limbs():
    """With 8-bit limbs Algorithm D's rare correction steps (the D3 trial
    quotient fix and the D6 add-back) occur often enough to be exercised."""
    oracle.reset_counters(8)
    rng = random.Random(11)
    for _ in range(20000):
        lu = rng.randint(3, 12)
        lv = rng.randint(2, lu)
        u = rng.getrandbits(8 * lu)
        v = rng.getrandbits(8 * lv) | (1 << (8 * lv - 1))
        if rng.random() < 0.5:          # divisors close to a power of the base
            v = (1 << (8 * lv - 1)) + rng.getrandbits(8 * (lv - 2))
        q, r = oracle.divmod_limbs(oracle.int_to_limbs(u, lu, 8), oracle.int_to_limbs(v, lv, 8), 8)
        assert oracle.limbs_to_int(q, 8) * v + oracle.limbs_to_int(r, 8) == u
        assert oracle.limbs_to_int(r, 8) < v
    assert oracle.addback_count(8) > 0
    assert oracle.qhat_fix_count(8) > 0


def test_modexp_8bit_build_agrees_with_pow():
    rng = random.Random(5)
    for _ in range(200):
        n = rng.getrandbits(rng.randint(9, 200)) | 1
        b = rng.getrandbits(220)
        e = rng.getrandbits(rng.randint(1, 64))
        ln, lb, le = (n.bit_length() + 7) // 8, max(1, (b.bit_length() + 7) // 8), max(1, (e.bit_length() + 7) // 8)
        out = oracle.modexp_batch(oracle.int_to_limbs(b, lb, 8)[None, :], oracle.int_to_limbs(e, le, 8),
                                  oracle.int_to_limbs(n, ln, 8), bits=8)
        assert oracle.limbs_to_int(out[0], 8) == pow(b, e, n)


def test_mul_schoolbook_against_python():
    rng = random.Random(3)
    for _ in range(500):
        la, lb = rng.randint(1, 70), rng.randint(1, 70)
        a, b = rng.getrandbits(32 * la), rng.getrandbits(32 * lb)
        w = oracle.mul_limbs(oracle.int_to_limbs(a, la), oracle.int_to_limbs(b, lb))
        assert oracle.limbs_to_int(w) == a * b


@pytest.mark.parametrize("bits", [512, 1024])
def test_fermat_on_seeded_primes(bits):
    rng = random.Random(bits)
    p = gen.random_prime(bits, rng)
    L = (bits + 31) // 32
    a = [rng.randrange(1, p) for _ in range(16)]
    out = oracle.modexp_batch(gen.to_limbs(a, L), gen.to_limbs(p - 1, L)[0], gen.to_limbs(p, L)[0])
    assert all(v == 1 for v in oracle.rows_to_ints(out))


def test_euler_and_round_trip_rsa1024():
    key = gen.rsa_key(1024, seed=gen.config_seed(1, 1))
    L = 32
    phi = (key.p - 1) * (key.q - 1)
    msgs = gen.uniform_below(key.n, 24, seed=4242)
    coprime = [m for m in msgs if math.gcd(m, key.n) == 1]
    out = oracle.modexp_batch(gen.to_limbs(coprime, L), gen.to_limbs(phi, L)[0], gen.to_limbs(key.n, L)[0])
    assert all(v == 1 for v in oracle.rows_to_ints(out))
    # m^(e d) == m for every m (n squarefree), including m not coprime to n
    msgs = msgs + [0, 1, key.n - 1, key.p, 2 * key.q]
    c = oracle.modexp_batch(gen.to_limbs(msgs, L), gen.to_limbs(key.e, 1)[0], gen.to_limbs(key.n, L)[0])
    m = oracle.modexp_batch(c, gen.to_limbs(key.d, L)[0], gen.to_limbs(key.n, L)[0])
    assert oracle.rows_to_ints(m) == msgs
    assert oracle.rows_to_ints(c) == [pow(x, key.e, key.n) for x in msgs]


def test_multiplicativity():
    rng = random.Random(99)
    n = rng.getrandbits(768) | (1 << 767) | 1
    L = 24
    for _ in range(10):
        a, b = rng.randrange(n), rng.randrange(n)
        e1, e2 = rng.getrandbits(100), rng.getrandbits(90)
        f = lambda x, e: oracle.modexp_int(x, e, n)
        assert f(a * b % n, e1) == f(a, e1) * f(b, e1) % n
        assert f(a, e1 + e2) == f(a, e1) * f(a, e2) % n


def test_per_element_exponents_and_cpython_pow():
    rng = random.Random(1234)
    for bits in (64, 96, 1024, 2048):
        n = rng.getrandbits(bits) | (1 << (bits - 1)) | rng.getrandbits(1)
        if n < 2:
            n = 3
        L = (bits + 31) // 32
        B = 12
        bases = [rng.getrandbits(32 * L) for _ in range(B)]
        exps = [rng.getrandbits(rng.randint(0, 200)) for _ in range(B)]
        out = oracle.modexp_batch(gen.to_limbs(bases, L), gen.to_limbs(exps, 7), gen.to_limbs(n, L)[0])
        assert oracle.rows_to_ints(out) == [pow(b, e, n) for b, e in zip(bases, exps)]


def test_crt_decryption_equals_plain():
    key = gen.rsa_key(2048, seed=gen.config_seed(2, 1))
    L = 64
    c = gen.uniform_below(key.n, 6, seed=77) + [0, 1, key.n - 1, key.p, 2 * key.q, key.q]
    cl = gen.to_limbs(c, L)
    crt = oracle.rsa_crt_batch(cl, key.p, key.q, key.dp, key.dq, key.qinv)
    assert oracle.rows_to_ints(crt) == [pow(x, key.d, key.n) for x in c]


def test_rns_ref_montgomery_identity():
    """The plain RNS Montgomery definition satisfies r*M == X*Y (mod N), its
    quotient is the Montgomery quotient -X*Y*N^-1 mod M up to a multiple of M
    below k*M, and r < (k+1)N whenever M >= (k+1)^2 N and X, Y < (k+1)N."""
    rng = random.Random(21)
    for trial in range(40):
        k = rng.randint(2, 9)
        B = gen.rns_primes(k, seed=trial)
        M = math.prod(B)
        nbits = max(8, M.bit_length() - 2 * (k + 1).bit_length() - 1)
        N = rng.getrandbits(nbits) | 1
        if N < 3 or math.gcd(N, M) != 1 or M < (k + 1) ** 2 * N:
            continue
        for _ in range(5):
            X, Y = rng.randrange((k + 1) * N), rng.randrange((k + 1) * N)
            qh = rns_ref.mont_qhat(X, Y, N, B)
            assert 0 <= qh < k * M
            assert qh % M == (-X * Y * pow(N, -1, M)) % M
            r = rns_ref.mont_mul(X, Y, N, B)
            assert r * M % N == X * Y % N
            assert 0 <= r < (k + 1) * N
            assert rns_ref.crt(rns_ref.residues(r, B), B) == r % M


# ---------------------------------------------------------------------------
# Primality steps of key generation (trial division, Miller-Rabin)

def test_small_primes_pins():
    from oracle import primality
    pr = primality.small_primes(10000)
    assert len(pr) == 10000 and pr[:10] == [2, 3, 5, 7, 11, 13, 17, 19, 23, 29]
    assert pr[-1] == 104729                       # the 10,000th prime
    # brute force below 2000
    brute = [n for n in range(2, 2000) if all(n % d for d in range(2, int(n ** 0.5) + 1))]
    assert pr[:len(brute)] == brute


def test_trial_division_pins():
    from oracle import primality
    pr = primality.small_primes(10000)
    assert primality.trial_division(104729, primes=pr)            # equal to a listed prime
    assert not primality.trial_division(104729 * 104723, primes=pr)
    assert primality.trial_division(104743 * 104759, primes=pr)   # smallest factors past the list
    big = (1 << 1023) + 1
    want = all(big % p for p in pr)
    assert primality.trial_division(big, primes=pr) == want
    assert not primality.trial_division(3 * ((1 << 1000) + 7), primes=pr)


def test_miller_rabin_pins():
    from oracle import primality
    # Mersenne primes pass every base
    for e in (61, 89, 107, 127, 521, 607):
        n = (1 << e) - 1
        assert primality.miller_rabin(n, [2, 3, 5, 7, 11, 1 << 40, n - 2])
    # Carmichael numbers fool Fermat but not the strong test to base 2
    for n in (561, 1105, 1729, 2465, 2821, 6601, 8911, 41041, 825265):
        assert pow(2, n - 1, n) == 1 or math.gcd(2, n) > 1
        assert not primality.miller_rabin(n, [2])
    # strong pseudoprimes: 2047 = 23 * 89 passes base 2 only; 3215031751 =
    # 151 * 751 * 28351 passes bases 2, 3, 5, 7 and fails 11
    assert primality.strong_probable_prime(2047, 2) and not primality.strong_probable_prime(2047, 3)
    assert 151 * 751 * 28351 == 3215031751
    assert primality.miller_rabin(3215031751, [2, 3, 5, 7])
    assert not primality.miller_rabin(3215031751, [2, 3, 5, 7, 11])
    # agreement with brute force for every odd n in [5, 3000) with bases 2, 3
    for n in range(5, 3000, 2):
        prime = all(n % d for d in range(3, int(n ** 0.5) + 1, 2))
        if prime:
            assert primality.miller_rabin(n, [2, 3])
        elif primality.miller_rabin(n, [2, 3]):
            raise AssertionError(n)                # no spsp(2, 3) below 1,373,653
    # a product of two 512-bit primes is composite for random bases
    p, q = (1 << 521) - 1, (1 << 607) - 1
    assert not primality.miller_rabin(p * q, [2, 3])


def test_first_prime_pins():
    from oracle import primality
    # small odd stream: the first prime with gcd(e, p - 1) = 1, by brute force
    stream = list(range(10001, 11001, 2))
    bases = [[2, 3] for _ in stream]
    isprime = lambda n: all(n % d for d in range(2, int(n ** 0.5) + 1))
    for e in (3, 17, 65537):
        want = next(c for c in stream if isprime(c) and math.gcd(e, c - 1) == 1)
        assert primality.first_prime(stream, bases, e, primes=primality.small_primes(10)) == want
    # exclude skips a prime; an all-composite stream gives 0
    p0 = primality.first_prime(stream, bases, 65537, primes=primality.small_primes(10))
    p1 = primality.first_prime(stream, bases, 65537, exclude=p0, primes=primality.small_primes(10))
    assert p1 > p0 and isprime(p1)
    assert primality.first_prime([9, 15, 21, 25], [[2]] * 4, 3) == 0
    # the key from two primes satisfies Euler's theorem for every tested m
    k = primality.rsa_key_from_primes((1 << 89) - 1, (1 << 61) - 1, 65537)
    for m in (2, 3, 12345678901234567, k["n"] - 1):
        assert pow(pow(m, 65537, k["n"]), k["d"], k["n"]) == m
    assert (k["qinv"] * ((1 << 61) - 1)) % ((1 << 89) - 1) == 1
