"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module draws the inputs of every test and benchmark: RSA keys, messages,
ciphertexts, exponents and, for tests that pin a base explicitly, 32-bit RNS
channel primes.  It holds none of the modular-exponentiation arithmetic of the
method itself: primality tests and inverses use CPython's built-in ``pow``.

Key generation follows the paper's description of the RSA layer (Sec. 3.3 and
Sec. 4.3): uniform odd candidates, trial division by the first 10,000 primes,
then Miller-Rabin rounds; the private exponent is the inverse of e modulo
(p-1)(q-1) (Sec. 3.3).  Bignums are drawn with ``random.Random(seed)`` (whose
``getrandbits`` is deterministic across platforms); all limb arrays are
little-endian uint32.
"""
from __future__ import annotations

import json
import math
import os
import random
import sys
from dataclasses import dataclass
from functools import lru_cache

import numpy as np

__all__ = [
    "first_primes", "is_probable_prime", "random_prime", "RsaKey", "rsa_key",
    "uniform_below", "random_exponent", "to_limbs", "limbs_needed",
    "rns_primes", "config_seed", "MixedOp", "mixed_batch_spec", "rsa_keys", "served_keys", "served_trace",
]

# Seed streams: config i uses 1000*i + s, s in {1: keys, 2: messages,
# 3: exponents, 4: RNS primes, 5: traces}.
def config_seed(config: int, stream: int) -> int:
    return 1000 * config + stream


@lru_cache(maxsize=None)
def first_primes(count: int = 10000) -> tuple:
    """The first ``count`` primes by a sieve of Eratosthenes."""
    limit = 16
    while True:
        sieve = bytearray([1]) * (limit + 1)
        sieve[0:2] = b"\x00\x00"
        for i in range(2, int(limit ** 0.5) + 1):
            if sieve[i]:
                sieve[i * i::i] = bytearray(len(sieve[i * i::i]))
        primes = [i for i in range(limit + 1) if sieve[i]]
        if len(primes) >= count:
            return tuple(primes[:count])
        limit *= 2


def is_probable_prime(n: int, rounds: int, rng: random.Random) -> bool:
    """Trial division by the first 10,000 primes, then Miller-Rabin."""
    if n < 2:
        return False
    for p in first_primes(10000):
        if n == p:
            return True
        if n % p == 0:
            return False
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for _ in range(rounds):
        a = rng.randrange(2, n - 1)
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def random_prime(bits: int, rng: random.Random, e: int = 65537, rounds: int = 40) -> int:
    """A prime of exactly ``bits`` bits with its top two bits set, p-1 coprime to e."""
    if bits < 4:
        raise ValueError("bits must be >= 4")
    while True:
        c = rng.getrandbits(bits) | (3 << (bits - 2)) | 1
        if math.gcd(e, c - 1) != 1:
            continue
        if is_probable_prime(c, rounds, rng):
            return c


@dataclass(frozen=True)
class RsaKey:
    n: int
    e: int
    d: int
    p: int
    q: int
    dp: int
    dq: int
    qinv: int          # q^-1 mod p

    @property
    def bits(self) -> int:
        return self.n.bit_length()


def _key_from_primes(p: int, q: int, e: int) -> RsaKey:
    n = p * q
    phi = (p - 1) * (q - 1)
    d = pow(e, -1, phi)
    return RsaKey(n=n, e=e, d=d, p=p, q=q, dp=d % (p - 1), dq=d % (q - 1),
                  qinv=pow(q, -1, p))


def _generate_key(bits: int, seed: int, e: int = 65537) -> RsaKey:
    """The seeded draw itself: p from the first half of the stream, then q."""
    rng = random.Random(seed)
    half = bits // 2
    p = random_prime(half, rng, e)
    while True:
        q = random_prime(bits - half, rng, e)
        if q != p:
            break
    return _key_from_primes(p, q, e)


# Keys of the mixed-size and served workloads, drawn once by _generate_key
# (gen/make_keys.py): "bits:seed" -> [p, q] in hex.
KEY_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "keys.json")


@lru_cache(maxsize=1)
def _key_cache() -> dict:
    if not os.path.exists(KEY_CACHE):
        return {}
    with open(KEY_CACHE) as fh:
        return json.load(fh).get("keys", {})


def rsa_key(bits: int, seed: int, e: int = 65537) -> RsaKey:
    """Seeded RSA key with an exactly ``bits``-bit modulus n = p*q (from the
    stored draw when gen/keys.json holds it, with e = 65537)."""
    hit = _key_cache().get("%d:%d" % (bits, seed)) if e == 65537 else None
    if hit is not None:
        k = _key_from_primes(int(hit[0], 16), int(hit[1], 16), e)
        if k.n.bit_length() != bits:
            raise ValueError("gen/keys.json entry %d:%d does not have %d bits" % (bits, seed, bits))
        return k
    return _generate_key(bits, seed, e)


def uniform_below(n: int, count: int, seed: int) -> list:
    """``count`` integers uniform in [0, n) by rejection on getrandbits."""
    rng = random.Random(seed)
    b = n.bit_length()
    out = []
    while len(out) < count:
        x = rng.getrandbits(b)
        if x < n:
            out.append(x)
    return out


def random_exponent(bits: int, seed: int) -> int:
    """Uniform random bits with the top bit set."""
    rng = random.Random(seed)
    return rng.getrandbits(bits) | (1 << (bits - 1))


def limbs_needed(x: int) -> int:
    return max(1, (x.bit_length() + 31) // 32)


def to_limbs(values, nlimbs: int) -> np.ndarray:
    """Pack non-negative ints into a [len, nlimbs] little-endian uint32 array."""
    if isinstance(values, int):
        values = [values]
    nbytes = 4 * nlimbs
    buf = bytearray()
    for v in values:
        if v < 0 or v.bit_length() > 32 * nlimbs:
            raise ValueError("value does not fit in %d limbs" % nlimbs)
        buf += v.to_bytes(nbytes, "little")
    return np.frombuffer(bytes(buf), dtype="<u4").reshape(len(values), nlimbs).copy()


def _is_prime_u32(n: int) -> bool:
    # Miller-Rabin with bases 2, 7, 61 is deterministic below 4,759,123,141.
    if n < 2:
        return False
    for p in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53, 59, 61):
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in (2, 7, 61):
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def rns_primes(count: int, seed: int, lo: int = 1 << 31, hi: int = 1 << 32,
               exclude=()) -> list:
    """``count`` distinct primes drawn uniformly from [lo, hi) (seeded)."""
    if hi > (1 << 32) or lo < 3:
        raise ValueError("channel primes must lie in [3, 2^32)")
    rng = random.Random(seed)
    seen = set(exclude)
    out = []
    while len(out) < count:
        c = rng.randrange(lo, hi) | 1
        if c >= hi or c in seen:
            continue
        if _is_prime_u32(c):
            seen.add(c)
            out.append(c)
    return out


# ---------------------------------------------------------------------------
# Mixed-size batch: keys of several sizes, per-key lognormal batch sizes,
# encryptions and CRT decryptions mixed.


@dataclass(frozen=True)
class MixedOp:
    key_index: int     # index into the key list
    bits: int          # modulus size
    kind: str          # "encrypt" or "decrypt"
    count: int
    msg_seed: int      # seed of the count messages, uniform in [0, n)


def mixed_batch_spec(n_keys: int = 64, sizes=(1024, 2048, 3072, 4096), median: float = 128.0,
                     sigma: float = 1.0, cap: int = 8192, p_decrypt: float = 0.5, config: int = 4):
    """Keys split evenly over ``sizes`` (key j has size sizes[j * len(sizes) //
    n_keys]); key j's batch is round(exp(ln(median) + sigma z_j)), z_j ~ N(0, 1),
    clipped to [1, cap]; each of its messages is a CRT decryption with
    probability p_decrypt, else an encryption.  Returns (key_specs, ops) with
    key_specs = [(bits, key_seed)] and ops a list of MixedOp (an encrypt and a
    decrypt op per key, either possibly with count 0 omitted)."""
    rng = np.random.default_rng(config_seed(config, 5))
    z = rng.standard_normal(n_keys)
    keys, ops = [], []
    for j in range(n_keys):
        bits = sizes[j * len(sizes) // n_keys]
        keys.append((bits, config_seed(config, 1) * 1000 + j))
        b = int(min(cap, max(1, round(math.exp(math.log(median) + sigma * z[j])))))
        n_dec = int(rng.binomial(b, p_decrypt))
        for kind, cnt in (("encrypt", b - n_dec), ("decrypt", n_dec)):
            if cnt:
                ops.append(MixedOp(j, bits, kind, cnt, config_seed(config, 2) * 100000 + 2 * j + (kind == "decrypt")))
    return keys, ops


def _key_job(args):
    bits, seed = args
    return _generate_key(bits, seed)


def _gpu_in_use() -> bool:
    torch = sys.modules.get("torch")
    try:
        return bool(torch is not None and torch.cuda.is_initialized())
    except Exception:
        return False


def rsa_keys(specs, processes: int = 1) -> list:
    """rsa_key for each (bits, seed) in specs.  Keys stored in gen/keys.json
    are read from it; the others are drawn, optionally in a process pool
    (pure Python: seconds per 4096-bit key).  A pool forks this process,
    which must not have touched the GPU yet (a forked copy of an initialised
    HIP runtime is not usable, and its exit can crash): that case raises."""
    specs = list(specs)
    cache = _key_cache()
    missing = [s for s in specs if "%d:%d" % s not in cache]
    if processes <= 1 or len(missing) < 2:
        return [rsa_key(b, s) for b, s in specs]
    if _gpu_in_use():
        raise RuntimeError("rsa_keys: %d keys are not in gen/keys.json and a process pool would fork a process "
                           "that already uses the GPU; draw them before the first GPU call or use processes=1"
                           % len(missing))
    import multiprocessing as mp
    with mp.get_context("fork").Pool(min(processes, len(missing))) as pool:
        drawn = dict(zip(missing, pool.map(_key_job, missing)))
    return [drawn[s] if s in drawn else rsa_key(*s) for s in specs]


# ---------------------------------------------------------------------------
# Served workload: resident keys and a Poisson request trace.

SERVED_SIZES = (2048, 1024, 3072, 4096)
SERVED_SIZE_P = (0.4, 0.3, 0.2, 0.1)


def served_keys(per_size: int = 64, sizes=SERVED_SIZES, config: int = 5) -> list:
    """(bits, seed) of the resident keys: per_size keys of each size, grouped
    by size in the order of ``sizes``."""
    return [(b, config_seed(config, 1) * 10000 + i * 1000 + j) for i, b in enumerate(sizes) for j in range(per_size)]


def served_trace(rate: float, duration: float, per_size: int = 64, p_decrypt: float = 0.7, sizes=SERVED_SIZES,
                 size_p=SERVED_SIZE_P, config: int = 5, seed_offset: int = 0):
    """Open-loop Poisson trace: exponential inter-arrival times of mean 1/rate
    over [0, duration); each request picks a key size with probabilities
    size_p, a key uniformly within that size, and is a CRT decryption with
    probability p_decrypt, else an encryption (e = 65537).  Returns numpy
    arrays (arrival seconds, key index into served_keys, kind 0 = encrypt /
    1 = decrypt, message seed)."""
    rng = np.random.default_rng(config_seed(config, 5) + seed_offset)
    n_max = int(rate * duration * 1.2 + 100)
    gaps = rng.exponential(1.0 / rate, n_max)
    arrival = np.cumsum(gaps)
    while arrival[-1] < duration:                      # extremely unlikely with the 20% margin
        arrival = np.concatenate([arrival, arrival[-1] + np.cumsum(rng.exponential(1.0 / rate, n_max))])
    arrival = arrival[arrival < duration]
    n = arrival.size
    size_idx = rng.choice(len(sizes), size=n, p=np.asarray(size_p) / np.sum(size_p))
    key = size_idx * per_size + rng.integers(0, per_size, size=n)
    kind = (rng.random(n) < p_decrypt).astype(np.int32)
    msg_seed = config_seed(config, 2) * 10_000_000 + seed_offset * 1_000_000 + np.arange(n)
    return arrival, key.astype(np.int32), kind, msg_seed


def uniform_below_fast(n: int, seed: int) -> int:
    """One integer uniform in [0, n) (rejection on getrandbits) for seed."""
    return uniform_below(n, 1, seed)[0]
