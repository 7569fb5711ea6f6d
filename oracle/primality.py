"""Primality steps of key generation -- test infrastructure only.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
import this module; it shares no code with the GPU library.  Plain Python
integers, each function the textbook definition:

* ``small_primes(count)``: the first ``count`` primes, sieve of
  Eratosthenes -- the trial-division list (the first 10,000 primes,
  Sec. 4.3).
* ``trial_division(n, count)``: False when one of the first ``count`` primes
  divides n and differs from it (n is then composite), else True.
* ``strong_probable_prime(n, a)`` and ``miller_rabin(n, bases)``: the
  Miller-Rabin test (Sec. 3.2, with the iteration counts of Sec. 4.3): write
  n - 1 = 2^s d with d odd; base a passes when a^d = 1 (mod n) or
  a^(2^j d) = n - 1 (mod n) for some 0 <= j < s.  n is declared a probable
  prime when every base passes; one failing base proves n composite.
"""
from __future__ import annotations

import math


def small_primes(count: int) -> list:
    """The first ``count`` primes (sieve of Eratosthenes over a bound from
    Rosser's theorem, p_n < n (ln n + ln ln n) for n >= 6)."""
    if count <= 0:
        return []
    bound = 15 if count < 6 else int(count * (math.log(count) + math.log(math.log(count)))) + 1
    sieve = bytearray([1]) * (bound + 1)
    sieve[0] = sieve[1] = 0
    for i in range(2, int(bound ** 0.5) + 1):
        if sieve[i]:
            sieve[i * i::i] = bytearray(len(range(i * i, bound + 1, i)))
    out = [i for i in range(bound + 1) if sieve[i]]
    return out[:count]


def trial_division(n: int, count: int = 10000, primes: list | None = None) -> bool:
    """False iff a prime among the first ``count`` divides n and is not n."""
    for p in primes if primes is not None else small_primes(count):
        if n % p == 0 and n != p:
            return False
    return True


def strong_probable_prime(n: int, a: int) -> bool:
    """Whether odd n > 2 passes the strong test to base a."""
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    x = pow(a, d, n)
    if x == 1 or x == n - 1:
        return True
    for _ in range(s - 1):
        x = x * x % n
        if x == n - 1:
            return True
    return False


def miller_rabin(n: int, bases) -> bool:
    """Probable prime iff every base passes the strong test."""
    return all(strong_probable_prime(n, a) for a in bases)


def first_prime(cands, bases, e: int, exclude: int = 0, primes: list | None = None) -> int:
    """The selection rule of key generation from a candidate stream: the
    first candidate, in order, that is odd and > 3, differs from
    ``exclude``, survives trial division by the first 10,000 primes, has
    gcd(e, c - 1) = 1 and passes the strong test to each of its bases.
    Returns 0 when none does."""
    pr = primes if primes is not None else small_primes(10000)
    for c, bs in zip(cands, bases):
        if c % 2 == 0 or c <= 3 or c == exclude:
            continue
        if not trial_division(c, primes=pr) or math.gcd(e, c - 1) != 1:
            continue
        if miller_rabin(c, bs):
            return c
    return 0


def rsa_key_from_primes(p: int, q: int, e: int) -> dict:
    """n = p q, d = e^-1 mod (p-1)(q-1) (the library's modular inverse), and
    the CRT parts dp, dq, qinv = q^-1 mod p."""
    d = pow(e, -1, (p - 1) * (q - 1))
    return {"n": p * q, "d": d, "dp": d % (p - 1), "dq": d % (q - 1), "qinv": pow(q, -1, p)}
