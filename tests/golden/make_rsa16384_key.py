"""Writes rsa16384_key.json: a seeded RSA-16384 key (two 8192-bit primes),
an input fixture for the CRT tests whose halves need bases of 257 channels.

Drawn from the seeded input generator's own prime test (trial division by the
first 10,000 primes, then Miller-Rabin); candidates are tested in a process
pool but taken in stream order, so the key depends on the seed only.  Pure
Python at these sizes takes a few minutes, hence the stored fixture.

    python3 tests/golden/make_rsa16384_key.py
"""
import json
import math
import multiprocessing as mp
import os
import random
import sys

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", ".."))
import gen  # noqa: E402

BITS = 16384
SEED = gen.config_seed(8, 16)
E = 65537
ROUNDS = 40


def _test(args):
    c, idx = args
    return gen.is_probable_prime(c, ROUNDS, random.Random(SEED * 1000003 + idx))


def _prime(rng, pool, start_idx, exclude=0):
    half = BITS // 2
    idx = start_idx
    while True:
        batch = []
        while len(batch) < 32:
            c = rng.getrandbits(half) | (3 << (half - 2)) | 1
            idx += 1
            if math.gcd(E, c - 1) == 1 and c != exclude:
                batch.append((c, idx))
        for (c, i), ok in zip(batch, pool.map(_test, batch)):
            if ok:
                return c, i


def main():
    rng = random.Random(SEED)
    with mp.get_context("fork").Pool(min(8, os.cpu_count() or 1)) as pool:
        p, i = _prime(rng, pool, 0)
        rng = random.Random(SEED + 1)
        q, _ = _prime(rng, pool, 10 ** 6, exclude=p)
    out = {"bits": BITS, "seed": SEED, "e": E, "p": hex(p), "q": hex(q),
           "source": "gen.is_probable_prime on seeded candidates (see this script)"}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rsa16384_key.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(path, (p * q).bit_length())


if __name__ == "__main__":
    main()
