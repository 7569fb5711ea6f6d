"""The seeded input generator: keys have the stated structure and are reproducible."""
import math

import numpy as np

import gen


def test_rsa_key_structure():
    for bits, cfg in ((1024, 1), (2048, 2)):
        key = gen.rsa_key(bits, seed=gen.config_seed(cfg, 1))
        assert key.n == key.p * key.q and key.n.bit_length() == bits
        assert key.p.bit_length() == key.q.bit_length() == bits // 2
        phi = (key.p - 1) * (key.q - 1)
        assert key.e * key.d % phi == 1            # inverse modulo (p-1)(q-1)
        assert key.dp == key.d % (key.p - 1) and key.dq == key.d % (key.q - 1)
        assert key.q * key.qinv % key.p == 1
        # Fermat witnesses with CPython pow, independent of the oracle
        for a in (2, 3, 5, 7):
            assert pow(a, key.p - 1, key.p) == 1 and pow(a, key.q - 1, key.q) == 1
        assert gen.rsa_key(bits, seed=gen.config_seed(cfg, 1)) == key


def test_arazi_inverse_formula_matches_euclid():
    # Sec. 3.1: d = (1 + f * (-f^-1 mod e)) / e is e^-1 mod f for coprime e, f
    for e, f in ((17, 3120), (65537, 2 ** 61 - 2), (3, 1000)):
        if math.gcd(e, f) != 1:
            continue
        t = (-pow(f, -1, e)) % e
        num = 1 + f * t
        assert num % e == 0 and num // e == pow(e, -1, f)
    assert (1 + 3120 * ((-pow(3120, -1, 17)) % 17)) // 17 == 2753


def test_uniform_below_and_limbs():
    n = (1 << 1000) + 12345
    xs = gen.uniform_below(n, 100, seed=3)
    assert all(0 <= x < n for x in xs) and xs == gen.uniform_below(n, 100, seed=3)
    a = gen.to_limbs(xs, 32)
    assert a.dtype == np.uint32 and a.shape == (100, 32)
    assert int.from_bytes(a[5].tobytes(), "little") == xs[5]


def test_rns_primes():
    ps = gen.rns_primes(66, seed=9)
    assert len(set(ps)) == 66 and all((1 << 31) <= p < (1 << 32) for p in ps)
    assert all(pow(2, p - 1, p) == 1 for p in ps)
    hi = gen.rns_primes(10, seed=9, lo=(1 << 32) - (1 << 24))
    assert all(p >= (1 << 32) - (1 << 24) for p in hi)


def test_mixed_batch_spec():
    keys, ops = gen.mixed_batch_spec()
    assert len(keys) == 64
    assert [b for b, _ in keys] == [1024] * 16 + [2048] * 16 + [3072] * 16 + [4096] * 16
    assert len({s for _, s in keys}) == 64
    per_key = {}
    for o in ops:
        per_key[o.key_index] = per_key.get(o.key_index, 0) + o.count
        assert o.count >= 1 and o.kind in ("encrypt", "decrypt") and o.bits == keys[o.key_index][0]
    sizes = sorted(per_key.values())
    assert 1 <= sizes[0] and sizes[-1] <= 8192
    assert 60 <= sizes[len(sizes) // 2] <= 260            # median 128 in distribution
    n_dec = sum(o.count for o in ops if o.kind == "decrypt")
    total = sum(o.count for o in ops)
    assert 0.4 < n_dec / total < 0.6
    assert gen.mixed_batch_spec() == (keys, ops)           # deterministic


def test_stored_keys_are_the_seeded_draws():
    """gen/keys.json holds the draws of gen/make_keys.py: a sample of its
    entries (all sizes of the mixed and served workloads) equals a fresh draw
    from the seeded generator, and every entry is an RSA key of its size."""
    import random

    cache = gen._key_cache()
    specs = [tuple(map(int, s.split(":"))) for s in cache]
    from gen.make_keys import standard_specs
    assert sorted(specs) == standard_specs()
    for bits, seed in random.Random(1).sample(sorted(s for s in specs if s[0] <= 2048), 6):
        assert gen.rsa_key(bits, seed) == gen._generate_key(bits, seed)
    for bits, seed in specs:
        k = gen.rsa_key(bits, seed)
        assert k.n.bit_length() == bits and k.p.bit_length() == k.q.bit_length() == bits // 2
        assert pow(3, k.p - 1, k.p) == 1 and pow(3, k.q - 1, k.q) == 1


def test_rsa_keys_refuses_to_fork_a_gpu_process(monkeypatch):
    """A process pool would fork the calling process: refused once the GPU is
    in use (keys missing from gen/keys.json); stored keys need no pool."""
    import pytest

    monkeypatch.setattr(gen, "_gpu_in_use", lambda: True)
    with pytest.raises(RuntimeError):
        gen.rsa_keys([(512, 11), (512, 12)], processes=4)
    specs, _ = gen.mixed_batch_spec()
    assert len(gen.rsa_keys(specs[:4], processes=4)) == 4
