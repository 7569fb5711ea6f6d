"""Write gen/keys.json: the seeded RSA keys of the mixed-size and served
workloads, drawn once by gen.rsa_key so that no test or benchmark has to run
the pure-Python key generator (seconds per 4096-bit key) or fork a process
pool after it has started using the GPU.

Each entry is keyed "bits:seed" and holds the primes p and q in hex; gen.rsa_key
rebuilds d, d_p, d_q and q^-1 mod p from them.  The file is input data: it is
written by this script from the seeded generator alone (no arithmetic of the
method under test).

  python -m gen.make_keys [-j N]
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import gen  # noqa: E402


def standard_specs() -> list:
    """(bits, seed) of every key the mixed-size workload (64 keys, and its
    8-key version in the GPU tests) and the served workload (256 keys) use."""
    specs, _ = gen.mixed_batch_spec()
    small, _ = gen.mixed_batch_spec(n_keys=8)
    return sorted(set(list(specs) + list(small) + list(gen.served_keys(per_size=64))))


def _one(spec):
    bits, seed = spec
    k = gen._generate_key(bits, seed)
    return "%d:%d" % (bits, seed), ["%x" % k.p, "%x" % k.q]


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("-j", type=int, default=os.cpu_count() or 4)
    a = ap.parse_args(argv)
    specs = standard_specs()
    # largest keys first so the pool finishes evenly
    specs.sort(key=lambda s: -s[0])
    with mp.get_context("fork").Pool(a.j) as pool:
        entries = dict(pool.map(_one, specs, chunksize=1))
    out = {"what": "seeded RSA keys (p, q in hex) of the mixed-size and served workloads, by gen.rsa_key",
           "keys": {k: entries[k] for k in sorted(entries, key=lambda s: tuple(map(int, s.split(":"))))}}
    with open(gen.KEY_CACHE, "w") as fh:
        json.dump(out, fh, indent=0)
        fh.write("\n")
    print("%d keys -> %s" % (len(entries), gen.KEY_CACHE))
    return 0


if __name__ == "__main__":
    sys.exit(main())
