"""RSA modular exponentiation in the Residue Number System on AMD MI355X.

The HIP library (``_lib/librnsrsa.so``, C ABI in ``include/rnsrsa.h``) does
all the arithmetic; ``rnsrsa`` is its ctypes binding.
"""
from .rnsrsa import (ENGINE_AUTO, ENGINE_CHANNEL, ENGINE_MATRIX, OP_DECRYPT, OP_ENCRYPT, PRIMES_FULL,  # noqa: F401
                     PRIMES_HIGH, Plan, RnsContext, RnsError, RsaBatch, RsaKey, RsaServer, int_to_limbs, lib,
                     keygen, miller_rabin, modexp_jobs, nlimbs, trial_division)
