"""RSA modular exponentiation in the Residue Number System on AMD MI355X.

The HIP library (``_lib/librnsrsa.so``, C ABI in ``include/rnsrsa.h``) does
all the arithmetic; ``rnsrsa`` is its ctypes binding.
"""
from .rnsrsa import (ENGINE_AUTO, ENGINE_CHANNEL, ENGINE_MATRIX, PRIMES_FULL, PRIMES_HIGH, Plan, RnsContext, RnsError, RsaKey,  # noqa: F401
                     int_to_limbs, lib, nlimbs)
