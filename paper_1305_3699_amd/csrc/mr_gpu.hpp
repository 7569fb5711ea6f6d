// Miller-Rabin with the per-candidate constants built on the GPU (mr_gpu.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace rnsrsa {
namespace api {

// The strong probable-prime test of every candidate (host, count x L limbs,
// odd, > 3) with its `rounds` bases (host, count x rounds x L, in [2, N - 2]):
// verdict[i] = 1 for a probable prime (host).  The candidates' tables are
// built on the device; every exponentiation runs on the matrix engine and
// every comparison on the device.  RNS_EUNSUPPORTED when the base for L-limb
// candidates has no matrix-engine kernel (the caller then takes the host
// path).  Synchronises s.
int miller_rabin_gpu(const uint32_t *cand, size_t count, int L, const uint32_t *bases, int rounds, uint8_t *verdict,
                     hipStream_t s);

}  // namespace api
}  // namespace rnsrsa
