// Host-side RNS planning: choice of the two bases and precomputation of every
// constant the RNS Montgomery product and its base extensions use.  The paper
// computes these once at initialisation and keeps them resident on the GPU
// (Sec. 3.1, last paragraph); the device upload lives in the C ABI layer.
#pragma once

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "arith.hpp"
#include "bn_host.hpp"

namespace rnsrsa {

// Supported (K, W) shapes: K channels per base, W waves per workgroup.  The
// kernels are instantiated for exactly this list (kernel_configs.inc).
struct Shape {
    int K, W;
};
const std::vector<Shape> &supported_shapes();
int default_waves(int K);              // 0 if K unsupported
bool shape_supported(int K, int W);    // a base of this shape can be planned
bool channel_kernel(int K, int W);     // the channel-engine kernels exist for it

enum PrimeRange { RANGE_HIGH = 0, RANGE_FULL = 1 };

// Two bases B (moduli m_i) and B' (m'_j), K primes each, plus the redundant
// channel 2^32, and all key-independent constants.
struct BaseSet {
    int K = 0, W = 0, KP = 0;
    std::vector<uint32_t> B, Bp;
    Limbs M, Mp;
    std::vector<uint32_t> blob;  // Layout{K,KP} base table
};

// One modulus N over a base set.
struct ModPlan {
    std::shared_ptr<const BaseSet> base;
    Limbs N;
    int L = 0;                   // limbs of the binary operands
    Limbs Mmod;                  // M mod N (Montgomery "one")
    Limbs R2;                    // M^2 mod N
    std::vector<uint32_t> blob;  // Layout{K,KP} per-modulus table
};

struct PlanOptions {
    int k = 0;                   // 0: smallest supported K meeting the bounds
    int waves = 0;               // 0: default for K
    int range = RANGE_HIGH;
    uint64_t seed = 0x5eed;
    const uint32_t *primes = nullptr;  // explicit 2K primes (B then B')
    size_t n_primes = 0;
    int engine = 0;              // 0 auto, 1 channel (VALU) kernel, 2 matrix-core kernel
};

// Returns 0 or a negative status (rnsrsa.h codes); err receives a message.
int make_modplan(const Limbs &N, int L, const PlanOptions &opt, ModPlan &out, std::string &err);

// Plan modulus N on an existing base set (both halves of a CRT key share one
// base set so that they run in one launch).
int make_modplan_on(const Limbs &N, int L, std::shared_ptr<const BaseSet> bs, ModPlan &out, std::string &err);

// Entry table for an input of nchunks*L limbs X = sum_h X_h 2^(32 L h),
// mapped to Z = sum_h X_h * Y_h: row j (input limb j), column = channel,
// value (2^(32 (j mod L)) * Y_(j div L)) mod m, scaled by R^2 for B and B'.
std::vector<uint32_t> make_entry_table(const ModPlan &mp, const std::vector<Limbs> &Y, int L);

// True when M >= (K+2)^2 N, M >= 2^(32 L + 1), M' >= (K+2) N and no channel
// prime of B divides N.
bool bounds_hold(const BaseSet &bs, const Limbs &N, int L);

}  // namespace rnsrsa
