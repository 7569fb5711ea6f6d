// Host model of the exponentiation kernels (emul.cpp).
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "plan.hpp"
#include "plan_mfma.hpp"

namespace rnsrsa {

// Same contract as the modexp kernel for one job: inputs of in_limbs limbs
// mapped through entry table E, outputs of mp.L limbs.
void emul_modexp(const ModPlan &mp, const std::vector<uint32_t> &E, int in_limbs, const uint32_t *base,
                 const uint32_t *exp, int exp_limbs, size_t exp_stride, int window, uint32_t *out,
                 size_t batch);

// Host model of the matrix-core kernel (emul_mfma.cpp), same contract.
// Returns false when a one-REDC step saw an input outside [0, m 2^32), where
// the kernel's result would be wrong.  scaled: keep the B residues scaled
// when T holds that form (the kernel's default), else the unscaled form.
bool emul_modexp_mfma(const ModPlan &mp, const MfmaTables &T, const std::vector<uint32_t> &E, int in_limbs,
                      const uint32_t *base, const uint32_t *exp, int exp_limbs, size_t exp_stride, int window,
                      uint32_t *out, size_t batch, bool scaled = true);

// One base extension of the matrix-core kernel (which = 1: first, 2:
// second) on raw digits xi [batch][K]: the byte partials of every slot row
// [batch][W*4MT][4] and S as the kernel combines them [batch][W*4MT].
// Returns false when a partial leaves int32 or the kernel's combination would
// wrap.
bool emul_mfma_extension(const MfmaTables &T, int which, const uint32_t *xi, size_t batch, int64_t *parts,
                         int64_t *value);

// The constant matrix of one extension as the matrix cores read it:
// [W*4MT rows][4 bytes][64*KSTEPS K indices] signed bytes.
void emul_mfma_matrix(const MfmaTables &T, int which, int8_t *A);

void emul_mont_mul(const ModPlan &mp, const uint32_t *x, const uint32_t *y, uint32_t *out, size_t batch);

}  // namespace rnsrsa
