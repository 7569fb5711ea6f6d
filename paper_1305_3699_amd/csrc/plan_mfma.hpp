// Host-side tables of the matrix-core (MFMA) exponentiation kernel.
//
// That kernel performs both base extensions of the RNS Montgomery product
// (Sec. 3.1) as int8 matrix products with exact int32 accumulation: every
// 32-bit quotient digit is split into four signed bytes (the B operand,
// staged through LDS) and every base-extension constant, pre-multiplied by
// 2^(8a) for digit a, into four signed bytes (the A operand, precomputed
// here in the exact lane layout of v_mfma_i32_16x16x64_i8).
//
// Lane layout of one wavefront (W per workgroup, 16*NT elements per
// workgroup): the wave's 4*MT "slots" per base are grouped in MT tiles of 4;
// lane l owns slot 4*mt + l/16 of every tile mt for elements 16*nt + l%16.
// Slot s < 4*MT-1 of wave w is channel w*(4*MT-1) + s of its base (if below
// K); slot 4*MT-1 carries the redundant modulus 2^32.
#pragma once

#include <cstdint>
#include <vector>

#include "mfma_layout.hpp"
#include "plan.hpp"

namespace rnsrsa {

using MfmaShape = MLayout;

struct MfmaTables {
    MfmaShape shape;
    std::vector<uint32_t> base;  // key-independent
    std::vector<uint32_t> key;   // per modulus
    // The key's B residues may be kept scaled (MLayout::sq_ok): every B
    // channel had a square root s_i of sigma_i c_i R^-1 for sigma_i = 1 or
    // -1.  Either way the key also serves the unscaled form.
    bool scaled = false;
};

// Matrix-core kernel shape for K: the first listed whose workgroup serves
// `group` elements, else (or for group 0) the first listed for K.
bool mfma_shape_for(int K, MfmaShape &out, int group = 0);

// with_base = false leaves `base` empty (for a base whose table is already
// resident) and builds the per-modulus part only; allow_scaled = false
// builds the unscaled form only (scaled stays false).
MfmaTables make_mfma_tables(const ModPlan &mp, const MfmaShape &sh, bool with_base = true, bool allow_scaled = true);

// Entry table: row j = input limb j (value 2^(32 (j mod L)) * Y_(j div L)),
// columns [B slots | B' slots | redundant], scaled for the representation the
// kernel keeps (B: x*2^32 mod m; B': x*2^32*M^-1 mod m'), reduced by two REDCs.
std::vector<uint32_t> make_mfma_entry_table(const ModPlan &mp, const MfmaShape &sh, const std::vector<Limbs> &Y,
                                            int L);

// Channel of slot (wave w, tile mt, group g): -1 for the redundant slot,
// K or more for unused slots.
inline int mfma_slot_channel(const MfmaShape &sh, int w, int mt, int g) {
    const int s = 4 * mt + g;
    if (s == 4 * sh.MT - 1) return -1;
    return w * sh.CH() + s;
}

}  // namespace rnsrsa
