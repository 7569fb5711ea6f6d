// Word layout of the matrix-core kernel's tables, shared by the host code that
// builds them (plan_mfma.cpp) and the kernel that reads them (kernels_mfma.hpp).
// All per-lane tables have rows of 64 words (one per lane) so each lane reads
// its own value with one coalesced load.
#pragma once

#include <cstddef>
#include <cstdint>

namespace rnsrsa {

// Digit bias: a residue v in [0, 2^32) is handed to the matrix core as the
// word v ^ kDigitBias, whose four bytes read as signed int8 are the balanced
// digits of v - kDigitBias (each byte b becomes b - 128).  The constant
// -kDigitBias * sum(C_i) this adds to an extension is cancelled by the offset
// column of the constant matrix.
constexpr uint32_t kDigitBias = 0x80808080u;

// Constants of the A matrices are stored balanced: the representative of a
// residue in [kDigitSplit - m, kDigitSplit), inside [-0x80808080, 0x7F7F7F7F],
// the range of four signed bytes.
constexpr uint32_t kDigitSplit = 0x7F7F7F80u;
// Largest B' prime the matrix engine accepts: step (iii) of a product reduces
// x' y' + S + m 2^17 in one REDC, whose input must stay below m 2^32; with
// |S| < 2^48 that holds for m <= 2^32 - 2^18.
constexpr uint32_t kMaxPrimeP = 0xFFFC0000u;

// Bound on |S|, the signed value of an extension output's four byte partials:
// 4K digit terms, each a constant of magnitude <= 0x80808080 times a digit
// byte of magnitude <= 128, plus the offset column (digit 1).
constexpr uint64_t mfma_sum_bound(int K) { return (uint64_t)4 * K * 0x80808080ull * 128u + 0x80808080ull; }

// Bound on one byte partial P_b of an extension output (the int32 the matrix
// core returns): 4K digit bytes times constant bytes, each of magnitude <= 128,
// plus the offset column (constant byte times digit 1).
constexpr int64_t mfma_partial_bound(int K) { return (int64_t)4 * K * 128 * 128 + 128; }

// Whether the pairwise combination P_0 + 2^8 P_1 (and P_2 + 2^8 P_3) of the
// four byte partials stays inside int32 for every input: 257 times the
// partial bound below 2^31, i.e. K <= 127.  Wider bases combine in 64 bits.
constexpr bool mfma_pair_fits_i32(int K) { return 257 * mfma_partial_bound(K) < ((int64_t)1 << 31); }

// Steps (iii) and (iv) add m 2^s to S so that the REDC input is positive:
// s = 17 up to 256 + 1 channels (|S| about 2^48), 18 beyond (about 2^49).
constexpr int mfma_offset_shift(int K) { return K > 257 ? 18 : 17; }

// Whether channel prime m keeps the one-REDC steps exact: S + m 2^s > 0 for
// a prime of B (step (iv) adds alpha nu < K m, far below m 2^32), and for a
// prime of B' also x' y' + S + m 2^s < m 2^32 with x', y' < m, i.e.
// m 2^s + |S| < m (2^32 - m) + 2m - 1 (every term below 2^63).
constexpr bool mfma_prime_fits(uint32_t m, int K, bool in_bprime) {
    const uint64_t off = (uint64_t)m << mfma_offset_shift(K), smax = mfma_sum_bound(K);
    if (off <= smax) return false;
    if (!in_bprime) return true;
    return m <= kMaxPrimeP && off + smax < (uint64_t)m * ((1ull << 32) - m) + 2ull * m - 1;
}

struct MLayout {
    int K, W, MT, NT;
    constexpr int CH() const { return 4 * MT - 1; }                 // prime channels per wave
    constexpr int KSTEPS() const { return (4 * K + 1 + 63) / 64; }  // 64-deep steps: 4 digits/channel + offset
    constexpr int KCH() const { return KSTEPS() * 16; }             // channels covered by the steps
    // LDS words per element row of digits: KCH + 8 (a row stride of 56 words
    // at k = 33) measured 2% faster than KCH + 4, and KCH + 12 .. KCH + 36
    // slower, on the 16-lane digit reads and writes of the exchange
    constexpr int BROW() const { return KCH() + 8; }
    constexpr int NM() const { return 16 * NT; }                    // elements per workgroup
    constexpr int SLOTS() const { return 2 * MT * NT + NT; }        // table words per lane per entry
    constexpr size_t tiles() const { return (size_t)W * MT * KSTEPS() * 64 * 4; }
    // key-independent table
    constexpr size_t a2() const { return 0; }                                  // [W][MT][KSTEPS][64][4] second extension
    constexpr size_t slotB() const { return tiles(); }                         // [W][MT][3][64] m, m^-1 mod 2^32, nu
    constexpr size_t slotP() const { return slotB() + (size_t)W * MT * 3 * 64; }  // [W][MT][4][64] m', m'^-1, H, kappa
    constexpr size_t mpj() const { return slotP() + (size_t)W * MT * 4 * 64; }  // [K] m'_j
    constexpr size_t mplo() const { return mpj() + K; }                        // [K] M'_j mod 2^32
    constexpr size_t MpL() const { return mplo() + K; }                        // [K][K+1] limbs of M'_j
    constexpr size_t MpF() const { return MpL() + (size_t)K * (K + 1); }        // [K+1] limbs of M'
    constexpr size_t bscal() const { return MpF() + K + 1; }                   // [4] M'^-1, M^-1 mod 2^32
    // [W][MT][3][64] conversions of the standalone product between plain
    // residues and the kept representation: R^2 mod m (into B), R^2 M^-1 mod m'
    // (into B'), M mod m' (out of B'; out of B is a REDC by 1)
    constexpr size_t mmconv() const { return bscal() + 4; }
    constexpr size_t base_size() const { return mmconv() + (size_t)W * MT * 3 * 64; }
    // per-modulus table
    constexpr size_t a1() const { return 0; }                                  // [W][MT][KSTEPS][64][4] first extension
    constexpr size_t slotC() const { return tiles(); }                         // [W][MT][64] c_i
    constexpr size_t one() const { return slotC() + (size_t)W * MT * 64; }     // [W][MT][2][64] + [1]: M mod N
    constexpr size_t Nl() const { return one() + (size_t)W * MT * 2 * 64 + 1; }  // [K] limbs of N
    constexpr size_t kscal() const { return Nl() + K; }                        // [4] N mod 2^32
    // Whether a key of this shape may keep its B residues scaled (x R s_i
    // instead of x R, with s_i^2 = sigma_i c_i R^-1 mod m_i, sigma_i = +-1):
    // a product's quotient digit is then one REDC of the two operands.  The
    // second extension's tiles and nu then carry the factor s_i and become
    // per key, so only shapes whose tiles sit in registers or LDS (at most
    // 5 k-steps) take it.
    constexpr bool sq_ok() const { return KSTEPS() <= 5; }
    // scaled form (sq_ok shapes): [W][MT][KSTEPS][64][4] second extension
    // with output row t times s_t, then [W][MT][3][64] nu s, R s (the unit),
    // (M mod N) R s (one)
    constexpr size_t a2s() const { return kscal() + 4; }
    constexpr size_t sqB() const { return a2s() + (sq_ok() ? tiles() : 0); }
    constexpr size_t key_size() const { return sqB() + (sq_ok() ? (size_t)W * MT * 3 * 64 : 0); }
    // entry table: per input limb [W*4*MT B slots | W*4*MT B' slots | redundant]
    constexpr size_t ecols() const { return (size_t)2 * W * 4 * MT + 1; }
};

}  // namespace rnsrsa
