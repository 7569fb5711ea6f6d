// Matrix-core (MFMA) variant of the exponentiation kernel.
//
// Same algorithm as kernels_impl.hpp (RNS Montgomery products with two base
// extensions, fixed-window exponent loop, CRT exit), but both base extensions
// run on the int8 matrix cores: each quotient digit xi (a residue below 2^32)
// is handed over as xi ^ 0x80808080, i.e. as the four signed bytes of
// xi - 0x80808080, and each extension is the product of a constant A matrix
// (rows = 4 bytes of each output channel, columns = 4 digits of each input
// channel, constants pre-multiplied by 2^(8 digit)) with the digit matrix B
// (columns = elements), accumulated exactly in int32 by
// v_mfma_i32_16x16x64_i8.  One extra column cancels the digit bias; one extra
// row per wave computes the redundant 2^32 channel.  The four byte partials of
// an output are recombined to a signed 64-bit integer and reduced by one REDC.
//
// Layout (plan_mfma.hpp): W waves serve 16*NT elements; lane l of a wave
// owns slot 4*mt + l/16 of tile mt for elements 16*nt + l%16, which is
// exactly where the matrix core leaves the outputs of that slot, so the
// per-channel steps run in place with no transposition.  Channel residues
// are kept scaled: x*2^32 mod m in B, x*2^32*M^-1 mod m' in B'; a key whose
// tables hold the scaled form (SQ) keeps x*2^32*s_i mod m_i in B instead,
// with s_i^2 = sigma_i c_i 2^-32, sigma_i = +-1 (see mfma_publish_xi).
#pragma once

#include "arith.hpp"
#include "kernels.hpp"
#include "mfma_layout.hpp"

namespace rnsrsa {

typedef int mfma_v4i __attribute__((ext_vector_type(4)));

template <int K, int W, int MT, int NT>
struct MShp {
    static constexpr MLayout LY{K, W, MT, NT};
    static constexpr int CH = LY.CH();
    static constexpr int KSTEPS = LY.KSTEPS();
    static constexpr int BROW = LY.BROW();
    static constexpr int NM = LY.NM();
    static constexpr int SLOTS = LY.SLOTS();
    static constexpr int ECOLS = (int)LY.ecols();
    static constexpr int OSH = mfma_offset_shift(K);   // REDC offset m 2^OSH of steps (iii) and (iv)
    static constexpr bool PAIR_I32 = mfma_pair_fits_i32(K);   // byte partials paired in int32 (K <= 127)
    // smallest b with 2^b > K+1: an exit value below (K+2)N has quotient < 2^b
    static constexpr int qbits() {
        int b = 0;
        while ((1 << b) <= K + 1) b++;
        return b;
    }
    // Exit: [K][NM] digits and 2 x [K+1][NM] limbs; with the split exit (from
    // 49 channels on, where it pays for itself) also the carries out of the
    // limb ranges that the 64 W / NM workers per element sum, [workers][2][NM].
    // Below that one lane per element sums all limbs, and the main loop keeps
    // its register allocation (the split exit measured 7% slower at k = 33).
    static constexpr bool SPLIT_EXIT = K >= 49;
    static constexpr int EXIT_CORE = (K + 2 * (K + 1)) * NM;
    static constexpr int EXIT_WORDS = EXIT_CORE + (SPLIT_EXIT ? 128 * W : 0);
    static constexpr int BUF_WORDS = 2 * NM * BROW;
    static constexpr int WORK_WORDS = EXIT_WORDS > BUF_WORDS ? EXIT_WORDS : BUF_WORDS;
    // Where the second extension's constant tiles (the same for every key of
    // the base pair) live: registers for 32-element tiles with few k-steps;
    // LDS for 16-element tiles (3 waves then share a SIMD) and wherever the
    // registers would overflow while the tiles still fit LDS; otherwise they
    // are read from global memory (L2) at each step.
    static constexpr int A2_TILE_WORDS = W * MT * KSTEPS * 64 * 4;
    static constexpr bool A2_FITS_LDS = (EXIT_WORDS > BUF_WORDS ? EXIT_WORDS : BUF_WORDS) + A2_TILE_WORDS <= 36 * 1024;
    static constexpr bool A2_GLOBAL = KSTEPS > 5 || (KSTEPS == 5 && !A2_FITS_LDS);
    static constexpr bool A2_LDS = !A2_GLOBAL && (NT == 1 || KSTEPS >= 5);
    // the per-key first-extension tiles follow the second ones to global
    // memory for those shapes (their workgroups of 9-12 waves leave 168
    // registers per lane)
    static constexpr bool A1_GLOBAL = A2_GLOBAL;
    static constexpr int A2_WORDS = A2_LDS ? A2_TILE_WORDS : 0;
    // The widest bases (more than 9 k-steps: 256 channels and up) leave too
    // few registers for the per-slot constants as well: those shapes keep
    // them in LDS, [W][MT][4 lane groups][8 words], read where they are used.
    static constexpr bool C_LDS = KSTEPS > 9;
    static constexpr int C_WORDS = C_LDS ? W * MT * 4 * 8 : 0;
    static constexpr int LDS_WORDS = WORK_WORDS + A2_WORDS + C_WORDS;
    // Each wave's second operand of the next window multiplication is
    // prefetched from the window table into LDS while the squarings before it
    // run: [SLOTS][64] words per wave, wherever that still fits the 160 KiB
    // a workgroup may hold (every shape but the 513-channel one).
    static constexpr int PF_WORDS = W * SLOTS * 64;
    static constexpr bool PREFETCH = (size_t)(LDS_WORDS + PF_WORDS) * 4 <= 160 * 1024;
    // Resident waves per SIMD the register allocation must allow (1: no
    // constraint).  The 32-element tile at k = 33 keeps both extensions'
    // tiles in registers (25 KB of LDS per workgroup) and would take 205
    // VGPRs, i.e. 2 waves per SIMD; held to 168 VGPRs (3 waves, 4 workgroups
    // and 128 elements per CU) it spills about 70 registers to scratch and
    // still runs the RSA-2048 CRT launch 6% faster than the 16-element tile
    // (4 waves per SIMD, 128 VGPRs, spilled in the hot loop: 2.5x slower).
    static constexpr int WAVES_PER_EU = (K == 33 && NT == 2) ? 3 : 1;
};

template <int MT, int NT>
struct MState {
    uint32_t b[MT][NT];  // slots of B (x * 2^32 mod m)
    uint32_t p[MT][NT];  // slots of B' (x * 2^32 * M^-1 mod m')
    uint32_t r[NT];      // redundant channel, replicated over the lane groups
};

// Pointers into global memory (address space 1): accesses through them are
// global loads and stores, not flat ones (which also count against the LDS
// wait counter, so every LDS wait would wait for them too).
#define RNS_GLOBAL __attribute__((address_space(1)))
typedef RNS_GLOBAL uint32_t gu32;
typedef const RNS_GLOBAL mfma_v4i gcv4i;

// Constants of one slot: its B prime with -m^-1 mod 2^32, nu = -M' R^2 (times
// s_i with scaled B residues) and
// c = sigma_i (-N^-1 M_i^-1) (unused with scaled B residues); its B' prime
// with -m^-1 mod 2^32 and H = M (M'_t)^-1.
struct MSlotB {
    uint32_t m, u, nu, c;
};
struct MSlotP {
    uint32_t m, u, H, pad;
};

// Per-lane constants: in registers for the whole kernel, except for the
// shapes whose per-slot constants live in LDS (CL; read at each use).
template <int MT, int KSTEPS, bool CL>
struct MConst {
    mfma_v4i A1[MT][KSTEPS], A2[MT][KSTEPS];
    const mfma_v4i *a2lds;   // the wave's second-extension tiles in LDS (A2_LDS), [MT][KSTEPS][64]
    gcv4i *a2mem;            // the same in global memory (A2_GLOBAL shapes)
    gcv4i *a1mem;            // its first-extension tiles in global memory (A1_GLOBAL shapes)
    uint32_t loff;           // lane * 16: the lane's byte offset in a tile
    uint32_t mB[MT], uB[MT], nuB[MT], cB[MT];
    uint32_t mP[MT], uP[MT], HP[MT];
    const uint32_t *cl;      // CL: this lane group's constants in LDS, tile mt at cl + 32 mt
    uint32_t Mpinv_r, Minv_r, N_r;
    int32_t kf[4];           // 1, 2^8, 2^16, 2^24, opaque to the compiler (see mfma_accumulate)

    __device__ __forceinline__ MSlotB slotB(int mt) const {
        if (CL) {
            const uint4 v = *(const uint4 *)(cl + 32 * mt);
            return MSlotB{v.x, v.y, v.z, v.w};
        }
        return MSlotB{mB[mt], uB[mt], nuB[mt], cB[mt]};
    }
    __device__ __forceinline__ MSlotP slotP(int mt) const {
        if (CL) {
            const uint4 v = *(const uint4 *)(cl + 32 * mt + 4);
            return MSlotP{v.x, v.y, v.z, 0u};
        }
        return MSlotP{mP[mt], uP[mt], HP[mt], 0u};
    }
};

template <int K, int W, int MT, int NT>
using MConstOf = MConst<MT, MShp<K, W, MT, NT>::KSTEPS, MShp<K, W, MT, NT>::C_LDS>;

// digit word of a residue: its bytes, read as signed int8, are those of v - kDigitBias
__device__ __forceinline__ uint32_t mfma_pack(uint32_t v) { return v ^ kDigitBias; }

// low word of the value of the four byte partials (the redundant row)
__device__ __forceinline__ uint32_t mfma_combine_lo(const mfma_v4i &d) {
    const uint32_t t1 = (uint32_t)d[0] + ((uint32_t)d[1] << 8);
    uint32_t t2 = (uint32_t)d[2] + ((uint32_t)d[3] << 8);
    asm volatile("" : "+v"(t2));   // keeps the three shift-adds from being reassociated into four ops
    return t1 + (t2 << 16);
}

// acc + the signed value S = sum_b 2^(8b) P_b of the four byte partials, mod
// 2^64.  |S| is at most mfma_sum_bound(K): 4K+1 terms of |A byte value| <=
// 0x80808080 times |digit byte| <= 128.  Callers add m 2^OSH > |S| so that
// the REDC input is positive (the host checks every channel prime).  The
// factors (1, 2^8, 2^16, 2^24) come from scalar registers the compiler cannot
// see through, so each step is one signed 32x32+64 multiply-add instead of a
// sign extension, a 64-bit shift and a 64-bit add.  Up to 127 channels the
// pairs P_0 + 2^8 P_1 and P_2 + 2^8 P_3 are formed in int32 first (exact:
// mfma_pair_fits_i32); wider bases could overflow there and take each
// partial into the 64-bit sum on its own.
template <bool PAIR_I32>
__device__ __forceinline__ uint64_t mfma_accumulate(const mfma_v4i &d, uint64_t acc, const int32_t (&kf)[4]) {
    if constexpr (PAIR_I32) {
        const int32_t t1 = d[0] + (d[1] << 8);
        const int32_t t2 = d[2] + (d[3] << 8);
        acc += (uint64_t)((int64_t)t2 * kf[2]);
        acc += (uint64_t)((int64_t)t1 * kf[0]);
    } else {
#pragma unroll
        for (int b = 3; b >= 0; b--) acc += (uint64_t)((int64_t)d[b] * kf[b]);
    }
    return acc;
}

// Tile t of a wave's constant tiles in global memory, this lane's 16 bytes:
// a uniform base plus the lane offset, so the load takes the scalar-base
// form and no per-tile 64-bit address is kept in vector registers.
__device__ __forceinline__ mfma_v4i mfma_tile_load(gcv4i *base, int t, uint32_t loff) {
    return *(gcv4i *)((const RNS_GLOBAL char *)(base + (size_t)t * 64) + loff);
}

template <int K, int W, int MT, int NT>
__device__ __forceinline__ void mfma_extension(const MConstOf<K, W, MT, NT> &C, bool second,
                                               const uint32_t *buf, int lane, mfma_v4i (&D)[MT][NT]) {
    using S = MShp<K, W, MT, NT>;
    // tiles in global memory: re-derive their base at every call (an opaque
    // zero offset), so the compiler cannot hoist one 64-bit address per tile
    // out of the exponent loop and keep them all live
    gcv4i *a1m = C.a1mem, *a2m = C.a2mem;
    if (S::A1_GLOBAL || S::A2_GLOBAL) {
        int zo;
        asm volatile("s_mov_b32 %0, 0" : "=s"(zo));
        a1m += zo;
        a2m += zo;
    }
#pragma unroll
    for (int mt = 0; mt < MT; mt++)
#pragma unroll
        for (int nt = 0; nt < NT; nt++) D[mt][nt] = mfma_v4i{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < S::KSTEPS; ks++) {
#pragma unroll
        for (int nt = 0; nt < NT; nt++) {
            const mfma_v4i bop =
                *(const mfma_v4i *)(buf + (16 * nt + (lane & 15)) * S::BROW + 16 * ks + 4 * (lane >> 4));
#pragma unroll
            for (int mt = 0; mt < MT; mt++)
                D[mt][nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(
                    second ? (S::A2_GLOBAL ? mfma_tile_load(a2m, mt * S::KSTEPS + ks, C.loff)
                              : S::A2_LDS  ? C.a2lds[(mt * S::KSTEPS + ks) * 64 + lane]
                                           : C.A2[mt][ks])
                           : (S::A1_GLOBAL ? mfma_tile_load(a1m, mt * S::KSTEPS + ks, C.loff) : C.A1[mt][ks]),
                    bop, D[mt][nt], 0, 0, 0);
        }
        // operands read from memory: keep at most one k-step of them in
        // flight, or the scheduler hoists all of them and the registers spill
        if (S::A1_GLOBAL) __builtin_amdgcn_sched_barrier(0);
    }
}

// LDS column of the digit of slot (wave, mt, lane group g): its channel, or
// for the redundant slot and channels >= K one of the four columns after the
// last k-step, which the matrix cores never read (so the store needs no mask).
template <int K, int W, int MT, int NT>
__device__ __forceinline__ int mfma_digit_col(int wave, int mt, int g) {
    using S = MShp<K, W, MT, NT>;
    const int ch = wave * S::CH + 4 * mt + g;
    const bool real = (4 * mt + g != 4 * MT - 1) && ch < K;
    return real ? ch : S::LY.KCH() + (wave & 3);
}

// Step (i) of a product: quotient digits xi = x y c_i of the B slots (times
// the channel's sign sigma_i), published as the B operand of the first
// extension.  With the B residues kept scaled (SQ: x R s_i, s_i^2 =
// sigma_i c_i R^-1) that is one REDC of the two operands, else two.
template <int K, int W, int MT, int NT, bool SQ = false>
__device__ __forceinline__ void mfma_publish_xi(const MConstOf<K, W, MT, NT> &C,
                                                const MState<MT, NT> &x, const MState<MT, NT> &y, uint32_t *buf1,
                                                int wave, int lane) {
    using S = MShp<K, W, MT, NT>;
    const int g = lane >> 4;
#pragma unroll
    for (int mt = 0; mt < MT; mt++) {
        const int col = mfma_digit_col<K, W, MT, NT>(wave, mt, g);
#pragma unroll
        for (int nt = 0; nt < NT; nt++) {
            const MSlotB sb = C.slotB(mt);
            const uint32_t t = mulredc(x.b[mt][nt], y.b[mt][nt], sb.m, sb.u);   // x y 2^32, or sigma x y c_i (SQ)
            const uint32_t xi = SQ ? t : mulredc(t, sb.c, sb.m, sb.u);         // sigma x y c_i
            buf1[(16 * nt + (lane & 15)) * S::BROW + col] = mfma_pack(xi);
        }
    }
}

// One RNS Montgomery product x <- x*y*M^-1 in the matrix-core layout.  With
// full == false the second extension is skipped (the caller leaves the RNS
// from the xi' digits in buf2).  x.r receives the new redundant residue.
// SQ: B residues kept scaled by s_i (C then holds the scaled second
// extension and nu, so the result comes out scaled as well).
template <int K, int W, int MT, int NT, bool SQ = false>
__device__ __forceinline__ void mfma_mm(const MConstOf<K, W, MT, NT> &C, MState<MT, NT> &x,
                                        const MState<MT, NT> &y, uint32_t *buf1, uint32_t *buf2, int wave, int lane,
                                        bool full) {
    using S = MShp<K, W, MT, NT>;
    const int g = lane >> 4;
    mfma_publish_xi<K, W, MT, NT, SQ>(C, x, y, buf1, wave, lane);
    __syncthreads();

    // (ii) first extension on the matrix cores: q^'' N M^-1 (scaled) in each B'
    // slot; the B' and redundant products below do not depend on it and can
    // issue while the matrix cores run
    mfma_v4i D[MT][NT];
    mfma_extension<K, W, MT, NT>(C, false, buf1, lane, D);
    uint32_t sr[NT];
#pragma unroll
    for (int nt = 0; nt < NT; nt++) sr[nt] = x.r[nt] * y.r[nt];
    const int rsrc = ((lane & 15) + 48) * 4;
    uint32_t rr[NT];
#pragma unroll
    for (int nt = 0; nt < NT; nt++) {
        const uint32_t lo = mfma_combine_lo(D[MT - 1][nt]);
        const uint32_t qr = (uint32_t)__builtin_amdgcn_ds_bpermute(rsrc, (int)lo);   // q^'' mod 2^32
        rr[nt] = (sr[nt] + qr * C.N_r) * C.Minv_r;
    }
    // (iii) r = (XY + q^'' N)/M in B'; publish xi' for the second extension
#pragma unroll
    for (int mt = 0; mt < MT; mt++) {
        const int col = mfma_digit_col<K, W, MT, NT>(wave, mt, g);
#pragma unroll
        for (int nt = 0; nt < NT; nt++) {
            const MSlotP sp = C.slotP(mt);
            const uint32_t m = sp.m;
            // x' y' + S in one REDC (S + m 2^OSH > 0; the sum stays below
            // m 2^32 for every B' prime that mfma_prime_fits accepts)
            const uint64_t T = mfma_accumulate<S::PAIR_I32>(
                D[mt][nt], (uint64_t)x.p[mt][nt] * y.p[mt][nt] + ((uint64_t)m << S::OSH), C.kf);
            const uint32_t r = redc((uint32_t)T, (uint32_t)(T >> 32), m, sp.u);
            x.p[mt][nt] = r;
            const uint32_t xip = mulredc(r, sp.H, m, sp.u);                            // r (M'_t)^-1
            buf2[(16 * nt + (lane & 15)) * S::BROW + col] = mfma_pack(xip);
        }
    }
#pragma unroll
    for (int nt = 0; nt < NT; nt++) x.r[nt] = rr[nt];
    __syncthreads();
    if (!full) return;

    // (iv) second extension, made exact by alpha from the redundant channel
    mfma_extension<K, W, MT, NT>(C, true, buf2, lane, D);
    uint32_t alpha[NT];
#pragma unroll
    for (int nt = 0; nt < NT; nt++) {
        const uint32_t lo = mfma_combine_lo(D[MT - 1][nt]);
        const uint32_t s2 = (uint32_t)__builtin_amdgcn_ds_bpermute(rsrc, (int)lo);
        alpha[nt] = (s2 - rr[nt]) * C.Mpinv_r;
    }
#pragma unroll
    for (int mt = 0; mt < MT; mt++)
#pragma unroll
        for (int nt = 0; nt < NT; nt++) {
            // S + alpha nu + m 2^OSH (alpha nu < 2^42): positive, below m 2^32
            const MSlotB sb = C.slotB(mt);
            const uint64_t T = mfma_accumulate<S::PAIR_I32>(
                D[mt][nt], (uint64_t)alpha[nt] * sb.nu + ((uint64_t)sb.m << S::OSH), C.kf);
            x.b[mt][nt] = redc((uint32_t)T, (uint32_t)(T >> 32), sb.m, sb.u);
        }
}

template <int MT, int NT>
__device__ __forceinline__ void mstate_store(gu32 *__restrict__ p, const MState<MT, NT> &a) {
#pragma unroll
    for (int mt = 0; mt < MT; mt++)
#pragma unroll
        for (int nt = 0; nt < NT; nt++) {
            p[(mt * NT + nt) * 64] = a.b[mt][nt];
            p[(MT * NT + mt * NT + nt) * 64] = a.p[mt][nt];
        }
#pragma unroll
    for (int nt = 0; nt < NT; nt++) p[(2 * MT * NT + nt) * 64] = a.r[nt];
}

template <int MT, int NT>
__device__ __forceinline__ void mstate_load(const gu32 *__restrict__ p, MState<MT, NT> &a) {
#pragma unroll
    for (int mt = 0; mt < MT; mt++)
#pragma unroll
        for (int nt = 0; nt < NT; nt++) {
            a.b[mt][nt] = p[(mt * NT + nt) * 64];
            a.p[mt][nt] = p[(MT * NT + mt * NT + nt) * 64];
        }
#pragma unroll
    for (int nt = 0; nt < NT; nt++) a.r[nt] = p[(2 * MT * NT + nt) * 64];
}

// The same in LDS (p = this wave's buffer + lane): each wave reads and
// writes only its own buffer, so program order (and, after the prefetch,
// vmem_drain) orders the accesses.
template <int MT, int NT>
__device__ __forceinline__ void mstate_store_lds(uint32_t *p, const MState<MT, NT> &a) {
#pragma unroll
    for (int mt = 0; mt < MT; mt++)
#pragma unroll
        for (int nt = 0; nt < NT; nt++) {
            p[(mt * NT + nt) * 64] = a.b[mt][nt];
            p[(MT * NT + mt * NT + nt) * 64] = a.p[mt][nt];
        }
#pragma unroll
    for (int nt = 0; nt < NT; nt++) p[(2 * MT * NT + nt) * 64] = a.r[nt];
}

template <int MT, int NT>
__device__ __forceinline__ void mstate_load_lds(const uint32_t *p, MState<MT, NT> &a) {
#pragma unroll
    for (int mt = 0; mt < MT; mt++)
#pragma unroll
        for (int nt = 0; nt < NT; nt++) {
            a.b[mt][nt] = p[(mt * NT + nt) * 64];
            a.p[mt][nt] = p[(MT * NT + mt * NT + nt) * 64];
        }
#pragma unroll
    for (int nt = 0; nt < NT; nt++) a.r[nt] = p[(2 * MT * NT + nt) * 64];
}

// y = 1 in the kept representation: 2^32 mod m in B, 2^32 M^-1 mod m' in B'
// (read from the table when needed rather than held in registers).  With
// scaled B residues (SQ) the B part is 2^32 s_i, except for the entry
// product, whose first operand comes from the entry table unscaled: there
// sigma_i c_i, so that its quotient digit is still one REDC and its result
// scaled.
template <int K, int W, int MT, int NT, bool SQ = false>
__device__ __forceinline__ void mstate_unit(const MConstOf<K, W, MT, NT> &C, const gu32 *__restrict__ mb,
                                            const gu32 *__restrict__ mk, bool entry, int wave, int lane,
                                            MState<MT, NT> &y) {
    using S = MShp<K, W, MT, NT>;
#pragma unroll
    for (int mt = 0; mt < MT; mt++) {
        const size_t sl = (size_t)wave * MT + mt;
        const uint32_t kap = mb[S::LY.slotP() + (sl * 4 + 3) * 64 + lane];
        uint32_t ub = 0u - C.slotB(mt).m;
        if (SQ) ub = entry ? mk[S::LY.slotC() + sl * 64 + lane] : mk[S::LY.sqB() + (sl * 3 + 1) * 64 + lane];
#pragma unroll
        for (int nt = 0; nt < NT; nt++) {
            y.b[mt][nt] = ub;
            y.p[mt][nt] = kap;
        }
    }
#pragma unroll
    for (int nt = 0; nt < NT; nt++) y.r[nt] = 1u;
}

// Limb l of a shared (wave-uniform) exponent, through the scalar unit: read
// through the constant address space at a uniform index it is a scalar load
// (its wait is on the scalar counter, so it never waits for the vector
// memory operations in flight, such as the operand prefetch).
typedef const __attribute__((address_space(4))) uint32_t ku32;
__device__ __forceinline__ uint32_t mexp_limb(const gu32 *__restrict__ e, int l) {
    return ((ku32 *)e)[__builtin_amdgcn_readfirstlane(l)];
}

// Wait until every vector memory operation of this wave has completed
// (s_waitcnt vmcnt(0): on this target the immediate holds vmcnt in bits 3:0
// and 15:14, expcnt in 6:4, lgkmcnt in 11:8; the others stay at their maximum).
__device__ __forceinline__ void vmem_drain() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// One row of the operand prefetch: lane l's word src[l] lands in LDS at
// dst[l] without passing through registers (global_load_lds_dword; M0 holds
// the wave-uniform LDS byte address of dst).  Issued as inline assembly so the
// compiler adds no waits of its own for it: its only reader waits with
// vmem_drain() first, and vector loads complete in issue order, so the
// compiler's counts for its own loads stay valid.
__device__ __forceinline__ void lds_dma_row(const gu32 *src, uint32_t *dst) {
    const uint32_t m0v = (uint32_t)(size_t)(__attribute__((address_space(3))) void *)dst;
    asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dword %1, off" ::"s"(m0v), "v"(src) : "memory");
}

// Bit i of a shared exponent.
__device__ __forceinline__ uint32_t mexp_bit(const gu32 *__restrict__ e, int i) {
    return (mexp_limb(e, i >> 5) >> (i & 31)) & 1u;
}

// Highest set bit of a shared exponent of n limbs, -1 if it is zero.
__device__ __forceinline__ int mexp_top_bit(const gu32 *__restrict__ e, int n) {
    for (int l = n - 1; l >= 0; l--) {
        const uint32_t v = mexp_limb(e, l);
        if (v) return 32 * l + 31 - __builtin_clz(v);
    }
    return -1;
}

// Sliding window of a shared exponent whose bit i is set: the bits i..low
// with low >= i - w + 1 the lowest set bit in that range; returns their value
// (odd, < 2^w) and low.
__device__ __forceinline__ uint32_t mexp_window(const gu32 *__restrict__ e, int n, int i, int w, int *low) {
    int lo = i - w + 1 > 0 ? i - w + 1 : 0;
    while (!mexp_bit(e, lo)) lo++;
    const int l = lo >> 5;
    uint64_t v = mexp_limb(e, l);
    if (l + 1 < n) v |= (uint64_t)mexp_limb(e, l + 1) << 32;
    *low = lo;
    return (uint32_t)(v >> (lo & 31)) & ((1u << (i - lo + 1)) - 1u);
}

__device__ __forceinline__ uint32_t mexp_digit(const gu32 *__restrict__ e, int nlimbs, int nd, int w, int di) {
    const int lo = (nd - 1 - di) * w;
    const int limb = lo >> 5, sh = lo & 31;
    uint64_t v = e[limb];
    if (limb + 1 < nlimbs) v |= (uint64_t)e[limb + 1] << 32;
    return (uint32_t)(v >> sh) & ((1u << w) - 1u);
}

// Elements the tile of job J serves: its first tile_elems columns (all 16*NT
// when tile_elems is 0).
__device__ __forceinline__ int mjob_tile_elems(const MJob &J, int NM) {
    return J.tile_elems > 0 && J.tile_elems < NM ? J.tile_elems : NM;
}

// End of the exit on wave 0, lane n (element n of the tile, message msg):
// acc holds the L+1 limbs of sum_j xi'_j M'_j; subtracts alpha M', takes the
// canonical representative mod N by conditional subtractions of N 2^b, and
// stores the L limbs (columns beyond the tile's elements store nothing).
template <int K, int W, int MT, int NT>
__device__ __forceinline__ void mfma_exit_tail(const gu32 *__restrict__ mb, const gu32 *__restrict__ mk, uint32_t *acc,
                                               uint32_t *tmp, uint32_t alpha, int L, int n, int msg, const MJob &J,
                                               gu32 *__restrict__ out) {
    using S = MShp<K, W, MT, NT>;
    constexpr int NM = S::NM;
    {
        uint64_t carry = 0;
        uint32_t borrow = 0;
        for (int l = 0; l <= L; l++) {
            const uint64_t p = (uint64_t)alpha * mb[S::LY.MpF() + l] + carry;
            carry = p >> 32;
            const uint32_t v = acc[l * NM + n], pl = (uint32_t)p;
            const uint32_t d = v - pl, d2 = d - borrow;
            borrow = (v < pl) | (d < borrow);
            acc[l * NM + n] = d2;
        }
    }
    for (int b = S::qbits() - 1; b >= 0; b--) {
        uint32_t borrow = 0;
        for (int l = 0; l <= L; l++) {
            const uint32_t nlo = l < L ? mk[S::LY.Nl() + l] : 0u;
            const uint32_t nhi = (b && l > 0) ? (mk[S::LY.Nl() + l - 1] >> (32 - b)) : 0u;
            const uint32_t nl = (nlo << b) | nhi;
            const uint32_t v = acc[l * NM + n];
            const uint32_t d = v - nl, d2 = d - borrow;
            borrow = (v < nl) | (d < borrow);
            tmp[l * NM + n] = d2;
        }
        if (!borrow)
            for (int l = 0; l <= L; l++) acc[l * NM + n] = tmp[l * NM + n];
    }
    if (msg < J.batch && n < mjob_tile_elems(J, NM))
        for (int l = 0; l < L; l++) out[(size_t)msg * J.out_stride + l] = acc[l * NM + n];
}

// Workgroup set-up shared by the kernels of the matrix-core engine: the
// constant digit rows of both exchange buffers (channel K holds the offset
// digit 1, the channels after it zero) and the per-lane constants of C (tiles
// in registers, LDS or global memory, per-slot constants, scalars).
template <int K, int W, int MT, int NT, bool SQ = false>
__device__ __forceinline__ void mfma_setup(const gu32 *__restrict__ mb, const gu32 *__restrict__ mk,
                                           uint32_t *__restrict__ lds, int wave, int lane,
                                           MConstOf<K, W, MT, NT> &C) {
    using S = MShp<K, W, MT, NT>;
    static_assert(!SQ || (S::LY.sq_ok() && !S::A2_GLOBAL && !S::C_LDS), "scaled B residues need per-key tiles in registers or LDS");
    // second extension's tiles and nu: the base's, or the key's scaled ones
    const gu32 *__restrict__ a2src = SQ ? mk + S::LY.a2s() : mb + S::LY.a2();
    uint32_t *buf1 = lds;
    uint32_t *buf2 = lds + S::NM * S::BROW;
    const int g = lane >> 4;
    // constant digit rows: channel K holds the offset digit 1, the rest zero
    for (int i = threadIdx.x; i < S::NM * (S::BROW - K); i += 64 * W) {
        const int n = i / (S::BROW - K), c = K + i % (S::BROW - K);
        const uint32_t v = c == K ? 1u : 0u;
        buf1[n * S::BROW + c] = v;
        buf2[n * S::BROW + c] = v;
    }

    // per-lane constants
#pragma unroll
    for (int mt = 0; mt < MT; mt++) {
        const size_t sl = (size_t)wave * MT + mt;
#pragma unroll
        for (int ks = 0; ks < S::KSTEPS; ks++) {
            const size_t ti = ((sl * S::KSTEPS + ks) * 64 + lane) * 4;
            if (!S::A1_GLOBAL) C.A1[mt][ks] = *(gcv4i *)(mk + S::LY.a1() + ti);
            if (!S::A2_LDS && !S::A2_GLOBAL) C.A2[mt][ks] = *(gcv4i *)(a2src + ti);
        }
        if (!S::C_LDS) {
            C.mB[mt] = mb[S::LY.slotB() + (sl * 3 + 0) * 64 + lane];
            C.uB[mt] = mb[S::LY.slotB() + (sl * 3 + 1) * 64 + lane];
            C.mP[mt] = mb[S::LY.slotP() + (sl * 4 + 0) * 64 + lane];
            C.uP[mt] = mb[S::LY.slotP() + (sl * 4 + 1) * 64 + lane];
            C.nuB[mt] = SQ ? mk[S::LY.sqB() + (sl * 3 + 0) * 64 + lane] : mb[S::LY.slotB() + (sl * 3 + 2) * 64 + lane];
            C.HP[mt] = mb[S::LY.slotP() + (sl * 4 + 2) * 64 + lane];
            if (!SQ) C.cB[mt] = mk[S::LY.slotC() + sl * 64 + lane];
        }
    }
    if (S::C_LDS) {
        // [W][MT][group][m, u, nu, c, m', u', H, 0]; a slot's constants are
        // the same for the 16 lanes of its lane group
        uint32_t *cl = lds + S::WORK_WORDS + S::A2_WORDS;
        for (int i = threadIdx.x; i < W * MT * 4 * 8; i += 64 * W) {
            const int f = i & 7, gi = (i >> 3) & 3;
            const size_t sl = (size_t)(i >> 5);
            const int ln = 16 * gi;
            uint32_t v = 0;
            if (f < 3) v = mb[S::LY.slotB() + (sl * 3 + f) * 64 + ln];
            else if (f == 3) v = mk[S::LY.slotC() + sl * 64 + ln];
            else if (f < 7) v = mb[S::LY.slotP() + (sl * 4 + (f - 4)) * 64 + ln];
            cl[i] = v;
        }
        C.cl = cl + ((size_t)wave * MT * 4 + g) * 8;
        __syncthreads();
    }
    if (S::A2_LDS) {
        // each wave copies its own tiles; it alone reads them, so program
        // order suffices (no barrier)
        mfma_v4i *dst = (mfma_v4i *)(lds + S::WORK_WORDS) + (size_t)wave * MT * S::KSTEPS * 64;
        gcv4i *src = (gcv4i *)a2src + (size_t)wave * MT * S::KSTEPS * 64;
        for (int i = lane; i < MT * S::KSTEPS * 64; i += 64) dst[i] = src[i];
        C.a2lds = dst;
    }
    if (S::A2_GLOBAL) C.a2mem = (gcv4i *)(mb + S::LY.a2()) + (size_t)wave * MT * S::KSTEPS * 64;
    if (S::A1_GLOBAL) C.a1mem = (gcv4i *)(mk + S::LY.a1()) + (size_t)wave * MT * S::KSTEPS * 64;
    C.loff = 16u * lane;
    asm volatile("" : "+v"(C.loff));   // one offset register for every tile load
    C.Mpinv_r = mb[S::LY.bscal() + 0];
    C.Minv_r = mb[S::LY.bscal() + 1];
    C.N_r = mk[S::LY.kscal() + 0];
#pragma unroll
    for (int b = 0; b < 4; b++) {
        C.kf[b] = 1 << (8 * b);
        asm volatile("" : "+s"(C.kf[b]));
    }

}

// One tile of exponentiation job J: columns n < 16*NT hold elements e0 + n
// of the job (those with n < mjob_tile_elems(J) are stored), with window
// table slot `slot` of the launch;
// ylds: the operand prefetch buffer (S::PF_WORDS words, if S::PREFETCH).
template <int K, int W, int MT, int NT, bool SQ = false>
__device__ __forceinline__ void modexp_mfma_tile(const MJob &J, int e0, uint32_t *__restrict__ lds,
                                                 uint32_t *__restrict__ table, size_t slot, int max_window,
                                                 uint32_t *__restrict__ ylds) {
    using S = MShp<K, W, MT, NT>;
    uint32_t *buf1 = lds;
    uint32_t *buf2 = lds + S::NM * S::BROW;
    const gu32 *__restrict__ mb = (const gu32 *)J.mb;
    const gu32 *__restrict__ mk = (const gu32 *)J.mk;
    const gu32 *__restrict__ E = (const gu32 *)J.E;
    const gu32 *__restrict__ ex = (const gu32 *)J.exp;
    const gu32 *__restrict__ in = (const gu32 *)J.in;
    gu32 *__restrict__ out = (gu32 *)J.out;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4;

    MConstOf<K, W, MT, NT> C;
    mfma_setup<K, W, MT, NT, SQ>(mb, mk, lds, wave, lane, C);

    // entry: residues of Z = sum_h X_h Y_h in the kept representation
    MState<MT, NT> a;
    {
        Acc ab[MT][NT], ap[MT][NT];
        uint32_t zr[NT];
        int msg[NT];
#pragma unroll
        for (int nt = 0; nt < NT; nt++) {
            msg[nt] = e0 + 16 * nt + (lane & 15);
            zr[nt] = 0;
        }
        const int colB = wave * 4 * MT + g, colP = W * 4 * MT + wave * 4 * MT + g;
        for (int l = 0; l < J.in_limbs; l++) {
            const gu32 *__restrict__ row = E + (size_t)l * S::ECOLS;
            uint32_t v[NT];
#pragma unroll
            for (int nt = 0; nt < NT; nt++)
                v[nt] = msg[nt] < J.batch ? in[(size_t)msg[nt] * J.in_stride + l] : 0u;
            const uint32_t er = row[S::ECOLS - 1];
#pragma unroll
            for (int mt = 0; mt < MT; mt++) {
                const uint32_t eb = row[colB + 4 * mt], ep = row[colP + 4 * mt];
#pragma unroll
                for (int nt = 0; nt < NT; nt++) {
                    acc_mac(ab[mt][nt], v[nt], eb);
                    acc_mac(ap[mt][nt], v[nt], ep);
                }
            }
#pragma unroll
            for (int nt = 0; nt < NT; nt++) zr[nt] += v[nt] * er;
        }
#pragma unroll
        for (int mt = 0; mt < MT; mt++)
#pragma unroll
            for (int nt = 0; nt < NT; nt++) {
                const MSlotB sb = C.slotB(mt);
                const MSlotP sp = C.slotP(mt);
                a.b[mt][nt] = acc_redc(ab[mt][nt], sb.m, sb.u);
                a.p[mt][nt] = acc_redc(ap[mt][nt], sp.m, sp.u);
            }
#pragma unroll
        for (int nt = 0; nt < NT; nt++) a.r[nt] = zr[nt];
    }
    const int w = J.window;
    const int T = 1 << w;
    const size_t estride = (size_t)W * S::SLOTS * 64;
    gu32 *__restrict__ tw = (gu32 *)table + ((slot << max_window) * W + wave) * (size_t)(S::SLOTS * 64) + lane;
    {
        MState<MT, NT> one;
#pragma unroll
        for (int mt = 0; mt < MT; mt++) {
            const size_t sl = (size_t)wave * MT + mt;
#pragma unroll
            for (int nt = 0; nt < NT; nt++) {
                one.b[mt][nt] = SQ ? mk[S::LY.sqB() + (sl * 3 + 2) * 64 + lane] : mk[S::LY.one() + (sl * 2 + 0) * 64 + lane];
                one.p[mt][nt] = mk[S::LY.one() + (sl * 2 + 1) * 64 + lane];
            }
        }
        const uint32_t onr = mk[S::LY.one() + (size_t)W * MT * 2 * 64];
#pragma unroll
        for (int nt = 0; nt < NT; nt++) one.r[nt] = onr;
        mstate_store<MT, NT>(tw, one);   // T[0] = M mod N
    }

    // Exponent schedule.  Shared exponent: left-to-right sliding windows of
    // at most w bits that start and end with a set bit, over a table of the
    // odd powers x, x^3, ..., x^(2^w - 1) (built with x^2); the windows are
    // found on the scalar unit.  Per-element exponents: fixed w-bit digits
    // over the full table x^0 .. x^(2^w - 1).  The control picks where the
    // next product's second operand comes from.  Squarings take their own
    // copy of the product (no operand copy).  With the prefetch buffer, the
    // constant operand of the table build (x^2, or x for per-element
    // exponents) stays in it, and the table entry of each window
    // multiplication is copied into it when the window is found, one or more
    // squarings ahead (Y_PREF_DMA waits for that copy).  Every other operand
    // load is drained where it is issued, so a product never waits for vector
    // memory and the copy in flight overlaps the squarings.
    const bool shared_exp = J.exp_stride == 0;
    const int nbits = 32 * J.exp_limbs;
    const int nd = (nbits + w - 1) / w;
    enum { ENTRY, SQX, BUILD, MAIN, EXIT };
    enum { Y_SQUARE, Y_UNIT, Y_TABLE, Y_ELEM, Y_PREF, Y_PREF_DMA };
    uint32_t *yb = ylds + (size_t)wave * S::SLOTS * 64;   // this wave's prefetch buffer, [slot][lane]
    int phase = ENTRY, j = 2, di = 0, s = 0;
    int bitpos = -1, sq = 0;
    uint32_t dm = 0;
    int ysrc = Y_UNIT, yidx = 0;
    for (;;) {
        if (ysrc == Y_SQUARE) {
            mfma_mm<K, W, MT, NT, SQ>(C, a, a, buf1, buf2, wave, lane, true);
        } else {
            MState<MT, NT> y;
            if (ysrc == Y_UNIT) {
                mstate_unit<K, W, MT, NT, SQ>(C, mb, mk, phase == ENTRY, wave, lane, y);
                vmem_drain();
            } else if (ysrc == Y_TABLE) {
                mstate_load<MT, NT>(tw + (size_t)yidx * estride, y);
                vmem_drain();
            } else if (ysrc == Y_PREF || ysrc == Y_PREF_DMA) {
                if (ysrc == Y_PREF_DMA) vmem_drain();   // the entry copied at the window's start has landed
                mstate_load_lds<MT, NT>(yb + lane, y);
            } else {
                // per-element exponents: each lane slot loads the entry of its own element
#pragma unroll
                for (int nt = 0; nt < NT; nt++) {
                    const int m = e0 + 16 * nt + (lane & 15);
                    const gu32 *__restrict__ ep = ex + (size_t)(m < J.batch ? m : 0) * J.exp_stride;
                    const uint32_t d = mexp_digit(ep, J.exp_limbs, nd, w, yidx);
                    const gu32 *__restrict__ pe = tw + (size_t)d * estride;
#pragma unroll
                    for (int mt = 0; mt < MT; mt++) {
                        y.b[mt][nt] = pe[(mt * NT + nt) * 64];
                        y.p[mt][nt] = pe[(MT * NT + mt * NT + nt) * 64];
                    }
                    y.r[nt] = pe[(2 * MT * NT + nt) * 64];
                }
                vmem_drain();
            }
            mfma_mm<K, W, MT, NT, SQ>(C, a, y, buf1, buf2, wave, lane, phase != EXIT);
        }
        if (phase == EXIT) break;
        if (phase == ENTRY) {
            mstate_store<MT, NT>(tw + estride, a);               // T[1] = x
            if (w > 1) {
                if (shared_exp) {
                    phase = SQX;
                    ysrc = Y_SQUARE;
                } else {
                    phase = BUILD;
                    j = 2;
                    if (S::PREFETCH) {
                        mstate_store_lds<MT, NT>(yb + lane, a);  // x, the build's constant operand
                        ysrc = Y_PREF;
                    } else {
                        ysrc = Y_TABLE;
                        yidx = 1;
                    }
                }
                continue;
            }
        } else if (phase == SQX) {
            if (S::PREFETCH) {
                mstate_store_lds<MT, NT>(yb + lane, a);          // x^2, the build's constant operand
            } else {
                mstate_store<MT, NT>(tw + 2 * estride, a);       // x^2, slot 2 (even: unused by the windows)
            }
            mstate_load<MT, NT>(tw + estride, a);
            vmem_drain();
            phase = BUILD;
            j = 3;
            ysrc = S::PREFETCH ? Y_PREF : Y_TABLE;
            yidx = 2;
            continue;
        } else if (phase == BUILD) {
            mstate_store<MT, NT>(tw + (size_t)j * estride, a);  // T[j] = T[j - step] * (x^2 or x)
            j += shared_exp ? 2 : 1;
            if (j < T) {
                ysrc = S::PREFETCH ? Y_PREF : Y_TABLE;
                yidx = shared_exp ? 2 : 1;
                continue;
            }
        }
        if (phase != MAIN) {
            phase = MAIN;
            if (shared_exp) {
                bitpos = mexp_top_bit(ex, J.exp_limbs);
                if (bitpos < 0) {
                    mstate_load<MT, NT>(tw, a);                   // e = 0: the result is 1
                } else {
                    int low;
                    const uint32_t d = mexp_window(ex, J.exp_limbs, bitpos, w, &low);
                    mstate_load<MT, NT>(tw + (size_t)d * estride, a);
                    bitpos = low - 1;
                }
            } else {
                mstate_load<MT, NT>(tw, a);
            }
            vmem_drain();
        }
        if (shared_exp) {
            if (sq > 0) {                                          // squarings of the current window
                ysrc = Y_SQUARE;
                sq--;
            } else if (dm) {                                       // its multiplication
                ysrc = S::PREFETCH ? Y_PREF_DMA : Y_TABLE;
                yidx = (int)dm;
                dm = 0;
            } else if (bitpos < 0) {
                phase = EXIT;
                ysrc = Y_UNIT;
            } else {
                ysrc = Y_SQUARE;                                   // a square in any case
                if (mexp_bit(ex, bitpos)) {
                    int low;
                    dm = mexp_window(ex, J.exp_limbs, bitpos, w, &low);
                    if (S::PREFETCH) {
                        const gu32 *src = tw + (size_t)dm * estride;
#pragma unroll
                        for (int r = 0; r < S::SLOTS; r++) lds_dma_row(src + r * 64, yb + r * 64);
                    }
                    sq = bitpos - low;
                    bitpos = low - 1;
                } else {
                    bitpos--;
                }
            }
        } else {
            if (di >= nd) {
                phase = EXIT;
                ysrc = Y_UNIT;
            } else if (s < w) {
                ysrc = Y_SQUARE;
                s++;
            } else {
                di++;
                s = 0;
                ysrc = Y_ELEM;
                yidx = di - 1;
            }
        }
    }

    // leave the RNS
    if constexpr (!S::SPLIT_EXIT) {
        // wave 0, lane n < NM handles element n of the workgroup alone
        __syncthreads();
        if (wave != 0 || lane >= S::NM) return;
        const int n = lane;
        const int msg = e0 + n;
        uint32_t rr = a.r[0];
#pragma unroll
        for (int nt = 1; nt < NT; nt++) rr = (n >> 4) == nt ? a.r[nt] : rr;   // lane n holds element n's r in slot n/16
        const int L = J.L;
        constexpr int NM = S::NM;
        uint32_t *X = lds;                               // [K][NM] xi'_j of the exit product
        uint32_t *acc = lds + K * NM;                    // [L+1][NM]
        uint32_t *tmp = acc + (L + 1) * NM;              // [L+1][NM]
        uint32_t s2 = 0;
        for (int jj = 0; jj < K; jj++) {
            const uint32_t v = buf2[n * S::BROW + jj] ^ kDigitBias;       // xi'_j in [0, m'_j)
            X[jj * NM + n] = v;
            s2 += v * mb[S::LY.mplo() + jj];
        }
        const uint32_t alpha = (s2 - rr) * C.Mpinv_r;                    // in [0, K)
        {
            uint64_t carry = 0;
            for (int l = 0; l <= L; l++) {
                Acc sum;
                sum.lo = carry;
                for (int jj = 0; jj < K; jj++) acc_mac(sum, X[jj * NM + n], mb[S::LY.MpL() + (size_t)jj * (K + 1) + l]);
                uint64_t lo;
                uint32_t top;
                acc_value(sum, lo, top);
                acc[l * NM + n] = (uint32_t)lo;
                carry = (lo >> 32) | ((uint64_t)top << 32);
            }
        }
        {
            uint64_t carry = 0;
            uint32_t borrow = 0;
            for (int l = 0; l <= L; l++) {
                const uint64_t p = (uint64_t)alpha * mb[S::LY.MpF() + l] + carry;
                carry = p >> 32;
                const uint32_t v = acc[l * NM + n], pl = (uint32_t)p;
                const uint32_t d = v - pl, d2 = d - borrow;
                borrow = (v < pl) | (d < borrow);
                acc[l * NM + n] = d2;
            }
        }
        for (int b = S::qbits() - 1; b >= 0; b--) {
            uint32_t borrow = 0;
            for (int l = 0; l <= L; l++) {
                const uint32_t nlo = l < L ? mk[S::LY.Nl() + l] : 0u;
                const uint32_t nhi = (b && l > 0) ? (mk[S::LY.Nl() + l - 1] >> (32 - b)) : 0u;
                const uint32_t nl = (nlo << b) | nhi;
                const uint32_t v = acc[l * NM + n];
                const uint32_t d = v - nl, d2 = d - borrow;
                borrow = (v < nl) | (d < borrow);
                tmp[l * NM + n] = d2;
            }
            if (!borrow)
                for (int l = 0; l <= L; l++) acc[l * NM + n] = tmp[l * NM + n];
        }
        if (msg < J.batch && n < mjob_tile_elems(J, NM))
            for (int l = 0; l < L; l++) out[(size_t)msg * J.out_stride + l] = acc[l * NM + n];
    } else {
        __syncthreads();
        const int L = J.L;
        constexpr int NM = S::NM;
        uint32_t *X = lds;                           // [K][NM] xi'_j of the exit product
        uint32_t *acc = lds + K * NM;                // [L+1][NM]
        uint32_t *tmp = acc + (L + 1) * NM;          // [L+1][NM]
        // wave 0 (lane n < NM: element n) gathers xi'_j and alpha; then every
        // wave and lane group sums a contiguous range of the limbs of
        // sum_j xi'_j M'_j (the range sums are independent); wave 0 adds the
        // carries between the ranges and finishes
        uint32_t *cout = lds + S::EXIT_CORE;         // [workers][2][NM]
        uint32_t alpha = 0;
        if (wave == 0 && lane < NM) {
            const int n = lane;
            uint32_t rr = a.r[0];
#pragma unroll
            for (int nt = 1; nt < NT; nt++) rr = (n >> 4) == nt ? a.r[nt] : rr;
            uint32_t s2 = 0;
            for (int jj = 0; jj < K; jj++) {
                const uint32_t v = buf2[n * S::BROW + jj] ^ kDigitBias;
                X[jj * NM + n] = v;
                s2 += v * mb[S::LY.mplo() + jj];
            }
            alpha = (s2 - rr) * C.Mpinv_r;
        }
        __syncthreads();
        constexpr int NW = W * (64 / NM);            // workers per element
        const int CW = (L + 1 + NW - 1) / NW;        // limbs per worker
        {
            const int n = lane % NM, wid = wave * (64 / NM) + lane / NM;
            const int l0 = wid * CW < L + 1 ? wid * CW : L + 1;
            const int l1 = l0 + CW < L + 1 ? l0 + CW : L + 1;
            uint64_t carry = 0;
            for (int l = l0; l < l1; l++) {
                Acc sum;
                sum.lo = carry;
                for (int jj = 0; jj < K; jj++)
                    acc_mac(sum, X[jj * NM + n], mb[S::LY.MpL() + (size_t)jj * (K + 1) + l]);
                uint64_t lo;
                uint32_t top;
                acc_value(sum, lo, top);
                acc[l * NM + n] = (uint32_t)lo;
                carry = (lo >> 32) | ((uint64_t)top << 32);
            }
            cout[2 * NM * wid + n] = (uint32_t)carry;
            cout[2 * NM * wid + NM + n] = (uint32_t)(carry >> 32);
        }
        __syncthreads();
        if (wave != 0 || lane >= NM) return;
        const int n = lane;
        ripple_carries(acc + n, NM, L + 1, cout + n, NM, NW, CW);
        mfma_exit_tail<K, W, MT, NT>(mb, mk, acc, tmp, alpha, L, n, e0 + n, J, out);
    }
}

// Exponentiation kernel, matrix-core variant: workgroup t runs tile t of the
// A.njobs jobs of one shape, which belongs to the job j with
// jobs[j].tile0 <= t < jobs[j+1].tile0.  (A resident loop that takes tiles
// from a counter costs 15-35 more VGPRs per lane here, as the compiler keeps
// the per-lane addresses of the tile body live across it; the hardware
// dispatcher refills the CUs as workgroups finish instead.)
template <int K, int W, int MT, int NT, bool SQ>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(MShp<K, W, MT, NT>::WAVES_PER_EU)))
void modexp_mfma_kernel(ModexpMfmaLaunch A) {
    using S = MShp<K, W, MT, NT>;
    __shared__ __attribute__((aligned(16))) uint32_t lds[S::LDS_WORDS];
    __shared__ __attribute__((aligned(16))) uint32_t ylds[S::PREFETCH ? S::PF_WORDS : 1];
    const int tile = blockIdx.x;
    MJob J;
    if (A.jobs) {
        int lo = 0, hi = A.njobs - 1;          // last job with tile0 <= tile
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (A.jobs[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
        }
        J = A.jobs[lo];
    } else {
        J = (A.njobs > 1 && tile >= A.inl[1].tile0) ? A.inl[1] : A.inl[0];
    }
    modexp_mfma_tile<K, W, MT, NT, SQ>(J, (tile - J.tile0) * mjob_tile_elems(J, S::NM), lds, A.table, blockIdx.x,
                                       A.max_window, ylds);
}

template <int K, int W, int MT, int NT>
hipError_t launch_modexp_mfma_t(const ModexpMfmaLaunch &a, hipStream_t s) {
    using S = MShp<K, W, MT, NT>;
    if (a.tiles <= 0) return hipSuccess;
    if constexpr (S::LY.sq_ok() && !S::A2_GLOBAL && !S::C_LDS) {
        if (a.scaled) {
            hipLaunchKernelGGL((modexp_mfma_kernel<K, W, MT, NT, true>), dim3((unsigned)a.tiles), dim3(64 * W), 0, s,
                               a);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((modexp_mfma_kernel<K, W, MT, NT, false>), dim3((unsigned)a.tiles), dim3(64 * W), 0, s, a);
    return hipGetLastError();
}

// One RNS Montgomery product per element on the matrix cores, for the
// standalone call: residues in and out channel-major ([2K+1][batch]: B, B',
// then the redundant channel), plain (each lane converts its slots to the
// kept representation and back with the base table's conversion factors).
// Workgroup t serves elements [t*E, (t+1)*E), E = A.tile_elems (0: 16*NT).
template <int K, int W, int MT, int NT>
__global__ __launch_bounds__(64 * W) void montmul_mfma_kernel(MontMulMfmaLaunch A) {
    using S = MShp<K, W, MT, NT>;
    __shared__ __attribute__((aligned(16))) uint32_t lds[S::LDS_WORDS];
    const gu32 *__restrict__ mb = (const gu32 *)A.mb;
    const gu32 *__restrict__ mk = (const gu32 *)A.mk;
    const gu32 *__restrict__ x = (const gu32 *)A.x;
    const gu32 *__restrict__ y = (const gu32 *)A.y;
    gu32 *__restrict__ out = (gu32 *)A.out;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4;
    MConstOf<K, W, MT, NT> C;
    mfma_setup<K, W, MT, NT>(mb, mk, lds, wave, lane, C);
    const int te = A.tile_elems > 0 && A.tile_elems < S::NM ? A.tile_elems : S::NM;
    const size_t B = (size_t)A.batch;
    int elem[NT];
    bool ok[NT];
#pragma unroll
    for (int nt = 0; nt < NT; nt++) {
        const int n = 16 * nt + (lane & 15);
        elem[nt] = (int)blockIdx.x * te + n;
        ok[nt] = n < te && elem[nt] < A.batch;
    }
    MState<MT, NT> a, b;
#pragma unroll
    for (int mt = 0; mt < MT; mt++) {
        const size_t sl = (size_t)wave * MT + mt;
        const int ch = wave * S::CH + 4 * mt + g;
        const bool real = (4 * mt + g != 4 * MT - 1) && ch < K;
        const uint32_t inB = mb[S::LY.mmconv() + (sl * 3 + 0) * 64 + lane];
        const uint32_t inP = mb[S::LY.mmconv() + (sl * 3 + 1) * 64 + lane];
        const MSlotB sb = C.slotB(mt);
        const MSlotP sp = C.slotP(mt);
#pragma unroll
        for (int nt = 0; nt < NT; nt++) {
            const bool ld = real && ok[nt];
            const size_t e = (size_t)elem[nt];
            a.b[mt][nt] = mulredc(ld ? x[(size_t)ch * B + e] : 0u, inB, sb.m, sb.u);   // x R mod m
            b.b[mt][nt] = mulredc(ld ? y[(size_t)ch * B + e] : 0u, inB, sb.m, sb.u);
            a.p[mt][nt] = mulredc(ld ? x[(size_t)(K + ch) * B + e] : 0u, inP, sp.m, sp.u);   // x R M^-1 mod m'
            b.p[mt][nt] = mulredc(ld ? y[(size_t)(K + ch) * B + e] : 0u, inP, sp.m, sp.u);
        }
    }
#pragma unroll
    for (int nt = 0; nt < NT; nt++) {
        a.r[nt] = ok[nt] ? x[(size_t)2 * K * B + elem[nt]] : 0u;
        b.r[nt] = ok[nt] ? y[(size_t)2 * K * B + elem[nt]] : 0u;
    }
    uint32_t *buf1 = lds;
    uint32_t *buf2 = lds + S::NM * S::BROW;
    mfma_mm<K, W, MT, NT>(C, a, b, buf1, buf2, wave, lane, true);
#pragma unroll
    for (int mt = 0; mt < MT; mt++) {
        const size_t sl = (size_t)wave * MT + mt;
        const int ch = wave * S::CH + 4 * mt + g;
        const bool real = (4 * mt + g != 4 * MT - 1) && ch < K;
        const uint32_t outP = mb[S::LY.mmconv() + (sl * 3 + 2) * 64 + lane];
        const MSlotB sb = C.slotB(mt);
        const MSlotP sp = C.slotP(mt);
#pragma unroll
        for (int nt = 0; nt < NT; nt++) {
            if (!real || !ok[nt]) continue;
            const size_t e = (size_t)elem[nt];
            out[(size_t)ch * B + e] = mulredc(a.b[mt][nt], 1u, sb.m, sb.u);
            out[(size_t)(K + ch) * B + e] = mulredc(a.p[mt][nt], outP, sp.m, sp.u);
        }
    }
    if (wave == 0 && g == 0)
#pragma unroll
        for (int nt = 0; nt < NT; nt++)
            if (ok[nt]) out[(size_t)2 * K * B + elem[nt]] = a.r[nt];
}

template <int K, int W, int MT, int NT>
hipError_t launch_montmul_mfma_t(const MontMulMfmaLaunch &a, hipStream_t s) {
    if (a.tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL((montmul_mfma_kernel<K, W, MT, NT>), dim3((unsigned)a.tiles), dim3(64 * W), 0, s, a);
    return hipGetLastError();
}

// Resident workgroups per CU of the kernel for this shape (occupancy).
template <int K, int W, int MT, int NT>
int mfma_blocks_per_cu_t() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, modexp_mfma_kernel<K, W, MT, NT, false>, 64 * W, 0) != hipSuccess)
        return 0;
    return n;
}

}  // namespace rnsrsa
