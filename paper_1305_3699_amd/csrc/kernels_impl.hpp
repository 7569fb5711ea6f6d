// RNS modular exponentiation kernels for gfx950.
//
// Data layout ("message per lane, channels split across waves"): a workgroup
// of W wavefronts serves 64 elements, one per lane index.  Wave w owns the
// channels [w*KS, (w+1)*KS) of each base (KS = ceil(K/W)), so the per-channel
// steps of the RNS Montgomery product and the rows of both base extensions
// are split over the W waves; every constant a wave touches is the same for
// all its lanes and is fetched with scalar loads.  The redundant 2^32 channel
// is carried by every wave.  Between the two halves of a product the waves
// exchange the quotient digits xi_i (and later xi'_j) through LDS, laid out
// [channel][lane] so every LDS access is conflict-free.
//
// RNS Montgomery product of X and Y over bases B, B' and the redundant
// channel m_r = 2^32 (Sec. 3.1, after Bajard et al. 2001):
//   (i)   xi_i  = |x_i y_i (-N^-1 M_i^-1)|_{m_i}                    in B
//   (ii)  q^_t  = |sum_i xi_i M_i|_{m_t}          first base extension to B', m_r
//   (iii) r_t   = |(x_t y_t + q^_t N) M^-1|_{m_t}                   in B', m_r
//   (iv)  xi'_t = |r_t (M'_t)^-1|_{m'_t};  alpha = |(sum_t xi'_t M'_t - r) M'^-1|_{2^32}
//         r_i   = |sum_t xi'_t M'_t - alpha M'|_{m_i}   exact second extension to B
// r = (XY + q^ N)/M is an exact integer below (k+1)N for inputs below (k+1)N.
#pragma once

#include "arith.hpp"
#include "kernels.hpp"

namespace rnsrsa {

template <int K, int W>
struct Shp {
    static constexpr int KS = (K + W - 1) / W;
    static constexpr int KP = KS * W;
    static constexpr int SLOTS = 2 * KS + 1;  // per-wave slots of one table entry
    static constexpr int NT = 64 * W;
    // smallest b with 2^b > K: an exit value below (K+1)N has quotient < 2^b
    static constexpr int qbits() {
        int b = 0;
        while ((1 << b) <= K) b++;
        return b;
    }
    // unroll factor of the K-long base-extension loops (bounds code size)
    static constexpr int UNR = 4;
    // output channels accumulated per pass over a base extension's inputs:
    // all of them, except in workgroups of more than 8 waves (at most 128
    // registers per lane), where 17 channels' accumulators would spill; those
    // make several passes, re-reading the digits from LDS
    static constexpr int KC = W > 8 ? 6 : KS;
};

template <int KS>
struct Res {
    uint32_t b[KS];  // owned channels of B
    uint32_t p[KS];  // owned channels of B'
    uint32_t r;      // redundant channel
};

template <int KS>
__device__ __forceinline__ void res_set_one(Res<KS> &y) {
#pragma unroll
    for (int c = 0; c < KS; c++) {
        y.b[c] = 1;
        y.p[c] = 1;
    }
    y.r = 1;
}

// One RNS Montgomery product x <- x*y*M^-1 on the owned channels.  With
// full == false the B outputs of the second base extension are skipped (the
// caller only needs xi' in LDS and alpha, to leave the RNS).  Returns alpha.
template <int K, int W>
__device__ __forceinline__ uint32_t rns_mm(const uint32_t *__restrict__ bc,
                                           const uint32_t *__restrict__ mc,
                                           Res<Shp<K, W>::KS> &x, const Res<Shp<K, W>::KS> &y,
                                           uint32_t *lds, int c0, int lane, bool full) {
    using S = Shp<K, W>;
    constexpr int KS = S::KS, KP = S::KP;
    constexpr Layout LY{K, KP};
    // Re-derive the table pointers at every product so the compiler cannot
    // hoist the (loop-invariant) constant loads out of the exponent loop and
    // keep hundreds of them live; per-wave bases let the scalar loads of a
    // channel slice merge into wide s_load_dwordxN.
    int zo;
    asm volatile("s_mov_b32 %0, 0" : "=s"(zo));
    bc += zo;
    mc += zo;
    const uint32_t *__restrict__ bw = bc + c0;   // per-wave slice of per-channel tables
    const uint32_t *__restrict__ mw = mc + c0;
    uint32_t *xi = lds;
    uint32_t *xip = lds + KP * 64;

    // (i) quotient digits in B, published for the first base extension
#pragma unroll
    for (int c = 0; c < KS; c++) {
        const uint32_t m = bw[LY.mB() + c], u = bw[LY.uB() + c];
        const uint32_t t = mulredc(x.b[c], y.b[c], m, u);              // x y R^-1
        xi[(c0 + c) * 64 + lane] = mulredc(t, mw[LY.c2B() + c], m, u); // x y c_i
    }
    // x y R^-1 in B', ahead of the barrier when one pass serves all channels
    constexpr int KC = S::KC;
    constexpr bool ONE_PASS = KC == KS;
    uint32_t a1pre[ONE_PASS ? KS : 1];
    if (ONE_PASS) {
#pragma unroll
        for (int c = 0; c < KS; c++)
            a1pre[c] = mulredc(x.p[c], y.p[c], bw[LY.mBp() + c], bw[LY.uBp() + c]);
    }
    const uint32_t sr = x.r * y.r;
    __syncthreads();

    // (ii) first base extension: q^ in the owned channels of B' and in m_r,
    // in passes of KC channels; (iii) r = (XY + q^ N)/M in B' and m_r,
    // publishing xi' for the second extension
    uint64_t qr = 0;
#pragma unroll
    for (int cc = 0; cc < KS; cc += KC) {
        Acc acc[KC];
#pragma unroll S::UNR
        for (int i = 0; i < K; i++) {
            const uint32_t v = xi[i * 64 + lane];
            const uint32_t *__restrict__ row = bw + LY.C1() + i * LY.crow() + cc;
#pragma unroll
            for (int c = 0; c < KC; c++)
                if (cc + c < KS) acc_mac(acc[c], v, row[c]);
            if (cc == 0) qr += (uint64_t)v * bc[LY.C1() + i * LY.crow() + KP];
        }
#pragma unroll
        for (int c = 0; c < KC; c++) {
            const int ch = cc + c;
            if (ch >= KS) break;
            const uint32_t m = bw[LY.mBp() + ch], u = bw[LY.uBp() + ch];
            const uint32_t a1 = ONE_PASS ? a1pre[ONE_PASS ? ch : 0] : mulredc(x.p[ch], y.p[ch], m, u);
            const uint32_t q = acc_redc(acc[c], m, u);                     // q^ mod m'_t
            const uint32_t a2 = mulredc(q, mw[LY.NnBp() + ch], m, u);      // -q^ N R^-1
            uint32_t s = a1 - a2;
            s = a1 < a2 ? s + m : s;                                        // (XY + q^ N) R^-1
            const uint32_t r = mulredc(s, mw[LY.MiBp() + ch], m, u);       // (XY + q^ N) M^-1
            x.p[ch] = r;
            xip[(c0 + ch) * 64 + lane] = mulredc(r, bw[LY.MpInv() + ch], m, u);  // r (M'_t)^-1
        }
    }
    const uint32_t rr = (sr + (uint32_t)qr * mc[LY.mscal()]) * bc[LY.scal() + 1];
    __syncthreads();

    // (iv) second base extension, exact thanks to alpha from m_r (the first
    // pass also sums the redundant channel, which fixes alpha)
    uint32_t alpha = 0;
    if (full) {
#pragma unroll
        for (int cc = 0; cc < KS; cc += KC) {
            Acc acc2[KC];
            uint64_t s2 = 0;
#pragma unroll S::UNR
            for (int j = 0; j < K; j++) {
                const uint32_t v = xip[j * 64 + lane];
                const uint32_t *__restrict__ row = bw + LY.C2() + j * LY.crow() + cc;
#pragma unroll
                for (int c = 0; c < KC; c++)
                    if (cc + c < KS) acc_mac(acc2[c], v, row[c]);
                if (cc == 0) s2 += (uint64_t)v * bc[LY.C2() + j * LY.crow() + KP];
            }
            if (cc == 0) alpha = ((uint32_t)s2 - rr) * bc[LY.scal()];
#pragma unroll
            for (int c = 0; c < KC; c++) {
                const int ch = cc + c;
                if (ch >= KS) break;
                acc_mac16(acc2[c], alpha, bw[LY.negMp() + ch]);         // alpha < K < 2^16
                x.b[ch] = acc_redc(acc2[c], bw[LY.mB() + ch], bw[LY.uB() + ch]);
            }
        }
    } else {
        uint64_t s2 = 0;
#pragma unroll S::UNR
        for (int j = 0; j < K; j++) s2 += (uint64_t)xip[j * 64 + lane] * bc[LY.C2() + j * LY.crow() + KP];
        alpha = ((uint32_t)s2 - rr) * bc[LY.scal()];
    }
    x.r = rr;
    return alpha;
}

// Z residues of an input of nl limbs: z_t = sum_l in_l E[l][t] (Sec. 3.1's
// binary-to-RNS conversion fused with the multiplication by the entry factors).
template <int K, int W>
__device__ __forceinline__ void rns_entry(const uint32_t *__restrict__ bc, const uint32_t *__restrict__ E,
                                          const uint32_t *__restrict__ src, int nl, bool active,
                                          Res<Shp<K, W>::KS> &a, int c0) {
    using S = Shp<K, W>;
    constexpr int KS = S::KS, KP = S::KP;
    constexpr Layout LY{K, KP};
    Acc ab[KS], ap[KS];
    uint64_t zr = 0;
    const uint32_t *__restrict__ Ew = E + c0;
    for (int l = 0; l < nl; l++) {
        const uint32_t v = active ? src[l] : 0u;
        const uint32_t *__restrict__ row = Ew + l * LY.ecols();
#pragma unroll
        for (int c = 0; c < KS; c++) {
            acc_mac(ab[c], v, row[c]);
            acc_mac(ap[c], v, row[KP + c]);
        }
        zr += (uint64_t)v * E[l * LY.ecols() + 2 * KP];
    }
    const uint32_t *__restrict__ bw = bc + c0;
#pragma unroll
    for (int c = 0; c < KS; c++) {
        a.b[c] = acc_redc(ab[c], bw[LY.mB() + c], bw[LY.uB() + c]);
        a.p[c] = acc_redc(ap[c], bw[LY.mBp() + c], bw[LY.uBp() + c]);
    }
    a.r = (uint32_t)zr;
}

// Limbs [l0, l1) of sum_j xi'_j M'_j into acc[l*64 + lane], carries
// propagated inside the range; returns the carry out of limb l1 - 1.
template <int K, int W>
__device__ __forceinline__ uint64_t exit_columns(const uint32_t *__restrict__ bc, const uint32_t *xip, uint32_t *acc,
                                                 int l0, int l1, int lane) {
    using S = Shp<K, W>;
    constexpr Layout LY{K, S::KP};
    uint64_t carry = 0;
    for (int l = l0; l < l1; l++) {
        const uint32_t *__restrict__ col = bc + LY.MpL() + l;
        Acc s;
        s.lo = carry;
#pragma unroll 8
        for (int j = 0; j < K; j++) acc_mac(s, xip[j * 64 + lane], col[j * (K + 1)]);
        uint64_t lo;
        uint32_t top;
        acc_value(s, lo, top);
        acc[l * 64 + lane] = (uint32_t)lo;
        carry = (lo >> 32) | ((uint64_t)top << 32);
    }
    return carry;
}

// Given acc = sum_j xi'_j M'_j (L+1 limbs): subtracts alpha M', then takes the
// canonical representative mod N (the value is below (K+1) N) by conditional
// subtractions of N 2^b, b = qbits-1 .. 0.  tmp: L+1 rows of scratch.
template <int K, int W>
__device__ __forceinline__ void exit_reduce(const uint32_t *__restrict__ bc, const uint32_t *__restrict__ mc,
                                            uint32_t *acc, uint32_t *tmp, uint32_t alpha, int L, int lane) {
    using S = Shp<K, W>;
    constexpr Layout LY{K, S::KP};
    {
        uint64_t carry = 0;
        uint32_t borrow = 0;
        for (int l = 0; l <= L; l++) {
            const uint64_t p = (uint64_t)alpha * bc[LY.MpF() + l] + carry;
            carry = p >> 32;
            const uint32_t v = acc[l * 64 + lane], pl = (uint32_t)p;
            const uint32_t d = v - pl, d2 = d - borrow;
            borrow = (v < pl) | (d < borrow);
            acc[l * 64 + lane] = d2;
        }
    }
    for (int b = S::qbits() - 1; b >= 0; b--) {
        uint32_t borrow = 0;
        for (int l = 0; l <= L; l++) {
            const uint32_t nlo = l < L ? mc[LY.Nl() + l] : 0u;
            const uint32_t nhi = (b && l > 0) ? (mc[LY.Nl() + l - 1] >> (32 - b)) : 0u;
            const uint32_t nl = (nlo << b) | nhi;
            const uint32_t v = acc[l * 64 + lane];
            const uint32_t d = v - nl, d2 = d - borrow;
            borrow = (v < nl) | (d < borrow);
            tmp[l * 64 + lane] = d2;
        }
        if (!borrow)
            for (int l = 0; l <= L; l++) acc[l * 64 + lane] = tmp[l * 64 + lane];
    }
}

// RNS -> binary for the value whose xi' (LDS) and alpha the last product left:
//   A = sum_j xi'_j M'_j - alpha M'   (CRT with the redundant modulus, Sec. 3.1)
// then the canonical representative A mod N (A < (K+1) N).  Result: L limbs
// in acc[l*64 + lane] (acc has room for L+1 rows).  Wave-local (no barrier).
template <int K, int W>
__device__ __forceinline__ void rns_exit(const uint32_t *__restrict__ bc, const uint32_t *__restrict__ mc,
                                         uint32_t *acc, uint32_t *tmp, const uint32_t *xip, uint32_t alpha,
                                         int L, int lane) {
    exit_columns<K, W>(bc, xip, acc, 0, L + 1, lane);
    exit_reduce<K, W>(bc, mc, acc, tmp, alpha, L, lane);
}

template <int KS>
__device__ __forceinline__ void tbl_store(uint32_t *__restrict__ p, const Res<KS> &a) {
#pragma unroll
    for (int c = 0; c < KS; c++) {
        p[c * 64] = a.b[c];
        p[(KS + c) * 64] = a.p[c];
    }
    p[2 * KS * 64] = a.r;
}

template <int KS>
__device__ __forceinline__ void tbl_load(const uint32_t *__restrict__ p, Res<KS> &a) {
#pragma unroll
    for (int c = 0; c < KS; c++) {
        a.b[c] = p[c * 64];
        a.p[c] = p[(KS + c) * 64];
    }
    a.r = p[2 * KS * 64];
}

__device__ __forceinline__ uint32_t exp_digit(const uint32_t *__restrict__ e, int nlimbs, int nd, int w, int di) {
    const int lo = (nd - 1 - di) * w;
    const int limb = lo >> 5, sh = lo & 31;
    uint64_t v = e[limb];
    if (limb + 1 < nlimbs) v |= (uint64_t)e[limb + 1] << 32;
    return (uint32_t)(v >> sh) & ((1u << w) - 1u);
}

// Left-to-right fixed-window exponentiation in the Montgomery domain (Sec. 3.1:
// square-and-multiply chaining RNS Montgomery products; the domain is entered
// and left once).  Table T[0] = M mod N ("one"), T[1] = X~ = X M mod N,
// T[j] = T[j-1] X~.  Every product runs through the single rns_mm call site of
// the loop below, which keeps the instruction footprint of the kernel small.
template <int K, int W>
__global__ __launch_bounds__(64 * W) void modexp_kernel(
    const uint32_t *__restrict__ bc, const uint32_t *__restrict__ mc0, const uint32_t *__restrict__ mc1,
    const uint32_t *__restrict__ E0, const uint32_t *__restrict__ E1, const uint32_t *__restrict__ ex0,
    const uint32_t *__restrict__ ex1, const uint32_t *__restrict__ in, uint32_t *__restrict__ out0,
    uint32_t *__restrict__ out1, uint32_t *__restrict__ table, ModexpParams P) {
    using S = Shp<K, W>;
    constexpr int KS = S::KS, KP = S::KP;
    constexpr Layout LY{K, KP};
    __shared__ uint32_t lds[2 * KP * 64];

    const int job = blockIdx.y;
    const uint32_t *__restrict__ mc = job ? mc1 : mc0;
    const uint32_t *__restrict__ E = job ? E1 : E0;
    const uint32_t *__restrict__ ex = job ? ex1 : ex0;
    uint32_t *__restrict__ out = job ? out1 : out0;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int c0 = wave * KS;
    const int msg = blockIdx.x * 64 + lane;
    const bool active = msg < P.batch;
    const size_t msafe = active ? (size_t)msg : 0;

    Res<KS> a, y;
    rns_entry<K, W>(bc, E, in + msafe * P.in_stride, P.in_limbs, active, a, c0);

    const int w = P.window;
    const int T = 1 << w;
    const size_t wg = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
    const size_t estride = (size_t)W * S::SLOTS * 64;
    uint32_t *__restrict__ tw = table + (wg * T * W + wave) * (size_t)(S::SLOTS * 64) + lane;

    {
        Res<KS> one;
#pragma unroll
        for (int c = 0; c < KS; c++) {
            one.b[c] = mc[LY.one() + c0 + c];
            one.p[c] = mc[LY.one() + KP + c0 + c];
        }
        one.r = mc[LY.one() + 2 * KP];
        tbl_store<KS>(tw, one);   // T[0] = M mod N
    }

    const int nd = (32 * P.exp_limbs + w - 1) / w;
    const bool shared_exp = P.exp_stride == 0;
    const uint32_t *__restrict__ ep = shared_exp ? ex : ex + msafe * P.exp_stride;

    enum { ENTRY, BUILD, MAIN, EXIT };
    int phase = ENTRY, j = 2, di = 0, s = 0;
    uint32_t alpha = 0;
    res_set_one<KS>(y);
    for (;;) {
        alpha = rns_mm<K, W>(bc, mc, a, y, lds, c0, lane, phase != EXIT);
        if (phase == EXIT) break;
        if (phase == ENTRY) {
            tbl_store<KS>(tw + estride, a);
            phase = BUILD;
        } else if (phase == BUILD) {
            tbl_store<KS>(tw + (size_t)j * estride, a);
            j++;
        }
        if (phase == BUILD) {
            if (j < T) {
                tbl_load<KS>(tw + estride, y);
                continue;
            }
            phase = MAIN;
            s = 0;
            if (shared_exp) {
                uint32_t d = 0;
                while (di < nd) {
                    d = __builtin_amdgcn_readfirstlane(exp_digit(ep, P.exp_limbs, nd, w, di));
                    if (d) break;
                    di++;
                }
                if (di < nd) {
                    tbl_load<KS>(tw + (size_t)d * estride, a);
                    di++;
                } else {
                    tbl_load<KS>(tw, a);
                }
            } else {
                tbl_load<KS>(tw, a);
            }
        }
        // choose the next product of the main loop
        for (;;) {
            if (di >= nd) {
                phase = EXIT;
                res_set_one<KS>(y);
                break;
            }
            if (s < w) {
                y = a;
                s++;
                break;
            }
            const uint32_t d = shared_exp ? __builtin_amdgcn_readfirstlane(exp_digit(ep, P.exp_limbs, nd, w, di))
                                          : exp_digit(ep, P.exp_limbs, nd, w, di);
            di++;
            s = 0;
            if (!shared_exp || d != 0) {
                tbl_load<KS>(tw + (size_t)d * estride, y);
                break;
            }
        }
    }
    __syncthreads();                // every wave has read xi' for alpha; LDS is wave 0's now
    if (wave != 0) return;
    uint32_t *acc = lds;
    const uint32_t *xip = lds + KP * 64;
    rns_exit<K, W>(bc, mc, acc, acc + (P.L + 1) * 64, xip, alpha, P.L, lane);
    if (active)
        for (int l = 0; l < P.L; l++) out[(size_t)msg * P.out_stride + l] = acc[l * 64 + lane];
}

// Garner recombination for CRT decryption over the p-modulus tables:
//   h = ((m_p - m_q) qinv) mod p as one RNS Montgomery product of the entry
//   value Z = m_p A + m_q (p - A), A = qinv M mod p, then m = m_q + h q.
template <int K, int W>
struct GarnerLds {
    static constexpr int WORDS = 2 * Shp<K, W>::KP * 64 + 2 * W * 64;
};

// Elements [e0, e0 + 64) of one Garner step (lds: GarnerLds<K, W>::WORDS).
template <int K, int W>
__device__ __forceinline__ void garner_tile(const GarnerLaunch &G, int e0, uint32_t *lds) {
    using S = Shp<K, W>;
    constexpr int KS = S::KS, KP = S::KP;
    const uint32_t *__restrict__ bc = G.bc;
    const uint32_t *__restrict__ mc = G.mc;
    const uint32_t *__restrict__ E = G.E;
    const uint32_t *__restrict__ ql = G.qlimbs;
    const uint32_t *__restrict__ in = G.in;
    uint32_t *__restrict__ out = G.out;
    const int L = G.L, out_limbs = G.out_limbs, out_stride = G.out_stride, batch = G.batch;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int c0 = wave * KS;
    const int msg = e0 + lane;
    const bool active = msg < batch;
    const size_t msafe = active ? (size_t)msg : 0;
    const uint32_t *src = in + msafe * (size_t)(2 * L);
    uint32_t *cout = lds + 2 * KP * 64;   // [W][2][64] carries out of each wave's limb range

    Res<KS> a, y;
    rns_entry<K, W>(bc, E, src, 2 * L, active, a, c0);
    res_set_one<KS>(y);
    const uint32_t alpha = rns_mm<K, W>(bc, mc, a, y, lds, c0, lane, false);
    __syncthreads();
    // leaving the RNS: the L+1 limbs of sum_j xi'_j M'_j in W ranges, one per
    // wave (the range sums are independent), then the carries between ranges,
    // alpha M' and the reduction mod p on wave 0
    uint32_t *h = lds;
    {
        const int C = (L + 1 + W - 1) / W;
        const int l0 = wave * C < L + 1 ? wave * C : L + 1;
        const int l1 = l0 + C < L + 1 ? l0 + C : L + 1;
        const uint64_t c = exit_columns<K, W>(bc, lds + KP * 64, h, l0, l1, lane);
        cout[wave * 128 + lane] = (uint32_t)c;
        cout[wave * 128 + 64 + lane] = (uint32_t)(c >> 32);
        __syncthreads();
        if (wave == 0) {
            ripple_carries(h + lane, 64, L + 1, cout + lane, 64, W, C);
            exit_reduce<K, W>(bc, mc, h, h + (L + 1) * 64, alpha, L, lane);
        }
        __syncthreads();
    }
    // m = m_q + h q: each wave its range of output limbs, then wave 0 adds the
    // carries between ranges (in the output buffer)
    const int C = (out_limbs + W - 1) / W;
    const int o0 = wave * C < out_limbs ? wave * C : out_limbs;
    const int o1 = o0 + C < out_limbs ? o0 + C : out_limbs;
    uint32_t *dst = out + msafe * (size_t)out_stride;
    uint64_t carry = 0;
    for (int l = o0; l < o1; l++) {
        const int i0 = l - L + 1 > 0 ? l - L + 1 : 0;
        const int i1 = l < L - 1 ? l : L - 1;
        Acc s;
        s.lo = carry + (l < L && active ? src[L + l] : 0u);   // + m_q
        for (int i = i0; i <= i1; i++) acc_mac(s, h[i * 64 + lane], ql[l - i]);
        uint64_t lo;
        uint32_t top;
        acc_value(s, lo, top);
        if (active) dst[l] = (uint32_t)lo;
        carry = (lo >> 32) | ((uint64_t)top << 32);
    }
    cout[wave * 128 + lane] = (uint32_t)carry;
    cout[wave * 128 + 64 + lane] = (uint32_t)(carry >> 32);
    __syncthreads();
    if (wave == 0 && active) ripple_carries(dst, 1, out_limbs, cout + lane, 64, W, C);
}

template <int K, int W>
__global__ __launch_bounds__(64 * W) void garner_kernel(GarnerLaunch G) {
    __shared__ uint32_t lds[GarnerLds<K, W>::WORDS];
    garner_tile<K, W>(G, blockIdx.x * 64, lds);
}

// Grouped Garner steps: workgroup t serves the job j with
// jobs[j].tile0 <= t < jobs[j+1].tile0 (binary search; jobs sorted).
template <int K, int W>
__global__ __launch_bounds__(64 * W) void garner_jobs_kernel(const GJob *__restrict__ jobs, int njobs) {
    __shared__ uint32_t lds[GarnerLds<K, W>::WORDS];
    const int t = blockIdx.x;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].tile0 <= t) lo = mid; else hi = mid - 1;
    }
    const GJob J = jobs[lo];
    garner_tile<K, W>(J.g, (t - J.tile0) * 64, lds);
}

// One RNS Montgomery product per element on channel-major residues.
template <int K, int W>
__global__ __launch_bounds__(64 * W) void montmul_kernel(const uint32_t *__restrict__ bc,
                                                           const uint32_t *__restrict__ mc,
                                                           const uint32_t *__restrict__ x,
                                                           const uint32_t *__restrict__ y,
                                                           uint32_t *__restrict__ out, int batch) {
    using S = Shp<K, W>;
    constexpr int KS = S::KS, KP = S::KP;
    __shared__ uint32_t lds[2 * KP * 64];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int c0 = wave * KS;
    const int msg = blockIdx.x * 64 + lane;
    const bool active = msg < batch;
    const size_t nb = (size_t)batch;
    Res<KS> a, b;
#pragma unroll
    for (int c = 0; c < KS; c++) {
        const int i = c0 + c;
        const bool ok = active && i < K;
        a.b[c] = ok ? x[(size_t)i * nb + msg] : 0u;
        b.b[c] = ok ? y[(size_t)i * nb + msg] : 0u;
        a.p[c] = ok ? x[(size_t)(K + i) * nb + msg] : 0u;
        b.p[c] = ok ? y[(size_t)(K + i) * nb + msg] : 0u;
    }
    a.r = active ? x[(size_t)(2 * K) * nb + msg] : 0u;
    b.r = active ? y[(size_t)(2 * K) * nb + msg] : 0u;
    rns_mm<K, W>(bc, mc, a, b, lds, c0, lane, true);
    if (!active) return;
#pragma unroll
    for (int c = 0; c < KS; c++) {
        const int i = c0 + c;
        if (i < K) {
            out[(size_t)i * nb + msg] = a.b[c];
            out[(size_t)(K + i) * nb + msg] = a.p[c];
        }
    }
    if (wave == 0) out[(size_t)(2 * K) * nb + msg] = a.r;
}

template <int K, int W>
hipError_t launch_modexp_t(const ModexpLaunch &a, hipStream_t s) {
    const unsigned gx = (unsigned)((a.P.batch + 63) / 64);
    hipLaunchKernelGGL((modexp_kernel<K, W>), dim3(gx, (unsigned)a.njobs), dim3(64 * W), 0, s, a.bc, a.mc[0],
                       a.mc[1], a.E[0], a.E[1], a.exp[0], a.exp[1], a.in, a.out[0], a.out[1], a.table, a.P);
    return hipGetLastError();
}

template <int K, int W>
hipError_t launch_garner_t(const GarnerLaunch &a, hipStream_t s) {
    const unsigned gx = (unsigned)((a.batch + 63) / 64);
    hipLaunchKernelGGL((garner_kernel<K, W>), dim3(gx), dim3(64 * W), 0, s, a);
    return hipGetLastError();
}

template <int K, int W>
hipError_t launch_garner_jobs_t(const GJob *jobs, int njobs, int tiles, hipStream_t s) {
    if (tiles <= 0 || njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL((garner_jobs_kernel<K, W>), dim3((unsigned)tiles), dim3(64 * W), 0, s, jobs, njobs);
    return hipGetLastError();
}

template <int K, int W>
hipError_t launch_montmul_t(const MontMulLaunch &a, hipStream_t s) {
    const unsigned gx = (unsigned)((a.batch + 63) / 64);
    hipLaunchKernelGGL((montmul_kernel<K, W>), dim3(gx), dim3(64 * W), 0, s, a.bc, a.mc, a.x, a.y, a.out,
                       a.batch);
    return hipGetLastError();
}

}  // namespace rnsrsa
