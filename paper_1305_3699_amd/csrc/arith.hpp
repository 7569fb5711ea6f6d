// Per-channel residue arithmetic shared by the device kernels and the host
// emulator, and the constant-table layout both of them read.
//
// Every RNS channel modulus is an odd prime m with 2^31 < m < 2^32 (the
// paper's "32-bit prime integers", Sec. 3.1); the redundant channel is
// 2^32 and uses plain wrap-around arithmetic.  Channel reductions use
// Montgomery's REDC with R = 2^32 in its subtractive form, which needs no
// 65-bit intermediate:  for x = xh*2^32 + xl with xh < m,
//     u = xl * m^-1 mod 2^32,  h = floor(u*m / 2^32),  t = xh - h  (+m if < 0)
// gives t = x * 2^-32 mod m, fully reduced.  Constants that meet a REDC are
// stored pre-multiplied by the matching power of 2^32, so every product
// leaves the channel arithmetic with no stray factor.
#pragma once

#include <cstdint>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define RNS_HD __host__ __device__ __forceinline__
#else
#define RNS_HD inline
#endif

namespace rnsrsa {

// t = x * 2^-32 mod m for x = xh:xl, xh < m; minv = m^-1 mod 2^32.
RNS_HD uint32_t redc(uint32_t xl, uint32_t xh, uint32_t m, uint32_t minv) {
    const uint32_t u = xl * minv;
#if defined(__HIP_DEVICE_COMPILE__)
    const uint32_t h = __umulhi(u, m);
#else
    const uint32_t h = (uint32_t)(((uint64_t)u * m) >> 32);
#endif
    uint32_t t;
    const bool borrow = __builtin_sub_overflow(xh, h, &t);
    return t + (borrow ? m : 0u);
}

// a * b * 2^-32 mod m for a, b < m.
RNS_HD uint32_t mulredc(uint32_t a, uint32_t b, uint32_t m, uint32_t minv) {
    const uint64_t p = (uint64_t)a * b;
    return redc((uint32_t)p, (uint32_t)(p >> 32), m, minv);
}

// Accumulator for sums of up to 255 products of 32-bit factors, kept as two
// 64-bit partial sums over the 16-bit halves of the per-lane factor:
//   value = lo + hi * 2^16,  with lo, hi < 255 * 2^48 < 2^56.
// Each product is one carry-free 32x32->64 multiply-add (v_mad_u64_u32).
struct Acc {
    uint64_t lo = 0, hi = 0;
};

// acc += v * c
RNS_HD void acc_mac(Acc &a, uint32_t v, uint32_t c) {
    a.lo += (uint64_t)(v & 0xFFFFu) * c;
    a.hi += (uint64_t)(v >> 16) * c;
}

// acc += v * c for a per-lane v below 2^16 (no upper half)
RNS_HD void acc_mac16(Acc &a, uint32_t v, uint32_t c) { a.lo += (uint64_t)v * c; }

// The 96-bit value of an accumulator as (w0:w1 in lo64, w2).
RNS_HD void acc_value(const Acc &a, uint64_t &lo64, uint32_t &top) {
    const uint64_t sh = a.hi << 16;
    lo64 = a.lo + sh;
    top = (uint32_t)(a.hi >> 48) + (lo64 < sh ? 1u : 0u);
}

// (hi:lo) * 2^-64 mod m for a 96-bit value whose top word is below m.
RNS_HD uint32_t redc96(uint64_t lo, uint32_t hi, uint32_t m, uint32_t minv) {
    uint32_t mid = (uint32_t)(lo >> 32);
    mid = mid >= m ? mid - m : mid;            // m > 2^31, so one step suffices
    const uint32_t t1 = redc((uint32_t)lo, mid, m, minv);
    return redc(t1, hi, m, minv);
}

// acc * 2^-64 mod m
RNS_HD uint32_t acc_redc(const Acc &a, uint32_t m, uint32_t minv) {
    uint64_t lo;
    uint32_t top;
    acc_value(a, lo, top);
    return redc96(lo, top, m, minv);
}

// Constant-table layout.  K = channels per base, KP = K padded to a multiple
// of the waves per workgroup (padding channels carry zero constants).
struct Layout {
    int K, KP;
    // key-independent ("base") table
    constexpr int mB() const { return 0; }             // [KP] moduli of B
    constexpr int uB() const { return KP; }            // [KP] m^-1 mod 2^32
    constexpr int mBp() const { return 2 * KP; }       // [KP] moduli of B'
    constexpr int uBp() const { return 3 * KP; }       // [KP]
    constexpr int negMp() const { return 4 * KP; }     // [KP] (-M' mod m_i) R^2 mod m_i
    constexpr int MpInv() const { return 5 * KP; }     // [KP] (M'/m'_t)^-1 R mod m'_t
    constexpr int scal() const { return 6 * KP; }      // [4]  M'^-1, M^-1 mod 2^32
    constexpr int C1() const { return 6 * KP + 4; }    // [K][KP+1]
    constexpr int C2() const { return C1() + K * (KP + 1); }  // [K][KP+1]
    constexpr int MpL() const { return C2() + K * (KP + 1); } // [K][K+1] limbs of M'/m'_j
    constexpr int MpF() const { return MpL() + K * (K + 1); } // [K+1] limbs of M'
    constexpr int base_size() const { return MpF() + K + 1; }
    constexpr int crow() const { return KP + 1; }      // row stride of C1, C2
    // per-modulus table
    constexpr int c2B() const { return 0; }            // [KP] c_i R^2 mod m_i
    constexpr int NnBp() const { return KP; }          // [KP] (-N) mod m'_t
    constexpr int MiBp() const { return 2 * KP; }      // [KP] M^-1 R^2 mod m'_t
    constexpr int one() const { return 3 * KP; }       // [2KP+1] residues of M mod N
    constexpr int mscal() const { return 5 * KP + 1; } // [4] N mod 2^32, L
    constexpr int Nl() const { return 5 * KP + 5; }    // [K] limbs of N
    constexpr int mod_size() const { return 5 * KP + 5 + K; }
    // entry table: [in_limbs][ecols]
    constexpr int ecols() const { return 2 * KP + 1; }
};

#ifdef __HIPCC__
// The limbs of a sum computed as n consecutive ranges of C limbs each, range r
// starting at limb r*C, whose carries out are cout[2*cs*r] (low word) and
// cout[2*cs*r + cs] (high word): adds each range's carry into the limbs that
// follow it, in order (v[l*vs] is limb l; nl limbs in all; a carry past limb
// nl-1 is dropped, the sum being taken mod 2^(32 nl)).
template <typename P>
__device__ __forceinline__ void ripple_carries(P v, size_t vs, int nl, const uint32_t *cout, int cs, int n, int C) {
    uint64_t c = 0;
    for (int r = 1; r < n; r++) {
        c += (uint64_t)cout[2 * cs * (r - 1)] | ((uint64_t)cout[2 * cs * (r - 1) + cs] << 32);
        const int end = (r + 1) * C < nl ? (r + 1) * C : nl;
        for (int l = r * C; c != 0 && l < end; l++) {
            const uint64_t t = (uint64_t)v[l * vs] + (uint32_t)c;
            v[l * vs] = (uint32_t)t;
            c = (c >> 32) + (t >> 32);
        }
    }
}
#endif

}  // namespace rnsrsa
