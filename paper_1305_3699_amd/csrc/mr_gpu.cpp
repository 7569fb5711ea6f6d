// Miller-Rabin with every per-candidate constant built on the GPU (Sec. 3.2:
// primality tests whose exponentiations run in RNS in the Montgomery domain;
// Sec. 4.3: key material stays on the GPU).  All candidates of one size share
// one base pair.  A table kernel derives each candidate's matrix-engine
// tables from N alone: N's residues, the first extension's constant tiles,
// c_i = -N^-1 M_i^-1, M mod N and M^2 mod N (a one-thread long division by
// N), the entry table, and d, s with N - 1 = 2^s d.  The exponentiations
// a^d and the squarings run as grouped matrix-core launches on those tables,
// and a check kernel takes each decision (1, N - 1) on the device; the host
// only plans the launches and reads the verdicts once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "capi_internal.hpp"
#include "jobs.hpp"
#include "mr_gpu.hpp"

namespace rnsrsa {
namespace {

// Key-independent constants the table kernel combines with N, per base pair
// and shape, by channel c (B: c < K, B': K <= c < 2K).
struct MrLayout {
    int K;
    constexpr size_t m() const { return 0; }                               // [2K] moduli
    constexpr size_t u() const { return 2 * (size_t)K; }                   // [2K] m^-1 mod 2^32
    constexpr size_t r2() const { return 4 * (size_t)K; }                  // [2K] R^2 mod m
    constexpr size_t r4() const { return 6 * (size_t)K; }                  // [2K] R^4 mod m_i; R^4 M^-1 mod m'_t
    constexpr size_t cinv() const { return 8 * (size_t)K; }                // [K] (M_i mod m_i)^-1 R mod m_i
    constexpr size_t g0() const { return 9 * (size_t)K; }                  // [K] R^3 M^-2 mod m'_t
    constexpr size_t kap() const { return 10 * (size_t)K; }                // [K] R^2 M^-1 mod m'_t
    constexpr size_t p1() const { return 11 * (size_t)K; }                 // [K][K+1][4] (M_i mod m'_t) 2^8a R mod m'_t
    constexpr size_t vred() const { return p1() + (size_t)K * (K + 1) * 4; }  // [K+1][4] redundant row, raw words
    constexpr size_t size() const { return vred() + (size_t)(K + 1) * 4; }
};

std::vector<uint32_t> make_mr_consts(const BaseSet &bs) {
    const int K = bs.K;
    const MrLayout ly{K};
    std::vector<uint32_t> v(ly.size(), 0);
    for (int c = 0; c < 2 * K; c++) {
        const uint32_t m = c < K ? bs.B[c] : bs.Bp[c - K];
        v[ly.m() + c] = m;
        v[ly.u() + c] = inv2_32(m);
        const uint32_t r2 = pow2_64_mod(m);
        v[ly.r2() + c] = r2;
        const uint32_t r4 = mulmod32(r2, r2, m);
        v[ly.r4() + c] = c < K ? r4 : mulmod32(r4, invmod32(prod_mod32(bs.B, m), m), m);
    }
    for (int i = 0; i < K; i++) {
        const uint32_t m = bs.B[i];
        std::vector<uint32_t> others;
        for (int j = 0; j < K; j++)
            if (j != i) others.push_back(bs.B[j]);
        v[ly.cinv() + i] = mulmod32(invmod32(prod_mod32(others, m), m), pow2_32_mod(m), m);
    }
    for (int t = 0; t < K; t++) {
        const uint32_t m = bs.Bp[t], R = pow2_32_mod(m), R2 = pow2_64_mod(m);
        const uint32_t minv = invmod32(prod_mod32(bs.B, m), m);
        v[ly.g0() + t] = mulmod32(mulmod32(mulmod32(R2, R, m), minv, m), minv, m);
        v[ly.kap() + t] = mulmod32(R2, minv, m);
        const uint32_t P = prod_mod32(bs.B, m);
        uint64_t sum = 0;
        for (int i = 0; i < K; i++) {
            const uint32_t mi = mulmod32(P, invmod32(bs.B[i] % m, m), m);
            sum = (sum + mi) % m;
            for (int a = 0; a < 4; a++)
                v[ly.p1() + ((size_t)t * (K + 1) + i) * 4 + a] =
                    mulmod32(mulmod32(mi, powmod32(2, 8 * a, m), m), R, m);
        }
        v[ly.p1() + ((size_t)t * (K + 1) + K) * 4] = mulmod32(mulmod32(kDigitBias % m, (uint32_t)sum, m), R, m);
    }
    uint32_t prod_lo = 1;
    for (uint32_t m : bs.B) prod_lo *= m;
    uint32_t sum_lo = 0;
    for (int i = 0; i < K; i++) {
        const uint32_t mi_lo = prod_lo * inv2_32(bs.B[i]);
        sum_lo += mi_lo;
        for (int a = 0; a < 4; a++) v[ly.vred() + (size_t)i * 4 + a] = mi_lo << (8 * a);
    }
    v[ly.vred() + (size_t)K * 4] = kDigitBias * sum_lo;
    return v;
}

struct MrTablesArgs {
    const uint32_t *cand;   // count x L limbs
    const uint32_t *cst;    // MrLayout constants
    uint32_t *keys;         // count x key_size: the matrix engine's per-modulus tables
    uint32_t *entry;        // count x (L x ecols): entry tables for L-limb inputs
    uint32_t *dexp;         // count x L: d
    uint8_t *flag;          // count: 0 N coprime to every channel, 1 a channel prime divides N, 2 N is one
    MLayout sh;
    int L;
};

constexpr int kMrThreads = 256;

__device__ __forceinline__ uint32_t residue_of(const uint32_t *x, int n, uint32_t m, uint32_t u, uint32_t r2) {
    uint32_t acc = 0;
    for (int l = n - 1; l >= 0; l--) {
        acc = mulredc(acc, r2, m, u);                           // acc 2^32 mod m
        const uint32_t v = x[l] >= m ? x[l] - m : x[l];         // m > 2^31: one step
        const uint64_t s = (uint64_t)acc + v;
        acc = s >= m ? (uint32_t)(s - m) : (uint32_t)s;
    }
    return acc;
}

// a^-1 mod m (prime m, a != 0) by Fermat's little theorem, in Montgomery form.
__device__ __forceinline__ uint32_t inv_mod_prime(uint32_t a, uint32_t m, uint32_t u, uint32_t r2) {
    const uint32_t aR = mulredc(a, r2, m, u);
    uint32_t x = mulredc(1u, r2, m, u);                         // 1 R
    const uint32_t e = m - 2;
    for (int b = 31; b >= 0; b--) {
        x = mulredc(x, x, m, u);
        if ((e >> b) & 1u) x = mulredc(x, aR, m, u);
    }
    return mulredc(x, 1u, m, u);
}

// Channel of slot (wave w, tile mt, lane group g) of the shape: -1 for the
// redundant slot, K or more for unused slots (the layout of plan_mfma.hpp).
__device__ __forceinline__ int slot_channel_dev(const MLayout &sh, int w, int mt, int g) {
    const int s = 4 * mt + g;
    return s == 4 * sh.MT - 1 ? -1 : w * sh.CH() + s;
}

__device__ __forceinline__ int64_t balanced_dev(uint32_t v, uint32_t m) {
    return v >= kDigitSplit ? (int64_t)v - m : (int64_t)v;
}
__device__ __forceinline__ int64_t balanced32_dev(uint32_t v) {
    return v > 0x7F7F7F7Fu ? (int64_t)v - ((int64_t)1 << 32) : (int64_t)v;
}
__device__ __forceinline__ uint32_t digit_dev(int64_t V, int b) {
    const uint32_t w = (uint32_t)(V + 0x80808080ll);
    return (uint32_t)(uint8_t)(int8_t)((int)((w >> (8 * b)) & 0xFFu) - 128);
}

// t (n + 1 limbs, below Nn 2^32) <- t mod Nn; Nn normalised (top bit of limb
// n - 1 set).  The quotient digit from the top two limbs over Nn's top limb
// overshoots by at most 2 (Knuth, Vol. 2, 4.3.1), corrected by adding Nn back.
__device__ void reduce_one(uint32_t *t, const uint32_t *Nn, int n) {
    const uint64_t num = ((uint64_t)t[n] << 32) | t[n - 1];
    uint64_t q = num / Nn[n - 1];
    if (q > 0xFFFFFFFFull) q = 0xFFFFFFFFull;
    uint64_t mul = 0;
    uint32_t borrow = 0;
    for (int l = 0; l <= n; l++) {
        const uint64_t p = (l < n ? q * Nn[l] : 0) + mul;
        mul = p >> 32;
        const uint32_t pl = (uint32_t)p, v = t[l];
        const uint32_t d = v - pl, d2 = d - borrow;
        borrow = (v < pl) | (d < borrow);
        t[l] = d2;
    }
    while (borrow) {                                            // negative: add Nn back
        uint32_t c = 0;
        for (int l = 0; l <= n; l++) {
            const uint64_t s = (uint64_t)t[l] + (l < n ? Nn[l] : 0) + c;
            t[l] = (uint32_t)s;
            c = (uint32_t)(s >> 32);
        }
        borrow = c ? 0u : 1u;                                   // a carry out of the top limb ends the deficit
    }
}

// x = a * w (n limbs times one word) into t (n + 1 limbs).
__device__ void mul_word(uint32_t *t, const uint32_t *a, uint32_t w, int n) {
    uint64_t c = 0;
    for (int l = 0; l < n; l++) {
        const uint64_t p = (uint64_t)a[l] * w + c;
        t[l] = (uint32_t)p;
        c = p >> 32;
    }
    t[n] = (uint32_t)c;
}

// One workgroup per candidate.  LDS: N, the normalised Nn, two (n + 2)-limb
// work rows, M mod N and M^2 mod N (shifted), residues of N, of M mod N and
// of M^2 mod N per channel, G_t and c_i.
__global__ __launch_bounds__(kMrThreads) void mr_tables_kernel(MrTablesArgs A) {
    extern __shared__ uint32_t sm[];
    const int K = A.sh.K, L = A.L, tid = threadIdx.x;
    const MrLayout cl{K};
    const uint32_t *__restrict__ cst = A.cst;
    uint32_t *N = sm, *Nn = N + L, *T1 = Nn + L + 1, *T2 = T1 + L + 2, *Mm = T2 + L + 2, *Yv = Mm + L + 1;
    uint32_t *nres = Yv + L + 1, *mres = nres + 2 * K, *yres = mres + 2 * K, *G = yres + 2 * K, *cv = G + K;
    __shared__ int s_flag;
    const size_t ci = blockIdx.x;
    const uint32_t *src = A.cand + ci * L;
    for (int l = tid; l < L; l += kMrThreads) N[l] = src[l];
    if (tid == 0) s_flag = 0;
    __syncthreads();

    for (int c = tid; c < 2 * K; c += kMrThreads)
        nres[c] = residue_of(N, L, cst[cl.m() + c], cst[cl.u() + c], cst[cl.r2() + c]);
    if (tid == 0) {
        // M mod N and M^2 mod N by long division in the normalised domain
        // (everything times 2^sh, Nn = N 2^sh with its top bit set), and d, s
        int n = L;
        while (n > 1 && N[n - 1] == 0) n--;
        const int sh = __builtin_clz(N[n - 1]);
        for (int l = n - 1; l >= 0; l--)
            Nn[l] = (N[l] << sh) | (sh && l > 0 ? N[l - 1] >> (32 - sh) : 0u);
        for (int l = 0; l <= n; l++) T1[l] = 0;
        T1[0] = 1u << sh;                                       // 1 (shifted); N > 1
        for (int i = 0; i < K; i++) {                           // times each prime of B: M = prod m_i
            mul_word(T2, T1, cst[cl.m() + i], n);
            reduce_one(T2, Nn, n);
            for (int l = 0; l < n; l++) T1[l] = T2[l];
        }
        for (int l = 0; l < n; l++) Mm[l] = T1[l];             // M mod N, shifted
        // M^2 mod N: Y = sum over the limbs z_l of M mod N, top first, of
        // Y 2^32 + (M mod N) z_l, each step reduced
        for (int l = 0; l <= n; l++) T1[l] = 0;
        for (int l = n - 1; l >= 0; l--) {
            const uint32_t z = (Mm[l] >> sh) | (sh && l + 1 < n ? Mm[l + 1] << (32 - sh) : 0u);   // limb l of M mod N
            for (int j = n; j > 0; j--) T1[j] = T1[j - 1];      // Y 2^32
            T1[0] = 0;
            reduce_one(T1, Nn, n);
            mul_word(T2, Mm, z, n);                             // (M mod N) z, shifted
            reduce_one(T2, Nn, n);
            uint32_t c = 0;
            for (int j = 0; j < n; j++) {
                const uint64_t s2 = (uint64_t)T1[j] + T2[j] + c;
                T1[j] = (uint32_t)s2;
                c = (uint32_t)(s2 >> 32);
            }
            // below 2 Nn: subtract Nn once if it is reached
            bool ge = c != 0;
            if (!ge) {
                ge = true;
                for (int j = n - 1; j >= 0; j--)
                    if (T1[j] != Nn[j]) {
                        ge = T1[j] > Nn[j];
                        break;
                    }
            }
            if (ge) {
                uint32_t b = 0;
                for (int j = 0; j < n; j++) {
                    const uint32_t v = T1[j], d = v - Nn[j], d2 = d - b;
                    b = (v < Nn[j]) | (d < b);
                    T1[j] = d2;
                }
            }
            T1[n] = 0;
        }
        // back from the shifted domain
        for (int l = 0; l < L; l++) {
            Yv[l] = l < n ? (T1[l] >> sh) | (sh && l + 1 < n ? T1[l + 1] << (32 - sh) : 0u) : 0u;
            const uint32_t mm = l < n ? (Mm[l] >> sh) | (sh && l + 1 < n ? Mm[l + 1] << (32 - sh) : 0u) : 0u;
            T2[l] = mm;
        }
        for (int l = 0; l < L; l++) Mm[l] = T2[l];
        // N - 1 = 2^s d (N odd)
        int s = 0;
        int l0 = 0;
        uint32_t w0 = N[0] & ~1u;
        while (w0 == 0 && l0 + 1 < L) w0 = N[++l0];
        s = 32 * l0 + (w0 ? __builtin_ctz(w0) : 0);
        uint32_t *d = A.dexp + ci * L;
        for (int l = 0; l < L; l++) {
            const int bit = 32 * l + s;
            const int lw = bit >> 5, sb = bit & 31;
            const uint32_t lo = lw < L ? (lw == 0 ? N[0] & ~1u : N[lw]) : 0u;
            const uint32_t hi = lw + 1 < L ? N[lw + 1] : 0u;
            d[l] = sb ? (lo >> sb) | (hi << (32 - sb)) : lo;
        }
    }
    __syncthreads();

    // G_t, c_i, residues of M mod N and M^2 mod N
    for (int t = tid; t < K; t += kMrThreads) {
        const int c = K + t;
        G[t] = mulredc(nres[c], cst[cl.g0() + t], cst[cl.m() + c], cst[cl.u() + c]);
    }
    for (int i = tid; i < K; i += kMrThreads) {
        const uint32_t m = cst[cl.m() + i], u = cst[cl.u() + i], r2 = cst[cl.r2() + i];
        const uint32_t n = nres[i];
        cv[i] = n ? mulredc(m - inv_mod_prime(n, m, u, r2), cst[cl.cinv() + i], m, u) : 0u;
    }
    for (int c = tid; c < 2 * K; c += kMrThreads) {
        const uint32_t m = cst[cl.m() + c], u = cst[cl.u() + c], r2 = cst[cl.r2() + c];
        mres[c] = residue_of(Mm, L, m, u, r2);
        yres[c] = residue_of(Yv, L, m, u, r2);
        if (nres[c] == 0) {
            // a channel prime divides N: N is composite unless it is that prime
            bool single = N[0] == m;
            for (int l = 1; l < L; l++) single = single && N[l] == 0;
            atomicMax(&s_flag, single ? 2 : 1);
        }
    }
    __syncthreads();

    const MLayout &sh = A.sh;
    const int KS = sh.KSTEPS(), SW = 4 * sh.MT;
    uint32_t *key = A.keys + ci * sh.key_size();
    // first-extension tiles: [W][MT][KSTEPS][64 lanes][16 bytes]
    const int quads = sh.W * sh.MT * KS * 64;
    for (int q = tid; q < quads; q += kMrThreads) {
        const int l = q % 64, ks = (q / 64) % KS, mt = (q / (64 * KS)) % sh.MT, w = q / (64 * KS * sh.MT);
        const int row = l % 16, g = row / 4, b = row % 4;
        const int t = slot_channel_dev(sh, w, mt, g);
        uint32_t words[4] = {0, 0, 0, 0};
        for (int j = 0; j < 16; j++) {
            const int kappa = 64 * ks + 16 * (l / 16) + j;
            const int ch = kappa / 4, a = kappa % 4;
            int64_t V = 0;
            if (t < K && ch <= K && (ch < K || a == 0)) {
                if (t < 0) {
                    V = balanced32_dev(cst[cl.vred() + (size_t)ch * 4 + a]);
                } else {
                    const int c = K + t;
                    const uint32_t m = cst[cl.m() + c];
                    V = balanced_dev(mulredc(cst[cl.p1() + ((size_t)t * (K + 1) + ch) * 4 + a], G[t], m,
                                             cst[cl.u() + c]), m);
                }
            }
            words[j / 4] |= digit_dev(V, b) << (8 * (j % 4));
        }
        uint32_t *p = key + sh.a1() + (size_t)q * 4;
        for (int z = 0; z < 4; z++) p[z] = words[z];
    }
    // c_i by slot, M mod N in the kept representation by slot
    const int slots = sh.W * sh.MT * 64;
    for (int q = tid; q < slots; q += kMrThreads) {
        const int l = q % 64, mt = (q / 64) % sh.MT, w = q / (64 * sh.MT);
        const int t = slot_channel_dev(sh, w, mt, l / 16);
        const bool ok = t >= 0 && t < K;
        key[sh.slotC() + q] = ok ? cv[t] : 0u;
        const size_t o = sh.one() + (((size_t)w * sh.MT + mt) * 2) * 64 + l;
        key[o] = ok ? mulredc(mres[t], cst[cl.r2() + t], cst[cl.m() + t], cst[cl.u() + t]) : 0u;   // (M mod N) R
        key[o + 64] = ok ? mulredc(mres[K + t], cst[cl.kap() + t], cst[cl.m() + K + t], cst[cl.u() + K + t])
                         : 0u;                                                                   // (M mod N) R M^-1
    }
    if (tid == 0) {
        key[sh.one() + (size_t)sh.W * sh.MT * 2 * 64] = Mm[0];
        for (int z = 0; z < 4; z++) key[sh.kscal() + z] = z == 0 ? N[0] : 0u;
        A.flag[ci] = (uint8_t)s_flag;
    }
    for (int l = tid; l < K; l += kMrThreads) key[sh.Nl() + l] = l < L ? N[l] : 0u;
    // entry table rows j < L: value 2^(32 j) (M^2 mod N), by slot column, in
    // the kept representation (R^3 with one REDC: B R^4; B' R^4 M^-1)
    const int cols = (int)sh.ecols();
    uint32_t *E = A.entry + ci * (size_t)L * cols;
    for (int q = tid; q < sh.W * SW; q += kMrThreads) {
        const int w = q / SW, s = q % SW;
        const int t = slot_channel_dev(sh, w, s / 4, s % 4);
        const bool ok = t >= 0 && t < K;
        uint32_t vm = 0, vp = 0;
        uint32_t m = 0, u = 0, r2 = 0, mp = 0, up = 0, r2p = 0;
        if (ok) {
            m = cst[cl.m() + t], u = cst[cl.u() + t], r2 = cst[cl.r2() + t];
            mp = cst[cl.m() + K + t], up = cst[cl.u() + K + t], r2p = cst[cl.r2() + K + t];
            vm = mulredc(yres[t], cst[cl.r4() + t], m, u);
            vp = mulredc(yres[K + t], cst[cl.r4() + K + t], mp, up);
        }
        for (int j = 0; j < L; j++) {
            E[(size_t)j * cols + (size_t)w * SW + s] = vm;
            E[(size_t)j * cols + (size_t)sh.W * SW + (size_t)w * SW + s] = vp;
            if (ok) {
                vm = mulredc(vm, r2, m, u);                     // times 2^32
                vp = mulredc(vp, r2p, mp, up);
            }
        }
    }
    for (int j = tid; j < L; j += kMrThreads) E[(size_t)j * cols + cols - 1] = j == 0 ? Yv[0] : 0u;
}

// state[c, r]: 0 undecided, 1 base passed, 2 base failed.  After the
// exponentiation of step j (j = 0: x = a^d, j > 0: x = x^2) compares each
// undecided x with 1 and N - 1.
__global__ void mr_check_kernel(const uint32_t *__restrict__ x, const uint32_t *__restrict__ cand, int L,
                                int rounds, int count, int step, uint8_t *__restrict__ state) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= count * rounds) return;
    if (state[idx]) return;
    const int c = idx / rounds;
    const uint32_t *xr = x + (size_t)idx * L, *N = cand + (size_t)c * L;
    bool one = xr[0] == 1u, nm1 = xr[0] == N[0] - 1u;   // N odd: N - 1 differs from N in limb 0 only
    for (int l = 1; l < L; l++) {
        one = one && xr[l] == 0u;
        nm1 = nm1 && xr[l] == N[l];
    }
    // s from N: the trailing zero bits of N - 1
    int s = 0;
    {
        int l0 = 0;
        uint32_t w0 = N[0] & ~1u;
        while (w0 == 0 && l0 + 1 < L) w0 = N[++l0];
        s = 32 * l0 + (w0 ? __builtin_ctz(w0) : 0);
    }
    uint8_t st = 0;
    if (nm1 || (step == 0 && one)) st = 1;              // a^(2^j d) = -1, or a^d = 1
    else if (one) st = 2;                               // 1 reached without passing -1
    else if (step + 1 >= s) st = 2;                     // no squaring left to reach -1
    state[idx] = st;
}

__global__ void mr_verdict_kernel(const uint8_t *__restrict__ state, const uint8_t *__restrict__ flag, int rounds,
                                  int count, uint8_t *__restrict__ verdict) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= count) return;
    uint8_t v = 1;
    for (int r = 0; r < rounds; r++) v &= state[(size_t)c * rounds + r] == 1;
    verdict[c] = flag[c] == 2 ? 1 : flag[c] == 1 ? 0 : v;
}

// Window with the fewest expected products for a random exponent of `bits`
// bits (sliding windows: 2^(w-1) table products and about bits / (w + 1)
// multiplications besides the squarings).
int window_for_bits(int bits) {
    int best = 1;
    double bc = 1e300;
    for (int w = 1; w <= 6; w++) {
        const double c = (w > 1 ? (double)(1 << (w - 1)) : 0.0) + (double)bits / (w + 1);
        if (c < bc) {
            bc = c;
            best = w;
        }
    }
    return best;
}

struct MrBase {
    std::shared_ptr<const BaseSet> bs;
    MfmaShape sh{};
    uint32_t *d_mbase = nullptr;   // shared, owned by the process-wide base cache
    uint32_t *d_consts = nullptr;
};

// The base pair, shape and device constants for candidates of L limbs (one
// per (L, device), kept for the process), or RNS_EUNSUPPORTED when that base
// does not run on the matrix engine.
int mr_base(int L, int dev, MrBase *out) {
    static std::mutex mu;
    static std::map<std::pair<int, int>, MrBase> cache;
    std::lock_guard<std::mutex> lk(mu);
    auto key = std::make_pair(L, dev);
    auto it = cache.find(key);
    if (it != cache.end()) {
        *out = it->second;
        return RNS_OK;
    }
    Limbs Nmax((size_t)L, 0xFFFFFFFFu);             // the largest L-limb value: bounds hold for every candidate
    ModPlan mp;
    std::string err;
    int rc = make_modplan(Nmax, L, PlanOptions{}, mp, err);
    if (rc) return api::fail(rc, err);
    MrBase b;
    b.bs = mp.base;
    const BaseSet &bs = *b.bs;
    bool fits = mfma_shape_for(bs.K, b.sh, 0);
    for (uint32_t m : bs.B) fits = fits && mfma_prime_fits(m, bs.K, false);
    for (uint32_t m : bs.Bp) fits = fits && mfma_prime_fits(m, bs.K, true);
    if (!fits) return api::fail(RNS_EUNSUPPORTED, "the base of these candidates has no matrix-engine kernel");
    uint32_t *resident = api::resident_mfma_base(b.bs.get(), b.sh);
    if (resident) {
        b.d_mbase = resident;
    } else {
        MfmaTables t = make_mfma_tables(mp, b.sh, true);
        if ((rc = api::device_mfma_base(b.bs, b.sh, t.base, &b.d_mbase))) return rc;
    }
    if ((rc = api::upload(make_mr_consts(bs), &b.d_consts))) return rc;
    cache[key] = b;
    *out = b;
    return RNS_OK;
}

}  // namespace

namespace api {

int miller_rabin_gpu(const uint32_t *cand, size_t count, int L, const uint32_t *bases, int rounds, uint8_t *verdict,
                     hipStream_t s) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    MrBase mb;
    int rc = mr_base(L, dev, &mb);
    if (rc) return rc;
    const MfmaShape &sh = mb.sh;
    const size_t row = (size_t)rounds * L, cols = sh.ecols();
    // s of each candidate (host copy: it sets the number of squaring steps)
    std::vector<int> sv(count);
    int smax = 0;
    for (size_t i = 0; i < count; i++) {
        const uint32_t *N = cand + i * L;
        int l0 = 0;
        uint32_t w0 = N[0] & ~1u;
        while (w0 == 0 && l0 + 1 < L) w0 = N[++l0];
        sv[i] = 32 * l0 + (w0 ? __builtin_ctz(w0) : 0);
        smax = std::max(smax, sv[i]);
    }
    Scratch d_cand, d_keys, d_entry, d_exp, d_x, d_two, d_flag, d_state, d_verdict;
    rc = scratch_alloc(d_cand, count * L * sizeof(uint32_t), s);
    if (!rc) rc = scratch_alloc(d_keys, count * sh.key_size() * sizeof(uint32_t), s);
    if (!rc) rc = scratch_alloc(d_entry, count * L * cols * sizeof(uint32_t), s);
    if (!rc) rc = scratch_alloc(d_exp, count * L * sizeof(uint32_t), s);
    if (!rc) rc = scratch_alloc(d_x, count * row * sizeof(uint32_t), s);
    if (!rc) rc = scratch_alloc(d_two, sizeof(uint32_t), s);
    if (!rc) rc = scratch_alloc(d_flag, count, s);
    if (!rc) rc = scratch_alloc(d_state, count * rounds, s);
    if (!rc) rc = scratch_alloc(d_verdict, count, s);
    if (rc) return rc;
    const uint32_t two = 2;
    e = hipMemcpyAsync(d_cand.p, cand, count * L * sizeof(uint32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_x.p, bases, count * row * sizeof(uint32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_two.p, &two, sizeof(uint32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(d_state.p, 0, count * rounds, s);
    if (e != hipSuccess) return hip_fail(e, "miller-rabin set-up copies");

    MrTablesArgs ta{};
    ta.cand = (const uint32_t *)d_cand.p;
    ta.cst = mb.d_consts;
    ta.keys = (uint32_t *)d_keys.p;
    ta.entry = (uint32_t *)d_entry.p;
    ta.dexp = (uint32_t *)d_exp.p;
    ta.flag = (uint8_t *)d_flag.p;
    ta.sh = sh;
    ta.L = L;
    // N, Nn, two work rows, M mod N, M^2 mod N; residues (3 x 2K), G, c
    const size_t lds = ((size_t)6 * L + 8 + (size_t)8 * sh.K) * sizeof(uint32_t);
    hipLaunchKernelGGL(mr_tables_kernel, dim3((unsigned)count), dim3(kMrThreads), lds, s, ta);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "miller-rabin table launch");

    std::vector<std::unique_ptr<Scratch>> keep;
    std::vector<std::vector<MJob>> host_jobs;
    const int w_d = window_for_bits(32 * L);
    for (int step = 0; step < std::max(1, smax); step++) {
        // x = a^d (step 0) or x = x^2 for the candidates that may square again
        JobGroup g;
        g.shape = sh;
        g.device = dev;
        for (size_t i = 0; i < count; i++) {
            if (step > 0 && sv[i] <= step) continue;
            PlannedJob J{};
            uint32_t *x = (uint32_t *)d_x.p + i * row;
            J.j.mb = mb.d_mbase;
            J.j.mk = (const uint32_t *)d_keys.p + i * sh.key_size();
            J.j.E = (const uint32_t *)d_entry.p + i * L * cols;
            J.j.exp = step == 0 ? (const uint32_t *)d_exp.p + i * L : (const uint32_t *)d_two.p;
            J.j.in = x;
            J.j.out = x;
            J.j.batch = rounds;
            J.j.in_limbs = L;
            J.j.in_stride = L;
            J.j.L = L;
            J.j.out_stride = L;
            J.j.exp_limbs = step == 0 ? L : 1;
            J.j.exp_stride = 0;
            J.j.window = step == 0 ? w_d : 1;
            J.cost = step == 0 ? (size_t)32 * L : 3;
            g.jobs.push_back(J);
        }
        if (g.jobs.empty()) break;
        finish_group(g);
        retile_group(g, dev);
        host_jobs.emplace_back();
        std::vector<MJob> &js = host_jobs.back();
        for (const PlannedJob &J : g.jobs) js.push_back(J.j);
        keep.emplace_back(new Scratch);
        Scratch &jt = *keep.back();
        if ((rc = scratch_alloc(jt, js.size() * sizeof(MJob), s))) return rc;
        if ((e = hipMemcpyAsync(jt.p, js.data(), js.size() * sizeof(MJob), hipMemcpyHostToDevice, s)) != hipSuccess)
            return hip_fail(e, "hipMemcpyAsync");
        keep.emplace_back(new Scratch);
        Scratch &tb = *keep.back();
        if ((rc = scratch_alloc(tb, g.table_words() * sizeof(uint32_t), s))) return rc;
        if ((e = launch_group(g, (const MJob *)jt.p, (uint32_t *)tb.p, s)) != hipSuccess)
            return hip_fail(e, "grouped modexp launch");
        const int n = (int)(count * rounds);
        hipLaunchKernelGGL(mr_check_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           (const uint32_t *)d_x.p, (const uint32_t *)d_cand.p, L, rounds, (int)count, step,
                           (uint8_t *)d_state.p);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "miller-rabin check launch");
    }
    hipLaunchKernelGGL(mr_verdict_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                       (const uint8_t *)d_state.p, (const uint8_t *)d_flag.p, rounds, (int)count,
                       (uint8_t *)d_verdict.p);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "miller-rabin verdict launch");
    if ((e = hipMemcpyAsync(verdict, d_verdict.p, count, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "miller-rabin verdict read-back");
    return RNS_OK;
}

}  // namespace api
}  // namespace rnsrsa
