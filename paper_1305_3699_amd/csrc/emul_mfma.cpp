// Host model of the matrix-core exponentiation kernel (kernels_mfma.hpp).
//
// It runs the kernel's steps on the same tables, element by element.  Each
// base-extension constant is rebuilt from the A-tile bytes through the
// hardware operand layout of v_mfma_i32_16x16x64_i8 (lane l holds row l%16
// and K indices 16*(l/16) + byte), independently of how the tables were
// packed, so a packing mistake shows up here before any GPU run.
#include <algorithm>
#include <climits>
#include <cstdint>

#include "emul.hpp"
#include "plan_mfma.hpp"

namespace rnsrsa {

namespace {

struct MCtx {
    const MfmaTables &T;
    const MLayout ly;
    int K;
    // [W][4MT][4 bytes][64*KSTEPS]: the A-row byte b of each slot, per K index
    // (A2s: the key's second extension for scaled B residues)
    std::vector<int16_t> A1, A2, A2s;
    bool sq;    // B residues kept scaled (x R s_i): the key holds the scaled form

    MCtx(const MfmaTables &t, bool scaled) : T(t), ly(t.shape), K(t.shape.K), sq(scaled && t.scaled) {
        const int SW = 4 * ly.MT, KK = 64 * ly.KSTEPS();
        A1.assign((size_t)ly.W * SW * 4 * KK, 0);
        A2.assign((size_t)ly.W * SW * 4 * KK, 0);
        if (sq) A2s.assign(A2.size(), 0);
        for (int w = 0; w < ly.W; w++)
            for (int s = 0; s < SW; s++)
                for (int b = 0; b < 4; b++)
                    for (int kap = 0; kap < KK; kap++) {
                        const size_t at = (((size_t)w * SW + s) * 4 + b) * KK + kap;
                        A1[at] = tile_byte(T.key.data() + ly.a1(), w, s, b, kap);
                        A2[at] = tile_byte(T.base.data() + ly.a2(), w, s, b, kap);
                        if (sq) A2s[at] = tile_byte(T.key.data() + ly.a2s(), w, s, b, kap);
                    }
    }
    // byte b of slot s's constant at K index kap, read through the hardware
    // operand layout: A row 4g+b of tile mt lives in lane (row + 16 lg), K
    // index 16 lg + j of the k-step in byte j of that lane's 16 bytes
    int16_t tile_byte(const uint32_t *tiles, int w, int s, int b, int kap) const {
        const int mt = s / 4, g = s % 4, ks = kap / 64, k = kap % 64, lg = k / 16, j = k % 16;
        const int lane = 16 * lg + 4 * g + b;
        const uint32_t word = tiles[((((size_t)w * ly.MT + mt) * ly.KSTEPS() + ks) * 64 + lane) * 4 + j / 4];
        return (int16_t)(int8_t)(word >> (8 * (j % 4)));
    }
    // per-lane constant of slot s in wave w: any lane of group s%4
    uint32_t slot(size_t off, size_t fields, int field, int w, int s) const {
        return T.base[off + (((size_t)w * ly.MT + s / 4) * fields + field) * 64 + 16 * (s % 4)];
    }
    uint32_t kslot(size_t off, size_t fields, int field, int w, int s) const {
        return T.key[off + (((size_t)w * ly.MT + s / 4) * fields + field) * 64 + 16 * (s % 4)];
    }
    int channel(int w, int s) const { return mfma_slot_channel(ly, w, s / 4, s % 4); }
    bool real(int w, int s) const {
        const int c = channel(w, s);
        return c >= 0 && c < K;
    }
};

struct MSt {
    std::vector<uint32_t> b, p;  // [W][4MT][NM]
    std::vector<uint32_t> r;     // [NM]
};

uint32_t pack_digits(uint32_t v) { return v ^ kDigitBias; }

// cleared when a REDC input of steps (iii)/(iv) leaves [0, m 2^32), where the
// kernel's one-step reduction would be wrong
thread_local bool t_in_range = true;

// REDC of P + S + m 2^sh, the kernel's reduction of an extension output
uint32_t reduce_offset(uint64_t P, int64_t S, uint32_t m, uint32_t u, int sh) {
    const __int128 T = (__int128)P + S + ((__int128)m << sh);
    if (T < 0 || T >= ((__int128)m << 32)) t_in_range = false;
    const uint64_t x = (uint64_t)T;
    return redc((uint32_t)x, (uint32_t)(x >> 32), m, u);
}

// The four byte partials P_b of slot row `row` ([W][4MT] index) for element
// e: exact sums over K indices of A byte times digit byte, the int32 values
// the matrix core accumulates (the host checks they fit).
void partials(const std::vector<int16_t> &A, size_t row, const std::vector<uint32_t> &dig, int e, int KK, int BROW,
              int64_t P[4]) {
    for (int b = 0; b < 4; b++) {
        const int16_t *a = A.data() + (row * 4 + b) * KK;
        int64_t s = 0;
        for (int kap = 0; kap < KK; kap++) {
            const uint32_t word = dig[(size_t)e * BROW + kap / 4];
            s += (int64_t)a[kap] * (int8_t)(word >> (8 * (kap % 4)));
        }
        if (s < INT32_MIN || s > INT32_MAX) t_in_range = false;
        P[b] = s;
    }
}

// S = sum_b 2^(8b) P_b as the kernel forms it: up to 127 channels the pairs
// P_0 + 2^8 P_1 and P_2 + 2^8 P_3 in int32 (a wrap there would change S by a
// multiple of 2^32 and is flagged), wider bases every partial in 64 bits.
int64_t combine(const int64_t P[4], int K) {
    if (mfma_pair_fits_i32(K)) {
        const int64_t t1 = P[0] + 256 * P[1], t2 = P[2] + 256 * P[3];
        if (t1 < INT32_MIN || t1 > INT32_MAX || t2 < INT32_MIN || t2 > INT32_MAX) t_in_range = false;
        return (int64_t)(int32_t)(uint32_t)t1 + (int64_t)(int32_t)(uint32_t)t2 * 65536;
    }
    return P[0] + 256 * P[1] + 65536 * P[2] + 16777216 * P[3];
}

int64_t extension(const std::vector<int16_t> &A, size_t row, const std::vector<uint32_t> &dig, int e, int KK, int BROW,
                  int K) {
    int64_t P[4];
    partials(A, row, dig, e, KK, BROW, P);
    return combine(P, K);
}

// One product x <- x*y*M^-1 for the NM elements of one workgroup; fills dig2
// (xi' digits) and returns nothing; with full == false skips the second extension.
void mm(const MCtx &c, MSt &x, const MSt &y, std::vector<uint32_t> &dig1, std::vector<uint32_t> &dig2, bool full) {
    const MLayout &ly = c.ly;
    const int SW = 4 * ly.MT, NM = ly.NM(), KK = 64 * ly.KSTEPS(), BROW = ly.BROW();
    const int sh = mfma_offset_shift(c.K);
    const uint32_t Mpinv_r = c.T.base[ly.bscal()], Minv_r = c.T.base[ly.bscal() + 1], N_r = c.T.key[ly.kscal()];
    auto idx = [&](int w, int s, int e) { return ((size_t)w * SW + s) * NM + e; };
    for (int w = 0; w < ly.W; w++)
        for (int s = 0; s < SW; s++) {
            const uint32_t m = c.slot(ly.slotB(), 3, 0, w, s), u = c.slot(ly.slotB(), 3, 1, w, s);
            const uint32_t ci = c.kslot(ly.slotC(), 1, 0, w, s);
            for (int e = 0; e < NM; e++) {
                // sigma_i x y c_i: one REDC of the operands when they are scaled
                const uint32_t t = mulredc(x.b[idx(w, s, e)], y.b[idx(w, s, e)], m, u);
                const uint32_t xi = c.sq ? t : mulredc(t, ci, m, u);
                if (c.real(w, s)) dig1[(size_t)e * BROW + c.channel(w, s)] = pack_digits(xi);
            }
        }
    std::vector<uint32_t> rr(NM);
    for (int e = 0; e < NM; e++) {
        // every wave carries the same redundant row; take wave 0's
        const int64_t S = extension(c.A1, (size_t)0 * SW + SW - 1, dig1, e, KK, BROW, c.K);
        rr[e] = (x.r[e] * y.r[e] + (uint32_t)S * N_r) * Minv_r;
    }
    for (int w = 0; w < ly.W; w++)
        for (int s = 0; s < SW; s++) {
            const uint32_t m = c.slot(ly.slotP(), 4, 0, w, s), u = c.slot(ly.slotP(), 4, 1, w, s);
            const uint32_t H = c.slot(ly.slotP(), 4, 2, w, s);
            for (int e = 0; e < NM; e++) {
                const int64_t S = extension(c.A1, (size_t)w * SW + s, dig1, e, KK, BROW, c.K);
                // x' y' + S + m 2^sh in one REDC
                const uint32_t r = reduce_offset((uint64_t)x.p[idx(w, s, e)] * y.p[idx(w, s, e)], S, m, u, sh);
                x.p[idx(w, s, e)] = r;
                if (c.real(w, s)) dig2[(size_t)e * BROW + c.channel(w, s)] = pack_digits(mulredc(r, H, m, u));
            }
        }
    for (int e = 0; e < NM; e++) x.r[e] = rr[e];
    if (!full) return;
    const std::vector<int16_t> &A2 = c.sq ? c.A2s : c.A2;
    for (int w = 0; w < ly.W; w++) {
        std::vector<uint32_t> alpha(NM);
        for (int e = 0; e < NM; e++) {
            const int64_t S = extension(A2, (size_t)w * SW + SW - 1, dig2, e, KK, BROW, c.K);
            alpha[e] = ((uint32_t)S - rr[e]) * Mpinv_r;
        }
        for (int s = 0; s < SW; s++) {
            const uint32_t m = c.slot(ly.slotB(), 3, 0, w, s), u = c.slot(ly.slotB(), 3, 1, w, s);
            const uint32_t nu = c.sq ? c.kslot(ly.sqB(), 3, 0, w, s) : c.slot(ly.slotB(), 3, 2, w, s);
            for (int e = 0; e < NM; e++) {
                const int64_t S = extension(A2, (size_t)w * SW + s, dig2, e, KK, BROW, c.K);
                x.b[idx(w, s, e)] = reduce_offset((uint64_t)alpha[e] * nu, S, m, u, sh);
            }
        }
    }
}

uint32_t digit_of(const uint32_t *e, int nlimbs, int nd, int w, int di) {
    const int lo = (nd - 1 - di) * w;
    const int limb = lo >> 5, sh = lo & 31;
    uint64_t v = e[limb];
    if (limb + 1 < nlimbs) v |= (uint64_t)e[limb + 1] << 32;
    return (uint32_t)(v >> sh) & ((1u << w) - 1u);
}

}  // namespace

bool emul_modexp_mfma(const ModPlan &mp, const MfmaTables &T, const std::vector<uint32_t> &E, int in_limbs,
                      const uint32_t *base, const uint32_t *exp, int exp_limbs, size_t exp_stride, int window,
                      uint32_t *out, size_t batch, bool scaled) {
    t_in_range = true;
    const MCtx c(T, scaled);
    const MLayout &ly = c.ly;
    const int K = c.K, SW = 4 * ly.MT, NM = ly.NM(), BROW = ly.BROW(), L = mp.L;
    const int w = window, TT = 1 << w;
    const int nd = (32 * exp_limbs + w - 1) / w;
    const size_t ecols = ly.ecols();
    auto idx = [&](int wv, int s, int e) { return ((size_t)wv * SW + s) * NM + e; };
    for (size_t g0 = 0; g0 < batch; g0 += NM) {
        std::vector<uint32_t> dig1((size_t)NM * BROW, 0), dig2((size_t)NM * BROW, 0);
        for (int e = 0; e < NM; e++) {
            dig1[(size_t)e * BROW + K] = 1;
            dig2[(size_t)e * BROW + K] = 1;
        }
        // unit: y = 1 for the exit product; unit_in for the entry product,
        // whose first operand comes from the entry table unscaled (with
        // scaled B residues its B part is sigma_i c_i, so the one-REDC
        // quotient digit is right and the result comes out scaled)
        MSt a, unit, unit_in, one;
        for (MSt *st : {&a, &unit, &unit_in, &one}) {
            st->b.assign((size_t)ly.W * SW * NM, 0);
            st->p.assign((size_t)ly.W * SW * NM, 0);
            st->r.assign(NM, 0);
        }
        for (int wv = 0; wv < ly.W; wv++)
            for (int s = 0; s < SW; s++) {
                const uint32_t m = c.slot(ly.slotB(), 3, 0, wv, s), u = c.slot(ly.slotB(), 3, 1, wv, s);
                const uint32_t mpp = c.slot(ly.slotP(), 4, 0, wv, s), up = c.slot(ly.slotP(), 4, 1, wv, s);
                const uint32_t kap = c.slot(ly.slotP(), 4, 3, wv, s);
                const size_t colB = (size_t)wv * SW + s, colP = (size_t)ly.W * SW + wv * SW + s;
                for (int e = 0; e < NM; e++) {
                    const size_t el = g0 + e;
                    Acc sb, sp;
                    for (int l = 0; l < in_limbs; l++) {
                        const uint32_t v = el < batch ? base[el * in_limbs + l] : 0u;
                        acc_mac(sb, v, E[(size_t)l * ecols + colB]);
                        acc_mac(sp, v, E[(size_t)l * ecols + colP]);
                    }
                    a.b[idx(wv, s, e)] = acc_redc(sb, m, u);
                    a.p[idx(wv, s, e)] = acc_redc(sp, mpp, up);
                    unit.b[idx(wv, s, e)] = c.sq ? c.kslot(ly.sqB(), 3, 1, wv, s) : 0u - m;
                    unit.p[idx(wv, s, e)] = kap;
                    unit_in.b[idx(wv, s, e)] = c.sq ? c.kslot(ly.slotC(), 1, 0, wv, s) : 0u - m;
                    unit_in.p[idx(wv, s, e)] = kap;
                    one.b[idx(wv, s, e)] = c.sq ? c.kslot(ly.sqB(), 3, 2, wv, s) : c.kslot(ly.one(), 2, 0, wv, s);
                    one.p[idx(wv, s, e)] = c.kslot(ly.one(), 2, 1, wv, s);
                }
            }
        for (int e = 0; e < NM; e++) {
            const size_t el = g0 + e;
            uint32_t z = 0;
            for (int l = 0; l < in_limbs; l++) z += (el < batch ? base[el * in_limbs + l] : 0u) * E[(size_t)l * ecols + ecols - 1];
            a.r[e] = z;
            unit.r[e] = 1;
            unit_in.r[e] = 1;
            one.r[e] = T.key[ly.one() + (size_t)ly.W * ly.MT * 2 * 64];
        }
        mm(c, a, unit_in, dig1, dig2, true);
        std::vector<MSt> tbl(TT);
        tbl[0] = one;
        tbl[1] = a;
        if (exp_stride == 0) {
            // sliding windows over odd powers (x^2 kept in slot 2)
            if (w > 1) {
                MSt x2 = a, sqr = a;
                mm(c, x2, sqr, dig1, dig2, true);
                tbl[2] = x2;
                for (int j = 3; j < TT; j += 2) {
                    MSt t = tbl[j - 2];
                    mm(c, t, x2, dig1, dig2, true);
                    tbl[j] = t;
                }
            }
            auto bit = [&](int i) { return (exp[i >> 5] >> (i & 31)) & 1u; };
            int top = -1;
            for (int i = 32 * exp_limbs - 1; i >= 0 && top < 0; i--)
                if (bit(i)) top = i;
            auto window = [&](int i, int *low) {
                int lo = std::max(i - w + 1, 0);
                while (!bit(lo)) lo++;
                uint32_t d = 0;
                for (int b = i; b >= lo; b--) d = 2 * d + bit(b);
                *low = lo;
                return d;
            };
            if (top < 0) {
                a = one;
            } else {
                int low;
                a = tbl[window(top, &low)];
                int i = low - 1;
                while (i >= 0) {
                    if (!bit(i)) {
                        MSt sqr = a;
                        mm(c, a, sqr, dig1, dig2, true);
                        i--;
                        continue;
                    }
                    const uint32_t d = window(i, &low);
                    for (int q = 0; q < i - low + 1; q++) {
                        MSt sqr = a;
                        mm(c, a, sqr, dig1, dig2, true);
                    }
                    mm(c, a, tbl[d], dig1, dig2, true);
                    i = low - 1;
                }
            }
        } else {
            for (int j = 2; j < TT; j++) {
                tbl[j] = tbl[j - 1];
                mm(c, tbl[j], tbl[1], dig1, dig2, true);
            }
            a = one;
            for (int di = 0; di < nd; di++) {
                for (int s = 0; s < w; s++) {
                    MSt sq = a;
                    mm(c, a, sq, dig1, dig2, true);
                }
                MSt y = one;
                for (int e = 0; e < NM; e++) {
                    const size_t el = std::min(g0 + e, batch - 1);
                    const uint32_t d = digit_of(exp + el * exp_stride, exp_limbs, nd, w, di);
                    for (size_t q = 0; q < y.b.size(); q++)
                        if ((int)(q % NM) == e) {
                            y.b[q] = tbl[d].b[q];
                            y.p[q] = tbl[d].p[q];
                        }
                    y.r[e] = tbl[d].r[e];
                }
                mm(c, a, y, dig1, dig2, true);
            }
        }
        mm(c, a, unit, dig1, dig2, false);
        // leave the RNS, element by element
        for (int e = 0; e < NM && g0 + e < batch; e++) {
            std::vector<uint32_t> X(K), acc(L + 1), tmp(L + 1);
            uint32_t s2 = 0;
            for (int j = 0; j < K; j++) {
                const uint32_t v = dig2[(size_t)e * BROW + j] ^ kDigitBias;
                X[j] = v;
                s2 += v * T.base[ly.mplo() + j];
            }
            const uint32_t alpha = (s2 - a.r[e]) * T.base[ly.bscal()];
            uint64_t cy = 0;
            for (int l = 0; l <= L; l++) {
                Acc sum;
                sum.lo = cy;
                for (int j = 0; j < K; j++) acc_mac(sum, X[j], T.base[ly.MpL() + (size_t)j * (K + 1) + l]);
                uint64_t lo;
                uint32_t top;
                acc_value(sum, lo, top);
                acc[l] = (uint32_t)lo;
                cy = (lo >> 32) | ((uint64_t)top << 32);
            }
            uint64_t carry = 0;
            uint32_t borrow = 0;
            for (int l = 0; l <= L; l++) {
                const uint64_t p = (uint64_t)alpha * T.base[ly.MpF() + l] + carry;
                carry = p >> 32;
                const uint32_t v = acc[l], pl = (uint32_t)p;
                const uint32_t d = v - pl, d2 = d - borrow;
                borrow = (v < pl) | (d < borrow);
                acc[l] = d2;
            }
            int qb = 0;
            while ((1 << qb) <= K + 1) qb++;
            for (int b = qb - 1; b >= 0; b--) {
                uint32_t br = 0;
                for (int l = 0; l <= L; l++) {
                    const uint32_t nlo = l < L ? T.key[ly.Nl() + l] : 0u;
                    const uint32_t nhi = (b && l > 0) ? (T.key[ly.Nl() + l - 1] >> (32 - b)) : 0u;
                    const uint32_t nl = (nlo << b) | nhi;
                    const uint32_t v = acc[l];
                    const uint32_t d = v - nl, d2 = d - br;
                    br = (v < nl) | (d < br);
                    tmp[l] = d2;
                }
                if (!br) acc = tmp;
            }
            std::copy(acc.begin(), acc.begin() + L, out + (g0 + e) * (size_t)L);
        }
    }
    return t_in_range;
}

bool emul_mfma_extension(const MfmaTables &T, int which, const uint32_t *xi, size_t batch, int64_t *parts,
                         int64_t *value) {
    t_in_range = true;
    const MCtx c(T, false);
    const MLayout &ly = c.ly;
    const int K = c.K, SW = 4 * ly.MT, BROW = ly.BROW(), KK = 64 * ly.KSTEPS(), rows = ly.W * SW;
    std::vector<uint32_t> dig((size_t)BROW, 0);
    dig[K] = 1;
    for (size_t e = 0; e < batch; e++) {
        for (int i = 0; i < K; i++) dig[i] = pack_digits(xi[e * K + i]);
        for (int r = 0; r < rows; r++) {
            int64_t P[4];
            partials(which == 1 ? c.A1 : c.A2, (size_t)r, dig, 0, KK, BROW, P);
            for (int b = 0; b < 4; b++) parts[(e * rows + r) * 4 + b] = P[b];
            value[e * rows + r] = combine(P, K);
        }
    }
    return t_in_range;
}

void emul_mfma_matrix(const MfmaTables &T, int which, int8_t *A) {
    const MCtx c(T, false);
    const std::vector<int16_t> &src = which == 1 ? c.A1 : c.A2;
    for (size_t i = 0; i < src.size(); i++) A[i] = (int8_t)src[i];
}

}  // namespace rnsrsa
