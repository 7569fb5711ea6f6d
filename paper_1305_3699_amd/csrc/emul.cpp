// Host model of the exponentiation kernels: the same constant tables, channel
// reductions and exponent schedule as kernels.hip, run sequentially over all
// channels of one element at a time.  Used by tests on machines without a
// GPU to check the planning and the arithmetic; the device entry points never
// call it.
#include "emul.hpp"

#include <algorithm>

namespace rnsrsa {

namespace {

struct State {
    std::vector<uint32_t> b, p;  // K residues in B and in B'
    uint32_t r = 0;              // redundant channel
};

struct Ctx {
    const BaseSet &bs;
    const std::vector<uint32_t> &bc;
    const std::vector<uint32_t> &mc;
    Layout ly;
    std::vector<uint32_t> xip;  // xi' of the last product
};

// One RNS Montgomery product x <- x*y*M^-1, steps (i)-(iv) of kernels.hip.
uint32_t mm(Ctx &c, State &x, const State &y, bool full) {
    const int K = c.bs.K, KP = c.bs.KP;
    const Layout &LY = c.ly;
    const auto &bc = c.bc;
    const auto &mc = c.mc;
    std::vector<uint32_t> xi(K), a1(K);
    for (int i = 0; i < K; i++) {
        uint32_t m = bc[LY.mB() + i], u = bc[LY.uB() + i];
        xi[i] = mulredc(mulredc(x.b[i], y.b[i], m, u), mc[LY.c2B() + i], m, u);
    }
    for (int t = 0; t < K; t++) a1[t] = mulredc(x.p[t], y.p[t], bc[LY.mBp() + t], bc[LY.uBp() + t]);
    const uint32_t sr = x.r * y.r;
    uint32_t qr = 0;
    for (int i = 0; i < K; i++) qr += xi[i] * bc[LY.C1() + i * LY.crow() + KP];
    c.xip.assign(K, 0);
    for (int t = 0; t < K; t++) {
        Acc sum;
        for (int i = 0; i < K; i++) acc_mac(sum, xi[i], bc[LY.C1() + i * LY.crow() + t]);
        uint32_t m = bc[LY.mBp() + t], u = bc[LY.uBp() + t];
        uint32_t q = acc_redc(sum, m, u);
        uint32_t a2 = mulredc(q, mc[LY.NnBp() + t], m, u);
        uint32_t s = a1[t] - a2;
        s = a1[t] < a2 ? s + m : s;
        uint32_t r = mulredc(s, mc[LY.MiBp() + t], m, u);
        x.p[t] = r;
        c.xip[t] = mulredc(r, bc[LY.MpInv() + t], m, u);
    }
    const uint32_t rr = (sr + qr * mc[LY.mscal()]) * bc[LY.scal() + 1];
    uint32_t s2 = 0;
    for (int j = 0; j < K; j++) s2 += c.xip[j] * bc[LY.C2() + j * LY.crow() + KP];
    const uint32_t alpha = (s2 - rr) * bc[LY.scal()];
    if (full) {
        for (int i = 0; i < K; i++) {
            Acc s;
            for (int j = 0; j < K; j++) acc_mac(s, c.xip[j], bc[LY.C2() + j * LY.crow() + i]);
            acc_mac16(s, alpha, bc[LY.negMp() + i]);
            x.b[i] = acc_redc(s, bc[LY.mB() + i], bc[LY.uB() + i]);
        }
    }
    x.r = rr;
    return alpha;
}

State entry(const Ctx &c, const std::vector<uint32_t> &E, const uint32_t *src, int nl) {
    const int K = c.bs.K, KP = c.bs.KP;
    const Layout &LY = c.ly;
    State a;
    a.b.resize(K);
    a.p.resize(K);
    for (int t = 0; t < K; t++) {
        Acc sb, sp;
        for (int l = 0; l < nl; l++) {
            acc_mac(sb, src[l], E[(size_t)l * LY.ecols() + t]);
            acc_mac(sp, src[l], E[(size_t)l * LY.ecols() + KP + t]);
        }
        a.b[t] = acc_redc(sb, c.bc[LY.mB() + t], c.bc[LY.uB() + t]);
        a.p[t] = acc_redc(sp, c.bc[LY.mBp() + t], c.bc[LY.uBp() + t]);
    }
    uint32_t zr = 0;
    for (int l = 0; l < nl; l++) zr += src[l] * E[(size_t)l * LY.ecols() + 2 * KP];
    a.r = zr;
    return a;
}

// RNS -> binary from xi' and alpha, then reduction to [0, N): L limbs.
std::vector<uint32_t> leave(const Ctx &c, uint32_t alpha, int L) {
    const int K = c.bs.K;
    const Layout &LY = c.ly;
    std::vector<uint32_t> acc(L + 1), tmp(L + 1);
    uint64_t cy = 0;
    for (int l = 0; l <= L; l++) {
        Acc s;
        s.lo = cy;
        for (int j = 0; j < K; j++) acc_mac(s, c.xip[j], c.bc[LY.MpL() + j * (K + 1) + l]);
        uint64_t lo;
        uint32_t top;
        acc_value(s, lo, top);
        acc[l] = (uint32_t)lo;
        cy = (lo >> 32) | ((uint64_t)top << 32);
    }
    uint64_t carry = 0;
    uint32_t borrow = 0;
    for (int l = 0; l <= L; l++) {
        uint64_t p = (uint64_t)alpha * c.bc[LY.MpF() + l] + carry;
        carry = p >> 32;
        uint32_t v = acc[l], pl = (uint32_t)p;
        uint32_t d = v - pl, d2 = d - borrow;
        borrow = (v < pl) | (d < borrow);
        acc[l] = d2;
    }
    int qb = 0;
    while ((1 << qb) <= K) qb++;
    for (int b = qb - 1; b >= 0; b--) {
        uint32_t br = 0;
        for (int l = 0; l <= L; l++) {
            uint32_t nlo = l < L ? c.mc[LY.Nl() + l] : 0u;
            uint32_t nhi = (b && l > 0) ? (c.mc[LY.Nl() + l - 1] >> (32 - b)) : 0u;
            uint32_t nl = (nlo << b) | nhi;
            uint32_t v = acc[l];
            uint32_t d = v - nl, d2 = d - br;
            br = (v < nl) | (d < br);
            tmp[l] = d2;
        }
        if (!br) acc = tmp;
    }
    acc.resize(L);
    return acc;
}

uint32_t digit(const uint32_t *e, int nlimbs, int nd, int w, int di) {
    int lo = (nd - 1 - di) * w;
    int limb = lo >> 5, sh = lo & 31;
    uint64_t v = e[limb];
    if (limb + 1 < nlimbs) v |= (uint64_t)e[limb + 1] << 32;
    return (uint32_t)(v >> sh) & ((1u << w) - 1u);
}

State one_state(const Ctx &c) {
    const int K = c.bs.K, KP = c.bs.KP;
    State s;
    s.b.assign(c.mc.begin() + c.ly.one(), c.mc.begin() + c.ly.one() + K);
    s.p.assign(c.mc.begin() + c.ly.one() + KP, c.mc.begin() + c.ly.one() + KP + K);
    s.r = c.mc[c.ly.one() + 2 * KP];
    return s;
}

State unit_state(int K) {
    State s;
    s.b.assign(K, 1);
    s.p.assign(K, 1);
    s.r = 1;
    return s;
}

}  // namespace

void emul_modexp(const ModPlan &mp, const std::vector<uint32_t> &E, int in_limbs, const uint32_t *base,
                 const uint32_t *exp, int exp_limbs, size_t exp_stride, int window, uint32_t *out,
                 size_t batch) {
    const BaseSet &bs = *mp.base;
    const int K = bs.K;
    Ctx c{bs, bs.blob, mp.blob, Layout{K, bs.KP}, {}};
    const int w = window, T = 1 << w;
    const int nd = (32 * exp_limbs + w - 1) / w;
    const State one = one_state(c), unit = unit_state(K);
    for (size_t e = 0; e < batch; e++) {
        const uint32_t *ep = exp + e * exp_stride;
        State a = entry(c, E, base + e * (size_t)in_limbs, in_limbs);
        mm(c, a, unit, true);
        std::vector<State> tbl(T);
        tbl[0] = one;
        tbl[1] = a;
        for (int j = 2; j < T; j++) {
            mm(c, a, tbl[1], true);
            tbl[j] = a;
        }
        int di = 0;
        if (exp_stride == 0) {
            while (di < nd && digit(ep, exp_limbs, nd, w, di) == 0) di++;
            if (di < nd) {
                a = tbl[digit(ep, exp_limbs, nd, w, di)];
                di++;
            } else {
                a = one;
            }
        } else {
            a = one;
        }
        for (; di < nd; di++) {
            for (int s = 0; s < w; s++) {
                State sq = a;
                mm(c, a, sq, true);
            }
            uint32_t d = digit(ep, exp_limbs, nd, w, di);
            if (exp_stride != 0 || d != 0) mm(c, a, tbl[d], true);
        }
        uint32_t alpha = mm(c, a, unit, false);
        std::vector<uint32_t> r = leave(c, alpha, mp.L);
        std::copy(r.begin(), r.end(), out + e * (size_t)mp.L);
    }
}

void emul_mont_mul(const ModPlan &mp, const uint32_t *x, const uint32_t *y, uint32_t *out, size_t batch) {
    const BaseSet &bs = *mp.base;
    const int K = bs.K;
    Ctx c{bs, bs.blob, mp.blob, Layout{K, bs.KP}, {}};
    for (size_t e = 0; e < batch; e++) {
        State a, b;
        a.b.resize(K);
        a.p.resize(K);
        b.b.resize(K);
        b.p.resize(K);
        for (int i = 0; i < K; i++) {
            a.b[i] = x[(size_t)i * batch + e];
            b.b[i] = y[(size_t)i * batch + e];
            a.p[i] = x[(size_t)(K + i) * batch + e];
            b.p[i] = y[(size_t)(K + i) * batch + e];
        }
        a.r = x[(size_t)(2 * K) * batch + e];
        b.r = y[(size_t)(2 * K) * batch + e];
        mm(c, a, b, true);
        for (int i = 0; i < K; i++) {
            out[(size_t)i * batch + e] = a.b[i];
            out[(size_t)(K + i) * batch + e] = a.p[i];
        }
        out[(size_t)(2 * K) * batch + e] = a.r;
    }
}

}  // namespace rnsrsa
