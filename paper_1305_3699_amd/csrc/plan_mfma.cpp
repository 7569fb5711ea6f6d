// Host-side tables of the matrix-core exponentiation kernel (plan_mfma.hpp).
#include "plan_mfma.hpp"


namespace rnsrsa {

bool mfma_shape_for(int K, MfmaShape &out, int group) {
    // the first shape listed for K with the preferred group, else the first for K
    for (int pass = group ? 0 : 1; pass < 2; pass++) {
#define RNSRSA_MSHAPE(k, w, mt, nt)                                    \
    if (K == k && (pass == 1 || group == 16 * (nt))) {               \
        out = MfmaShape{k, w, mt, nt};                                 \
        return true;                                                   \
    }
#include "kernel_configs_mfma.inc"
#undef RNSRSA_MSHAPE
    }
    return false;
}

namespace {

// Representative of v mod m in [kDigitSplit - m, kDigitSplit): four balanced bytes.
int64_t balanced(uint32_t v, uint32_t m) { return v >= kDigitSplit ? (int64_t)v - m : (int64_t)v; }

// Representative of v mod 2^32 in [-0x80808080, 0x7F7F7F7F].
int64_t balanced32(uint32_t v) { return v > 0x7F7F7F7Fu ? (int64_t)v - ((int64_t)1 << 32) : (int64_t)v; }

// Signed byte b of a balanced value V = sum_b d_b 256^b, d_b in [-128, 127].
int8_t digit(int64_t V, int b) {
    uint32_t u = (uint32_t)(V + 0x80808080ll);
    return (int8_t)((int)((u >> (8 * b)) & 0xFFu) - 128);
}

uint32_t pow2_mod(uint32_t e, uint32_t m) { return powmod32(2, e, m); }

// A square root of a modulo the odd prime p (Tonelli-Shanks; p = 3 mod 4 in
// one step), or false when a is not a square mod p.
bool sqrt_mod(uint32_t a, uint32_t p, uint32_t *root) {
    a %= p;
    if (a == 0) {
        *root = 0;
        return true;
    }
    if (powmod32(a, (p - 1) / 2, p) != 1) return false;   // Euler's criterion
    if (p % 4 == 3) {
        *root = powmod32(a, ((uint64_t)p + 1) / 4, p);
        return true;
    }
    uint32_t q = p - 1;
    int s = 0;
    while (!(q & 1)) {
        q >>= 1;
        s++;
    }
    uint32_t z = 2;
    while (powmod32(z, (p - 1) / 2, p) != p - 1) z++;     // a non-residue
    uint32_t c = powmod32(z, q, p), x = powmod32(a, ((uint64_t)q + 1) / 2, p), t = powmod32(a, q, p);
    int m = s;
    while (t != 1) {
        int i = 0;
        uint32_t t2 = t;
        while (t2 != 1) {
            t2 = mulmod32(t2, t2, p);
            i++;
        }
        uint32_t b = c;
        for (int j = 0; j < m - i - 1; j++) b = mulmod32(b, b, p);
        x = mulmod32(x, b, p);
        c = mulmod32(b, b, p);
        t = mulmod32(t, c, p);
        m = i;
    }
    *root = x;
    return true;
}

// One matrix of A tiles [W][MT][KSTEPS][64 lanes][16 bytes] from a value
// function V(slot channel t (-1: redundant), input channel i (K: offset slot), digit a).
template <class F>
void fill_tiles(const MfmaShape &sh, uint32_t *dst, F value) {
    const int KS = sh.KSTEPS();
    for (int w = 0; w < sh.W; w++)
        for (int mt = 0; mt < sh.MT; mt++)
            for (int ks = 0; ks < KS; ks++)
                for (int l = 0; l < 64; l++) {
                    uint32_t words[4] = {0, 0, 0, 0};
                    const int row = l % 16, g = row / 4, b = row % 4;
                    const int t = mfma_slot_channel(sh, w, mt, g);
                    for (int j = 0; j < 16; j++) {
                        const int kappa = 64 * ks + 16 * (l / 16) + j;
                        const int ch = kappa / 4, a = kappa % 4;
                        int64_t V = 0;
                        if (t < sh.K && ch <= sh.K && (ch < sh.K || a == 0)) V = value(t, ch, a);
                        words[j / 4] |= (uint32_t)(uint8_t)digit(V, b) << (8 * (j % 4));
                    }
                    uint32_t *p = dst + ((((size_t)w * sh.MT + mt) * KS + ks) * 64 + l) * 4;
                    for (int q = 0; q < 4; q++) p[q] = words[q];
                }
}

// Per-lane slot table [W][MT][64] of f(channel) (channel -1 or >= K: junk).
template <class F>
void fill_slots(const MfmaShape &sh, uint32_t *dst, size_t field_stride, F f) {
    for (int w = 0; w < sh.W; w++)
        for (int mt = 0; mt < sh.MT; mt++)
            for (int l = 0; l < 64; l++) dst[((size_t)w * sh.MT + mt) * field_stride + l] = f(mfma_slot_channel(sh, w, mt, l / 16));
}

}  // namespace

MfmaTables make_mfma_tables(const ModPlan &mp, const MfmaShape &sh, bool with_base, bool allow_scaled) {
    const BaseSet &bs = *mp.base;
    const int K = bs.K;
    const MLayout &ly = sh;
    MfmaTables out;
    out.shape = sh;
    if (with_base) out.base.assign(ly.base_size(), 0);
    out.key.assign(ly.key_size(), 0);
    const Limbs &N = mp.N;

    // c_i = -N^-1 M_i^-1 mod m_i, and for the scaled form a sign sigma_i and
    // a root s_i with s_i^2 = sigma_i c_i R^-1 (mod m_i).  A product's
    // quotient digit x y c_i is then REDC(x R s_i * y R s_i) = sigma_i x y c_i:
    // the digit published for channel i is sigma_i xi_i mod m_i, so the first
    // extension takes sigma_i C_i as input i's constants and adds
    // sum_{sigma_i = -1} m_i C_i through its offset column.  (A zero digit
    // then stands for xi_i = m_i: the extension's q lies in [0, K M] instead
    // of [0, K M), which the bounds on the base already cover.)  For a
    // prime = 3 mod 4 one of c_i R^-1 and -c_i R^-1 is a square; the default
    // bases draw such primes.  Without a root for every channel the key keeps
    // sigma_i = 1 and the unscaled form only.
    std::vector<uint32_t> cB(K), sB(K, 1u);
    std::vector<int> sgn(K, 1);
    for (int i = 0; i < K; i++) {
        const uint32_t m = bs.B[i];
        std::vector<uint32_t> others;                                  // M_i mod m_i: product of the other primes
        for (int j = 0; j < K; j++)
            if (j != i) others.push_back(bs.B[j]);
        cB[i] = mulmod32(m - invmod32(bn_mod_word(N, m), m), invmod32(prod_mod32(others, m), m), m);
    }
    out.scaled = allow_scaled && ly.sq_ok();
    for (int i = 0; i < K && out.scaled; i++) {
        const uint32_t m = bs.B[i];
        const uint32_t a = mulmod32(cB[i], invmod32(pow2_32_mod(m), m), m);   // c_i R^-1
        if (sqrt_mod(a, m, &sB[i])) sgn[i] = 1;
        else if (sqrt_mod(m - a, m, &sB[i])) sgn[i] = -1;
        else out.scaled = false;
    }
    if (!out.scaled) {
        std::fill(sgn.begin(), sgn.end(), 1);
        std::fill(sB.begin(), sB.end(), 1u);
    }

    // Values of the two extensions' constant matrices, [t + 1][i][a] for output
    // channel t (-1: the redundant row), input channel i (K: the offset
    // column, digit a = 0 only) and digit a, computed once: the residues of
    // M_i = M / m_i modulo a prime m are prod(B) mod m times (m_i mod m)^-1,
    // and modulo 2^32 prod(B) times m_i^-1 (m_i odd).
    //
    // The digit words carry xi - kDigitBias; the offset column (input channel K,
    // digit value 1) adds kDigitBias * sum_i C_i back, so each extension is the
    // exact integer sum_i xi_i C_i.
    //
    // BE1 (key table): slot t of B' gets sum_i xi_i M_i * G_t with
    // G_t = N R^2 M^-2 mod m'_t, so that one REDC yields q N M^-1 * (R M^-1);
    // the redundant row gets sum_i xi_i M_i mod 2^32.
    // BE2 (base table): slot i of B gets sum_j xi'_j M'_j R^2 mod m_i; the
    // redundant row sum_j xi'_j M'_j mod 2^32.
    // With input signs sig (the first extension of the scaled form) input i's
    // constants are sig_i C_i and the offset column adds
    // kDigitBias sum_i sig_i C_i + sum_{sig_i = -1} m_i C_i.
    const size_t KK = (size_t)(K + 1) * 4;
    auto ext_values = [&](const std::vector<uint32_t> &in, const std::vector<uint32_t> &outm, auto scale,
                          const std::vector<int> &sig) {
        std::vector<int64_t> V((size_t)(K + 1) * KK, 0);
        uint32_t prod_lo = 1;
        for (uint32_t m : in) prod_lo *= m;
        uint32_t off_lo = 0;
        for (int i = 0; i < K; i++) {
            const uint32_t mi_lo = prod_lo * inv2_32(in[i]);
            const uint32_t ci_lo = sig[i] < 0 ? 0u - mi_lo : mi_lo;
            off_lo += kDigitBias * ci_lo + (sig[i] < 0 ? in[i] * mi_lo : 0u);
            for (int a = 0; a < 4; a++) V[(size_t)i * 4 + a] = balanced32(ci_lo << (8 * a));
        }
        V[(size_t)K * 4] = balanced32(off_lo);
        for (int t = 0; t < K; t++) {
            const uint32_t m = outm[t], f = scale(t);
            const uint32_t P = prod_mod32(in, m);
            uint64_t off = 0;
            int64_t *row = V.data() + (size_t)(t + 1) * KK;
            for (int i = 0; i < K; i++) {
                const uint32_t mi = mulmod32(P, invmod32(in[i] % m, m), m);
                const uint32_t ci = sig[i] < 0 && mi ? m - mi : mi;
                off = (off + mulmod32(kDigitBias % m, ci, m)) % m;
                if (sig[i] < 0) off = (off + mulmod32(in[i] % m, mi, m)) % m;
                for (int a = 0; a < 4; a++)
                    row[(size_t)i * 4 + a] = balanced(mulmod32(mulmod32(ci, pow2_mod(8 * a, m), m), f, m), m);
            }
            row[(size_t)K * 4] = balanced(mulmod32((uint32_t)off, f, m), m);
        }
        return V;
    };
    const std::vector<int> plus(K, 1);
    std::vector<uint32_t> G(K);
    for (int t = 0; t < K; t++) {
        uint32_t m = bs.Bp[t];
        uint32_t minv = invmod32(prod_mod32(bs.B, m), m);
        G[t] = mulmod32(mulmod32(bn_mod_word(N, m), pow2_64_mod(m), m), mulmod32(minv, minv, m), m);
    }
    const std::vector<int64_t> V1 = ext_values(bs.B, bs.Bp, [&](int t) { return G[t]; }, sgn);
    fill_tiles(sh, out.key.data() + ly.a1(),
               [&](int t, int i, int a) -> int64_t { return V1[(size_t)(t + 1) * KK + (size_t)i * 4 + a]; });
    auto okc = [&](int t) { return t >= 0 && t < K; };
    if (with_base) {
    const std::vector<int64_t> V2 = ext_values(bs.Bp, bs.B, [&](int t) { return pow2_64_mod(bs.B[t]); }, plus);
    fill_tiles(sh, out.base.data() + ly.a2(),
               [&](int t, int j, int a) -> int64_t { return V2[(size_t)(t + 1) * KK + (size_t)j * 4 + a]; });
    auto Mpj_lo = [&](int j) {
        uint32_t w = 1;
        for (int t = 0; t < K; t++)
            if (t != j) w *= bs.Bp[t];
        return w;
    };

    // per-slot constants; junk slots use a valid modulus and zero constants
    const uint32_t mB0 = bs.B[K - 1], mP0 = bs.Bp[K - 1];
    const size_t fs = (size_t)3 * 64;      // [W][MT][3][64]
    fill_slots(sh, out.base.data() + ly.slotB() + 0 * 64, fs, [&](int t) { return okc(t) ? bs.B[t] : mB0; });
    fill_slots(sh, out.base.data() + ly.slotB() + 1 * 64, fs, [&](int t) { return inv2_32(okc(t) ? bs.B[t] : mB0); });
    fill_slots(sh, out.base.data() + ly.slotB() + 2 * 64, fs, [&](int t) -> uint32_t {
        if (!okc(t)) return 0;
        uint32_t m = bs.B[t], mpm = prod_mod32(bs.Bp, m);
        return mulmod32(mpm ? m - mpm : 0, pow2_64_mod(m), m);   // nu = -M' R^2 mod m_i
    });
    const size_t fp = (size_t)4 * 64;      // [W][MT][4][64]
    fill_slots(sh, out.base.data() + ly.slotP() + 0 * 64, fp, [&](int t) { return okc(t) ? bs.Bp[t] : mP0; });
    fill_slots(sh, out.base.data() + ly.slotP() + 1 * 64, fp, [&](int t) { return inv2_32(okc(t) ? bs.Bp[t] : mP0); });
    fill_slots(sh, out.base.data() + ly.slotP() + 3 * 64, fp, [&](int t) -> uint32_t {
        if (!okc(t)) return 0;
        uint32_t m = bs.Bp[t];
        return mulmod32(pow2_32_mod(m), invmod32(prod_mod32(bs.B, m), m), m);     // kappa = R M^-1
    });
    fill_slots(sh, out.base.data() + ly.slotP() + 2 * 64, fp, [&](int t) -> uint32_t {
        if (!okc(t)) return 0;
        uint32_t m = bs.Bp[t];
        std::vector<uint32_t> others;
        for (int j = 0; j < K; j++)
            if (j != t) others.push_back(bs.Bp[j]);
        return mulmod32(prod_mod32(bs.B, m), invmod32(prod_mod32(others, m), m), m);   // H = M (M'_t)^-1
    });
    // leaving the RNS: m'_j, M'_j mod 2^32, limbs of M'_j and of M'
    for (int j = 0; j < K; j++) {
        out.base[ly.mpj() + j] = bs.Bp[j];
        out.base[ly.mplo() + j] = Mpj_lo(j);
        std::vector<uint32_t> others;
        for (int t = 0; t < K; t++)
            if (t != j) others.push_back(bs.Bp[t]);
        Limbs Mj{1};
        for (uint32_t x : others) Mj = bn_mul_word(Mj, x);
        for (int l = 0; l <= K && l < (int)Mj.size(); l++) out.base[ly.MpL() + (size_t)j * (K + 1) + l] = Mj[l];
    }
    for (int l = 0; l <= K && l < (int)bs.Mp.size(); l++) out.base[ly.MpF() + l] = bs.Mp[l];
    out.base[ly.bscal() + 0] = inv2_32(bn_low(bs.Mp));
    out.base[ly.bscal() + 1] = inv2_32(bn_low(bs.M));
    const size_t fc = (size_t)3 * 64;      // [W][MT][3][64]
    fill_slots(sh, out.base.data() + ly.mmconv() + 0 * 64, fc,
               [&](int t) -> uint32_t { return okc(t) ? pow2_64_mod(bs.B[t]) : 0; });
    fill_slots(sh, out.base.data() + ly.mmconv() + 1 * 64, fc, [&](int t) -> uint32_t {
        if (!okc(t)) return 0;
        const uint32_t m = bs.Bp[t];
        return mulmod32(pow2_64_mod(m), invmod32(prod_mod32(bs.B, m), m), m);
    });
    fill_slots(sh, out.base.data() + ly.mmconv() + 2 * 64, fc,
               [&](int t) -> uint32_t { return okc(t) ? prod_mod32(bs.B, bs.Bp[t]) : 0; });
    }

    // key: sigma_i c_i mod m_i; "one" = M mod N in the kept representation
    fill_slots(sh, out.key.data() + ly.slotC(), 64, [&](int t) -> uint32_t {
        if (!okc(t)) return 0;
        return sgn[t] < 0 && cB[t] ? bs.B[t] - cB[t] : cB[t];
    });
    const size_t os = (size_t)2 * 64;      // [W][MT][2][64]
    fill_slots(sh, out.key.data() + ly.one(), os, [&](int t) -> uint32_t {
        if (!okc(t)) return 0;
        uint32_t m = bs.B[t];
        return mulmod32(bn_mod_word(mp.Mmod, m), pow2_32_mod(m), m);
    });
    fill_slots(sh, out.key.data() + ly.one() + 64, os, [&](int t) -> uint32_t {
        if (!okc(t)) return 0;
        uint32_t m = bs.Bp[t];
        uint32_t kappa = mulmod32(pow2_32_mod(m), invmod32(prod_mod32(bs.B, m), m), m);   // R M^-1
        return mulmod32(bn_mod_word(mp.Mmod, m), kappa, m);
    });
    out.key[ly.one() + (size_t)sh.W * sh.MT * 2 * 64] = bn_low(mp.Mmod);
    for (int l = 0; l < K && l < (int)N.size(); l++) out.key[ly.Nl() + l] = N[l];
    out.key[ly.kscal() + 0] = bn_low(N);
    if (out.scaled) {
        // second extension with row t scaled by s_t (R^2 s_t mod m_t)
        const std::vector<int64_t> V2s = ext_values(
            bs.Bp, bs.B, [&](int t) { return mulmod32(pow2_64_mod(bs.B[t]), sB[t], bs.B[t]); }, plus);
        fill_tiles(sh, out.key.data() + ly.a2s(),
                   [&](int t, int j, int a) -> int64_t { return V2s[(size_t)(t + 1) * KK + (size_t)j * 4 + a]; });
        const size_t fq = (size_t)3 * 64;      // [W][MT][3][64]
        fill_slots(sh, out.key.data() + ly.sqB() + 0 * 64, fq, [&](int t) -> uint32_t {
            if (!okc(t)) return 0;
            const uint32_t m = bs.B[t], mpm = prod_mod32(bs.Bp, m);
            return mulmod32(mulmod32(mpm ? m - mpm : 0, pow2_64_mod(m), m), sB[t], m);   // nu s_t
        });
        fill_slots(sh, out.key.data() + ly.sqB() + 1 * 64, fq, [&](int t) -> uint32_t {
            return okc(t) ? mulmod32(pow2_32_mod(bs.B[t]), sB[t], bs.B[t]) : 0;      // R s_t
        });
        fill_slots(sh, out.key.data() + ly.sqB() + 2 * 64, fq, [&](int t) -> uint32_t {
            if (!okc(t)) return 0;
            const uint32_t m = bs.B[t];
            return mulmod32(mulmod32(bn_mod_word(mp.Mmod, m), pow2_32_mod(m), m), sB[t], m);   // one s_t
        });
    }
    return out;
}

std::vector<uint32_t> make_mfma_entry_table(const ModPlan &mp, const MfmaShape &sh, const std::vector<Limbs> &Y,
                                            int L) {
    const BaseSet &bs = *mp.base;
    const int K = bs.K;
    const MLayout &ly = sh;
    const size_t cols = ly.ecols();
    const int rows = (int)Y.size() * L;
    const int SW = 4 * sh.MT;    // slots per wave
    std::vector<uint32_t> e((size_t)rows * cols, 0);
    // row j holds the residues of v = Y_h 2^(32 (j mod L)), h = j / L: per
    // channel, (Y_h mod m) times (2^32 mod m)^(j mod L), times the channel's
    // constant factor
    for (int w = 0; w < sh.W; w++)
        for (int s = 0; s < SW; s++) {
            const int t = mfma_slot_channel(sh, w, s / 4, s % 4);
            if (t < 0 || t >= K) continue;
            const uint32_t m = bs.B[t], mp2 = bs.Bp[t];
            const uint32_t r3 = mulmod32(pow2_64_mod(m), pow2_32_mod(m), m);
            const uint32_t r3p = mulmod32(mulmod32(pow2_64_mod(mp2), pow2_32_mod(mp2), mp2),
                                          invmod32(prod_mod32(bs.B, mp2), mp2), mp2);
            const uint32_t w32 = pow2_32_mod(m), w32p = pow2_32_mod(mp2);
            for (size_t h = 0; h < Y.size(); h++) {
                uint32_t vm = mulmod32(bn_mod_word(Y[h], m), r3, m);
                uint32_t vp = mulmod32(bn_mod_word(Y[h], mp2), r3p, mp2);
                for (int l = 0; l < L; l++) {
                    const size_t j = h * (size_t)L + l;
                    e[j * cols + (size_t)w * SW + s] = vm;
                    e[j * cols + (size_t)sh.W * SW + (size_t)w * SW + s] = vp;
                    vm = mulmod32(vm, w32, m);
                    vp = mulmod32(vp, w32p, mp2);
                }
            }
        }
    for (int j = 0; j < rows; j++) e[(size_t)j * cols + cols - 1] = (j % L) ? 0u : bn_low(Y[j / L]);
    return e;
}

}  // namespace rnsrsa
