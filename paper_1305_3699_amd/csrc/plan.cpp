// Host-side RNS planning (see plan.hpp).
#include "plan.hpp"

#include <algorithm>
#include <map>
#include <mutex>
#include <set>
#include <tuple>

#include "rnsrsa.h"

namespace rnsrsa {

const std::vector<Shape> &supported_shapes() {
    static const std::vector<Shape> shapes = {
#define RNSRSA_SHAPE(K, W) {K, W},
#define RNSRSA_BASE_SHAPE(K, W) {K, W},
#include "kernel_configs.inc"
#undef RNSRSA_BASE_SHAPE
#undef RNSRSA_SHAPE
    };
    return shapes;
}

bool channel_kernel(int K, int W) {
#define RNSRSA_SHAPE(k, w) \
    if (K == k && W == w) return true;
#include "kernel_configs.inc"
#undef RNSRSA_SHAPE
    return false;
}

int default_waves(int K) {
    for (const Shape &s : supported_shapes())
        if (s.K == K) return s.W;
    return 0;
}

bool shape_supported(int K, int W) {
    for (const Shape &s : supported_shapes())
        if (s.K == K && s.W == W) return true;
    return false;
}

static uint64_t splitmix64(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// 2K distinct primes from the chosen range, deterministic in (seed, K, attempt).
static std::vector<uint32_t> draw_primes(int K, int range, uint64_t seed, int attempt) {
    uint64_t s = seed ^ ((uint64_t)K << 40) ^ ((uint64_t)attempt << 20) ^ ((uint64_t)range << 60);
    uint64_t lo = range == RANGE_FULL ? (1ull << 31) + 1 : (1ull << 32) - (1ull << 24);
    uint64_t span = (1ull << 32) - lo;
    std::set<uint32_t> seen;
    std::vector<uint32_t> out;
    while ((int)out.size() < 2 * K) {
        // primes = 3 mod 4: for each of them one of +-a is a square for any
        // a != 0, which the matrix engine's scaled B residues rely on
        uint32_t c = (uint32_t)(lo + splitmix64(s) % span) | 3u;
        if (c <= (1u << 31) || seen.count(c) || !is_prime32(c)) continue;
        seen.insert(c);
        out.push_back(c);
    }
    return out;
}

static Limbs product(const std::vector<uint32_t> &ms) {
    Limbs r{1};
    for (uint32_t m : ms) r = bn_mul_word(r, m);
    return r;
}

static uint32_t prod_mod(const std::vector<uint32_t> &ms, uint32_t m) { return prod_mod32(ms, m); }

static std::shared_ptr<BaseSet> build_base(int K, int W, const std::vector<uint32_t> &primes) {
    auto bs = std::make_shared<BaseSet>();
    bs->K = K;
    bs->W = W;
    int KS = (K + W - 1) / W;
    bs->KP = KS * W;
    bs->B.assign(primes.begin(), primes.begin() + K);
    bs->Bp.assign(primes.begin() + K, primes.begin() + 2 * K);
    bs->M = product(bs->B);
    bs->Mp = product(bs->Bp);
    const Layout ly{K, bs->KP};
    const int KP = bs->KP;
    std::vector<uint32_t> &b = bs->blob;
    b.assign(ly.base_size(), 0);
    for (int c = 0; c < KP; c++) {
        uint32_t mi = bs->B[std::min(c, K - 1)], mj = bs->Bp[std::min(c, K - 1)];
        b[ly.mB() + c] = mi;
        b[ly.uB() + c] = inv2_32(mi);
        b[ly.mBp() + c] = mj;
        b[ly.uBp() + c] = inv2_32(mj);
    }
    for (int i = 0; i < K; i++) {
        uint32_t m = bs->B[i];
        uint32_t mp_mod = prod_mod(bs->Bp, m);                      // M' mod m_i
        uint32_t neg = mp_mod ? m - mp_mod : 0;
        b[ly.negMp() + i] = mulmod32(neg, pow2_64_mod(m), m);
    }
    for (int t = 0; t < K; t++) {
        uint32_t m = bs->Bp[t];
        std::vector<uint32_t> others;
        for (int j = 0; j < K; j++)
            if (j != t) others.push_back(bs->Bp[j]);
        uint32_t Mpt = prod_mod(others, m);                          // M'_t mod m'_t
        b[ly.MpInv() + t] = mulmod32(invmod32(Mpt, m), pow2_32_mod(m), m);
    }
    b[ly.scal() + 0] = inv2_32(bn_low(bs->Mp));
    b[ly.scal() + 1] = inv2_32(bn_low(bs->M));
    // C1[i][t] = (M_i mod m'_t) R^2 mod m'_t;  C1[i][KP] = M_i mod 2^32
    for (int i = 0; i < K; i++) {
        for (int t = 0; t < K; t++) {
            uint32_t m = bs->Bp[t];
            uint32_t Mi = mulmod32(prod_mod(bs->B, m), invmod32(bs->B[i] % m, m), m);
            b[ly.C1() + i * ly.crow() + t] = mulmod32(Mi, pow2_64_mod(m), m);
        }
        uint32_t w = 1;
        for (int j = 0; j < K; j++)
            if (j != i) w *= bs->B[j];
        b[ly.C1() + i * ly.crow() + KP] = w;
    }
    // C2[j][i] = (M'_j mod m_i) R^2 mod m_i;  C2[j][KP] = M'_j mod 2^32
    for (int j = 0; j < K; j++) {
        for (int i = 0; i < K; i++) {
            uint32_t m = bs->B[i];
            uint32_t Mj = mulmod32(prod_mod(bs->Bp, m), invmod32(bs->Bp[j] % m, m), m);
            b[ly.C2() + j * ly.crow() + i] = mulmod32(Mj, pow2_64_mod(m), m);
        }
        uint32_t w = 1;
        for (int t = 0; t < K; t++)
            if (t != j) w *= bs->Bp[t];
        b[ly.C2() + j * ly.crow() + KP] = w;
    }
    // limbs of M'_j and of M'
    for (int j = 0; j < K; j++) {
        std::vector<uint32_t> others;
        for (int t = 0; t < K; t++)
            if (t != j) others.push_back(bs->Bp[t]);
        Limbs Mj = product(others);
        for (int l = 0; l <= K && l < (int)Mj.size(); l++) b[ly.MpL() + j * (K + 1) + l] = Mj[l];
    }
    for (int l = 0; l <= K && l < (int)bs->Mp.size(); l++) b[ly.MpF() + l] = bs->Mp[l];
    return bs;
}

bool bounds_hold(const BaseSet &bs, const Limbs &N, int L) {
    Limbs k1 = bn_from_u64((uint64_t)bs.K + 1);
    if (bn_cmp(bn_mul(bn_mul(k1, k1), N), bs.M) > 0) return false;        // M >= (K+1)^2 N
    if (bn_cmp(bn_shl(Limbs{1}, 32u * L + 1), bs.M) > 0) return false;    // M >= 2^(32L+1)
    if (bn_cmp(bn_mul(k1, N), bs.Mp) > 0) return false;                   // M' >= (K+1) N
    for (uint32_t m : bs.B)
        if (bn_mod_word(N, m) == 0) return false;
    return true;
}

static std::mutex g_base_mu;
static std::map<std::tuple<int, int, int, uint64_t, int>, std::shared_ptr<BaseSet>> g_bases;

static std::shared_ptr<const BaseSet> cached_base(int K, int W, int range, uint64_t seed, int attempt) {
    std::lock_guard<std::mutex> lk(g_base_mu);
    auto key = std::make_tuple(K, W, range, seed, attempt);
    auto it = g_bases.find(key);
    if (it != g_bases.end()) return it->second;
    std::vector<uint32_t> pr = draw_primes(K, range, seed, attempt);
    std::sort(pr.begin(), pr.end(), [](uint32_t a, uint32_t b) { return a > b; });  // B gets the larger primes
    auto bs = build_base(K, W, pr);
    g_bases[key] = bs;
    return bs;
}

static void fill_modplan(const Limbs &N, int L, std::shared_ptr<const BaseSet> bs, ModPlan &mp) {
    const int K = bs->K, KP = bs->KP;
    const Layout ly{K, KP};
    mp.base = bs;
    mp.N = N;
    mp.L = L;
    mp.Mmod = bn_mod(bs->M, N);
    mp.R2 = bn_mod(bn_mul(mp.Mmod, mp.Mmod), N);
    std::vector<uint32_t> &b = mp.blob;
    b.assign(ly.mod_size(), 0);
    for (int i = 0; i < K; i++) {
        uint32_t m = bs->B[i];
        uint32_t ninv = invmod32(bn_mod_word(N, m), m);
        std::vector<uint32_t> others;
        for (int j = 0; j < K; j++)
            if (j != i) others.push_back(bs->B[j]);
        uint32_t Mi_inv = invmod32(prod_mod(others, m), m);
        uint32_t c = mulmod32(m - ninv, Mi_inv, m);                    // -N^-1 M_i^-1
        b[ly.c2B() + i] = mulmod32(c, pow2_64_mod(m), m);
    }
    for (int t = 0; t < K; t++) {
        uint32_t m = bs->Bp[t];
        uint32_t nm = bn_mod_word(N, m);
        b[ly.NnBp() + t] = nm ? m - nm : 0;
        uint32_t minv = invmod32(prod_mod(bs->B, m), m);
        b[ly.MiBp() + t] = mulmod32(minv, pow2_64_mod(m), m);
    }
    for (int i = 0; i < K; i++) b[ly.one() + i] = bn_mod_word(mp.Mmod, bs->B[i]);
    for (int t = 0; t < K; t++) b[ly.one() + KP + t] = bn_mod_word(mp.Mmod, bs->Bp[t]);
    b[ly.one() + 2 * KP] = bn_low(mp.Mmod);
    b[ly.mscal() + 0] = bn_low(N);
    b[ly.mscal() + 1] = (uint32_t)L;
    for (int l = 0; l < L && l < K; l++) b[ly.Nl() + l] = l < (int)N.size() ? N[l] : 0;
}

int make_modplan(const Limbs &Nin, int L, const PlanOptions &opt, ModPlan &out, std::string &err) {
    Limbs N = Nin;
    bn_trim(N);
    if (bn_cmp(N, Limbs{2}) < 0) { err = "modulus must be >= 2"; return RNS_ERANGE; }
    if (L <= 0 || (int)N.size() > L) { err = "modulus does not fit its limb count"; return RNS_EINVAL; }
    if (opt.waves && !opt.k && !opt.primes) { err = "waves needs an explicit k"; return RNS_EINVAL; }
    if (opt.primes) {
        if (opt.n_primes % 2 || opt.n_primes == 0) { err = "explicit base needs 2k primes"; return RNS_EINVAL; }
        int K = (int)(opt.n_primes / 2);
        int W = opt.waves ? opt.waves : default_waves(K);
        if (!shape_supported(K, W)) { err = "no kernel for this k / waves"; return RNS_EUNSUPPORTED; }
        std::vector<uint32_t> pr(opt.primes, opt.primes + opt.n_primes);
        std::set<uint32_t> uniq(pr.begin(), pr.end());
        if ((int)uniq.size() != 2 * K) { err = "explicit primes must be distinct"; return RNS_EINVAL; }
        for (uint32_t p : pr)
            if (p <= (1u << 31) || !is_prime32(p)) { err = "explicit primes must be primes in (2^31, 2^32)"; return RNS_EINVAL; }
        auto bs = build_base(K, W, pr);
        for (uint32_t m : bs->B)
            if (bn_mod_word(N, m) == 0) { err = "a channel prime divides the modulus"; return RNS_EFACTOR; }
        if (!bounds_hold(*bs, N, L)) { err = "explicit base too small for this modulus"; return RNS_ERANGE; }
        fill_modplan(N, L, bs, out);
        return RNS_OK;
    }
    if (opt.range != RANGE_HIGH && opt.range != RANGE_FULL) { err = "bad prime range"; return RNS_EINVAL; }
    std::vector<int> ks;
    if (opt.k) {
        ks.push_back(opt.k);
    } else {
        for (const Shape &s : supported_shapes())
            if (ks.empty() || ks.back() != s.K) ks.push_back(s.K);
        std::sort(ks.begin(), ks.end());
        ks.erase(std::unique(ks.begin(), ks.end()), ks.end());
    }
    for (int K : ks) {
        if (K < L + 1) continue;
        int W = opt.waves ? opt.waves : default_waves(K);
        if (!shape_supported(K, W)) { err = "no kernel for this k / waves"; return RNS_EUNSUPPORTED; }
        for (int attempt = 0; attempt < 8; attempt++) {
            auto bs = cached_base(K, W, opt.range, opt.seed, attempt);
            if (bounds_hold(*bs, N, L)) {
                fill_modplan(N, L, bs, out);
                return RNS_OK;
            }
        }
    }
    err = "no supported base size satisfies the RNS bounds for this modulus";
    return RNS_ERANGE;
}

int make_modplan_on(const Limbs &Nin, int L, std::shared_ptr<const BaseSet> bs, ModPlan &out, std::string &err) {
    Limbs N = Nin;
    bn_trim(N);
    if (bn_cmp(N, Limbs{2}) < 0) { err = "modulus must be >= 2"; return RNS_ERANGE; }
    if (L <= 0 || (int)N.size() > L) { err = "modulus does not fit its limb count"; return RNS_EINVAL; }
    for (uint32_t m : bs->B)
        if (bn_mod_word(N, m) == 0) { err = "a channel prime divides the modulus"; return RNS_EFACTOR; }
    if (!bounds_hold(*bs, N, L)) { err = "base set too small for this modulus"; return RNS_ERANGE; }
    fill_modplan(N, L, bs, out);
    return RNS_OK;
}

std::vector<uint32_t> make_entry_table(const ModPlan &mp, const std::vector<Limbs> &Y, int L) {
    const BaseSet &bs = *mp.base;
    const int K = bs.K, KP = bs.KP;
    const Layout ly{K, KP};
    const int rows = (int)Y.size() * L, cols = ly.ecols();
    std::vector<uint32_t> e((size_t)rows * cols, 0);
    // row j: residues of 2^(32 (j mod L)) Y_h (h = j / L) times 2^64, chained
    // per channel through the factor 2^32 mod m
    auto fill = [&](uint32_t m, size_t col) {
        const uint32_t w32 = pow2_32_mod(m), r2 = pow2_64_mod(m);
        for (size_t h = 0; h < Y.size(); h++) {
            uint32_t v = mulmod32(bn_mod_word(Y[h], m), r2, m);
            for (int l = 0; l < L; l++) {
                e[(h * (size_t)L + l) * cols + col] = v;
                v = mulmod32(v, w32, m);
            }
        }
    };
    for (int i = 0; i < K; i++) fill(bs.B[i], (size_t)i);
    for (int t = 0; t < K; t++) fill(bs.Bp[t], (size_t)KP + t);
    for (int j = 0; j < rows; j++) e[(size_t)j * cols + 2 * KP] = (j % L) ? 0u : bn_low(Y[j / L]);
    return e;
}

}  // namespace rnsrsa
