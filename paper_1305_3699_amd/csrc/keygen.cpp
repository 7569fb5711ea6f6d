// Primality steps of key generation on the GPU (include/rnsrsa.h): trial
// division by the first small primes (Sec. 4.3) and Miller-Rabin tests whose
// exponentiations run in RNS in the Montgomery domain (Sec. 3.2), one
// modulus per candidate, all candidates in grouped launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "bn_host.hpp"
#include "jobs.hpp"
#include "kernels_impl.hpp"
#include "mr_gpu.hpp"

using namespace rnsrsa;
using namespace rnsrsa::api;

namespace {

constexpr int kMaxSmallPrimes = 10000;   // the 10,000th prime is 104729
constexpr int kMaxRounds = 64;

// The first `count` primes, sieve of Eratosthenes below 104730.
std::vector<uint32_t> first_primes(int count) {
    const uint32_t bound = 104730;
    std::vector<uint8_t> composite(bound, 0);
    std::vector<uint32_t> out;
    for (uint32_t i = 2; i < bound && (int)out.size() < count; i++) {
        if (composite[i]) continue;
        out.push_back(i);
        for (uint64_t j = (uint64_t)i * i; j < bound; j += i) composite[j] = 1;
    }
    return out;
}

struct SmallPrimes {
    uint32_t *p = nullptr;   // the primes
    double *inv = nullptr;   // 1/p rounded to double
};

// Device tables of the small primes and their reciprocals, per device, kept
// for the life of the process.
int small_primes(int dev, SmallPrimes *out) {
    static std::mutex mu;
    static std::map<int, SmallPrimes> tables;
    std::lock_guard<std::mutex> lk(mu);
    auto it = tables.find(dev);
    if (it == tables.end()) {
        const std::vector<uint32_t> pr = first_primes(kMaxSmallPrimes);
        std::vector<double> inv(pr.size());
        for (size_t i = 0; i < pr.size(); i++) inv[i] = 1.0 / (double)pr[i];
        SmallPrimes t;
        hipError_t e = hipMalloc((void **)&t.p, pr.size() * sizeof(uint32_t));
        if (e == hipSuccess) e = hipMalloc((void **)&t.inv, inv.size() * sizeof(double));
        if (e == hipSuccess) e = hipMemcpy(t.p, pr.data(), pr.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(t.inv, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            if (t.p) hipFree(t.p);
            if (t.inv) hipFree(t.inv);
            return hip_fail(e, "small-prime tables");
        }
        it = tables.emplace(dev, t).first;
    }
    *out = it->second;
    return RNS_OK;
}

constexpr int kTdThreads = 256;

// One workgroup per candidate (its limbs in LDS); lane t reduces the
// candidate modulo primes t, t + 256, ... by Horner's rule over the 32-bit
// limbs.  Each step divides x = r 2^32 + limb < p 2^32 < 2^49 by p through
// the double reciprocal: the estimate is off by at most one (relative error
// below 2^-51 on a quotient below 2^48), fixed by one add or subtract.
__global__ __launch_bounds__(kTdThreads) void trial_division_kernel(const uint32_t *__restrict__ cand, int limbs,
                                                                     const uint32_t *__restrict__ primes,
                                                                     const double *__restrict__ inv, int n_primes,
                                                                     uint8_t *__restrict__ flags) {
    extern __shared__ uint32_t c[];
    const uint32_t *__restrict__ src = cand + (size_t)blockIdx.x * limbs;
    for (int l = threadIdx.x; l < limbs; l += kTdThreads) c[l] = src[l];
    __syncthreads();
    int top = limbs - 1;
    while (top > 0 && c[top] == 0) top--;
    int divisible = 0;
    for (int t = threadIdx.x; t < n_primes; t += kTdThreads) {
        const uint32_t p = primes[t];
        const double ip = inv[t];
        int64_t r = 0;
        for (int l = top; l >= 0; l--) {
            const int64_t x = (int64_t)(((uint64_t)r << 32) | c[l]);
            const int64_t q = (int64_t)((double)x * ip);
            r = x - q * (int64_t)p;
            if (r < 0) r += p;
            else if (r >= (int64_t)p) r -= p;
        }
        if (r == 0 && !(top == 0 && c[0] == p)) divisible = 1;
    }
    const int any = __syncthreads_or(divisible);
    if (threadIdx.x == 0) flags[blockIdx.x] = any ? 0 : 1;
}

struct Candidate {
    std::unique_ptr<rns_ctx> ctx;
    Limbs nm1;       // N - 1
    int s = 0;       // N - 1 = 2^s d, d odd
    Limbs d;
};

// Launch x <- x^e (mod each candidate's N) for the listed candidates, x rows
// of `rounds` elements in place; exponent e: per candidate (exps, L limbs
// each) or the shared `shared_exp` of one limb.
int exponentiate(const std::vector<Candidate> &cs, const std::vector<size_t> &which, uint32_t *d_x,
                 const uint32_t *d_exps, const uint32_t *d_shared_exp, uint32_t shared_exp, int L, int rounds,
                 hipStream_t s, std::vector<std::unique_ptr<Scratch>> &keep,
                 std::vector<std::vector<MJob>> &host_jobs) {
    std::map<std::tuple<int, int, int>, JobGroup> groups;
    for (size_t i : which) {
        const rns_ctx *c = cs[i].ctx.get();
        uint32_t *x = d_x + i * (size_t)rounds * L;
        const bool shared = d_exps == nullptr;
        const uint32_t *exp = shared ? d_shared_exp : d_exps + i * (size_t)L;
        const int exp_limbs = shared ? 1 : L;
        if (c->engine != RNS_ENGINE_MATRIX) {
            int rc = run_modexp(c, nullptr, entry_of(c), nullptr, x, L, exp, nullptr, exp_limbs, 0, x, nullptr, L,
                                (size_t)rounds, s);
            if (rc) return rc;
            continue;
        }
        const MLayout &sh = c->mshape;
        JobGroup &g = groups[std::make_tuple(sh.K, sh.W, sh.MT)];
        if (g.jobs.empty()) {
            g.shape = sh;
            g.device = c->device;
            g.scaled = true;
        }
        g.scaled = g.scaled && c->mscaled;
        const std::vector<uint32_t> eh = shared ? std::vector<uint32_t>{shared_exp} : cs[i].d;
        PlannedJob J{};
        J.j.mb = c->d_mbase;
        J.j.mk = c->d_mkey;
        J.j.E = c->d_mentry;
        J.j.exp = exp;
        J.j.in = x;
        J.j.out = x;
        J.j.batch = rounds;
        J.j.in_limbs = L;
        J.j.in_stride = L;
        J.j.L = c->plan.L;
        J.j.out_stride = L;
        J.j.exp_limbs = exp_limbs;
        J.j.exp_stride = 0;
        J.j.window = best_window(eh, 0);
        J.cost = mm_count(eh, J.j.window);
        g.jobs.push_back(J);
    }
    for (auto &kv : groups) {
        JobGroup &g = kv.second;
        finish_group(g);
        retile_group(g, g.device);
        // the job table's host copy lives until the caller synchronises
        host_jobs.emplace_back();
        std::vector<MJob> &js = host_jobs.back();
        for (const PlannedJob &J : g.jobs) js.push_back(J.j);
        keep.emplace_back(new Scratch);
        Scratch &jt = *keep.back();
        int rc = scratch_alloc(jt, js.size() * sizeof(MJob), s);
        if (rc) return rc;
        hipError_t e = hipMemcpyAsync(jt.p, js.data(), js.size() * sizeof(MJob), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
        keep.emplace_back(new Scratch);
        Scratch &tb = *keep.back();
        if ((rc = scratch_alloc(tb, g.table_words() * sizeof(uint32_t), s))) return rc;
        if ((e = launch_group(g, (const MJob *)jt.p, (uint32_t *)tb.p, s)) != hipSuccess)
            return hip_fail(e, "grouped modexp launch");
    }
    return RNS_OK;
}

// Arazi's inversion in RNS (Sec. 3.1): d = (1 + f t) / e with t = -f^-1 mod e
// (a scalar), channel by channel on the owned B' channels and the redundant
// one: d_j = (1 + f_j t) e^-1 mod m'_j, then d in binary through the base's
// exit (CRT over B' with alpha from the redundant channel; exact since
// d < n).  One element per lane (f of fl limbs, d of L limbs).
template <int K, int W>
__global__ __launch_bounds__(64 * W) void arazi_kernel(const uint32_t *__restrict__ bc, const uint32_t *__restrict__ mc,
                                                       const uint32_t *__restrict__ f, int fl, uint32_t t, uint32_t e,
                                                       uint32_t einv32, int L, uint32_t *__restrict__ d, int batch) {
    using S = Shp<K, W>;
    constexpr int KS = S::KS, KP = S::KP;
    constexpr Layout LY{K, KP};
    __shared__ uint32_t lds[2 * KP * 64];
    uint32_t *xip = lds + KP * 64;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int msg = blockIdx.x * 64 + lane;
    const bool active = msg < batch;
    const uint32_t *__restrict__ fr = f + (size_t)(active ? msg : 0) * fl;
    for (int c = 0; c < KS; c++) {
        const int j = wave * KS + c;
        if (j >= K) break;
        const uint32_t m = bc[LY.mBp() + j];
        uint64_t r = 0;
        for (int l = fl - 1; l >= 0; l--) r = ((r << 32) | fr[l]) % m;
        // e^-1 mod m' by Fermat (m' prime, e not a multiple of it)
        uint64_t inv = 1, b = e % m;
        for (uint32_t x = m - 2; x; x >>= 1) {
            if (x & 1u) inv = inv * b % m;
            b = b * b % m;
        }
        const uint64_t dj = (1 + r * t % m) % m * inv % m;
        xip[j * 64 + lane] = mulredc((uint32_t)dj, bc[LY.MpInv() + j], m, bc[LY.uBp() + j]);   // d_j (M'_j)^-1
    }
    const uint32_t dr = (1u + fr[0] * t) * einv32;                                               // d mod 2^32
    __syncthreads();
    uint64_t s2 = 0;
    for (int j = 0; j < K; j++) s2 += (uint64_t)xip[j * 64 + lane] * bc[LY.C2() + j * LY.crow() + KP];
    const uint32_t alpha = ((uint32_t)s2 - dr) * bc[LY.scal()];
    __syncthreads();
    if (wave != 0) return;
    rns_exit<K, W>(bc, mc, lds, lds + (L + 1) * 64, xip, alpha, L, lane);
    if (active)
        for (int l = 0; l < L; l++) d[(size_t)msg * L + l] = lds[l * 64 + lane];
}

// d = e^-1 mod f by arazi_kernel on the channel tables of context c (whose
// modulus exceeds f).  Returns RNS_OK or the error code (also recorded for
// rns_last_error).
int arazi_inverse(const rns_ctx *c, const Limbs &f, uint32_t e, Limbs &d, hipStream_t s) {
    const int K = c->plan.base->K, W = c->plan.base->W, L = c->plan.L;
    for (uint32_t m : c->plan.base->Bp)
        if (e % m == 0) return fail(RNS_EUNSUPPORTED, "e is a channel prime");
    const uint32_t fe = bn_mod_word(f, e), fi = invmod32(fe, e);
    if (!fi) return fail(RNS_EINVAL, "e not coprime to (p-1)(q-1)");
    const uint32_t t = (e - fi) % e;
    Limbs fl = f;
    fl.resize((size_t)L, 0u);
    Scratch df, dd;
    int rc = scratch_alloc(df, (size_t)L * sizeof(uint32_t), s);
    if (!rc) rc = scratch_alloc(dd, (size_t)L * sizeof(uint32_t), s);
    if (rc) return rc;
    hipError_t he = hipMemcpyAsync(df.p, fl.data(), (size_t)L * sizeof(uint32_t), hipMemcpyHostToDevice, s);
    if (he != hipSuccess) return hip_fail(he, "hipMemcpyAsync");
    bool launched = false;
#define RNSRSA_SHAPE(k, w)                                                                                        \
    if (!launched && K == k && W == w) {                                                                      \
        hipLaunchKernelGGL((arazi_kernel<k, w>), dim3(1), dim3(64 * w), 0, s, c->d_base, c->d_mod,              \
                           (const uint32_t *)df.p, L, t, e, inv2_32(e), L, (uint32_t *)dd.p, 1);               \
        launched = true;                                                                                          \
    }
#include "kernel_configs.inc"
#undef RNSRSA_SHAPE
    if (!launched) return fail(RNS_EUNSUPPORTED, "no channel kernel for this k");
    if ((he = hipGetLastError()) != hipSuccess) return hip_fail(he, "arazi launch");
    d.assign((size_t)L, 0u);
    if ((he = hipMemcpyAsync(d.data(), dd.p, (size_t)L * sizeof(uint32_t), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (he = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(he, "arazi read-back");
    bn_trim(d);
    return RNS_OK;
}

// a^-1 mod p for odd p > 1 by the binary extended Euclidean algorithm
// (invariants x1 a = u and x2 a = v mod p); false when gcd(a, p) > 1.
bool bn_modinv_odd(const Limbs &a, const Limbs &p, Limbs &out) {
    const Limbs one{1};
    Limbs u = bn_mod(a, p), v = p, x1 = one, x2;
    auto half = [&](Limbs &x) {
        if (bn_low(x) & 1u) x = bn_add(x, p);
        x = bn_shr1(x);
    };
    auto sub_mod = [&](const Limbs &x, const Limbs &y) {
        return bn_cmp(x, y) >= 0 ? bn_sub(x, y) : bn_sub(bn_add(x, p), y);
    };
    if (bn_is_zero(u)) return false;
    while (bn_cmp(u, one) != 0 && bn_cmp(v, one) != 0) {
        while (!(bn_low(u) & 1u)) {
            u = bn_shr1(u);
            half(x1);
        }
        while (!(bn_low(v) & 1u)) {
            v = bn_shr1(v);
            half(x2);
        }
        if (bn_cmp(u, v) >= 0) {
            u = bn_sub(u, v);
            x1 = sub_mod(x1, x2);
        } else {
            v = bn_sub(v, u);
            x2 = sub_mod(x2, x1);
        }
        if (bn_is_zero(u) || bn_is_zero(v)) return false;
    }
    out = bn_cmp(u, one) == 0 ? x1 : x2;
    return true;
}

bool rows_equal(const uint32_t *a, const Limbs &b, int L) {
    for (int l = 0; l < L; l++)
        if (a[l] != (l < (int)b.size() ? b[l] : 0u)) return false;
    return true;
}

}  // namespace

extern "C" {

int rsa_trial_division(const uint32_t *cand, size_t count, int limbs, int n_primes, uint8_t *flags,
                       void *hip_stream) {
    if (count == 0) return ok();
    if (!cand || !flags) return fail(RNS_EINVAL, "null buffer");
    if (limbs <= 0 || limbs > 4096) return fail(RNS_EINVAL, "limbs must be in 1..4096");
    if (n_primes <= 0 || n_primes > kMaxSmallPrimes) return fail(RNS_EINVAL, "n_primes must be in 1..10000");
    if (count > (size_t)INT32_MAX) return fail(RNS_EINVAL, "count too large");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    SmallPrimes sp;
    int rc = RNS_OK;
    try {
        rc = small_primes(dev, &sp);
    } catch (const std::bad_alloc &) {
        rc = fail(RNS_ENOMEM, "out of host memory");
    }
    if (rc) return rc;
    hipLaunchKernelGGL(trial_division_kernel, dim3((unsigned)count), dim3(kTdThreads), limbs * sizeof(uint32_t),
                       (hipStream_t)hip_stream, cand, limbs, sp.p, sp.inv, n_primes, flags);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "trial division launch");
    return ok();
}

int rsa_miller_rabin(const uint32_t *cand, size_t count, int limbs, const uint32_t *bases, int rounds,
                     uint8_t *verdict, void *hip_stream) {
    if (count == 0) return ok();
    if (!cand || !bases || !verdict) return fail(RNS_EINVAL, "null buffer");
    if (limbs <= 0 || limbs > 4096) return fail(RNS_EINVAL, "limbs must be in 1..4096");
    if (rounds <= 0 || rounds > kMaxRounds) return fail(RNS_EINVAL, "rounds must be in 1..64");
    if (count > (size_t)INT32_MAX / kMaxRounds) return fail(RNS_EINVAL, "count too large");
    hipStream_t s = (hipStream_t)hip_stream;
    const int L = limbs;
    const size_t row = (size_t)rounds * L;
    try {
        std::vector<Candidate> cs(count);
        for (size_t i = 0; i < count; i++) {
            Limbs N = bn_from_ptr(cand + i * L, (size_t)L);
            bn_trim(N);
            if (bn_low(N) % 2 == 0 || bn_cmp(N, Limbs{3}) <= 0) return fail(RNS_EINVAL, "candidates must be odd and > 3");
            Candidate &c = cs[i];
            c.nm1 = bn_sub(N, Limbs{1});
            for (int r = 0; r < rounds; r++) {
                Limbs a = bn_from_ptr(bases + i * row + (size_t)r * L, (size_t)L);
                bn_trim(a);
                if (bn_cmp(a, Limbs{2}) < 0 || bn_cmp(a, bn_sub(N, Limbs{2})) > 0)
                    return fail(RNS_EINVAL, "bases must lie in [2, N - 2]");
            }
            c.d = c.nm1;
            while (bn_low(c.d) % 2 == 0) {
                c.d = bn_shr1(c.d);
                c.s++;
            }
            c.d.resize((size_t)L, 0u);
        }
        // every candidate's tables built on the device when its base runs on
        // the matrix engine (the default bases do)
        {
            const int grc = miller_rabin_gpu(cand, count, L, bases, rounds, verdict, s);
            if (grc != RNS_EUNSUPPORTED) return grc ? grc : ok();
        }
        // otherwise one context per candidate, built on a pool of host
        // threads (each on the caller's device); errors are reported on this
        // thread
        int dev = 0;
        hipError_t de = hipGetDevice(&dev);
        if (de != hipSuccess) return hip_fail(de, "hipGetDevice");
        std::vector<int> crc(count, RNS_OK);
        std::atomic<size_t> next{0};
        auto work = [&] {
            if (hipSetDevice(dev) != hipSuccess) return;
            for (size_t i; (i = next.fetch_add(1)) < count;) {
                Limbs N = bn_from_ptr(cand + i * L, (size_t)L);
                bn_trim(N);
                rns_ctx *ctx = nullptr;
                crc[i] = make_context(N, L, &ctx);
                cs[i].ctx.reset(ctx);
            }
        };
        const unsigned nthreads =
            (unsigned)std::min<size_t>(count, std::min(16u, std::max(1u, std::thread::hardware_concurrency())));
        std::vector<std::thread> pool;
        for (unsigned t = 1; t < nthreads; t++) pool.emplace_back(work);
        work();
        for (std::thread &t : pool) t.join();
        for (size_t i = 0; i < count; i++) {
            if (crc[i] == RNS_OK && !cs[i].ctx) crc[i] = RNS_EDEVICE;
            if (crc[i] != RNS_OK) return fail(crc[i], "context set-up failed for candidate " + std::to_string(i));
        }
        // device: per-candidate exponents d, the rows of x (the bases first)
        std::vector<uint32_t> hd(count * (size_t)L);
        for (size_t i = 0; i < count; i++) std::copy(cs[i].d.begin(), cs[i].d.end(), hd.begin() + i * L);
        Scratch d_exps, d_x, d_two;
        int rc = scratch_alloc(d_exps, hd.size() * sizeof(uint32_t), s);
        if (!rc) rc = scratch_alloc(d_x, count * row * sizeof(uint32_t), s);
        if (!rc) rc = scratch_alloc(d_two, sizeof(uint32_t), s);
        if (rc) return rc;
        const uint32_t two = 2;
        hipError_t e = hipMemcpyAsync(d_exps.p, hd.data(), hd.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_x.p, bases, count * row * sizeof(uint32_t), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(d_two.p, &two, sizeof(uint32_t), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");

        // state per (candidate, base): 0 undecided, 1 passed, 2 failed
        std::vector<uint8_t> st(count * (size_t)rounds, 0);
        std::vector<uint32_t> hx(count * row);
        std::vector<std::unique_ptr<Scratch>> keep;
        std::vector<std::vector<MJob>> host_jobs;
        std::vector<size_t> which(count);
        for (size_t i = 0; i < count; i++) which[i] = i;
        for (int j = 0; !which.empty(); j++) {
            // j = 0: x = a^d; j > 0: x = x^2
            rc = j == 0 ? exponentiate(cs, which, (uint32_t *)d_x.p, (const uint32_t *)d_exps.p, nullptr, 0, L,
                                       rounds, s, keep, host_jobs)
                        : exponentiate(cs, which, (uint32_t *)d_x.p, nullptr, (const uint32_t *)d_two.p, 2u, L,
                                       rounds, s, keep, host_jobs);
            if (rc) return rc;
            if ((e = hipMemcpyAsync(hx.data(), d_x.p, hx.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s)) !=
                    hipSuccess ||
                (e = hipStreamSynchronize(s)) != hipSuccess)
                return hip_fail(e, "miller-rabin read-back");
            keep.clear();
            host_jobs.clear();
            std::vector<size_t> next;
            for (size_t i : which) {
                const Candidate &c = cs[i];
                bool open = false;
                for (int r = 0; r < rounds; r++) {
                    uint8_t &z = st[i * rounds + r];
                    if (z) continue;
                    const uint32_t *x = hx.data() + i * row + (size_t)r * L;
                    if (rows_equal(x, c.nm1, L) || (j == 0 && rows_equal(x, Limbs{1}, L)))
                        z = 1;                                      // a^(2^j d) = -1, or a^d = 1
                    else if (j > 0 && rows_equal(x, Limbs{1}, L))
                        z = 2;                                      // 1 reached without passing -1
                    else if (j + 1 >= c.s)
                        z = 2;                                      // no square left to reach -1
                    if (!z) open = true;
                }
                if (open) next.push_back(i);
            }
            which.swap(next);
        }
        for (size_t i = 0; i < count; i++) {
            uint8_t v = 1;
            for (int r = 0; r < rounds; r++) v &= st[i * rounds + r] == 1;
            verdict[i] = v;
        }
    } catch (const std::bad_alloc &) {
        return fail(RNS_ENOMEM, "out of host memory");
    }
    return ok();
}


}  // extern "C"

namespace {

constexpr size_t kMrChunk = 64;

// The first candidate of a stream (host, count x L limbs, in order) that
// passes trial division on the GPU, has gcd(e, c - 1) = 1, differs from
// `exclude` and passes Miller-Rabin with its bases (chunks of up to 64
// eligible candidates, in order).
int first_prime(const uint32_t *cand, const uint32_t *bases, size_t count, int L, int rounds, uint32_t e,
                const Limbs &exclude, hipStream_t s, Limbs &out) {
    Scratch dc, df;
    int rc = scratch_alloc(dc, count * (size_t)L * sizeof(uint32_t), s);
    if (!rc) rc = scratch_alloc(df, count, s);
    if (rc) return rc;
    hipError_t he = hipMemcpyAsync(dc.p, cand, count * (size_t)L * sizeof(uint32_t), hipMemcpyHostToDevice, s);
    if (he != hipSuccess) return hip_fail(he, "hipMemcpyAsync");
    if ((rc = rsa_trial_division((const uint32_t *)dc.p, count, L, kMaxSmallPrimes, (uint8_t *)df.p, s))) return rc;
    std::vector<uint8_t> flags(count);
    if ((he = hipMemcpyAsync(flags.data(), df.p, count, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (he = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(he, "trial division read-back");
    std::vector<size_t> elig;
    for (size_t i = 0; i < count; i++) {
        if (!flags[i]) continue;
        Limbs c = bn_from_ptr(cand + i * L, (size_t)L);
        bn_trim(c);
        if (!(bn_low(c) & 1u) || bn_cmp(c, Limbs{3}) <= 0 || bn_cmp(c, exclude) == 0) continue;
        const uint32_t cm1 = bn_mod_word(bn_sub(c, Limbs{1}), e);
        uint32_t a = e, b = cm1;
        while (b) {
            const uint32_t t = a % b;
            a = b;
            b = t;
        }
        if (a == 1) elig.push_back(i);
    }
    const size_t row = (size_t)rounds * L;
    for (size_t start = 0; start < elig.size(); start += kMrChunk) {
        const size_t n = std::min(kMrChunk, elig.size() - start);
        std::vector<uint32_t> cc(n * (size_t)L), bb(n * row);
        for (size_t k = 0; k < n; k++) {
            std::copy(cand + elig[start + k] * L, cand + (elig[start + k] + 1) * L, cc.begin() + k * L);
            std::copy(bases + elig[start + k] * row, bases + (elig[start + k] + 1) * row, bb.begin() + k * row);
        }
        std::vector<uint8_t> verdict(n);
        if ((rc = rsa_miller_rabin(cc.data(), n, L, bb.data(), rounds, verdict.data(), s))) return rc;
        for (size_t k = 0; k < n; k++)
            if (verdict[k]) {
                out = bn_from_ptr(cc.data() + k * L, (size_t)L);
                bn_trim(out);
                return RNS_OK;
            }
    }
    return fail(RNS_ERANGE, "no probable prime among the candidates");
}

}  // namespace

extern "C" {

int rsa_keygen(const uint32_t *cand_p, const uint32_t *bases_p, const uint32_t *cand_q, const uint32_t *bases_q,
               size_t count, int half_limbs, int rounds, uint32_t e, const rns_opts *opts, uint32_t *n_out,
               rsa_key **out, void *hip_stream) {
    if (!out) return fail(RNS_EINVAL, "null output handle");
    *out = nullptr;
    if (!cand_p || !bases_p || !cand_q || !bases_q || !n_out || count == 0)
        return fail(RNS_EINVAL, "null buffer or empty candidate streams");
    if (half_limbs <= 0 || half_limbs > 2048) return fail(RNS_EINVAL, "half_limbs must be in 1..2048");
    if (rounds <= 0 || rounds > kMaxRounds) return fail(RNS_EINVAL, "rounds must be in 1..64");
    if (e < 3 || !(e & 1u)) return fail(RNS_EINVAL, "e must be odd and >= 3");
    hipStream_t s = (hipStream_t)hip_stream;
    const int H = half_limbs;
    try {
        Limbs p, q;
        int rc = first_prime(cand_p, bases_p, count, H, rounds, e, Limbs{}, s, p);
        if (!rc) rc = first_prime(cand_q, bases_q, count, H, rounds, e, p, s, q);
        if (rc) return rc;
        const Limbs one{1};
        const Limbs pm1 = bn_sub(p, one), qm1 = bn_sub(q, one);
        const Limbs n = bn_mul(p, q), f = bn_mul(pm1, qm1);
        // d = e^-1 mod f by Arazi's formula in RNS on the GPU, on the channel
        // tables of a context for n (n > f > d), checked on the host
        rns_ctx *nc = nullptr;
        if ((rc = make_context(n, 2 * H, &nc))) return rc;
        std::unique_ptr<rns_ctx> nctx(nc);
        Limbs d;
        if ((rc = arazi_inverse(nc, f, e, d, s))) return rc;
        if (bn_cmp(bn_mod(bn_mul_word(d, e), f), one) != 0)
            return fail(RNS_EVERIFY, "d e != 1 mod (p-1)(q-1)");
        const Limbs dp = bn_mod(d, pm1), dq = bn_mod(d, qm1);
        Limbs qinv;
        if (!bn_modinv_odd(q, p, qinv)) return fail(RNS_EINVAL, "q not invertible mod p");
        auto limbs = [](const Limbs &x, int k) {
            Limbs r = x;
            r.resize((size_t)k, 0u);
            return r;
        };
        const Limbs nl = limbs(n, 2 * H), dl = limbs(d, 2 * H);
        const Limbs pl = limbs(p, H), ql = limbs(q, H), dpl = limbs(dp, H), dql = limbs(dq, H), qil = limbs(qinv, H);
        const uint32_t el[1] = {e};
        if ((rc = rsa_key_load(nl.data(), (size_t)(2 * H), el, 1, dl.data(), pl.data(), ql.data(), dpl.data(),
                               dql.data(), qil.data(), (size_t)H, opts, out)))
            return rc;
        std::copy(nl.begin(), nl.end(), n_out);
    } catch (const std::bad_alloc &) {
        return fail(RNS_ENOMEM, "out of host memory");
    }
    return ok();
}

}  // extern "C"
