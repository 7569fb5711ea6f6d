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
        }
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
        const MfmaShape t = auto_tile(g.shape, (size_t)g.tiles, g.device);
        if (t.NT != g.shape.NT) {
            g.shape = t;
            finish_group(g);
        }
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
    int rc = small_primes(dev, &sp);
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
        // one context per candidate, built on a pool of host threads (each
        // on the caller's device); errors are reported on this thread
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
