// The exported C ABI of librnsrsa (include/rnsrsa.h, include/rnsrsa_host.h).
#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <tuple>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "capi_internal.hpp"
#include "emul.hpp"
#include "jobs.hpp"
#include "range.hpp"
#include "rnsrsa_host.h"

using namespace rnsrsa;
using namespace rnsrsa::api;

namespace rnsrsa {
namespace api {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int ok() {
    g_err.clear();
    return RNS_OK;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(RNS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

int window_or_default(const rns_opts *o) { return (o && o->window) ? o->window : 5; }

PlanOptions plan_options(const rns_opts *o) {
    PlanOptions p;
    if (!o) return p;
    p.k = o->k;
    p.waves = o->waves;
    p.range = o->prime_range;
    if (o->prime_seed) p.seed = o->prime_seed;
    p.primes = o->primes;
    p.n_primes = o->n_primes;
    p.engine = o->engine;
    return p;
}

// Device copies of base tables, one per (base set, device), kept for the life
// of the process: a handful of distinct base sets exist per process.
std::mutex g_dev_mu;
std::map<std::pair<const BaseSet *, int>, std::pair<std::shared_ptr<const BaseSet>, uint32_t *>> g_dev_bases;

int upload(const std::vector<uint32_t> &v, uint32_t **out) {
    *out = nullptr;
    if (v.empty()) return RNS_OK;
    hipError_t e = hipMalloc((void **)out, v.size() * sizeof(uint32_t));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    e = hipMemcpy(*out, v.data(), v.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        hipFree(*out);
        *out = nullptr;
        return hip_fail(e, "hipMemcpy");
    }
    return RNS_OK;
}

// Device copies of the matrix-core base tables, per (base set, device).
// keyed by (base set, device, W, MT): the table's layout depends on the
// kernel shape's waves and tiles per wave (not on its elements per tile)
std::map<std::tuple<const BaseSet *, int, int, int>, std::pair<std::shared_ptr<const BaseSet>, uint32_t *>>
    g_dev_mbases;

int device_mfma_base(const std::shared_ptr<const BaseSet> &bs, const MLayout &sh, const std::vector<uint32_t> &blob,
                     uint32_t **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_dev_mu);
    auto key = std::make_tuple(bs.get(), dev, sh.W, sh.MT);
    auto it = g_dev_mbases.find(key);
    if (it != g_dev_mbases.end()) {
        *out = it->second.second;
        return RNS_OK;
    }
    uint32_t *d = nullptr;
    int rc = upload(blob, &d);
    if (rc) return rc;
    g_dev_mbases[key] = std::make_pair(bs, d);
    *out = d;
    return RNS_OK;
}

// The device's copy of a base's matrix-engine table, if one was uploaded.
uint32_t *resident_mfma_base(const BaseSet *bs, const MLayout &sh) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    auto it = g_dev_mbases.find(std::make_tuple(bs, dev, sh.W, sh.MT));
    return it == g_dev_mbases.end() ? nullptr : it->second.second;
}

int device_base(const std::shared_ptr<const BaseSet> &bs, uint32_t **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_dev_mu);
    auto key = std::make_pair(bs.get(), dev);
    auto it = g_dev_bases.find(key);
    if (it != g_dev_bases.end()) {
        *out = it->second.second;
        return RNS_OK;
    }
    uint32_t *d = nullptr;
    int rc = upload(bs->blob, &d);
    if (rc) return rc;
    g_dev_bases[key] = std::make_pair(bs, d);
    *out = d;
    return RNS_OK;
}

// Stream-ordered allocations keep scratch out of the caller's way; the pool
// keeps freed blocks so repeated calls do not go back to the driver.
void configure_pool_once() {
    static std::once_flag flag;
    std::call_once(flag, [] {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return;
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, dev) != hipSuccess) return;
        uint64_t thr = UINT64_MAX;
        hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    });
}

int scratch_alloc(Scratch &sc, size_t bytes, hipStream_t s) {
    sc.s = s;
    if (bytes == 0) return RNS_OK;
    configure_pool_once();
    hipError_t e = hipMallocAsync(&sc.p, bytes, s);
    if (e != hipSuccess) {
        sc.p = nullptr;
        return fail(RNS_ENOMEM, std::string("hipMallocAsync: ") + hipGetErrorString(e));
    }
    return RNS_OK;
}

}  // namespace api
}  // namespace rnsrsa

namespace {

// Engine for a plan: the matrix-core kernel when one exists for k (unless the
// channel engine was asked for).
int choose_engine(const BaseSet &bs, int requested, int group, int *engine) {
    const int K = bs.K;
    if (requested < 0 || requested > RNS_ENGINE_MATRIX) return fail(RNS_EINVAL, "bad engine");
    if (group != 0 && group != 16 && group != 32) return fail(RNS_EINVAL, "group must be 0, 16 or 32");
    const bool channel_ok = channel_kernel(K, bs.W);
    if (requested == RNS_ENGINE_CHANNEL) {
        if (!channel_ok) return fail(RNS_EUNSUPPORTED, "no channel-engine kernel for this k (matrix cores only)");
        *engine = RNS_ENGINE_CHANNEL;
        return RNS_OK;
    }
    MfmaShape sh;
    bool primes_ok = true;
    for (uint32_t m : bs.B) primes_ok = primes_ok && mfma_prime_fits(m, K, false);
    for (uint32_t m : bs.Bp) primes_ok = primes_ok && mfma_prime_fits(m, K, true);
    if (mfma_shape_for(K, sh, group) && primes_ok) {
        *engine = RNS_ENGINE_MATRIX;
        return RNS_OK;
    }
    if (requested == RNS_ENGINE_MATRIX || !channel_ok)
        return fail(RNS_EUNSUPPORTED, primes_ok ? "no matrix-core kernel for this k"
                                                : "a channel prime is outside the matrix engine's one-step reduction "
                                                  "bounds (B' primes <= 2^32 - 2^18, all primes large enough)");
    *engine = RNS_ENGINE_CHANNEL;
    return RNS_OK;
}

int ctx_from_plan(ModPlan &&mp, int window, int engine_req, int group, rns_ctx **out, bool allow_scaled = true) {
    std::unique_ptr<rns_ctx> c(new (std::nothrow) rns_ctx);
    if (!c) return fail(RNS_ENOMEM, "out of host memory");
    c->plan = std::move(mp);
    c->window = window;
    int rc = choose_engine(*c->plan.base, engine_req, group, &c->engine);
    if (rc) return rc;
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if ((rc = device_base(c->plan.base, &c->d_base))) return rc;
    if ((rc = upload(c->plan.blob, &c->d_mod))) return rc;
    std::vector<uint32_t> E = make_entry_table(c->plan, {c->plan.R2}, c->plan.L);
    if ((rc = upload(E, &c->d_entry))) return rc;
    if (c->engine == RNS_ENGINE_MATRIX) {
        mfma_shape_for(c->plan.base->K, c->mshape, group);
        // the base table is built only when no context has uploaded it yet
        uint32_t *resident = resident_mfma_base(c->plan.base.get(), c->mshape);
        MfmaTables t = make_mfma_tables(c->plan, c->mshape, resident == nullptr, allow_scaled);
        if (resident)
            c->d_mbase = resident;
        else if ((rc = device_mfma_base(c->plan.base, c->mshape, t.base, &c->d_mbase)))
            return rc;
        if ((rc = upload(t.key, &c->d_mkey))) return rc;
        c->mscaled = t.scaled;
        std::vector<uint32_t> Em = make_mfma_entry_table(c->plan, c->mshape, {c->plan.R2}, c->plan.L);
        if ((rc = upload(Em, &c->d_mentry))) return rc;
    }
    c->group_req = group;
    *out = c.release();
    return RNS_OK;
}

bool valid_window(int w) { return w >= 1 && w <= 6; }

int check_opts(const rns_opts *o) {
    if (o && o->window && !valid_window(o->window)) return fail(RNS_EINVAL, "window must be in 1..6");
    if (o && o->primes && o->n_primes == 0) return fail(RNS_EINVAL, "primes given with n_primes = 0");
    return RNS_OK;
}

}  // namespace

namespace rnsrsa {
namespace api {

int device_simds(int dev) {
    static std::mutex mu;
    static std::map<int, int> simds_of;
    std::lock_guard<std::mutex> lk(mu);
    auto it = simds_of.find(dev);
    if (it == simds_of.end()) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            return 0;
        it = simds_of.emplace(dev, 4 * cus).first;
    }
    return it->second;
}

// Resident workgroups per CU of the exponentiation kernel of shape sh (the
// occupancy query, once per shape and device; 0 if it fails).
static int resident_per_cu(const MLayout &sh, int dev) {
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int, int>, int> cache;
    const auto key = std::make_tuple(sh.K, sh.W, sh.MT, sh.NT, dev);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it == cache.end()) it = cache.emplace(key, mfma_blocks_per_cu(sh)).first;
    return it->second;
}

MfmaShape auto_tile(const MfmaShape &sh, size_t tiles, int dev, bool small_jobs) {
    if (sh.NT != 2) return sh;
    MfmaShape alt;
    if (!mfma_shape_for(sh.K, alt, 16) || alt.NT != 1 || alt.W != sh.W || alt.MT != sh.MT) return sh;
    // jobs of a few elements each: the 16-element tile needs hardly more
    // workgroups, and each does half the work
    if (small_jobs) return alt;
    const int simds = device_simds(dev);
    if (!simds) return sh;
    // the 32-element tile unless its workgroups cannot fill the resident
    // slots of every CU: then the 16-element tile's twice as many
    // workgroups give the SIMDs more waves
    const int per_cu = resident_per_cu(sh, dev);
    if (per_cu <= 0) return 2 * tiles * (size_t)sh.W < 3 * (size_t)simds ? alt : sh;
    return tiles < (size_t)(simds / 4) * per_cu ? alt : sh;
}

int spread_tile_elems(const MfmaShape &sh, size_t tiles, int dev) {
    const int simds = device_simds(dev);
    int e = sh.NM();
    while (simds && e > kMinTileElems && tiles * (size_t)sh.W < (size_t)simds) {
        e /= 2;
        tiles *= 2;
    }
    return e == sh.NM() ? 0 : e;
}

// Kernel shape and elements per tile of a plain launch of njobs jobs of
// `batch` elements on c0 (spread: a small launch may use fewer elements per
// tile, i.e. more workgroups and window tables).
static MfmaShape plain_shape(const rns_ctx *c0, int njobs, size_t batch, bool spread, int *tile_elems) {
    MfmaShape sh = c0->mshape;
    if (!c0->group_req) sh = auto_tile(sh, (size_t)mfma_tiles(sh, batch) * njobs, c0->device);
    *tile_elems = spread ? spread_tile_elems(sh, (size_t)mfma_tiles(sh, batch) * njobs, c0->device) : 0;
    return sh;
}

size_t modexp_scratch_bytes(const rns_ctx *c0, int njobs, size_t batch, bool spread) {
    if (c0->engine == RNS_ENGINE_MATRIX) {
        int te = 0;
        const MfmaShape sh = plain_shape(c0, njobs, batch, spread, &te);
        return modexp_mfma_table_words(sh, c0->window, (size_t)mfma_job_tiles(sh, batch, te) * njobs) *
               sizeof(uint32_t);
    }
    const BaseSet &bs = *c0->plan.base;
    return modexp_table_words(bs.K, bs.W, c0->window, (batch + 63) / 64 * njobs) * sizeof(uint32_t);
}

int run_modexp(const rns_ctx *c0, const rns_ctx *c1, const uint32_t *E0, const uint32_t *E1, const uint32_t *in,
               int in_limbs, const uint32_t *x0, const uint32_t *x1, int exp_limbs, int exp_stride, uint32_t *out0,
               uint32_t *out1, int out_stride, size_t batch, hipStream_t s, uint32_t *table_buf, bool spread) {
    const BaseSet &bs = *c0->plan.base;
    const int njobs = c1 ? 2 : 1;
    ModexpParams P{};
    P.in_limbs = in_limbs;
    P.in_stride = in_limbs;
    P.L = c0->plan.L;
    P.out_stride = out_stride;
    P.exp_limbs = exp_limbs;
    P.exp_stride = exp_stride;
    P.window = c0->window;
    P.batch = (int)batch;
    if (c0->engine == RNS_ENGINE_MATRIX) {
        int te = 0;
        const MfmaShape sh = plain_shape(c0, njobs, batch, spread, &te);
        ModexpMfmaLaunch a{};
        const int per_job = mfma_job_tiles(sh, batch, te);
        for (int j = 0; j < njobs; j++) {
            const rns_ctx *c = j ? c1 : c0;
            MJob &J = a.inl[j];
            J.mb = c->d_mbase;
            J.mk = c->d_mkey;
            J.E = j ? E1 : E0;
            J.exp = j ? x1 : x0;
            J.in = in;
            J.out = j ? out1 : out0;
            J.batch = (int)batch;
            J.in_limbs = in_limbs;
            J.in_stride = in_limbs;
            J.L = c->plan.L;
            J.out_stride = out_stride;
            J.exp_limbs = exp_limbs;
            J.exp_stride = exp_stride;
            J.window = c0->window;
            J.tile0 = j * per_job;
            J.tile_elems = te;
        }
        a.njobs = njobs;
        a.tiles = per_job * njobs;
        a.max_window = c0->window;
        a.scaled = c0->mscaled && (njobs < 2 || c1->mscaled);
        Scratch table;
        if (!table_buf) {
            int rc = scratch_alloc(table, modexp_scratch_bytes(c0, njobs, batch, spread), s);
            if (rc) return rc;
        }
        a.table = table_buf ? table_buf : (uint32_t *)table.p;
        hipError_t e = launch_modexp_mfma(sh, a, s);
        if (e != hipSuccess) return hip_fail(e, "modexp (matrix cores) launch");
        return RNS_OK;
    }
    Scratch table;
    if (!table_buf) {
        int rc = scratch_alloc(table, modexp_scratch_bytes(c0, njobs, batch), s);
        if (rc) return rc;
    }
    ModexpLaunch a{};
    a.bc = c0->d_base;
    a.mc[0] = c0->d_mod;
    a.mc[1] = c1 ? c1->d_mod : c0->d_mod;
    a.E[0] = E0;
    a.E[1] = E1 ? E1 : E0;
    a.exp[0] = x0;
    a.exp[1] = x1 ? x1 : x0;
    a.in = in;
    a.out[0] = out0;
    a.out[1] = out1 ? out1 : out0;
    a.table = table_buf ? table_buf : (uint32_t *)table.p;
    a.P.in_limbs = in_limbs;
    a.P.in_stride = in_limbs;
    a.P.L = c0->plan.L;
    a.P.out_stride = out_stride;
    a.P.exp_limbs = exp_limbs;
    a.P.exp_stride = exp_stride;
    a.P.window = c0->window;
    a.P.batch = (int)batch;
    a.njobs = njobs;
    hipError_t e = launch_modexp(bs.K, bs.W, a, s);
    if (e != hipSuccess) return hip_fail(e, "modexp launch");
    return RNS_OK;
}

Limbs limbs_of(const uint32_t *p, size_t n) { return bn_from_ptr(p, n); }

const uint32_t *entry_of(const rns_ctx *c) { return c->engine == RNS_ENGINE_MATRIX ? c->d_mentry : c->d_entry; }

// Both half-size exponentiations of a CRT decryption in one launch.
int crt_halves(const rsa_key *key, const uint32_t *c, uint32_t *mpq, size_t batch, hipStream_t s, uint32_t *table,
               bool spread) {
    const int L = (int)key->half;
    const bool m = key->p->engine == RNS_ENGINE_MATRIX;
    return run_modexp(key->p, key->q, m ? key->d_mcentry_p : key->d_centry_p, m ? key->d_mcentry_q : key->d_centry_q,
                      c, (int)key->n_limbs, key->d_dp, key->d_dq, L, 0, mpq, mpq + L, 2 * L, batch, s, table, spread);
}

// Garner recombination over the p-modulus tables.
GarnerLaunch garner_launch_of(const rsa_key *key, const uint32_t *mpq, uint32_t *m, size_t batch) {
    GarnerLaunch g{};
    g.bc = key->p->d_base;
    g.mc = key->p->d_mod;
    g.E = key->d_gentry;
    g.qlimbs = key->d_qlimbs;
    g.in = mpq;
    g.out = m;
    g.L = (int)key->half;
    g.out_limbs = (int)key->n_limbs;
    g.out_stride = (int)key->n_limbs;
    g.batch = (int)batch;
    return g;
}

int crt_combine(const rsa_key *key, const uint32_t *mpq, uint32_t *m, size_t batch, hipStream_t s) {
    const BaseSet &bs = *key->p->plan.base;
    hipError_t e = launch_garner(bs.K, bs.W, garner_launch_of(key, mpq, m, batch), s);
    if (e != hipSuccess) return hip_fail(e, "garner launch");
    return RNS_OK;
}

int make_context(const Limbs &N, int L, rns_ctx **out) {
    *out = nullptr;
    ModPlan mp;
    std::string err;
    int rc = make_modplan(N, L, PlanOptions{}, mp, err);
    if (rc) return fail(rc, err);
    return ctx_from_plan(std::move(mp), 5, 0, 0, out);
}

}  // namespace api
}  // namespace rnsrsa

extern "C" {

const char *rns_last_error(void) { return g_err.c_str(); }

int rns_abi_version(void) { return 6; }

int rns_setup(const uint32_t *mod, size_t mod_limbs, const rns_opts *opts, rns_ctx **out) {
    if (!mod || !out || mod_limbs == 0 || mod_limbs > 4096) return fail(RNS_EINVAL, "bad modulus arguments");
    *out = nullptr;
    int rc = check_opts(opts);
    if (rc) return rc;
    try {
        ModPlan mp;
        std::string err;
        rc = make_modplan(limbs_of(mod, mod_limbs), (int)mod_limbs, plan_options(opts), mp, err);
        if (rc) return fail(rc, err);
        rc = ctx_from_plan(std::move(mp), window_or_default(opts), opts ? opts->engine : 0, opts ? opts->group : 0,
                           out, !(opts && opts->unscaled));
        if (rc) return rc;
    } catch (const std::bad_alloc &) {
        return fail(RNS_ENOMEM, "out of host memory");
    } catch (...) {
        return fail(RNS_EINVAL, "internal error during setup");
    }
    return ok();
}

void rns_free(rns_ctx *ctx) { delete ctx; }

int rns_get_info(const rns_ctx *ctx, rns_info *info) {
    if (!ctx || !info) return fail(RNS_EINVAL, "null argument");
    info->k = ctx->plan.base->K;
    info->waves = ctx->plan.base->W;
    info->window = ctx->window;
    info->mod_limbs = ctx->plan.L;
    info->mod_bits = (int)bn_bits(ctx->plan.N);
    info->engine = ctx->engine;
    info->group = 64;
    info->scaled = ctx->mscaled ? 1 : 0;
    if (ctx->engine == RNS_ENGINE_MATRIX) {
        info->waves = ctx->mshape.W;
        info->group = ctx->mshape.NM();
    }
    return ok();
}

int rns_get_primes(const rns_ctx *ctx, uint32_t *primes, size_t n) {
    if (!ctx || !primes) return fail(RNS_EINVAL, "null argument");
    const BaseSet &bs = *ctx->plan.base;
    if (n < (size_t)(2 * bs.K)) return fail(RNS_EINVAL, "buffer shorter than 2k");
    std::copy(bs.B.begin(), bs.B.end(), primes);
    std::copy(bs.Bp.begin(), bs.Bp.end(), primes + bs.K);
    return ok();
}

int rns_modexp_batch(rns_ctx *ctx, const uint32_t *base, const uint32_t *exp, size_t exp_limbs, size_t exp_stride,
                     uint32_t *out, size_t batch, void *hip_stream) {
    if (!ctx) return fail(RNS_EINVAL, "null context");
    if (batch == 0) return ok();
    if (!base || !exp || !out || exp_limbs == 0) return fail(RNS_EINVAL, "null buffer or zero exponent limbs");
    if (exp_stride != 0 && exp_stride < exp_limbs) return fail(RNS_EINVAL, "exp_stride below exp_limbs");
    if (batch > (size_t)INT32_MAX - 64 || exp_limbs > 1u << 20 || exp_stride > 1u << 24)
        return fail(RNS_EINVAL, "batch or exponent too large");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != ctx->device) return fail(RNS_EINVAL, "context belongs to another device");
    int rc = run_modexp(ctx, nullptr, entry_of(ctx), nullptr, base, ctx->plan.L, exp, nullptr, (int)exp_limbs, (int)exp_stride,
                        out, nullptr, ctx->plan.L, batch, (hipStream_t)hip_stream);
    return rc ? rc : ok();
}

int rns_modexp_jobs(const rns_job *jobs, size_t njobs, void *hip_stream) {
    if (njobs == 0) return ok();
    if (!jobs) return fail(RNS_EINVAL, "null job array");
    if (njobs > (1u << 20)) return fail(RNS_EINVAL, "more than 2^20 jobs");
    for (size_t i = 0; i < njobs; i++) {
        const rns_job &j = jobs[i];
        const std::string at = "job " + std::to_string(i) + ": ";
        if (!j.ctx) return fail(RNS_EINVAL, at + "null context");
        if (j.count == 0) continue;
        if (!j.base || !j.exp || !j.out || j.exp_limbs == 0)
            return fail(RNS_EINVAL, at + "null buffer or zero exponent limbs");
        if (j.exp_stride != 0 && j.exp_stride < j.exp_limbs) return fail(RNS_EINVAL, at + "exp_stride below exp_limbs");
        if (j.count > (size_t)INT32_MAX - 64 || j.exp_limbs > 1u << 20 || j.exp_stride > 1u << 24)
            return fail(RNS_EINVAL, at + "count or exponent too large");
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    for (size_t i = 0; i < njobs; i++)
        if (jobs[i].count && jobs[i].ctx->device != dev)
            return fail(RNS_EINVAL, "job " + std::to_string(i) + ": context belongs to another device");
    hipStream_t s = (hipStream_t)hip_stream;
    try {
        // matrix-core jobs of one kernel shape (and requested tile) share a launch
        std::map<std::tuple<int, int, int, int>, JobGroup> groups;
        for (size_t i = 0; i < njobs; i++) {
            const rns_job &j = jobs[i];
            const rns_ctx *c = j.ctx;
            if (j.count == 0) continue;
            const int L = c->plan.L;
            if (c->engine != RNS_ENGINE_MATRIX) {
                int rc = run_modexp(c, nullptr, entry_of(c), nullptr, j.base, L, j.exp, nullptr, (int)j.exp_limbs,
                                    (int)j.exp_stride, j.out, nullptr, L, j.count, s);
                if (rc) return rc;
                continue;
            }
            const MfmaShape &sh = c->mshape;
            JobGroup &g = groups[std::make_tuple(sh.K, sh.W, sh.MT, c->group_req)];
            if (g.jobs.empty()) {
                g.shape = sh;
                g.device = dev;
                g.auto_tile = c->group_req == 0;
                g.scaled = true;
            }
            g.scaled = g.scaled && c->mscaled;
            PlannedJob J{};
            J.j.mb = c->d_mbase;
            J.j.mk = c->d_mkey;
            J.j.E = entry_of(c);
            J.j.exp = j.exp;
            J.j.in = j.base;
            J.j.out = j.out;
            J.j.batch = (int)j.count;
            J.j.in_limbs = L;
            J.j.in_stride = L;
            J.j.L = L;
            J.j.out_stride = L;
            J.j.exp_limbs = (int)j.exp_limbs;
            J.j.exp_stride = (int)j.exp_stride;
            J.j.window = c->window;
            J.cost = 32 * j.exp_limbs;   // the exponents stay on the device: their length orders the tiles
            g.jobs.push_back(J);
        }
        for (auto &kv : groups) {
            JobGroup &g = kv.second;
            finish_group(g);
            if (g.auto_tile) retile_group(g, dev);
            // the job table's host copy is released by the stream once copied
            std::unique_ptr<std::vector<MJob>> host(new std::vector<MJob>());
            for (const PlannedJob &J : g.jobs) host->push_back(J.j);
            const size_t bytes = host->size() * sizeof(MJob);
            Scratch jt, tb;
            int rc = scratch_alloc(jt, bytes, s);
            if (!rc) rc = scratch_alloc(tb, g.table_words() * sizeof(uint32_t), s);
            if (rc) return rc;
            if ((e = hipMemcpyAsync(jt.p, host->data(), bytes, hipMemcpyHostToDevice, s)) != hipSuccess)
                return hip_fail(e, "hipMemcpyAsync");
            std::vector<MJob> *h = host.get();
            if (hipLaunchHostFunc(s, [](void *p) { delete (std::vector<MJob> *)p; }, h) == hipSuccess) {
                host.release();
            } else if ((e = hipStreamSynchronize(s)) != hipSuccess) {
                host.release();   // the copy may still read it: leaked rather than freed early
                return hip_fail(e, "hipStreamSynchronize");
            }
            if ((e = launch_group(g, (const MJob *)jt.p, (uint32_t *)tb.p, s)) != hipSuccess)
                return hip_fail(e, "grouped modexp launch");
        }
    } catch (const std::bad_alloc &) {
        return fail(RNS_ENOMEM, "out of host memory");
    }
    return ok();
}

int rns_mont_mul_batch(rns_ctx *ctx, const uint32_t *x, const uint32_t *y, uint32_t *out, size_t batch,
                       void *hip_stream) {
    if (!ctx) return fail(RNS_EINVAL, "null context");
    if (batch == 0) return ok();
    if (!x || !y || !out) return fail(RNS_EINVAL, "null buffer");
    if (batch > (size_t)INT32_MAX - 64) return fail(RNS_EINVAL, "batch too large");
    const BaseSet &bs = *ctx->plan.base;
    if (ctx->engine == RNS_ENGINE_MATRIX) {
        MfmaShape sh = ctx->mshape;
        if (!ctx->group_req) sh = auto_tile(sh, (size_t)mfma_tiles(sh, batch), ctx->device);
        MontMulMfmaLaunch a{};
        a.mb = ctx->d_mbase;
        a.mk = ctx->d_mkey;
        a.x = x;
        a.y = y;
        a.out = out;
        a.batch = (int)batch;
        a.tile_elems = spread_tile_elems(sh, (size_t)mfma_tiles(sh, batch), ctx->device);
        a.tiles = mfma_job_tiles(sh, batch, a.tile_elems);
        hipError_t e = launch_montmul_mfma(sh, a, (hipStream_t)hip_stream);
        if (e != hipSuccess) return hip_fail(e, "montmul (matrix cores) launch");
        return ok();
    }
    if (!channel_kernel(bs.K, bs.W)) return fail(RNS_EUNSUPPORTED, "no single-product kernel for this k");
    MontMulLaunch a{ctx->d_base, ctx->d_mod, x, y, out, (int)batch};
    hipError_t e = launch_montmul(bs.K, bs.W, a, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "montmul launch");
    return ok();
}

int rsa_key_load(const uint32_t *n, size_t n_limbs, const uint32_t *e, size_t e_limbs, const uint32_t *d,
                 const uint32_t *p, const uint32_t *q, const uint32_t *dp, const uint32_t *dq, const uint32_t *qinv,
                 size_t half_limbs, const rns_opts *opts, rsa_key **out) {
    if (!n || !e || !out || n_limbs == 0 || e_limbs == 0 || n_limbs > 4096 || e_limbs > 4096)
        return fail(RNS_EINVAL, "bad key arguments");
    *out = nullptr;
    int rc = check_opts(opts);
    if (rc) return rc;
    const bool any_crt = p || q || dp || dq || qinv;
    const bool all_crt = p && q && dp && dq && qinv;
    if (any_crt && !all_crt) return fail(RNS_EINVAL, "CRT parts must be all present or all NULL");
    if (all_crt && (half_limbs == 0 || 2 * half_limbs < n_limbs)) return fail(RNS_EINVAL, "bad half_limbs");
    if (opts && opts->primes && all_crt) return fail(RNS_EINVAL, "explicit primes apply to one modulus only");
    try {
        std::unique_ptr<rsa_key> key(new rsa_key);
        key->n_limbs = n_limbs;
        key->e_limbs = e_limbs;
        key->half = half_limbs;
        const int window = window_or_default(opts);
        const int engine = opts ? opts->engine : 0;
        const int group = opts ? opts->group : 0;
        const bool scaled = !(opts && opts->unscaled);
        std::string err;
        {
            ModPlan mp;
            PlanOptions po = plan_options(opts);
            rc = make_modplan(limbs_of(n, n_limbs), (int)n_limbs, po, mp, err);
            if (rc == RNS_ERANGE && all_crt && po.k) {
                // an explicit k sized for the CRT halves: size the full modulus automatically
                po.k = 0;
                po.waves = 0;
                rc = make_modplan(limbs_of(n, n_limbs), (int)n_limbs, po, mp, err);
            }
            // a CRT-only key when no base covers the full modulus or no kernel
            // of the requested engine runs it: decryption through the halves,
            // encryption unsupported
            if (rc) {
                if (!(rc == RNS_ERANGE && all_crt)) return fail(rc, err);
            } else if ((rc = ctx_from_plan(std::move(mp), window, engine, group, &key->n, scaled))) {
                if (!(rc == RNS_EUNSUPPORTED && all_crt)) return rc;   // message recorded by ctx_from_plan
            }
            rc = RNS_OK;
        }
        key->h_n.assign(n, n + n_limbs);
        if ((rc = upload(key->h_n, &key->d_n))) return rc;
        {
            hipError_t he = hipMalloc((void **)&key->d_status, sizeof(unsigned long long));
            if (he == hipSuccess) he = hipMemset(key->d_status, 0, sizeof(unsigned long long));
            if (he != hipSuccess) return hip_fail(he, "status word");
        }
        key->h_e.assign(e, e + e_limbs);
        if (d) key->h_d.assign(d, d + n_limbs);
        key->wc_e = window_costs(key->h_e);
        if (d) key->wc_d = window_costs(key->h_d);
        if ((rc = upload(key->h_e, &key->d_e))) return rc;
        if (d && (rc = upload(key->h_d, &key->d_d))) return rc;
        if (all_crt) {
            const int L = (int)half_limbs;
            Limbs P = limbs_of(p, half_limbs), Q = limbs_of(q, half_limbs);
            Limbs big = bn_cmp(P, Q) >= 0 ? P : Q;
            ModPlan pp, qp;
            rc = make_modplan(big, L, plan_options(opts), pp, err);  // base set fitting both halves
            if (rc) return fail(rc, err);
            std::shared_ptr<const BaseSet> bs = pp.base;
            if ((rc = make_modplan_on(P, L, bs, pp, err))) return fail(rc, err);
            if ((rc = make_modplan_on(Q, L, bs, qp, err))) return fail(rc, err);
            // inputs of n_limbs limbs enter as sum_h c_h (2^(32 L h) M^2 mod p)
            const int chunks = (int)((n_limbs + half_limbs - 1) / half_limbs);
            std::vector<Limbs> Yp, Yq;
            for (int h = 0; h < chunks; h++) {
                Yp.push_back(bn_mod(bn_mul(bn_shl(Limbs{1}, 32u * L * h), pp.R2), P));
                Yq.push_back(bn_mod(bn_mul(bn_shl(Limbs{1}, 32u * L * h), qp.R2), Q));
            }
            std::vector<uint32_t> Ep = make_entry_table(pp, Yp, L), Eq = make_entry_table(qp, Yq, L);
            Ep.resize((size_t)n_limbs * Layout{bs->K, bs->KP}.ecols());
            Eq.resize((size_t)n_limbs * Layout{bs->K, bs->KP}.ecols());
            // Garner: Z = m_p A + m_q (p - A), A = qinv M mod p
            Limbs A = bn_mod(bn_mul(limbs_of(qinv, half_limbs), pp.Mmod), P);
            Limbs Bv = bn_is_zero(A) ? Limbs{} : bn_sub(P, A);
            std::vector<uint32_t> Eg = make_entry_table(pp, {A, Bv}, L);
            std::vector<uint32_t> Epm, Eqm;
            MfmaShape msh;
            const bool mfma = mfma_shape_for(bs->K, msh, group);
            if (mfma) {
                Epm = make_mfma_entry_table(pp, msh, Yp, L);
                Eqm = make_mfma_entry_table(qp, msh, Yq, L);
                Epm.resize((size_t)n_limbs * msh.ecols());
                Eqm.resize((size_t)n_limbs * msh.ecols());
            }
            if ((rc = ctx_from_plan(std::move(pp), window, engine, group, &key->p, scaled))) return rc;
            if ((rc = ctx_from_plan(std::move(qp), window, engine, group, &key->q, scaled))) return rc;
            if ((rc = upload(Ep, &key->d_centry_p))) return rc;
            if ((rc = upload(Eq, &key->d_centry_q))) return rc;
            if (key->p->engine == RNS_ENGINE_MATRIX) {
                if ((rc = upload(Epm, &key->d_mcentry_p))) return rc;
                if ((rc = upload(Eqm, &key->d_mcentry_q))) return rc;
            }
            if ((rc = upload(Eg, &key->d_gentry))) return rc;
            key->h_dp.assign(dp, dp + half_limbs);
            key->h_dq.assign(dq, dq + half_limbs);
            key->wc_dp = window_costs(key->h_dp);
            key->wc_dq = window_costs(key->h_dq);
            if ((rc = upload(key->h_dp, &key->d_dp))) return rc;
            if ((rc = upload(key->h_dq, &key->d_dq))) return rc;
            if ((rc = upload(std::vector<uint32_t>(q, q + half_limbs), &key->d_qlimbs))) return rc;
            key->has_crt = true;
        }
        *out = key.release();
    } catch (const std::bad_alloc &) {
        return fail(RNS_ENOMEM, "out of host memory");
    } catch (...) {
        return fail(RNS_EINVAL, "internal error during key load");
    }
    return ok();
}

void rsa_key_free(rsa_key *key) { delete key; }

int rsa_key_info(const rsa_key *key, int which, rns_info *info) {
    if (!key || !info) return fail(RNS_EINVAL, "null argument");
    if (which == 0 && !key->n) return fail(RNS_EUNSUPPORTED, "CRT-only key: no context for the full modulus");
    const rns_ctx *c = which == 0 ? key->n : which == 1 ? key->p : which == 2 ? key->q : nullptr;
    if (!c) return fail(RNS_EINVAL, "no such context in this key");
    return rns_get_info(c, info);
}

int rsa_encrypt(const rsa_key *key, const uint32_t *m, uint32_t *c, size_t batch, void *hip_stream) {
    if (!key) return fail(RNS_EINVAL, "null key");
    if (batch == 0) return ok();
    if (!m || !c) return fail(RNS_EINVAL, "null buffer");
    if (batch > (size_t)INT32_MAX - 64) return fail(RNS_EINVAL, "batch too large");
    if (!key->n) return fail(RNS_EUNSUPPORTED, "CRT-only key: no context for the full modulus");
    const rns_ctx *x = key->n;
    int rc = check_inputs(key, m, batch, (hipStream_t)hip_stream);
    if (!rc)
        rc = run_modexp(x, nullptr, entry_of(x), nullptr, m, x->plan.L, key->d_e, nullptr, (int)key->e_limbs, 0, c,
                        nullptr, x->plan.L, batch, (hipStream_t)hip_stream);
    return rc ? rc : ok();
}

int rsa_decrypt(const rsa_key *key, const uint32_t *c, uint32_t *m, size_t batch, int use_crt, void *hip_stream) {
    if (!key) return fail(RNS_EINVAL, "null key");
    if (batch == 0) return ok();
    if (!c || !m) return fail(RNS_EINVAL, "null buffer");
    if (batch > (size_t)INT32_MAX - 64) return fail(RNS_EINVAL, "batch too large");
    hipStream_t s = (hipStream_t)hip_stream;
    if (!use_crt) {
        if (!key->d_d) return fail(RNS_EINVAL, "key has no private exponent");
        if (!key->n) return fail(RNS_EUNSUPPORTED, "CRT-only key: no context for the full modulus");
        const rns_ctx *x = key->n;
        int rc = check_inputs(key, c, batch, s);
        if (!rc)
            rc = run_modexp(x, nullptr, entry_of(x), nullptr, c, x->plan.L, key->d_d, nullptr, (int)key->n_limbs, 0, m,
                            nullptr, x->plan.L, batch, s);
        return rc ? rc : ok();
    }
    if (!key->has_crt) return fail(RNS_EINVAL, "key has no CRT parts");
    Scratch ws;  // [m_p | m_q] per element
    int rc = scratch_alloc(ws, batch * 2 * key->half * sizeof(uint32_t), s);
    if (rc) return rc;
    if ((rc = check_inputs(key, c, batch, s))) return rc;
    if ((rc = crt_halves(key, c, (uint32_t *)ws.p, batch, s))) return rc;
    if ((rc = crt_combine(key, (uint32_t *)ws.p, m, batch, s))) return rc;
    return ok();
}

int rsa_crt_halves(const rsa_key *key, const uint32_t *c, uint32_t *mpq, size_t batch, void *hip_stream) {
    if (!key) return fail(RNS_EINVAL, "null key");
    if (batch == 0) return ok();
    if (!c || !mpq) return fail(RNS_EINVAL, "null buffer");
    if (batch > (size_t)INT32_MAX - 64) return fail(RNS_EINVAL, "batch too large");
    if (!key->has_crt) return fail(RNS_EINVAL, "key has no CRT parts");
    int rc = check_inputs(key, c, batch, (hipStream_t)hip_stream);
    if (!rc) rc = crt_halves(key, c, mpq, batch, (hipStream_t)hip_stream);
    return rc ? rc : ok();
}

int rsa_crt_combine(const rsa_key *key, const uint32_t *mpq, uint32_t *m, size_t batch, void *hip_stream) {
    if (!key) return fail(RNS_EINVAL, "null key");
    if (batch == 0) return ok();
    if (!mpq || !m) return fail(RNS_EINVAL, "null buffer");
    if (batch > (size_t)INT32_MAX - 64) return fail(RNS_EINVAL, "batch too large");
    if (!key->has_crt) return fail(RNS_EINVAL, "key has no CRT parts");
    int rc = crt_combine(key, mpq, m, batch, (hipStream_t)hip_stream);
    return rc ? rc : ok();
}

// ---- host-side planning and model ---------------------------------------

int rns_plan_create(const uint32_t *mod, size_t mod_limbs, const rns_opts *opts, rns_plan **out) {
    if (!mod || !out || mod_limbs == 0 || mod_limbs > 4096) return fail(RNS_EINVAL, "bad modulus arguments");
    *out = nullptr;
    int rc = check_opts(opts);
    if (rc) return rc;
    try {
        std::unique_ptr<rns_plan> p(new rns_plan);
        std::string err;
        rc = make_modplan(limbs_of(mod, mod_limbs), (int)mod_limbs, plan_options(opts), p->plan, err);
        if (rc) return fail(rc, err);
        p->window = window_or_default(opts);
        const int group = opts ? opts->group : 0;
        if ((rc = choose_engine(*p->plan.base, opts ? opts->engine : 0, group, &p->engine))) return rc;
        if (p->engine == RNS_ENGINE_MATRIX) {
            MfmaShape sh;
            mfma_shape_for(p->plan.base->K, sh, group);
            p->mt = make_mfma_tables(p->plan, sh, true, !(opts && opts->unscaled));
        }
        *out = p.release();
    } catch (const std::bad_alloc &) {
        return fail(RNS_ENOMEM, "out of host memory");
    }
    return ok();
}

void rns_plan_free(rns_plan *plan) { delete plan; }

int rns_plan_info(const rns_plan *plan, rns_info *info) {
    if (!plan || !info) return fail(RNS_EINVAL, "null argument");
    info->k = plan->plan.base->K;
    info->waves = plan->plan.base->W;
    info->window = plan->window;
    info->mod_limbs = plan->plan.L;
    info->mod_bits = (int)bn_bits(plan->plan.N);
    info->engine = plan->engine;
    info->group = 64;
    info->scaled = plan->mt.scaled ? 1 : 0;
    if (plan->engine == RNS_ENGINE_MATRIX) {
        info->waves = plan->mt.shape.W;
        info->group = plan->mt.shape.NM();
    }
    return ok();
}

int rns_plan_primes(const rns_plan *plan, uint32_t *primes, size_t n) {
    if (!plan || !primes) return fail(RNS_EINVAL, "null argument");
    const BaseSet &bs = *plan->plan.base;
    if (n < (size_t)(2 * bs.K)) return fail(RNS_EINVAL, "buffer shorter than 2k");
    std::copy(bs.B.begin(), bs.B.end(), primes);
    std::copy(bs.Bp.begin(), bs.Bp.end(), primes + bs.K);
    return ok();
}

int rns_emul_modexp(const rns_plan *plan, const uint32_t *base, const uint32_t *exp, size_t exp_limbs,
                    size_t exp_stride, uint32_t *out, size_t batch) {
    if (!plan) return fail(RNS_EINVAL, "null plan");
    if (batch == 0) return ok();
    if (!base || !exp || !out || exp_limbs == 0) return fail(RNS_EINVAL, "null buffer or zero exponent limbs");
    if (exp_stride != 0 && exp_stride < exp_limbs) return fail(RNS_EINVAL, "exp_stride below exp_limbs");
    try {
        if (plan->engine == RNS_ENGINE_MATRIX) {
            std::vector<uint32_t> E = make_mfma_entry_table(plan->plan, plan->mt.shape, {plan->plan.R2}, plan->plan.L);
            if (!emul_modexp_mfma(plan->plan, plan->mt, E, plan->plan.L, base, exp, (int)exp_limbs, exp_stride,
                                  plan->window, out, batch))
                return fail(RNS_EVERIFY, "a one-step reduction of the matrix-engine model left [0, m 2^32)");
            return ok();
        }
        std::vector<uint32_t> E = make_entry_table(plan->plan, {plan->plan.R2}, plan->plan.L);
        emul_modexp(plan->plan, E, plan->plan.L, base, exp, (int)exp_limbs, exp_stride, plan->window, out, batch);
    } catch (const std::bad_alloc &) {
        return fail(RNS_ENOMEM, "out of host memory");
    }
    return ok();
}

int rns_emul_mfma_extension(const rns_plan *plan, int which, const uint32_t *xi, size_t batch, size_t *rows,
                            int64_t *partials, int64_t *value) {
    if (!plan || !rows) return fail(RNS_EINVAL, "null plan or rows");
    if (plan->engine != RNS_ENGINE_MATRIX) return fail(RNS_EUNSUPPORTED, "the plan does not use the matrix engine");
    if (which != 1 && which != 2) return fail(RNS_EINVAL, "which must be 1 or 2");
    const MfmaShape &sh = plan->mt.shape;
    *rows = (size_t)sh.W * 4 * sh.MT;
    if (batch == 0 || (!partials && !value)) return ok();
    if (!xi || !partials || !value) return fail(RNS_EINVAL, "null buffer");
    if (!emul_mfma_extension(plan->mt, which, xi, batch, partials, value))
        return fail(RNS_EVERIFY, "a byte partial or the kernel's combination of them left its integer range");
    return ok();
}

int rns_emul_mfma_matrix(const rns_plan *plan, int which, size_t *rows, size_t *kdim, int8_t *A) {
    if (!plan || !rows || !kdim) return fail(RNS_EINVAL, "null argument");
    if (plan->engine != RNS_ENGINE_MATRIX) return fail(RNS_EUNSUPPORTED, "the plan does not use the matrix engine");
    if (which != 1 && which != 2) return fail(RNS_EINVAL, "which must be 1 or 2");
    const MfmaShape &sh = plan->mt.shape;
    *rows = (size_t)sh.W * 4 * sh.MT;
    *kdim = (size_t)64 * MLayout{sh.K, sh.W, sh.MT, sh.NT}.KSTEPS();
    if (A) emul_mfma_matrix(plan->mt, which, A);
    return ok();
}

int rns_emul_mont_mul(const rns_plan *plan, const uint32_t *x, const uint32_t *y, uint32_t *out, size_t batch) {
    if (!plan) return fail(RNS_EINVAL, "null plan");
    if (batch == 0) return ok();
    if (!x || !y || !out) return fail(RNS_EINVAL, "null buffer");
    emul_mont_mul(plan->plan, x, y, out, batch);
    return ok();
}

}  // extern "C"
