// Batched RSA operations over many keys (include/rnsrsa.h, rsa_batch_*).
//
// Planning, done once per batch: every operation becomes exponentiation jobs
// (a CRT decryption is two half-size jobs plus a Garner step); each job gets
// the window width that minimises its number of Montgomery products for its
// own exponent; jobs on contexts with the same matrix-core kernel shape form
// one launch, with the tiles of the most expensive jobs first so the
// workgroup dispatcher starts the long ones early.  The launches of different
// shapes run concurrently on internal streams; the Garner steps follow them.
// With use_graph the whole sequence is captured into a hipGraph at creation.
#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "capi_internal.hpp"

using namespace rnsrsa;
using namespace rnsrsa::api;

namespace {

// Montgomery products of one exponentiation as the kernels schedule them:
// entry, 2^w - 2 table products, w squarings and one product per non-zero
// digit after the leading non-zero one, exit.
size_t mm_count(const std::vector<uint32_t> &e, int w) {
    const int nbits = 32 * (int)e.size();
    const int nd = (nbits + w - 1) / w;
    size_t n = 1 + ((size_t)1 << w) - 2 + 1;
    bool started = false;
    for (int di = 0; di < nd; di++) {
        const int lo = (nd - 1 - di) * w;
        uint64_t v = e[lo >> 5];
        if ((lo >> 5) + 1 < (int)e.size()) v |= (uint64_t)e[(lo >> 5) + 1] << 32;
        const uint32_t d = (uint32_t)(v >> (lo & 31)) & ((1u << w) - 1u);
        if (!started) {
            started = d != 0;
            continue;
        }
        n += (size_t)w + (d ? 1 : 0);
    }
    return n;
}

int best_window(const std::vector<uint32_t> &e, int fixed) {
    if (fixed) return fixed;
    int best = 1;
    size_t bn = mm_count(e, 1);
    for (int w = 2; w <= 6; w++) {
        const size_t n = mm_count(e, w);
        if (n < bn) {
            bn = n;
            best = w;
        }
    }
    return best;
}

// Tile (elements per workgroup) chosen per (K, W, MT) by timing, per process.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, int> g_tuned_nt;

struct Job {
    MJob j;
    size_t cost;  // Montgomery products per element
};

struct Group {
    MLayout shape{};
    std::vector<Job> jobs;
    MJob *d_jobs = nullptr;
    uint32_t *d_table = nullptr;
    int tiles = 0;
    int max_window = 1;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
};

// Exponentiations on channel-engine contexts, launched one at a time.
struct PlainJob {
    const rns_ctx *c0, *c1;
    const uint32_t *E0, *E1, *in, *x0, *x1;
    int in_limbs, exp_limbs;
    uint32_t *out0, *out1;
    int out_stride;
    size_t count;
};

struct GarnerJob {
    const rsa_key *key;
    const uint32_t *mpq;
    uint32_t *out;
    size_t count;
};

ModexpMfmaLaunch group_launch(const Group &g) {
    ModexpMfmaLaunch a{};
    a.jobs = g.d_jobs;
    a.njobs = (int)g.jobs.size();
    a.tiles = g.tiles;
    a.max_window = g.max_window;
    a.table = g.d_table;
    return a;
}

}  // namespace

struct rsa_batch {
    std::vector<Group> groups;
    std::vector<PlainJob> plain;
    std::vector<GarnerJob> garners;
    uint32_t *d_mpq = nullptr;
    hipEvent_t fork = nullptr;
    hipStream_t capture = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    rsa_batch_info info{};
    ~rsa_batch() {
        hipDeviceSynchronize();
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        for (Group &g : groups) {
            if (g.d_jobs) hipFree(g.d_jobs);
            if (g.d_table) hipFree(g.d_table);
            if (g.done) hipEventDestroy(g.done);
            if (g.stream) hipStreamDestroy(g.stream);
        }
        if (d_mpq) hipFree(d_mpq);
        if (fork) hipEventDestroy(fork);
        if (capture) hipStreamDestroy(capture);
    }
};

namespace {

int dmalloc(void **p, size_t bytes, size_t *total) {
    *p = nullptr;
    if (bytes == 0) return RNS_OK;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return fail(RNS_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    *total += bytes;
    return RNS_OK;
}

// Everything one run enqueues, on stream s (which the run's work follows).
int enqueue(rsa_batch *b, hipStream_t s) {
    hipError_t e = hipEventRecord(b->fork, s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    for (Group &g : b->groups) {
        if ((e = hipStreamWaitEvent(g.stream, b->fork, 0)) != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
        if ((e = launch_modexp_mfma(g.shape, group_launch(g), g.stream)) != hipSuccess)
            return hip_fail(e, "grouped modexp launch");
        if ((e = hipEventRecord(g.done, g.stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    }
    for (const PlainJob &p : b->plain) {
        int rc = run_modexp(p.c0, p.c1, p.E0, p.E1, p.in, p.in_limbs, p.x0, p.x1, p.exp_limbs, 0, p.out0, p.out1,
                            p.out_stride, p.count, s);
        if (rc) return rc;
    }
    for (Group &g : b->groups)
        if ((e = hipStreamWaitEvent(s, g.done, 0)) != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
    for (const GarnerJob &gj : b->garners) {
        int rc = crt_combine(gj.key, gj.mpq, gj.out, gj.count, s);
        if (rc) return rc;
    }
    return RNS_OK;
}

// Times each candidate tile of a group's shape class on copies of its most
// expensive job (outputs to scratch) and returns the faster NT.
int tune_tile(const Group &g, const std::vector<MLayout> &cands, hipStream_t s, int *nt_out) {
    const Job &heavy = *std::max_element(g.jobs.begin(), g.jobs.end(),
                                         [](const Job &a, const Job &b) { return a.cost < b.cost; });
    const int copies = std::max(1, (int)(16384 / std::max(1, heavy.j.batch)));
    const size_t out_words = (size_t)copies * heavy.j.batch * heavy.j.L;
    uint32_t *d_out = nullptr;
    MJob *d_jobs = nullptr;
    uint32_t *d_table = nullptr;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    int rc = RNS_OK;
    float best = 0;
    *nt_out = cands[0].NT;
    auto cleanup = [&] {
        if (d_out) hipFree(d_out);
        if (d_jobs) hipFree(d_jobs);
        if (d_table) hipFree(d_table);
        if (t0) hipEventDestroy(t0);
        if (t1) hipEventDestroy(t1);
    };
    hipError_t e = hipMalloc((void **)&d_out, out_words * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc((void **)&d_jobs, (size_t)copies * sizeof(MJob));
    if (e == hipSuccess) e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    if (e != hipSuccess) {
        cleanup();
        return hip_fail(e, "autotune set-up");
    }
    for (const MLayout &sh : cands) {
        std::vector<MJob> js(copies, heavy.j);
        const int per = mfma_tiles(sh, (size_t)heavy.j.batch);
        for (int c = 0; c < copies; c++) {
            js[c].out = d_out + (size_t)c * heavy.j.batch * heavy.j.L;
            js[c].out_stride = heavy.j.L;
            js[c].tile0 = c * per;
        }
        ModexpMfmaLaunch a{};
        a.jobs = d_jobs;
        a.njobs = copies;
        a.tiles = per * copies;
        a.max_window = heavy.j.window;
        if (d_table) hipFree(d_table);
        d_table = nullptr;
        e = hipMalloc((void **)&d_table, modexp_mfma_table_words(sh, a.max_window, (size_t)a.tiles) * sizeof(uint32_t));
        if (e == hipSuccess) e = hipMemcpy(d_jobs, js.data(), js.size() * sizeof(MJob), hipMemcpyHostToDevice);
        a.table = d_table;
        float ms = 0;
        for (int rep = 0; rep < 2 && e == hipSuccess; rep++) {
            if ((e = hipEventRecord(t0, s)) != hipSuccess) break;
            if ((e = launch_modexp_mfma(sh, a, s)) != hipSuccess) break;
            if ((e = hipEventRecord(t1, s)) != hipSuccess) break;
            if ((e = hipEventSynchronize(t1)) != hipSuccess) break;
            e = hipEventElapsedTime(&ms, t0, t1);
        }
        if (e != hipSuccess) {
            rc = hip_fail(e, "autotune run");
            break;
        }
        if (best == 0 || ms < best) {
            best = ms;
            *nt_out = sh.NT;
        }
    }
    cleanup();
    return rc;
}

}  // namespace

extern "C" {

int rsa_batch_create(const rsa_op *ops, size_t n_ops, const rsa_batch_opts *opts, void *hip_stream, rsa_batch **out) {
    if (!out) return fail(RNS_EINVAL, "null output handle");
    *out = nullptr;
    if (n_ops && !ops) return fail(RNS_EINVAL, "null op list");
    const int autotune = opts ? opts->autotune : 0;
    const int use_graph = opts ? opts->use_graph : 1;
    const int fixed_w = opts ? opts->window : 0;
    if (fixed_w < 0 || fixed_w > 6) return fail(RNS_EINVAL, "window must be in 0..6");
    hipStream_t s = (hipStream_t)hip_stream;
    std::unique_ptr<rsa_batch> b(new (std::nothrow) rsa_batch);
    if (!b) return fail(RNS_ENOMEM, "out of host memory");
    try {
        // 1. CRT intermediates
        size_t mpq_words = 0;
        for (size_t i = 0; i < n_ops; i++) {
            const rsa_op &o = ops[i];
            if (!o.key || (o.kind != RSA_OP_ENCRYPT && o.kind != RSA_OP_DECRYPT))
                return fail(RNS_EINVAL, "bad operation");
            if (o.count && (!o.in || !o.out)) return fail(RNS_EINVAL, "null buffer");
            if (o.count > (size_t)INT32_MAX - 64) return fail(RNS_EINVAL, "count too large");
            if (o.kind == RSA_OP_DECRYPT && !o.key->has_crt && !o.key->d_d)
                return fail(RNS_EINVAL, "key has no private exponent");
            if (o.kind == RSA_OP_DECRYPT && o.key->has_crt) mpq_words += o.count * 2 * o.key->half;
        }
        int rc = dmalloc((void **)&b->d_mpq, mpq_words * sizeof(uint32_t), &b->info.workspace_bytes);
        if (rc) return rc;

        // 2. jobs
        std::map<std::tuple<int, int, int>, size_t> group_of;
        auto add_job = [&](const rns_ctx *c, const uint32_t *E, const uint32_t *x, const std::vector<uint32_t> &hx,
                           const uint32_t *in, int in_limbs, uint32_t *o, int out_stride, size_t count) {
            Job J{};
            J.j.mb = c->d_mbase;
            J.j.mk = c->d_mkey;
            J.j.E = E;
            J.j.exp = x;
            J.j.in = in;
            J.j.out = o;
            J.j.batch = (int)count;
            J.j.in_limbs = in_limbs;
            J.j.in_stride = in_limbs;
            J.j.L = c->plan.L;
            J.j.out_stride = out_stride;
            J.j.exp_limbs = (int)hx.size();
            J.j.exp_stride = 0;
            J.j.window = best_window(hx, fixed_w);
            J.cost = mm_count(hx, J.j.window);
            b->info.modmuls += J.cost * count;
            b->info.jobs++;
            const MLayout &sh = c->mshape;
            auto key = std::make_tuple(sh.K, sh.W, sh.MT);
            auto it = group_of.find(key);
            if (it == group_of.end()) {
                it = group_of.emplace(key, b->groups.size()).first;
                b->groups.emplace_back();
                b->groups.back().shape = sh;
            }
            b->groups[it->second].jobs.push_back(J);
        };
        size_t mpq_off = 0;
        for (size_t i = 0; i < n_ops; i++) {
            const rsa_op &o = ops[i];
            if (!o.count) continue;
            const rsa_key *k = o.key;
            const int nl = (int)k->n_limbs;
            if (o.kind == RSA_OP_DECRYPT && k->has_crt) {
                const int h = (int)k->half;
                uint32_t *mpq = b->d_mpq + mpq_off;
                mpq_off += o.count * 2 * h;
                if (k->p->engine == RNS_ENGINE_MATRIX) {
                    add_job(k->p, k->d_mcentry_p, k->d_dp, k->h_dp, o.in, nl, mpq, 2 * h, o.count);
                    add_job(k->q, k->d_mcentry_q, k->d_dq, k->h_dq, o.in, nl, mpq + h, 2 * h, o.count);
                } else {
                    b->plain.push_back(PlainJob{k->p, k->q, k->d_centry_p, k->d_centry_q, o.in, k->d_dp, k->d_dq, nl, h,
                                                mpq, mpq + h, 2 * h, o.count});
                    b->info.jobs += 2;
                }
                b->garners.push_back(GarnerJob{k, mpq, o.out, o.count});
            } else {
                const bool enc = o.kind == RSA_OP_ENCRYPT;
                const rns_ctx *c = k->n;
                const uint32_t *x = enc ? k->d_e : k->d_d;
                const std::vector<uint32_t> &hx = enc ? k->h_e : k->h_d;
                if (c->engine == RNS_ENGINE_MATRIX) {
                    add_job(c, c->d_mentry, x, hx, o.in, nl, o.out, nl, o.count);
                } else {
                    b->plain.push_back(PlainJob{c, nullptr, entry_of(c), nullptr, o.in, x, nullptr, nl, (int)hx.size(),
                                                o.out, nullptr, nl, o.count});
                    b->info.jobs++;
                }
            }
        }

        // 3. per group: tile choice, tile order, device job table, window tables
        for (Group &g : b->groups) {
            std::vector<MLayout> cands;
            for (int nt : {1, 2}) {
                MfmaShape sh;
                if (mfma_shape_for(g.shape.K, sh, 16 * nt) && sh.W == g.shape.W && sh.MT == g.shape.MT &&
                    sh.NT == nt)
                    cands.push_back(sh);
            }
            if (autotune && cands.size() > 1) {
                const auto key = std::make_tuple(g.shape.K, g.shape.W, g.shape.MT);
                int nt = 0;
                {
                    std::lock_guard<std::mutex> lk(g_tune_mu);
                    auto it = g_tuned_nt.find(key);
                    if (it != g_tuned_nt.end()) nt = it->second;
                }
                if (!nt) {
                    if ((rc = tune_tile(g, cands, s, &nt))) return rc;
                    std::lock_guard<std::mutex> lk(g_tune_mu);
                    g_tuned_nt[key] = nt;
                }
                for (const MLayout &c : cands)
                    if (c.NT == nt) g.shape = c;
            }
            std::stable_sort(g.jobs.begin(), g.jobs.end(), [](const Job &x, const Job &y) { return x.cost > y.cost; });
            std::vector<MJob> js;
            for (Job &J : g.jobs) {
                J.j.tile0 = g.tiles;
                g.tiles += mfma_tiles(g.shape, (size_t)J.j.batch);
                g.max_window = std::max(g.max_window, J.j.window);
                js.push_back(J.j);
            }
            if ((rc = dmalloc((void **)&g.d_jobs, js.size() * sizeof(MJob), &b->info.workspace_bytes))) return rc;
            hipError_t e = hipMemcpy(g.d_jobs, js.data(), js.size() * sizeof(MJob), hipMemcpyHostToDevice);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
            const size_t tw = modexp_mfma_table_words(g.shape, g.max_window, (size_t)g.tiles);
            if ((rc = dmalloc((void **)&g.d_table, tw * sizeof(uint32_t), &b->info.workspace_bytes))) return rc;
            if ((e = hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking)) != hipSuccess)
                return hip_fail(e, "hipStreamCreate");
            if ((e = hipEventCreateWithFlags(&g.done, hipEventDisableTiming)) != hipSuccess)
                return hip_fail(e, "hipEventCreate");
        }
        hipError_t e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
        b->info.launches = (int)(b->groups.size() + b->plain.size());
        b->info.garner_launches = (int)b->garners.size();

        // 4. optional graph (channel-engine jobs allocate stream-ordered scratch
        // per launch, so a batch holding any runs without one)
        if (use_graph && b->plain.empty()) {
            if ((e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking)) != hipSuccess)
                return hip_fail(e, "hipStreamCreate");
            if ((e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal)) != hipSuccess)
                return hip_fail(e, "hipStreamBeginCapture");
            rc = enqueue(b.get(), b->capture);
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(b->capture, &graph);
            b->graph = graph;
            if (rc) return rc;
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess)
                return hip_fail(e, "hipGraphInstantiate");
        }
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    } catch (const std::bad_alloc &) {
        return fail(RNS_ENOMEM, "out of host memory");
    }
    *out = b.release();
    return ok();
}

int rsa_batch_run(rsa_batch *b, void *hip_stream) {
    if (!b) return fail(RNS_EINVAL, "null batch");
    hipStream_t s = (hipStream_t)hip_stream;
    if (b->exec) {
        hipError_t e = hipGraphLaunch(b->exec, s);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        return ok();
    }
    int rc = enqueue(b, s);
    return rc ? rc : ok();
}

int rsa_batch_info_get(const rsa_batch *b, rsa_batch_info *info) {
    if (!b || !info) return fail(RNS_EINVAL, "null argument");
    *info = b->info;
    return ok();
}

void rsa_batch_free(rsa_batch *b) { delete b; }

}  // extern "C"
