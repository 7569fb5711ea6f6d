// Batched RSA operations over many keys (include/rnsrsa.h, rsa_batch_*).
//
// Planning, done once per batch (jobs.cpp): every operation becomes
// exponentiation jobs (a CRT decryption is two half-size jobs plus a Garner
// step); each job gets the window width that minimises its number of
// Montgomery products for its own exponent; jobs on contexts with the same
// matrix-core kernel shape form one launch, with the tiles of the most
// expensive jobs first so the workgroup dispatcher starts the long ones
// early.  The launches of different shapes run concurrently on internal
// streams; the Garner steps follow them.  With use_graph the whole sequence
// is captured into a hipGraph at creation.
#include <algorithm>
#include <climits>
#include <map>
#include <string>
#include <memory>
#include <new>
#include <vector>

#include "jobs.hpp"
#include "range.hpp"

using namespace rnsrsa;
using namespace rnsrsa::api;

struct rsa_batch {
    JobPlan plan;
    std::vector<MJob *> d_jobs;
    std::vector<uint32_t *> d_tables;
    std::vector<hipStream_t> streams;   // one per branch
    std::vector<hipEvent_t> done;       // one per branch
    std::vector<GarnerGroup> ggroups;   // Garner steps, one grouped launch per base shape
    std::vector<GJob *> d_gjobs;
    std::vector<int> gdep;              // the one exponentiation group a Garner group waits for, or -1
    uint32_t *d_mpq = nullptr;
    RangeLaunch range{};                // input check of every operation: one launch
    RangeJob *d_rjobs = nullptr;
    hipEvent_t fork = nullptr;
    hipStream_t capture = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    rsa_batch_info info{};
    std::vector<float> group_ms;        // autotune: time of each group's launch as tuned (ms)
    std::vector<std::vector<size_t>> branches;   // exponentiation groups per branch, in launch order
    ~rsa_batch() {
        hipDeviceSynchronize();
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        for (MJob *p : d_jobs)
            if (p) hipFree(p);
        for (uint32_t *p : d_tables)
            if (p) hipFree(p);
        for (GJob *p : d_gjobs)
            if (p) hipFree(p);
        for (hipEvent_t e : done)
            if (e) hipEventDestroy(e);
        for (hipStream_t s : streams)
            if (s) hipStreamDestroy(s);
        if (d_mpq) hipFree(d_mpq);
        if (d_rjobs) hipFree(d_rjobs);
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
    // each branch's exponentiation groups in turn on its stream, each
    // followed there by the Garner groups that need only its results; the
    // others follow the join on s.  Branches are enqueued longest first, so
    // the longest group's workgroups take their CUs before the shorter
    // groups' fill the rest.
    for (size_t br = 0; br < b->branches.size(); br++) {
        hipStream_t bs = b->streams[br];
        if ((e = hipStreamWaitEvent(bs, b->fork, 0)) != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
        for (size_t i : b->branches[br]) {
            if ((e = launch_group(b->plan.groups[i], b->d_jobs[i], b->d_tables[i], bs)) != hipSuccess)
                return hip_fail(e, "grouped modexp launch");
            for (size_t j = 0; j < b->ggroups.size(); j++)
                if (b->gdep[j] == (int)i && (e = launch_garner_group(b->ggroups[j], b->d_gjobs[j], bs)) != hipSuccess)
                    return hip_fail(e, "grouped Garner launch");
        }
        if ((e = hipEventRecord(b->done[br], bs)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    }
    if ((e = launch_range_check(b->range, s)) != hipSuccess) return hip_fail(e, "range check launch");
    int rc = launch_plain_and_garner(b->plan, s, true, false);
    if (rc) return rc;
    for (hipEvent_t d : b->done)
        if ((e = hipStreamWaitEvent(s, d, 0)) != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
    for (size_t j = 0; j < b->ggroups.size(); j++)
        if (b->gdep[j] < 0 && (e = launch_garner_group(b->ggroups[j], b->d_gjobs[j], s)) != hipSuccess)
            return hip_fail(e, "grouped Garner launch");
    return RNS_OK;
}

// Times launches of one exponentiation group as it would run (every job,
// outputs redirected to scratch so the caller's buffers are not written) for
// the autotuner.  The scratch grows as needed and is released by release().
struct GroupTimer {
    hipStream_t s = nullptr;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    uint32_t *out = nullptr, *table = nullptr;
    MJob *jobs = nullptr;
    size_t out_words = 0, table_words = 0, njobs = 0;
    int launches = 0;

    int init() {
        hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreate(&t0);
        if (e == hipSuccess) e = hipEventCreate(&t1);
        return e == hipSuccess ? RNS_OK : hip_fail(e, "autotune set-up");
    }
    void release() {
        if (out) hipFree(out);
        if (table) hipFree(table);
        if (jobs) hipFree(jobs);
        if (t0) hipEventDestroy(t0);
        if (t1) hipEventDestroy(t1);
        if (s) hipStreamDestroy(s);
    }
    template <class T>
    static hipError_t grow(T **p, size_t *have, size_t need) {
        if (need <= *have) return hipSuccess;
        if (*p) hipFree(*p);
        *p = nullptr;
        *have = 0;
        hipError_t e = hipMalloc((void **)p, need * sizeof(T));
        if (e == hipSuccess) *have = need;
        return e;
    }
    // Best of `reps` launch times of g (its shape, windows and tile order) in ms.
    int time(const JobGroup &g, int reps, float *best) {
        std::vector<MJob> js;
        size_t words = 0;
        for (const PlannedJob &J : g.jobs) words += (size_t)J.j.batch * J.j.out_stride;
        hipError_t e = grow(&out, &out_words, words);
        if (e == hipSuccess) e = grow(&table, &table_words, g.table_words());
        if (e == hipSuccess) e = grow(&jobs, &njobs, g.jobs.size());
        if (e != hipSuccess) return fail(RNS_ENOMEM, std::string("autotune scratch: ") + hipGetErrorString(e));
        size_t off = 0;
        for (const PlannedJob &J : g.jobs) {
            js.push_back(J.j);
            js.back().out = out + off;
            off += (size_t)J.j.batch * J.j.out_stride;
        }
        if ((e = hipMemcpy(jobs, js.data(), js.size() * sizeof(MJob), hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "hipMemcpy");
        *best = 0;
        for (int rep = 0; rep < reps; rep++) {
            float ms = 0;
            if ((e = hipEventRecord(t0, s)) != hipSuccess) break;
            if ((e = launch_group(g, jobs, table, s)) != hipSuccess) break;
            if ((e = hipEventRecord(t1, s)) != hipSuccess) break;
            if ((e = hipEventSynchronize(t1)) != hipSuccess) break;
            if ((e = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess) break;
            launches++;
            if (*best == 0 || ms < *best) *best = ms;
        }
        return e == hipSuccess ? RNS_OK : hip_fail(e, "autotune run");
    }
};

// Autotuner of one exponentiation group: first the tile (elements per
// workgroup) among the shapes of its class, with every job at the window
// that minimises its product count; then, for each exponent length in the
// group (longest total work first), the window offset -1 / 0 / +1 from each
// job's own best, kept when it is at least 1% faster.  Each candidate is
// timed on the whole group (best of 3 launches).  Choices already made in
// this process for the class are reused without timing.
int tune_group(JobGroup &g, bool fixed_window, GroupTimer &tm, float *ms_out) {
    constexpr int kReps = 3;
    std::vector<MLayout> cands;
    for (int nt : {1, 2}) {
        MfmaShape sh;
        if (mfma_shape_for(g.shape.K, sh, 16 * nt) && sh.W == g.shape.W && sh.MT == g.shape.MT && sh.NT == nt)
            cands.push_back(sh);
    }
    float best = 0;
    int rc = RNS_OK;
    const int cached_nt = tuned_nt(g.shape);
    if (cands.size() > 1 && !cached_nt) {
        MLayout pick = g.shape;
        for (const MLayout &c : cands) {
            JobGroup trial = g;
            trial.shape = c;
            finish_group(trial);
            float ms = 0;
            if ((rc = tm.time(trial, kReps, &ms))) return rc;
            if (best == 0 || ms < best) {
                best = ms;
                pick = c;
            }
        }
        g.shape = pick;
        set_tuned_nt(g.shape, g.shape.NT);
    } else if (cached_nt) {
        for (const MLayout &c : cands)
            if (c.NT == cached_nt) g.shape = c;
    }
    finish_group(g);
    g.auto_tile = false;
    if (!fixed_window) {
        // exponent lengths of the group, by total products (largest first)
        std::map<int, size_t> work;
        for (const PlannedJob &J : g.jobs) work[J.j.exp_limbs] += J.cost * (size_t)J.j.batch;
        std::vector<std::pair<size_t, int>> order;
        for (auto &kv : work) order.push_back({kv.second, kv.first});
        std::sort(order.rbegin(), order.rend());
        for (auto &o : order) {
            const int el = o.second;
            bool known = false;
            int dw = tuned_dw(g.shape, el, &known);
            if (!known) {
                if (best == 0 && (rc = tm.time(g, kReps, &best))) return rc;
                dw = 0;
                for (int cand : {-1, 1}) {
                    JobGroup trial = g;
                    bool changed = false;
                    for (PlannedJob &J : trial.jobs)
                        if (J.j.exp_limbs == el) {
                            const int before = J.j.window;
                            set_job_window(J, cand);
                            changed = changed || J.j.window != before;
                        }
                    if (!changed) continue;
                    finish_group(trial);
                    float ms = 0;
                    if ((rc = tm.time(trial, kReps, &ms))) return rc;
                    if (ms < 0.99f * best) {
                        best = ms;
                        dw = cand;
                    }
                }
                set_tuned_dw(g.shape, el, dw);
            }
            for (PlannedJob &J : g.jobs)
                if (J.j.exp_limbs == el) set_job_window(J, dw);
        }
        finish_group(g);
    }
    if (best == 0 && (rc = tm.time(g, kReps, &best))) return rc;
    *ms_out = best;
    return RNS_OK;
}

// Per (kernel shape, exponent length) class of a batch: k, waves, tile,
// window, offset and the tuned launch time; returns the class count (the
// first `cap` are written).
size_t batch_classes(const rsa_batch *b, rsa_batch_class *out, size_t cap) {
    size_t i = 0;
    for (size_t gi = 0; gi < b->plan.groups.size(); gi++) {
        const JobGroup &g = b->plan.groups[gi];
        std::map<int, std::vector<const PlannedJob *>> by_len;   // exponent limbs -> jobs
        for (const PlannedJob &J : g.jobs) by_len[J.j.exp_limbs].push_back(&J);
        for (auto it = by_len.rbegin(); it != by_len.rend(); ++it, ++i) {
            if (i >= cap) continue;
            const PlannedJob *heavy = *std::max_element(
                it->second.begin(), it->second.end(),
                [](const PlannedJob *x, const PlannedJob *y) { return x->cost < y->cost; });
            rsa_batch_class &c = out[i];
            c.k = g.shape.K;
            c.waves = g.shape.W;
            c.group = g.shape.NM();
            c.exp_bits = 32 * it->first;
            c.window = heavy->j.window;
            c.window_offset = heavy->j.window - heavy->w0;
            c.jobs = (int)it->second.size();
            c.tuned = gi < b->group_ms.size() ? 1 : 0;
            c.launch_ms = gi < b->group_ms.size() ? b->group_ms[gi] : 0.0;
        }
    }
    return i;
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
        // CRT intermediates, then the jobs
        size_t mpq_words = 0;
        for (size_t i = 0; i < n_ops; i++) {
            if (!ops[i].key) return fail(RNS_EINVAL, "bad operation");
            mpq_words += op_mpq_words(ops[i].key, ops[i].kind, ops[i].count);
        }
        int rc = dmalloc((void **)&b->d_mpq, mpq_words * sizeof(uint32_t), &b->info.workspace_bytes);
        if (rc) return rc;
        std::vector<PlannedOp> pops;
        size_t off = 0;
        for (size_t i = 0; i < n_ops; i++) {
            const rsa_op &o = ops[i];
            pops.push_back(PlannedOp{o.key, o.kind, o.in, o.out, o.count, b->d_mpq ? b->d_mpq + off : nullptr});
            off += op_mpq_words(o.key, o.kind, o.count);
        }
        if ((rc = plan_jobs(pops, fixed_w, b->plan))) return rc;

        // tile and window choice, device job tables, window tables, streams
        if (autotune) {
            GroupTimer tm;
            rc = tm.init();
            for (JobGroup &g : b->plan.groups) {
                if (rc) break;
                float ms = 0;
                rc = tune_group(g, fixed_w != 0, tm, &ms);
                if (!rc) b->group_ms.push_back(ms);
            }
            b->info.tuning_launches = tm.launches;
            tm.release();
            if (rc) return rc;
            b->plan.modmuls = 0;
            for (const JobGroup &g : b->plan.groups)
                for (const PlannedJob &J : g.jobs) b->plan.modmuls += J.cost * (size_t)J.j.batch;
        }
        // Branches: at most kBranches concurrent streams (the device runs a
        // few hardware queues, and two streams on one queue serialise in
        // whatever order they were enqueued).  The groups are taken longest
        // first (by tuned launch time, else by longest chain of products
        // times the base size), each onto the branch with the least work so
        // far, so short groups follow the short ones instead of waiting
        // behind the longest.
        {
            constexpr size_t kBranches = 4;
            std::vector<std::pair<double, size_t>> key;
            for (size_t i = 0; i < b->plan.groups.size(); i++) {
                const JobGroup &g = b->plan.groups[i];
                double est = 0;
                for (const PlannedJob &J : g.jobs) est = std::max(est, (double)J.cost * g.shape.K);
                key.push_back({i < b->group_ms.size() ? (double)b->group_ms[i] : est, i});
            }
            std::stable_sort(key.begin(), key.end(), [](const auto &x, const auto &y) { return x.first > y.first; });
            const size_t nb = std::min(kBranches, key.size());
            b->branches.assign(nb, {});
            std::vector<double> load(nb, 0.0);
            for (auto &kv : key) {
                const size_t br = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
                b->branches[br].push_back(kv.second);
                load[br] += kv.first;
            }
            for (size_t br = 0; br < nb; br++) {
                hipStream_t gs = nullptr;
                hipEvent_t ge = nullptr;
                hipError_t e = hipStreamCreateWithFlags(&gs, hipStreamNonBlocking);
                b->streams.push_back(gs);
                if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
                e = hipEventCreateWithFlags(&ge, hipEventDisableTiming);
                b->done.push_back(ge);
                if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
            }
        }
        for (JobGroup &g : b->plan.groups) {
            std::vector<MJob> js;
            for (const PlannedJob &J : g.jobs) js.push_back(J.j);
            MJob *dj = nullptr;
            uint32_t *dt = nullptr;
            rc = dmalloc((void **)&dj, js.size() * sizeof(MJob), &b->info.workspace_bytes);
            b->d_jobs.push_back(dj);
            if (rc) return rc;
            hipError_t e = hipMemcpy(dj, js.data(), js.size() * sizeof(MJob), hipMemcpyHostToDevice);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
            rc = dmalloc((void **)&dt, g.table_words() * sizeof(uint32_t), &b->info.workspace_bytes);
            b->d_tables.push_back(dt);
            if (rc) return rc;
        }
        // Garner steps: one grouped launch per base shape, job tables on the
        // device; a group whose halves all come from one matrix-core
        // exponentiation group (same k, no channel-engine jobs of that k)
        // runs right after it on its stream
        b->ggroups = garner_groups(b->plan);
        for (const GarnerGroup &g : b->ggroups) {
            int dep = -1, n = 0;
            for (size_t i = 0; i < b->plan.groups.size(); i++)
                if (b->plan.groups[i].shape.K == g.K) {
                    dep = (int)i;
                    n++;
                }
            for (const PlainJob &pj : b->plan.plain)
                if (pj.c0->plan.base->K == g.K) n = 2;
            b->gdep.push_back(n == 1 ? dep : -1);
        }
        for (const GarnerGroup &g : b->ggroups) {
            GJob *dj = nullptr;
            rc = dmalloc((void **)&dj, g.jobs.size() * sizeof(GJob), &b->info.workspace_bytes);
            b->d_gjobs.push_back(dj);
            if (rc) return rc;
            hipError_t e = hipMemcpy(dj, g.jobs.data(), g.jobs.size() * sizeof(GJob), hipMemcpyHostToDevice);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
        }
        // input range check: one job per operation
        std::vector<RangeJob> rj;
        int elems = 0;
        for (size_t i = 0; i < n_ops; i++) {
            if (!ops[i].count) continue;
            if (ops[i].count > (size_t)(INT32_MAX - 256 - elems)) return fail(RNS_EINVAL, "more than 2^31 elements");
            RangeJob j = range_job(ops[i].key, ops[i].in, ops[i].count);
            j.elem0 = elems;
            elems += (int)ops[i].count;
            rj.push_back(j);
        }
        if (!rj.empty()) {
            rc = dmalloc((void **)&b->d_rjobs, rj.size() * sizeof(RangeJob), &b->info.workspace_bytes);
            if (rc) return rc;
            hipError_t he = hipMemcpy(b->d_rjobs, rj.data(), rj.size() * sizeof(RangeJob), hipMemcpyHostToDevice);
            if (he != hipSuccess) return hip_fail(he, "hipMemcpy");
            b->range.jobs = b->d_rjobs;
            b->range.njobs = (int)rj.size();
            b->range.total = elems;
        }
        hipError_t e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
        b->info.launches = (int)(b->plan.groups.size() + b->plan.plain.size());
        b->info.garner_launches = (int)b->ggroups.size();
        b->info.jobs = (int)b->plan.jobs;
        b->info.modmuls = b->plan.modmuls;

        // optional graph (channel-engine jobs allocate stream-ordered scratch
        // per launch, so a batch holding any runs without one)
        if (use_graph && b->plan.plain.empty()) {
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

int rsa_batch_classes(const rsa_batch *b, rsa_batch_class *out, size_t cap, size_t *n) {
    if (!b || !n || (cap && !out)) return fail(RNS_EINVAL, "null argument");
    try {
        *n = batch_classes(b, out, cap);
    } catch (const std::bad_alloc &) {
        return fail(RNS_ENOMEM, "out of host memory");
    }
    return ok();
}

void rsa_batch_free(rsa_batch *b) { delete b; }

}  // extern "C"
