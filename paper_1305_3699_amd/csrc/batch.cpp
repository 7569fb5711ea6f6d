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
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> done;
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
    // each exponentiation group on its stream, followed there by the Garner
    // groups that need only its results; the others follow the join on s
    for (size_t i = 0; i < b->plan.groups.size(); i++) {
        if ((e = hipStreamWaitEvent(b->streams[i], b->fork, 0)) != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
        if ((e = launch_group(b->plan.groups[i], b->d_jobs[i], b->d_tables[i], b->streams[i])) != hipSuccess)
            return hip_fail(e, "grouped modexp launch");
        for (size_t j = 0; j < b->ggroups.size(); j++)
            if (b->gdep[j] == (int)i && (e = launch_garner_group(b->ggroups[j], b->d_gjobs[j], b->streams[i])) != hipSuccess)
                return hip_fail(e, "grouped Garner launch");
        if ((e = hipEventRecord(b->done[i], b->streams[i])) != hipSuccess) return hip_fail(e, "hipEventRecord");
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

// Times each candidate tile of a group's shape class on copies of its most
// expensive job (outputs to scratch) and returns the faster NT.
int tune_tile(const JobGroup &g, const std::vector<MLayout> &cands, int *nt_out) {
    const PlannedJob &heavy = *std::max_element(
        g.jobs.begin(), g.jobs.end(), [](const PlannedJob &a, const PlannedJob &b) { return a.cost < b.cost; });
    const int copies = std::max(1, (int)(16384 / std::max(1, heavy.j.batch)));
    const size_t out_words = (size_t)copies * heavy.j.batch * heavy.j.L;
    uint32_t *d_out = nullptr;
    MJob *d_jobs = nullptr;
    uint32_t *d_table = nullptr;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    hipStream_t s = nullptr;
    int rc = RNS_OK;
    float best = 0;
    *nt_out = cands[0].NT;
    auto cleanup = [&] {
        if (d_out) hipFree(d_out);
        if (d_jobs) hipFree(d_jobs);
        if (d_table) hipFree(d_table);
        if (t0) hipEventDestroy(t0);
        if (t1) hipEventDestroy(t1);
        if (s) hipStreamDestroy(s);
    };
    hipError_t e = hipMalloc((void **)&d_out, out_words * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc((void **)&d_jobs, (size_t)copies * sizeof(MJob));
    if (e == hipSuccess) e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
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

        // tile choice, device job tables, window tables, streams
        for (JobGroup &g : b->plan.groups) {
            std::vector<MLayout> cands;
            for (int nt : {1, 2}) {
                MfmaShape sh;
                if (mfma_shape_for(g.shape.K, sh, 16 * nt) && sh.W == g.shape.W && sh.MT == g.shape.MT && sh.NT == nt)
                    cands.push_back(sh);
            }
            if (autotune && cands.size() > 1) {
                int nt = tuned_nt(g.shape);
                if (!nt) {
                    if ((rc = tune_tile(g, cands, &nt))) return rc;
                    set_tuned_nt(g.shape, nt);
                }
                for (const MLayout &c : cands)
                    if (c.NT == nt) g.shape = c;
                finish_group(g);
            }
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
            hipStream_t gs = nullptr;
            hipEvent_t ge = nullptr;
            e = hipStreamCreateWithFlags(&gs, hipStreamNonBlocking);
            b->streams.push_back(gs);
            if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
            e = hipEventCreateWithFlags(&ge, hipEventDisableTiming);
            b->done.push_back(ge);
            if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
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

void rsa_batch_free(rsa_batch *b) { delete b; }

}  // extern "C"
