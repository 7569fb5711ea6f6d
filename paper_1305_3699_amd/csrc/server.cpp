// Request server over resident keys (include/rnsrsa.h, rsa_server_*).
//
// One host thread runs the loop: admit the requests whose arrival time has
// passed, retire dispatches whose completion event fired (results are copied
// out of pinned staging into the callers' buffers), and when a dispatch slot
// is free, pack as many pending requests as the device-memory budget allows
// into one dispatch.  A dispatch groups its requests by (key, kind) into RSA
// operations, plans them into grouped launches (jobs.cpp), and enqueues on the
// slot's stream: one host-to-device copy of the inputs and job tables, the
// launches, one device-to-host copy of the outputs, an event.  Each slot
// keeps one device arena across its dispatches (grown in stream order when a
// dispatch needs more), so a dispatch allocates nothing in the common case.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <deque>
#include <thread>
#include <tuple>
#include <utility>
#include <vector>

#include "jobs.hpp"
#include "range.hpp"

using namespace rnsrsa;
using namespace rnsrsa::api;

namespace {

constexpr size_t kDefaultBudget = (size_t)64 << 30;
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    uint32_t *h_in = nullptr;    // pinned staging: inputs, then job tables
    size_t h_in_bytes = 0;
    uint32_t *h_out = nullptr;   // pinned staging: outputs
    size_t h_out_bytes = 0;
    void *d_arena = nullptr;     // the slot's device arena, kept across its dispatches
    size_t arena_bytes = 0;
    size_t bytes = 0;            // device bytes the dispatch in flight uses
    bool busy = false;
    std::vector<size_t> reqs;              // request indices of the dispatch
    std::vector<size_t> out_word;          // their output offsets in h_out
};

int ensure_pinned(uint32_t **p, size_t *have, size_t need) {
    if (*have >= need) return RNS_OK;
    if (*p) hipHostFree(*p);
    *p = nullptr;
    *have = 0;
    size_t sz = std::max(need, (size_t)1 << 20);
    hipError_t e = hipHostMalloc((void **)p, sz, hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(e, "hipHostMalloc");
    *have = sz;
    return RNS_OK;
}

// Device bytes a dispatch needs for `count` requests of one (key, kind),
// with window tables sized for the widest window (2^6 entries) and the
// fewest elements per tile (a small launch is spread over more tiles).
size_t op_bytes(const rsa_key *k, int kind, size_t count) {
    size_t words = 2 * count * k->n_limbs + op_mpq_words(k, kind, count);
    const bool crt = kind == RSA_OP_DECRYPT && k->has_crt;
    const rns_ctx *ctxs[2] = {crt ? k->p : k->n, crt ? k->q : nullptr};
    for (const rns_ctx *c : ctxs) {
        if (!c || c->engine != RNS_ENGINE_MATRIX) continue;
        words += modexp_mfma_table_words(c->mshape, 6, (size_t)mfma_job_tiles(c->mshape, count, kMinTileElems));
    }
    // job descriptors (two exponentiations and a Garner step at most), plus
    // the alignment of the arena's regions (inputs, outputs, CRT scratch, one
    // table per group, job tables, Garner job tables: at most 7 per op)
    return words * sizeof(uint32_t) + 2 * sizeof(MJob) + sizeof(GJob) + 7 * kAlign;
}

// Kernel-shape class of a request: the context its exponentiations run on
// (the p-half for a CRT decryption).  Requests of one class have similar
// costs and share launches; classes are dispatched separately so that short
// requests do not wait for long ones.
std::tuple<int, int, int, int> request_class(const rsa_key *k, int kind) {
    const rns_ctx *c = (kind == RSA_OP_DECRYPT && k->has_crt) ? k->p : k->n;
    if (c->engine != RNS_ENGINE_MATRIX) return std::make_tuple(-c->plan.base->K, 0, 0, c->engine);
    return std::make_tuple(c->mshape.K, c->mshape.W, c->mshape.MT, c->engine);
}

double now_s(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct rsa_server {
    std::vector<const rsa_key *> keys;
    size_t budget = kDefaultBudget;
    size_t max_ops = 16384;
    size_t max_pending = 0;      // 0: no limit on requests waiting for admission
    std::vector<Slot> slots;
    ~rsa_server() {
        for (Slot &s : slots) {
            if (s.d_arena) hipFreeAsync(s.d_arena, s.stream);   // stream-ordered, as it was allocated
            if (s.stream) hipStreamSynchronize(s.stream);
            if (s.done) hipEventDestroy(s.done);
            if (s.stream) hipStreamDestroy(s.stream);
            if (s.h_in) hipHostFree(s.h_in);
            if (s.h_out) hipHostFree(s.h_out);
        }
    }
};

namespace {

// Packs the requests `ids` into one dispatch on slot `sl` and enqueues it.
int dispatch(rsa_server *srv, Slot &sl, const rsa_request *reqs, const std::vector<size_t> &ids) {
    // operations: requests grouped by (key, kind), in first-arrival order
    std::map<std::pair<int, int>, size_t> op_of;
    struct Op {
        int key, kind;
        std::vector<size_t> reqs;
    };
    std::vector<Op> ops;
    for (size_t id : ids) {
        auto k = std::make_pair(reqs[id].key, reqs[id].kind);
        auto it = op_of.find(k);
        if (it == op_of.end()) {
            it = op_of.emplace(k, ops.size()).first;
            ops.push_back(Op{k.first, k.second, {}});
        }
        ops[it->second].reqs.push_back(id);
    }
    // device layout: [inputs | job tables | Garner job tables | outputs | CRT
    // scratch | window tables]; the job regions are sized for the most jobs
    // the operations can make (two exponentiations and a Garner step each),
    // so the inputs and both job tables are one copy from staging
    size_t in_words = 0, out_words = 0, mpq_words = 0;
    for (const Op &o : ops) {
        const rsa_key *k = srv->keys[o.key];
        in_words += o.reqs.size() * k->n_limbs;
        mpq_words += op_mpq_words(k, o.kind, o.reqs.size());
    }
    out_words = in_words;
    const size_t mjob_cap = align_up(2 * ops.size() * sizeof(MJob)), gjob_cap = align_up(ops.size() * sizeof(GJob));
    const size_t in_off = 0, jobs_off = align_up(in_words * 4), gj_off = jobs_off + mjob_cap;
    const size_t out_off = gj_off + gjob_cap, mpq_off = out_off + align_up(out_words * 4);
    size_t tbl_off = mpq_off + align_up(mpq_words * 4);
    // plan with provisional device pointers relative to a null arena, then rebase
    std::vector<PlannedOp> pops;
    {
        size_t iw = 0, mw = 0;
        for (const Op &o : ops) {
            const rsa_key *k = srv->keys[o.key];
            const size_t cnt = o.reqs.size();
            PlannedOp p{k, o.kind, (const uint32_t *)(uintptr_t)(in_off + iw * 4 + 4),
                        (uint32_t *)(uintptr_t)(out_off + iw * 4 + 4), cnt,
                        (uint32_t *)(uintptr_t)(mpq_off + mw * 4 + 4)};
            pops.push_back(p);
            iw += cnt * k->n_limbs;
            mw += op_mpq_words(k, o.kind, cnt);
        }
    }
    JobPlan plan;
    int rc = plan_jobs(pops, 0, plan);
    if (rc) return rc;
    std::vector<size_t> g_tbl, g_jobs;
    for (const JobGroup &g : plan.groups) {
        g_tbl.push_back(tbl_off);
        tbl_off += align_up(g.table_words() * 4);
    }
    size_t njobs = 0;
    for (const JobGroup &g : plan.groups) {
        g_jobs.push_back(jobs_off + njobs * sizeof(MJob));
        njobs += g.jobs.size();
    }
    // at most one Garner job per planned Garner step
    const size_t ngj = plan.garners.size();
    if (njobs * sizeof(MJob) > mjob_cap || ngj * sizeof(GJob) > gjob_cap) return fail(RNS_EINVAL, "job table overflow");
    const size_t total = tbl_off;

    // pinned staging laid out as the first device regions: inputs, job
    // tables, Garner job tables; outputs
    if ((rc = ensure_pinned(&sl.h_in, &sl.h_in_bytes, out_off))) return rc;
    if ((rc = ensure_pinned(&sl.h_out, &sl.h_out_bytes, out_words * 4))) return rc;
    if (total > sl.arena_bytes) {
        // grow the slot's arena: the old one is released in stream order,
        // after the slot's earlier dispatches
        if (sl.d_arena) {
            hipError_t fe = hipFreeAsync(sl.d_arena, sl.stream);
            sl.d_arena = nullptr;
            sl.arena_bytes = 0;
            if (fe != hipSuccess) return hip_fail(fe, "hipFreeAsync");
        }
        const size_t want = std::max(total + total / 4, (size_t)1 << 20);
        hipError_t e = hipMallocAsync(&sl.d_arena, want, sl.stream);
        if (e != hipSuccess) {
            sl.d_arena = nullptr;
            return fail(RNS_ENOMEM, std::string("hipMallocAsync: ") + hipGetErrorString(e));
        }
        sl.arena_bytes = want;
    }
    char *base = (char *)sl.d_arena;
    hipError_t e = hipSuccess;
    auto rebase = [&](const void *p) -> uint32_t * { return (uint32_t *)(base + ((uintptr_t)p - 4)); };
    // inputs into staging, in op order; remember each request's output slot
    sl.reqs.clear();
    sl.out_word.clear();
    {
        size_t w = 0;
        for (const Op &o : ops) {
            const size_t nl = srv->keys[o.key]->n_limbs;
            for (size_t id : o.reqs) {
                std::memcpy(sl.h_in + w, reqs[id].in, nl * 4);
                sl.reqs.push_back(id);
                sl.out_word.push_back(w);
                w += nl;
            }
        }
    }
    // job tables with real pointers, after the inputs in staging
    MJob *hj = (MJob *)((char *)sl.h_in + jobs_off);
    size_t jn = 0;
    for (JobGroup &g : plan.groups)
        for (PlannedJob &J : g.jobs) {
            J.j.in = rebase(J.j.in);
            J.j.out = rebase(J.j.out);
            hj[jn++] = J.j;
        }
    for (PlainJob &p : plan.plain) {
        p.in = rebase(p.in);
        p.out0 = rebase(p.out0);
        if (p.out1) p.out1 = rebase(p.out1);
    }
    for (GarnerJob &gj : plan.garners) {
        gj.mpq = rebase(gj.mpq);
        gj.out = rebase(gj.out);
    }
    // Garner steps grouped by base shape (real pointers), after the job tables
    const std::vector<GarnerGroup> gg = garner_groups(plan);
    GJob *hg = (GJob *)((char *)sl.h_in + gj_off);
    std::vector<size_t> g_gj;
    size_t gn = 0;
    for (const GarnerGroup &g : gg) {
        g_gj.push_back(gj_off + gn * sizeof(GJob));
        for (const GJob &J : g.jobs) hg[gn++] = J;
    }
    // enqueue: inputs and job tables in one copy
    const size_t up = gn ? gj_off + gn * sizeof(GJob) : jobs_off + njobs * sizeof(MJob);
    if ((e = hipMemcpyAsync(base + in_off, sl.h_in, up, hipMemcpyHostToDevice, sl.stream)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync");
    for (size_t i = 0; i < plan.groups.size(); i++)
        if ((e = launch_group(plan.groups[i], (const MJob *)(base + g_jobs[i]), (uint32_t *)(base + g_tbl[i]),
                              sl.stream)) != hipSuccess)
            return hip_fail(e, "grouped modexp launch");
    if ((rc = launch_plain_and_garner(plan, sl.stream, true, false))) return rc;
    for (size_t i = 0; i < gg.size(); i++)
        if ((e = launch_garner_group(gg[i], (const GJob *)(base + g_gj[i]), sl.stream)) != hipSuccess)
            return hip_fail(e, "grouped Garner launch");
    if ((e = hipMemcpyAsync(sl.h_out, base + out_off, out_words * 4, hipMemcpyDeviceToHost, sl.stream)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync");
    if ((e = hipEventRecord(sl.done, sl.stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    sl.bytes = total;
    sl.busy = true;
    return RNS_OK;
}

}  // namespace

static int server_create(const rsa_key *const *keys, size_t n_keys, const rsa_server_opts *opts, rsa_server **out) {
    if (!out) return fail(RNS_EINVAL, "null output handle");
    *out = nullptr;
    if (!keys || !n_keys) return fail(RNS_EINVAL, "no keys");
    std::unique_ptr<rsa_server> s(new (std::nothrow) rsa_server);
    if (!s) return fail(RNS_ENOMEM, "out of host memory");
    for (size_t i = 0; i < n_keys; i++) {
        if (!keys[i]) return fail(RNS_EINVAL, "null key");
        s->keys.push_back(keys[i]);
    }
    if (opts && opts->hbm_budget) s->budget = opts->hbm_budget;
    if (opts && opts->max_dispatch_ops) s->max_ops = opts->max_dispatch_ops;
    if (opts) s->max_pending = opts->max_pending;
    // default: one slot per hardware queue the runtime gives a process (4):
    // a further stream shares a queue and its dispatch waits behind the one
    // enqueued there before it (measured: p99 latency up to 1.4x at 8 slots)
    const int inflight = (opts && opts->max_inflight > 0) ? opts->max_inflight : 4;
    if (inflight > 32) return fail(RNS_EINVAL, "max_inflight above 32");
    configure_pool_once();
    s->slots.resize((size_t)inflight);
    for (Slot &sl : s->slots) {
        hipError_t e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
        if ((e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess)
            return hip_fail(e, "hipEventCreate");
    }
    *out = s.release();
    return ok();
}

static int server_replay(rsa_server *srv, const rsa_request *reqs, size_t n, double *latency, rsa_server_stats *stats) {
    if (!srv) return fail(RNS_EINVAL, "null server");
    if (n && !reqs) return fail(RNS_EINVAL, "null request list");
    std::vector<size_t> need(n);
    for (size_t i = 0; i < n; i++) {
        const rsa_request &r = reqs[i];
        if (r.key < 0 || (size_t)r.key >= srv->keys.size()) return fail(RNS_EINVAL, "bad key index");
        if (r.kind != RSA_OP_ENCRYPT && r.kind != RSA_OP_DECRYPT) return fail(RNS_EINVAL, "bad request kind");
        if (!r.in || !r.out) return fail(RNS_EINVAL, "null request buffer");
        if (i && r.arrival < reqs[i - 1].arrival) return fail(RNS_EINVAL, "arrivals must be non-decreasing");
        const rsa_key *k = srv->keys[(size_t)r.key];
        if (r.kind == RSA_OP_DECRYPT && !k->has_crt && !k->d_d) return fail(RNS_EINVAL, "key has no private exponent");
        if ((r.kind == RSA_OP_ENCRYPT || !k->has_crt) && !k->n)
            return fail(RNS_EUNSUPPORTED, "CRT-only key: no context for the full modulus");
        if (!host_below_n(k, r.in))
            return fail(RNS_ERANGE, "request " + std::to_string(i) + ": input not below n (raw RSA works on [0, n))");
        need[i] = op_bytes(k, r.kind, 1);
        if (need[i] > srv->budget)
            return fail(RNS_EBUSY, "request " + std::to_string(i) + " alone exceeds the device-memory admission budget");
    }
    std::vector<double> lat(n, 0.0);
    // pending requests, one FIFO per kernel-shape class
    std::map<std::tuple<int, int, int, int>, int> class_id;
    std::vector<int> cls(n);
    for (size_t i = 0; i < n; i++) {
        auto c = request_class(srv->keys[(size_t)reqs[i].key], reqs[i].kind);
        auto it = class_id.emplace(c, (int)class_id.size()).first;
        cls[i] = it->second;
    }
    std::vector<std::deque<size_t>> pending(class_id.size());
    size_t n_pending = 0;
    size_t next = 0, done = 0, dispatches = 0, ops_sum = 0, inflight_bytes = 0, peak_bytes = 0, rejected = 0;
    int inflight = 0, peak_inflight = 0;
    const auto t0 = std::chrono::steady_clock::now();
    double last_done = 0;
    int rc = RNS_OK;
    while (done < n) {
        bool progress = false;
        const double now = now_s(t0);
        while (next < n && reqs[next].arrival <= now) {
            if (srv->max_pending && n_pending >= srv->max_pending) {
                // admission queue full: the request is refused (load shedding)
                lat[next] = -1.0;
                rejected++;
                done++;
            } else {
                pending[(size_t)cls[next]].push_back(next);
                n_pending++;
            }
            next++;
        }
        // retire finished dispatches
        for (Slot &sl : srv->slots) {
            if (!sl.busy) continue;
            hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) {
                rc = hip_fail(q, "dispatch");
                break;
            }
            const double t = now_s(t0);
            for (size_t i = 0; i < sl.reqs.size(); i++) {
                const rsa_request &r = reqs[sl.reqs[i]];
                std::memcpy(r.out, sl.h_out + sl.out_word[i], srv->keys[(size_t)r.key]->n_limbs * 4);
                lat[sl.reqs[i]] = t - r.arrival;
            }
            done += sl.reqs.size();
            last_done = t;
            inflight_bytes -= sl.bytes;
            inflight--;
            sl.busy = false;
            progress = true;
        }
        if (rc) break;
        // admit pending requests of one class into a free slot, within the
        // budget: the class whose oldest pending request arrived first
        if (n_pending) {
            Slot *free_slot = nullptr;
            for (Slot &sl : srv->slots)
                if (!sl.busy) {
                    free_slot = &sl;
                    break;
                }
            if (free_slot) {
                size_t c_best = pending.size();
                for (size_t c = 0; c < pending.size(); c++)
                    if (!pending[c].empty() &&
                        (c_best == pending.size() || pending[c].front() < pending[c_best].front()))
                        c_best = c;
                std::deque<size_t> &q = pending[c_best];
                // per (key, kind) request counts decide the bytes of a dispatch
                std::map<std::pair<int, int>, size_t> counts;
                size_t bytes = 0, take = 0;
                while (take < q.size() && take < srv->max_ops) {
                    const rsa_request &r = reqs[q[take]];
                    auto k = std::make_pair(r.key, r.kind);
                    const size_t c = counts[k];
                    const rsa_key *key = srv->keys[(size_t)r.key];
                    const size_t delta = op_bytes(key, r.kind, c + 1) - (c ? op_bytes(key, r.kind, c) : 0);
                    if (inflight_bytes + bytes + delta > srv->budget) break;
                    counts[k] = c + 1;
                    bytes += delta;
                    take++;
                }
                if (take) {
                    std::vector<size_t> ids(q.begin(), q.begin() + (long)take);
                    if ((rc = dispatch(srv, *free_slot, reqs, ids))) break;
                    q.erase(q.begin(), q.begin() + (long)take);
                    n_pending -= take;
                    dispatches++;
                    ops_sum += take;
                    inflight++;
                    inflight_bytes += free_slot->bytes;
                    peak_inflight = std::max(peak_inflight, inflight);
                    peak_bytes = std::max(peak_bytes, inflight_bytes);
                    progress = true;
                }
            }
        }
        if (!progress) {
            // spin while work is in flight or an arrival is near; otherwise sleep
            const double wait = next < n ? reqs[next].arrival - now_s(t0) : 0;
            if (inflight == 0 && wait > 2e-4)
                std::this_thread::sleep_for(std::chrono::microseconds((long)(wait * 1e6) - 100));
            else
                std::this_thread::yield();
        }
    }
    if (rc) {
        for (Slot &sl : srv->slots) {
            hipStreamSynchronize(sl.stream);
            sl.busy = false;
        }
        return rc;
    }
    if (latency) std::copy(lat.begin(), lat.end(), latency);
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->completed = done - rejected;
        stats->rejected = rejected;
        stats->dispatches = dispatches;
        stats->elapsed = n ? last_done - reqs[0].arrival : 0;
        std::vector<double> s;
        for (double v : lat)
            if (v >= 0) s.push_back(v);
        std::sort(s.begin(), s.end());
        const size_t m = s.size();
        if (m) {
            stats->p50_latency = s[(m - 1) / 2];
            stats->p99_latency = s[std::min(m - 1, (size_t)((double)(m - 1) * 0.99 + 0.5))];
            stats->max_latency = s[m - 1];
        }
        stats->mean_dispatch_ops = dispatches ? (double)ops_sum / (double)dispatches : 0;
        stats->peak_inflight_bytes = peak_bytes;
        stats->peak_inflight = peak_inflight;
    }
    if (rejected)
        return fail(RNS_EBUSY, std::to_string(rejected) + " request(s) refused: admission queue full (max_pending)");
    return ok();
}

extern "C" {

// No exception crosses the C ABI: host allocation failures become RNS_ENOMEM
// (after the replay's dispatches in flight have finished).
int rsa_server_create(const rsa_key *const *keys, size_t n_keys, const rsa_server_opts *opts, rsa_server **out) {
    try {
        return server_create(keys, n_keys, opts, out);
    } catch (const std::bad_alloc &) {
        return fail(RNS_ENOMEM, "out of host memory");
    }
}

int rsa_server_replay(rsa_server *srv, const rsa_request *reqs, size_t n, double *latency, rsa_server_stats *stats) {
    try {
        return server_replay(srv, reqs, n, latency, stats);
    } catch (const std::bad_alloc &) {
        for (Slot &sl : srv->slots) {
            hipStreamSynchronize(sl.stream);
            sl.busy = false;
        }
        return fail(RNS_ENOMEM, "out of host memory");
    }
}

void rsa_server_free(rsa_server *srv) { delete srv; }

}  // extern "C"
