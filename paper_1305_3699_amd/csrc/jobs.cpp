// Planning of grouped exponentiation launches (jobs.hpp).
#include "jobs.hpp"

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

namespace rnsrsa {
namespace api {

size_t mm_count(const std::vector<uint32_t> &e, int w) {
    auto bit = [&](int i) { return (e[(size_t)i >> 5] >> (i & 31)) & 1u; };
    size_t n = 2;                                       // entry and exit products
    if (w > 1) n += (size_t)1 << (w - 1);               // x^2 and the odd powers x^3 .. x^(2^w - 1)
    int i = 32 * (int)e.size() - 1;
    while (i >= 0 && !bit(i)) i--;
    bool first = true;
    while (i >= 0) {
        if (!bit(i)) {
            n++;                                        // a squaring
            i--;
            continue;
        }
        int lo = std::max(i - w + 1, 0);
        while (!bit(lo)) lo++;
        if (!first) n += (size_t)(i - lo + 1) + 1;      // its squarings and one multiplication
        first = false;
        i = lo - 1;
    }
    return n;
}

WindowCosts window_costs(const std::vector<uint32_t> &e) {
    WindowCosts c;
    for (int w = 1; w <= 6; w++) {
        c.mm[w] = mm_count(e, w);
        if (c.mm[w] < c.mm[c.best]) c.best = w;
    }
    return c;
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

namespace {
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, int> g_tuned_nt;
std::map<std::tuple<int, int, int, int>, int> g_tuned_dw;
}  // namespace

int tuned_dw(const MLayout &s, int exp_limbs, bool *known) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned_dw.find(std::make_tuple(s.K, s.W, s.MT, exp_limbs));
    *known = it != g_tuned_dw.end();
    return *known ? it->second : 0;
}

void set_tuned_dw(const MLayout &s, int exp_limbs, int dw) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned_dw[std::make_tuple(s.K, s.W, s.MT, exp_limbs)] = dw;
}

void set_job_window(PlannedJob &J, int dw) {
    J.j.window = std::min(6, std::max(1, J.w0 + dw));
    J.cost = J.wc->mm[J.j.window];
}

int tuned_nt(const MLayout &s) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned_nt.find(std::make_tuple(s.K, s.W, s.MT));
    return it == g_tuned_nt.end() ? 0 : it->second;
}

void set_tuned_nt(const MLayout &s, int nt) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned_nt[std::make_tuple(s.K, s.W, s.MT)] = nt;
}

size_t op_mpq_words(const rsa_key *key, int kind, size_t count) {
    return (kind == RSA_OP_DECRYPT && key->has_crt) ? count * 2 * key->half : 0;
}

int plan_jobs(const std::vector<PlannedOp> &ops, int fixed_w, JobPlan &P) {
    std::map<std::tuple<int, int, int>, size_t> group_of;
    auto add_job = [&](const rns_ctx *c, const uint32_t *E, const uint32_t *x, const std::vector<uint32_t> &hx,
                       const WindowCosts &wc, const uint32_t *in, int in_limbs, uint32_t *o, int out_stride,
                       size_t count) {
        PlannedJob J{};
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
        J.w0 = fixed_w ? fixed_w : wc.best;
        J.wc = &wc;
        bool known = false;
        const int dw = fixed_w ? 0 : tuned_dw(c->mshape, (int)hx.size(), &known);
        set_job_window(J, dw);
        P.modmuls += J.cost * count;
        P.jobs++;
        const MLayout &sh = c->mshape;
        auto key = std::make_tuple(sh.K, sh.W, sh.MT);
        auto it = group_of.find(key);
        if (it == group_of.end()) {
            it = group_of.emplace(key, P.groups.size()).first;
            P.groups.emplace_back();
            JobGroup &g = P.groups.back();
            g.shape = sh;
            g.device = c->device;
            g.scaled = true;
            if (const int nt = tuned_nt(sh)) {
                MfmaShape t;
                if (mfma_shape_for(sh.K, t, 16 * nt) && t.W == sh.W && t.MT == sh.MT && t.NT == nt) g.shape = t;
                g.auto_tile = false;
            }
        }
        JobGroup &g = P.groups[it->second];
        g.scaled = g.scaled && c->mscaled;
        if (c->group_req) {
            g.auto_tile = false;
            if (!tuned_nt(sh)) g.shape = sh;
        }
        g.jobs.push_back(J);
    };
    for (const PlannedOp &o : ops) {
        if (!o.key || (o.kind != RSA_OP_ENCRYPT && o.kind != RSA_OP_DECRYPT)) return fail(RNS_EINVAL, "bad operation");
        if (o.count && (!o.in || !o.out)) return fail(RNS_EINVAL, "null buffer");
        if (o.count > (size_t)INT32_MAX - 64) return fail(RNS_EINVAL, "count too large");
        const rsa_key *k = o.key;
        if (o.kind == RSA_OP_DECRYPT && !k->has_crt && !k->d_d) return fail(RNS_EINVAL, "key has no private exponent");
        if (!o.count) continue;
        const int nl = (int)k->n_limbs;
        if (o.kind == RSA_OP_DECRYPT && k->has_crt) {
            const int h = (int)k->half;
            if (!o.mpq) return fail(RNS_EINVAL, "no CRT scratch");
            if (k->p->engine == RNS_ENGINE_MATRIX) {
                add_job(k->p, k->d_mcentry_p, k->d_dp, k->h_dp, k->wc_dp, o.in, nl, o.mpq, 2 * h, o.count);
                add_job(k->q, k->d_mcentry_q, k->d_dq, k->h_dq, k->wc_dq, o.in, nl, o.mpq + h, 2 * h, o.count);
            } else {
                P.plain.push_back(PlainJob{k->p, k->q, k->d_centry_p, k->d_centry_q, o.in, k->d_dp, k->d_dq, nl, h,
                                           o.mpq, o.mpq + h, 2 * h, o.count});
                P.jobs += 2;
            }
            P.garners.push_back(GarnerJob{k, o.mpq, o.out, o.count});
        } else {
            const bool enc = o.kind == RSA_OP_ENCRYPT;
            if (!k->n) return fail(RNS_EUNSUPPORTED, "CRT-only key: no context for the full modulus");
            const rns_ctx *c = k->n;
            const uint32_t *x = enc ? k->d_e : k->d_d;
            const std::vector<uint32_t> &hx = enc ? k->h_e : k->h_d;
            const WindowCosts &wc = enc ? k->wc_e : k->wc_d;
            if (c->engine == RNS_ENGINE_MATRIX) {
                add_job(c, c->d_mentry, x, hx, wc, o.in, nl, o.out, nl, o.count);
            } else {
                P.plain.push_back(PlainJob{c, nullptr, entry_of(c), nullptr, o.in, x, nullptr, nl, (int)hx.size(),
                                           o.out, nullptr, nl, o.count});
                P.jobs++;
            }
        }
    }
    for (JobGroup &g : P.groups) {
        finish_group(g);
        if (g.auto_tile) retile_group(g, g.device);
    }
    return RNS_OK;
}

void retile_group(JobGroup &g, int dev) {
    size_t t32 = 0, t16 = 0;
    for (const PlannedJob &J : g.jobs) {
        t32 += ((size_t)J.j.batch + 31) / 32;
        t16 += ((size_t)J.j.batch + 15) / 16;
    }
    const MfmaShape t = auto_tile(g.shape, (size_t)g.tiles, dev, 4 * t16 <= 5 * t32);
    if (t.NT != g.shape.NT) {
        g.shape = t;
        finish_group(g);
    }
}

void finish_group(JobGroup &g) {
    std::stable_sort(g.jobs.begin(), g.jobs.end(),
                     [](const PlannedJob &x, const PlannedJob &y) { return x.cost > y.cost; });
    size_t full = 0;
    for (const PlannedJob &J : g.jobs) full += (size_t)mfma_tiles(g.shape, (size_t)J.j.batch);
    const int te = spread_tile_elems(g.shape, full, g.device);
    g.tiles = 0;
    g.max_window = 1;
    for (PlannedJob &J : g.jobs) {
        J.j.tile0 = g.tiles;
        J.j.tile_elems = te;
        g.tiles += mfma_job_tiles(g.shape, (size_t)J.j.batch, te);
        g.max_window = std::max(g.max_window, J.j.window);
    }
}

hipError_t launch_group(const JobGroup &g, const MJob *d_jobs, uint32_t *table, hipStream_t s) {
    ModexpMfmaLaunch a{};
    a.jobs = d_jobs;
    a.njobs = (int)g.jobs.size();
    a.tiles = g.tiles;
    a.max_window = g.max_window;
    a.table = table;
    a.scaled = g.scaled ? 1 : 0;
    return launch_modexp_mfma(g.shape, a, s);
}

std::vector<GarnerGroup> garner_groups(const JobPlan &p) {
    std::map<std::pair<int, int>, GarnerGroup> m;
    for (const GarnerJob &gj : p.garners) {
        if (gj.count == 0) continue;
        const BaseSet &bs = *gj.key->p->plan.base;
        GarnerGroup &g = m[std::make_pair(bs.K, bs.W)];
        g.K = bs.K;
        g.W = bs.W;
        GJob J{};
        J.g = garner_launch_of(gj.key, gj.mpq, gj.out, gj.count);
        J.tile0 = g.tiles;
        g.tiles += (int)((gj.count + 63) / 64);
        g.jobs.push_back(J);
    }
    std::vector<GarnerGroup> out;
    for (auto &kv : m) out.push_back(std::move(kv.second));
    return out;
}

hipError_t launch_garner_group(const GarnerGroup &g, const GJob *d_jobs, hipStream_t s) {
    return launch_garner_jobs(g.K, g.W, d_jobs, (int)g.jobs.size(), g.tiles, s);
}

int launch_plain_and_garner(const JobPlan &p, hipStream_t s, bool plain, bool garner) {
    if (plain)
        for (const PlainJob &j : p.plain) {
            int rc = run_modexp(j.c0, j.c1, j.E0, j.E1, j.in, j.in_limbs, j.x0, j.x1, j.exp_limbs, 0, j.out0, j.out1,
                                j.out_stride, j.count, s);
            if (rc) return rc;
        }
    if (garner)
        for (const GarnerJob &gj : p.garners) {
            int rc = crt_combine(gj.key, gj.mpq, gj.out, gj.count, s);
            if (rc) return rc;
        }
    return RNS_OK;
}

}  // namespace api
}  // namespace rnsrsa
