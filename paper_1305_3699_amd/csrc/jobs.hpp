// Planning of grouped exponentiation launches, shared by the batched form
// (batch.cpp) and the request server (server.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "capi_internal.hpp"

namespace rnsrsa {
namespace api {

// Montgomery products of one exponentiation with a shared exponent as the
// matrix-core kernel schedules it: entry, x^2 and the odd powers up to
// x^(2^w - 1) (w > 1), then sliding windows of at most w bits after the
// first (their squarings plus one multiplication each), one squaring per
// zero bit between windows, exit.
size_t mm_count(const std::vector<uint32_t> &e, int w);
// Window width in 1..6 with the fewest products for e (fixed > 0: fixed).
int best_window(const std::vector<uint32_t> &e, int fixed);

// One RSA operation with its buffers (device): mpq is the CRT scratch of
// count x 2 half limbs for a CRT decryption, else unused.
struct PlannedOp {
    const rsa_key *key;
    int kind;  // RSA_OP_ENCRYPT / RSA_OP_DECRYPT
    const uint32_t *in;
    uint32_t *out;
    size_t count;
    uint32_t *mpq;
};

struct PlannedJob {
    MJob j;
    size_t cost;                          // Montgomery products per element
    int w0 = 1;                           // window with the fewest products for the exponent
    const WindowCosts *wc = nullptr;      // products per window width for the exponent (owned by the key)
};

// Jobs of one matrix-core kernel shape: one launch.
struct JobGroup {
    MLayout shape{};
    bool auto_tile = true;  // no context asked for a tile and none was tuned
    int device = 0;
    std::vector<PlannedJob> jobs;
    int tiles = 0;
    int max_window = 1;
    bool scaled = false;    // every job's key holds the scaled form (the kernel keeps B residues scaled)
    size_t table_words() const { return modexp_mfma_table_words(shape, max_window, (size_t)tiles); }
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

struct JobPlan {
    std::vector<JobGroup> groups;
    std::vector<PlainJob> plain;
    std::vector<GarnerJob> garners;
    size_t jobs = 0;
    size_t modmuls = 0;
};

// CRT scratch words an operation needs (0 unless a CRT decryption).
size_t op_mpq_words(const rsa_key *key, int kind, size_t count);
// Jobs of `ops`, grouped by kernel shape (tile: the per-process tuned one for
// the shape class if any, else the contexts' if they asked for one, else the
// one auto_tile picks for the group's size), each group's tiles ordered by
// decreasing cost.  Validates the operations (RNS_EINVAL).
int plan_jobs(const std::vector<PlannedOp> &ops, int fixed_window, JobPlan &out);
// Assign tile0 in cost order and max_window for a group with its final shape.
void finish_group(JobGroup &g);
// The group's tile by auto_tile (the 16-element tile also when it needs at
// most 1.25x the 32-element tile's workgroups: jobs of a few elements), then
// finish_group again if it changed; g must be finished.
void retile_group(JobGroup &g, int dev);

// Per-process tile choice per (K, W, MT) from the batch autotuner (0: none).
int tuned_nt(const MLayout &s);
void set_tuned_nt(const MLayout &s, int nt);
// Per-process window offset from the batch autotuner for the jobs of shape
// class (K, W, MT) with exponents of exp_limbs limbs: the window is
// clamp(w0 + offset, 1, 6); *known = false when none was tuned.
int tuned_dw(const MLayout &s, int exp_limbs, bool *known);
void set_tuned_dw(const MLayout &s, int exp_limbs, int dw);
// Window of job J with offset dw from its own best; updates J.j.window and J.cost.
void set_job_window(PlannedJob &J, int dw);

// Enqueue one group's launch with device job table d_jobs and window table.
hipError_t launch_group(const JobGroup &g, const MJob *d_jobs, uint32_t *table, hipStream_t s);
// Enqueue the channel-engine jobs and the Garner steps of a plan on s.
int launch_plain_and_garner(const JobPlan &p, hipStream_t s, bool plain, bool garner);

// Garner steps of one base shape (K, W): one grouped launch whose
// workgroups serve every key's step of that shape at once.
struct GarnerGroup {
    int K = 0, W = 0;
    std::vector<GJob> jobs;
    int tiles = 0;
};
// The plan's Garner steps grouped by base shape, with the buffer pointers
// they hold in p.garners (so rebase those first).
std::vector<GarnerGroup> garner_groups(const JobPlan &p);
// Enqueue one grouped Garner launch with device job table d_jobs.
hipError_t launch_garner_group(const GarnerGroup &g, const GJob *d_jobs, hipStream_t s);

}  // namespace api
}  // namespace rnsrsa
