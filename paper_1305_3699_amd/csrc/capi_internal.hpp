// Internal interface shared by the C ABI translation units (capi.cpp,
// batch.cpp): error reporting, device uploads, stream-ordered scratch, and
// the objects behind the opaque handles of include/rnsrsa.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "plan.hpp"
#include "plan_mfma.hpp"
#include "rnsrsa.h"

namespace rnsrsa {
namespace api {

int fail(int code, const std::string &msg);   // records msg for rns_last_error, returns code
int ok();
int hip_fail(hipError_t e, const char *what);
int upload(const std::vector<uint32_t> &v, uint32_t **out);

// A stream-ordered device allocation released (stream-ordered) on destruction.
struct Scratch {
    void *p = nullptr;
    hipStream_t s = nullptr;
    ~Scratch() {
        if (p) hipFreeAsync(p, s);
    }
};
int scratch_alloc(Scratch &sc, size_t bytes, hipStream_t s);
// Keep freed stream-ordered blocks in the device pool (once per process).
void configure_pool_once();

// Montgomery products of an exponentiation by one exponent for each window
// width (mm[w], w = 1..6) and the width with the fewest, computed once when
// a key is loaded so that planning a launch does not rescan the exponent.
struct WindowCosts {
    size_t mm[7] = {};
    int best = 1;
};
WindowCosts window_costs(const std::vector<uint32_t> &e);

}  // namespace api
}  // namespace rnsrsa

// A modulus with its device tables.
struct rns_ctx {
    rnsrsa::ModPlan plan;
    int window = 5;
    int device = 0;
    int engine = RNS_ENGINE_CHANNEL;
    uint32_t *d_base = nullptr;  // shared, owned by the process-wide cache
    uint32_t *d_mod = nullptr;
    uint32_t *d_entry = nullptr;  // entry table for L-limb inputs (factor M^2 mod N)
    // matrix-core engine
    rnsrsa::MfmaShape mshape{};  // default tile
    int group_req = 0;            // tile asked for at set-up (0: chosen per launch)
    uint32_t *d_mbase = nullptr;  // shared, owned by the process-wide cache
    uint32_t *d_mkey = nullptr;
    uint32_t *d_mentry = nullptr;
    bool mscaled = false;         // the key table holds the scaled form (MfmaTables::scaled)
    ~rns_ctx() {
        for (uint32_t *x : {d_mod, d_entry, d_mkey, d_mentry})
            if (x) hipFree(x);
    }
};

struct rns_plan {
    rnsrsa::ModPlan plan;
    int window = 5;
    int engine = RNS_ENGINE_CHANNEL;
    rnsrsa::MfmaTables mt;
};

struct rsa_key {
    size_t n_limbs = 0, e_limbs = 0, half = 0;
    std::vector<uint32_t> h_n;                    // host copy of n
    std::vector<uint32_t> h_e, h_dp, h_dq, h_d;   // host copies of the exponents
    rnsrsa::api::WindowCosts wc_e, wc_dp, wc_dq, wc_d;   // their products per window width
    uint32_t *d_n = nullptr;                      // n on the device (input range check)
    unsigned long long *d_status = nullptr;       // inputs >= n seen since the last rsa_key_status
    rns_ctx *n = nullptr;
    uint32_t *d_e = nullptr, *d_d = nullptr;
    bool has_crt = false;
    rns_ctx *p = nullptr, *q = nullptr;
    uint32_t *d_dp = nullptr, *d_dq = nullptr;
    uint32_t *d_centry_p = nullptr, *d_centry_q = nullptr;  // entry tables for n_limbs-limb inputs
    uint32_t *d_mcentry_p = nullptr, *d_mcentry_q = nullptr;  // the same for the matrix-core engine
    uint32_t *d_gentry = nullptr;                           // Garner entry table (p-modulus)
    uint32_t *d_qlimbs = nullptr;
    ~rsa_key() {
        delete n;
        delete p;
        delete q;
        for (uint32_t *x : {d_n, d_e, d_d, d_dp, d_dq, d_centry_p, d_centry_q, d_mcentry_p, d_mcentry_q, d_gentry,
                            d_qlimbs})
            if (x) hipFree(x);
        if (d_status) hipFree(d_status);
    }
};


namespace rnsrsa {
namespace api {

// Entry table of a context for its own L-limb inputs.
const uint32_t *entry_of(const rns_ctx *c);
// The device copy of a base set's matrix-engine table: uploads `blob` on the
// first request per (base set, device, the shape's waves and tiles per wave);
// resident_mfma_base returns it if it is already there (else null).
int device_mfma_base(const std::shared_ptr<const BaseSet> &bs, const MLayout &sh, const std::vector<uint32_t> &blob,
                     uint32_t **out);
uint32_t *resident_mfma_base(const BaseSet *bs, const MLayout &sh);
// Garner recombination of [m_p | m_q] rows into m (n_limbs limbs).
int crt_combine(const rsa_key *key, const uint32_t *mpq, uint32_t *m, size_t batch, hipStream_t s);
// The Garner launch arguments of that recombination.
GarnerLaunch garner_launch_of(const rsa_key *key, const uint32_t *mpq, uint32_t *m, size_t batch);
// Tile of one matrix-core launch of `tiles` workgroups of shape sh on device
// dev: the 16-element tile of the same (K, W, MT) instead of the 32-element one
// when the latter would leave fewer than 1.5 resident waves per SIMD.  Below
// that the smaller tile's shorter per-wave work (and twice the workgroups)
// wins; above it the 32-element tile's shared constant loads do (measured for
// k = 17 .. 129).  Shapes without that alternative are returned unchanged.
MfmaShape auto_tile(const MfmaShape &sh, size_t tiles, int dev, bool small_jobs = false);
// SIMDs of device dev (4 per compute unit), cached; 0 if unknown.
int device_simds(int dev);
// Elements per tile for a matrix-core launch of `tiles` full tiles of shape
// sh on device dev: 0 (all 16*NT columns) unless the launch would leave
// SIMDs without a wave; then the largest of 16*NT/2, /4, ... down to
// kMinTileElems that gives every SIMD a wave.  A workgroup's time does not
// depend on how many of its columns are real, so on an underfilled GPU
// spreading the elements over more workgroups shortens the launch.
int spread_tile_elems(const MfmaShape &sh, size_t tiles, int dev);
// A context for odd modulus N of L limbs with the default options (smallest
// base, default engine and tile).  Owned by the caller (delete).
int make_context(const Limbs &N, int L, rns_ctx **out);
// One or two exponentiation jobs sharing their inputs (the plain launch).
// table_buf: device scratch of modexp_scratch_bytes(c0, njobs, batch, spread)
// bytes for the window tables, or null to allocate it stream-ordered.
// spread: a launch too small to give every SIMD a wave may use fewer
// elements per workgroup (more workgroups, more window-table scratch).
int run_modexp(const rns_ctx *c0, const rns_ctx *c1, const uint32_t *E0, const uint32_t *E1, const uint32_t *in,
               int in_limbs, const uint32_t *x0, const uint32_t *x1, int exp_limbs, int exp_stride, uint32_t *out0,
               uint32_t *out1, int out_stride, size_t batch, hipStream_t s, uint32_t *table_buf = nullptr,
               bool spread = true);
// Window-table bytes of a plain launch of njobs (1 or 2) jobs of `batch`
// elements on c0 (same base, window and tile for both jobs).
size_t modexp_scratch_bytes(const rns_ctx *c0, int njobs, size_t batch, bool spread = true);
// Both halves of a CRT decryption in one launch into mpq (table and spread as
// run_modexp).
int crt_halves(const rsa_key *key, const uint32_t *c, uint32_t *mpq, size_t batch, hipStream_t s,
               uint32_t *table = nullptr, bool spread = true);

}  // namespace api
}  // namespace rnsrsa
