// Launch interface of the RNS modular-exponentiation kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "mfma_layout.hpp"

namespace rnsrsa {

// Parameters shared by the two exponentiation jobs of one launch.
struct ModexpParams {
    int in_limbs;    // input limbs per element
    int in_stride;   // limbs between consecutive inputs
    int L;           // output limbs (modulus limbs)
    int out_stride;  // limbs between consecutive outputs
    int exp_limbs;   // exponent limbs
    int exp_stride;  // 0: one exponent shared by the batch
    int window;      // window width w, 1..6
    int batch;       // elements per job
};

// One launch runs njobs (1 or 2) exponentiation jobs with the same base set:
// job j uses modulus table mc[j], entry table E[j], exponent exp[j] and writes
// out[j]; all jobs read the same inputs (a CRT decryption runs its p- and
// q-halves as the two jobs of one launch).
struct ModexpLaunch {
    const uint32_t *bc;
    const uint32_t *mc[2];
    const uint32_t *E[2];
    const uint32_t *exp[2];
    const uint32_t *in;
    uint32_t *out[2];
    uint32_t *table;  // scratch, modexp_table_words(...) words
    ModexpParams P;
    int njobs;
};

// Garner recombination m = m_q + q * ((m_p - m_q) qinv mod p) over the
// p-modulus tables: in = [m_p | m_q] (2*L limbs per element).
struct GarnerLaunch {
    const uint32_t *bc;
    const uint32_t *mc;    // p-modulus table
    const uint32_t *E;     // entry table mapping (m_p, m_q) to (m_p - m_q) qinv M
    const uint32_t *qlimbs;  // L limbs of q
    const uint32_t *in;
    uint32_t *out;
    int L;          // half limbs
    int out_limbs;  // limbs written per result (<= 2L)
    int out_stride;
    int batch;
};

// One Garner step of a grouped launch (several keys of one base shape):
// the fields of GarnerLaunch plus the job's first workgroup (64 elements
// each) in the launch.  Jobs are ordered by tile0.
struct GJob {
    GarnerLaunch g;
    int tile0;
};

struct MontMulLaunch {
    const uint32_t *bc;
    const uint32_t *mc;
    const uint32_t *x, *y;
    uint32_t *out;
    int batch;
};

// One exponentiation job of the matrix-core kernel: `batch` elements
// out[i] = in[i]^exp mod N with the tables of one modulus: mb the
// key-independent table and mk the per-modulus table (plan_mfma.hpp), E the
// entry table of in_limbs rows.  tile0 is the job's first tile in its
// launch; each tile serves tile_elems consecutive elements (0: all 16*NT
// columns of the workgroup; fewer spread a small job over more workgroups,
// the other columns computing values that are not stored).
struct MJob {
    const uint32_t *mb, *mk, *E, *exp, *in;
    uint32_t *out;
    int batch, in_limbs, in_stride, L, out_stride, exp_limbs, exp_stride, window;
    int tile0;
    int tile_elems;
};

// A launch of the matrix-core kernel: njobs jobs of one shape, from the
// device array `jobs` or, when it is null, from inl (at most 2 jobs).
struct ModexpMfmaLaunch {
    MJob inl[2];
    const MJob *jobs;
    int njobs;
    int tiles;           // total tiles of all jobs = workgroups launched
    int max_window;      // window table slots hold 2^max_window entries
    uint32_t *table;     // scratch: modexp_mfma_table_words(shape, max_window, tiles) words
    int scaled;          // every job's key keeps scaled B residues (MfmaTables::scaled)
};

// One RNS Montgomery product per element on the matrix cores (the
// standalone product): residues channel-major, [2K+1][batch], plain.
struct MontMulMfmaLaunch {
    const uint32_t *mb, *mk;
    const uint32_t *x, *y;
    uint32_t *out;
    int batch;
    int tiles;        // workgroups launched
    int tile_elems;   // elements per workgroup (0: 16*NT)
};

size_t modexp_table_words(int K, int W, int window, size_t workgroups);
size_t modexp_mfma_table_words(const MLayout &shape, int max_window, size_t workgroups);
int mfma_tiles(const MLayout &shape, size_t elements);
// Tiles of a job of `elements` elements at tile_elems per tile (0: 16*NT).
int mfma_job_tiles(const MLayout &shape, size_t elements, int tile_elems);
// Fewest elements a tile is given when a small launch is spread out.
constexpr int kMinTileElems = 4;
bool mfma_supported(int K);
int mfma_blocks_per_cu(const MLayout &shape);
hipError_t launch_modexp_mfma(const MLayout &shape, const ModexpMfmaLaunch &a, hipStream_t s);
hipError_t launch_montmul_mfma(const MLayout &shape, const MontMulMfmaLaunch &a, hipStream_t s);
hipError_t launch_modexp(int K, int W, const ModexpLaunch &a, hipStream_t s);
hipError_t launch_garner(int K, int W, const GarnerLaunch &a, hipStream_t s);
// Grouped Garner steps: `tiles` workgroups over njobs jobs (device table).
hipError_t launch_garner_jobs(int K, int W, const GJob *jobs, int njobs, int tiles, hipStream_t s);
hipError_t launch_montmul(int K, int W, const MontMulLaunch &a, hipStream_t s);

}  // namespace rnsrsa
