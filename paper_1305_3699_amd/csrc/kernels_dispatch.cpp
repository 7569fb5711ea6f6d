// Dispatch from a runtime (K, W) shape to the kernel instantiations, which
// are compiled one shape per translation unit (see the build script).
#include "kernels.hpp"
#include "mfma_layout.hpp"

namespace rnsrsa {

template <int K, int W>
hipError_t launch_modexp_t(const ModexpLaunch &a, hipStream_t s);
template <int K, int W>
hipError_t launch_garner_t(const GarnerLaunch &a, hipStream_t s);
template <int K, int W>
hipError_t launch_montmul_t(const MontMulLaunch &a, hipStream_t s);
template <int K, int W>
hipError_t launch_garner_jobs_t(const GJob *jobs, int njobs, int tiles, hipStream_t s);

#define RNSRSA_SHAPE(k, w)                                                          \
    extern template hipError_t launch_modexp_t<k, w>(const ModexpLaunch &, hipStream_t); \
    extern template hipError_t launch_garner_t<k, w>(const GarnerLaunch &, hipStream_t); \
    extern template hipError_t launch_montmul_t<k, w>(const MontMulLaunch &, hipStream_t); \
    extern template hipError_t launch_garner_jobs_t<k, w>(const GJob *, int, int, hipStream_t);
#include "kernel_configs.inc"
#undef RNSRSA_SHAPE

template <int K, int W, int MT, int NT>
hipError_t launch_modexp_mfma_t(const ModexpMfmaLaunch &a, hipStream_t s);
template <int K, int W, int MT, int NT>
int mfma_blocks_per_cu_t();
template <int K, int W, int MT, int NT>
hipError_t launch_montmul_mfma_t(const MontMulMfmaLaunch &a, hipStream_t s);
#define RNSRSA_MSHAPE(k, w, mt, nt) \
    extern template hipError_t launch_modexp_mfma_t<k, w, mt, nt>(const ModexpMfmaLaunch &, hipStream_t); \
    extern template hipError_t launch_montmul_mfma_t<k, w, mt, nt>(const MontMulMfmaLaunch &, hipStream_t); \
    extern template int mfma_blocks_per_cu_t<k, w, mt, nt>();
#include "kernel_configs_mfma.inc"
#undef RNSRSA_MSHAPE

bool mfma_supported(int K) {
#define RNSRSA_MSHAPE(k, w, mt, nt) \
    if (K == k) return true;
#include "kernel_configs_mfma.inc"
#undef RNSRSA_MSHAPE
    return false;
}

size_t modexp_mfma_table_words(const MLayout &s, int max_window, size_t workgroups) {
    return workgroups * ((size_t)1 << max_window) * (size_t)s.W * s.SLOTS() * 64;
}

int mfma_tiles(const MLayout &s, size_t elements) { return (int)((elements + s.NM() - 1) / s.NM()); }

int mfma_job_tiles(const MLayout &s, size_t elements, int tile_elems) {
    const size_t e = tile_elems > 0 && tile_elems < s.NM() ? (size_t)tile_elems : (size_t)s.NM();
    return (int)((elements + e - 1) / e);
}

int mfma_blocks_per_cu(const MLayout &sh) {
#define RNSRSA_MSHAPE(k, w, mt, nt) \
    if (sh.K == k && sh.W == w && sh.MT == mt && sh.NT == nt) return mfma_blocks_per_cu_t<k, w, mt, nt>();
#include "kernel_configs_mfma.inc"
#undef RNSRSA_MSHAPE
    return 0;
}

hipError_t launch_modexp_mfma(const MLayout &sh, const ModexpMfmaLaunch &a, hipStream_t s) {
#define RNSRSA_MSHAPE(k, w, mt, nt) \
    if (sh.K == k && sh.W == w && sh.MT == mt && sh.NT == nt) return launch_modexp_mfma_t<k, w, mt, nt>(a, s);
#include "kernel_configs_mfma.inc"
#undef RNSRSA_MSHAPE
    return hipErrorInvalidValue;
}

hipError_t launch_montmul_mfma(const MLayout &sh, const MontMulMfmaLaunch &a, hipStream_t s) {
#define RNSRSA_MSHAPE(k, w, mt, nt) \
    if (sh.K == k && sh.W == w && sh.MT == mt && sh.NT == nt) return launch_montmul_mfma_t<k, w, mt, nt>(a, s);
#include "kernel_configs_mfma.inc"
#undef RNSRSA_MSHAPE
    return hipErrorInvalidValue;
}

size_t modexp_table_words(int K, int W, int window, size_t workgroups) {
    const int KS = (K + W - 1) / W;
    return workgroups * ((size_t)1 << window) * (size_t)W * (2 * KS + 1) * 64;
}

hipError_t launch_modexp(int K, int W, const ModexpLaunch &a, hipStream_t s) {
#define RNSRSA_SHAPE(k, w) \
    if (K == k && W == w) return launch_modexp_t<k, w>(a, s);
#include "kernel_configs.inc"
#undef RNSRSA_SHAPE
    return hipErrorInvalidValue;
}

hipError_t launch_garner(int K, int W, const GarnerLaunch &a, hipStream_t s) {
#define RNSRSA_SHAPE(k, w) \
    if (K == k && W == w) return launch_garner_t<k, w>(a, s);
#include "kernel_configs.inc"
#undef RNSRSA_SHAPE
    return hipErrorInvalidValue;
}

hipError_t launch_garner_jobs(int K, int W, const GJob *jobs, int njobs, int tiles, hipStream_t s) {
#define RNSRSA_SHAPE(k, w) \
    if (K == k && W == w) return launch_garner_jobs_t<k, w>(jobs, njobs, tiles, s);
#include "kernel_configs.inc"
#undef RNSRSA_SHAPE
    return hipErrorInvalidValue;
}

hipError_t launch_montmul(int K, int W, const MontMulLaunch &a, hipStream_t s) {
#define RNSRSA_SHAPE(k, w) \
    if (K == k && W == w) return launch_montmul_t<k, w>(a, s);
#include "kernel_configs.inc"
#undef RNSRSA_SHAPE
    return hipErrorInvalidValue;
}

}  // namespace rnsrsa
