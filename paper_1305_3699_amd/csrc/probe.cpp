// Throughput probes of the vector ALU's wide integer multiplies, the
// denominator of the per-channel arithmetic's roofline: each lane runs 8
// independent dependent chains of one instruction form; the grid fills
// every SIMD many times over.
#include <hip/hip_runtime.h>

#include "capi_internal.hpp"
#include "rnsrsa.h"

using namespace rnsrsa::api;

namespace {

constexpr int kProbeIter = 4096;
constexpr int kProbeChains = 8;
constexpr int kProbeThreads = 256;

template <int OP>
__global__ __launch_bounds__(kProbeThreads) void probe_kernel(uint32_t *__restrict__ out, uint32_t seed) {
    const uint32_t t = blockIdx.x * kProbeThreads + threadIdx.x;
    const uint32_t m = 0xFFFFFFC5u ^ (seed & 0xFFu);
    uint64_t w[kProbeChains];
#pragma unroll
    for (int c = 0; c < kProbeChains; c++) w[c] = (uint64_t)(t * 2654435761u + 97u * c + seed) << 7 | c;
    for (int i = 0; i < kProbeIter; i++) {
#pragma unroll
        for (int c = 0; c < kProbeChains; c++) {
            if (OP == RNS_PROBE_MAD_U64_U32) w[c] = (uint64_t)(uint32_t)w[c] * m + w[c];
            if (OP == RNS_PROBE_MAD_I64_I32)
                w[c] = (uint64_t)((int64_t)(int32_t)w[c] * (int32_t)m + (int64_t)w[c]);
        }
    }
    uint32_t s = 0;
#pragma unroll
    for (int c = 0; c < kProbeChains; c++) s += (uint32_t)w[c] ^ (uint32_t)(w[c] >> 32);
    out[t] = s;
}

}  // namespace

extern "C" int rns_probe_alu(int op, double *lane_ops_per_s, void *hip_stream) {
    if (!lane_ops_per_s) return fail(RNS_EINVAL, "null output");
    *lane_ops_per_s = 0;
    if (op != RNS_PROBE_MAD_U64_U32 && op != RNS_PROBE_MAD_I64_I32) return fail(RNS_EINVAL, "unknown probe");
    hipStream_t s = (hipStream_t)hip_stream;
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    const unsigned blocks = (unsigned)(cus > 0 ? cus : 1) * 32u;
    const size_t n = (size_t)blocks * kProbeThreads;
    Scratch buf;
    int rc = scratch_alloc(buf, n * sizeof(uint32_t), s);
    if (rc) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
        if (e0) hipEventDestroy(e0);
        return hip_fail(e, "hipEventCreate");
    }
    float ms = 0;
    for (int rep = 0; rep < 2 && e == hipSuccess; rep++) {   // the first launch warms up
        e = hipEventRecord(e0, s);
        if (e == hipSuccess) {
            if (op == RNS_PROBE_MAD_U64_U32)
                hipLaunchKernelGGL(probe_kernel<RNS_PROBE_MAD_U64_U32>, dim3(blocks), dim3(kProbeThreads), 0, s,
                                   (uint32_t *)buf.p, 7u + rep);
            else
                hipLaunchKernelGGL(probe_kernel<RNS_PROBE_MAD_I64_I32>, dim3(blocks), dim3(kProbeThreads), 0, s,
                                   (uint32_t *)buf.p, 7u + rep);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(e, "probe");
    if (ms <= 0) return fail(RNS_EDEVICE, "probe took no measurable time");
    *lane_ops_per_s = (double)n * kProbeIter * kProbeChains / (ms * 1e-3);
    return ok();
}
