// Input range check of the RSA operations (include/rnsrsa.h, rsa_key_status).
//
// Raw RSA works on integers below the modulus (Sec. 3.3).  The library still
// computes x^e mod n for a larger x (the exponentiation reduces its input),
// but counts such inputs in a per-key device word, which rsa_key_status reads
// and clears at the caller's synchronisation point.  The check is one thread
// per element comparing limbs from the top; for an input below n it usually
// stops at the first limb.
#include <hip/hip_runtime.h>

#include <cstring>

#include "range.hpp"

using namespace rnsrsa;
using namespace rnsrsa::api;

namespace rnsrsa {

namespace {

__global__ __launch_bounds__(256) void range_check_kernel(RangeLaunch a) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= a.total) return;
    RangeJob J = a.inl;
    if (a.jobs) {
        int lo = 0, hi = a.njobs - 1;   // last job with elem0 <= i
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.jobs[mid].elem0 <= i) lo = mid; else hi = mid - 1;
        }
        J = a.jobs[lo];
    }
    const uint32_t *x = J.in + (size_t)(i - J.elem0) * J.stride;
    bool ge = true;                      // x == n counts as out of range
    for (int l = J.limbs - 1; l >= 0; l--) {
        const uint32_t v = x[l], m = J.n[l];
        if (v != m) {
            ge = v > m;
            break;
        }
    }
    if (ge) atomicAdd(J.status, 1ull);
}

}  // namespace

hipError_t launch_range_check(const RangeLaunch &a, hipStream_t s) {
    if (a.total <= 0) return hipSuccess;
    hipLaunchKernelGGL(range_check_kernel, dim3((unsigned)((a.total + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

namespace api {

RangeJob range_job(const rsa_key *key, const uint32_t *in, size_t count) {
    RangeJob j{};
    j.in = in;
    j.n = key->d_n;
    j.status = key->d_status;
    j.limbs = (int)key->n_limbs;
    j.stride = (int)key->n_limbs;
    j.count = (int)count;
    j.elem0 = 0;
    return j;
}

int check_inputs(const rsa_key *key, const uint32_t *in, size_t count, hipStream_t s) {
    RangeLaunch a{};
    a.inl = range_job(key, in, count);
    a.total = (int)count;
    hipError_t e = launch_range_check(a, s);
    return e == hipSuccess ? RNS_OK : hip_fail(e, "range check launch");
}

bool host_below_n(const rsa_key *key, const uint32_t *x) {
    for (size_t l = key->n_limbs; l-- > 0;)
        if (x[l] != key->h_n[l]) return x[l] < key->h_n[l];
    return false;
}

}  // namespace api
}  // namespace rnsrsa

extern "C" {

int rsa_key_status(const rsa_key *key, size_t *n_out_of_range, void *hip_stream) {
    if (n_out_of_range) *n_out_of_range = 0;
    if (!key) return fail(RNS_EINVAL, "null key");
    hipStream_t s = (hipStream_t)hip_stream;
    unsigned long long count = 0;
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipMemcpyAsync(&count, key->d_status, sizeof(count), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && count) e = hipMemsetAsync(key->d_status, 0, sizeof(count), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "rsa_key_status");
    if (n_out_of_range) *n_out_of_range = (size_t)count;
    if (count)
        return fail(RNS_ERANGE, std::to_string(count) + " input(s) not below n since the last status read (reduced mod n)");
    return ok();
}

}  // extern "C"
