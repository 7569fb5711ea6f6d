// Check of CRT decryption results: m^e mod n must give the ciphertext back.
// A fault in either half of a CRT decryption yields an m whose re-encryption
// differs from c (and whose gcd with n reveals a factor), so failing results
// are zeroed before the caller can release them.
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "capi_internal.hpp"
#include "rnsrsa.h"

using namespace rnsrsa;
using namespace rnsrsa::api;

namespace {

// One wave per element: bad[i] = (t_i != c_i); a failing m_i is zeroed.
__global__ __launch_bounds__(64) void crt_check_kernel(const uint32_t *__restrict__ c, const uint32_t *__restrict__ t,
                                                       uint32_t *__restrict__ m, uint32_t *__restrict__ bad, int L) {
    const size_t row = (size_t)blockIdx.x * L;
    bool diff = false;
    for (int l = threadIdx.x; l < L; l += 64) diff |= c[row + l] != t[row + l];
    const bool any = __ballot(diff) != 0;
    if (any)
        for (int l = threadIdx.x; l < L; l += 64) m[row + l] = 0u;
    if (threadIdx.x == 0) bad[blockIdx.x] = any ? 1u : 0u;
}

}  // namespace

extern "C" int rsa_crt_verify(const rsa_key *key, const uint32_t *c, uint32_t *m, size_t batch, size_t *n_bad,
                              void *hip_stream) {
    if (n_bad) *n_bad = 0;
    if (!key) return fail(RNS_EINVAL, "null key");
    if (batch == 0) return ok();
    if (!c || !m) return fail(RNS_EINVAL, "null buffer");
    if (c == m) return fail(RNS_EINVAL, "c and m must not alias (c must still hold the ciphertexts)");
    if (batch > (size_t)INT32_MAX - 64) return fail(RNS_EINVAL, "batch too large");
    if (!key->n) return fail(RNS_EUNSUPPORTED, "CRT-only key: no context for the full modulus");
    const rns_ctx *x = key->n;
    const int L = x->plan.L;
    hipStream_t s = (hipStream_t)hip_stream;
    try {
        Scratch t, bad;
        int rc = scratch_alloc(t, batch * (size_t)L * sizeof(uint32_t), s);
        if (!rc) rc = scratch_alloc(bad, batch * sizeof(uint32_t), s);
        if (rc) return rc;
        if ((rc = run_modexp(x, nullptr, entry_of(x), nullptr, m, L, key->d_e, nullptr, (int)key->e_limbs, 0,
                             (uint32_t *)t.p, nullptr, L, batch, s)))
            return rc;
        hipLaunchKernelGGL(crt_check_kernel, dim3((unsigned)batch), dim3(64), 0, s, c, (const uint32_t *)t.p, m,
                           (uint32_t *)bad.p, L);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "check launch");
        std::vector<uint32_t> hb(batch);
        if ((e = hipMemcpyAsync(hb.data(), bad.p, batch * sizeof(uint32_t), hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return hip_fail(e, "check read-back");
        size_t cnt = 0;
        for (uint32_t v : hb) cnt += v;
        if (n_bad) *n_bad = cnt;
        if (cnt)
            return fail(RNS_EVERIFY, std::to_string(cnt) + " result(s) failed m^e = c; their outputs were zeroed");
    } catch (const std::bad_alloc &) {
        return fail(RNS_ENOMEM, "out of host memory");
    }
    return ok();
}
