// The decryption entry point that allocates nothing (include/rnsrsa.h,
// rsa_decrypt_noalloc): the same launches as rsa_decrypt, with the window
// tables and the CRT intermediates in a fixed device array of the library
// instead of stream-ordered allocations.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "capi_internal.hpp"
#include "range.hpp"

using namespace rnsrsa;
using namespace rnsrsa::api;

namespace {

// The fixed scratch array.  Each device the library runs on holds one copy at
// its own address until the process ends; host code reaches it only through
// the address hipGetSymbolAddress returns for that device (the name itself is
// a host-side stand-in, not a device address).
constexpr size_t kNoallocScratchBytes = RSA_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) uint32_t scratch[kNoallocScratchBytes / sizeof(uint32_t)];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint32_t *g_scratch_of[kMaxDevices];   // device -> address of its copy of scratch (null: not looked up yet)

// Address of the current device's copy of scratch, looked up once per device
// with that device current.
int scratch_address(int dev, uint32_t **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(RNS_EUNSUPPORTED, "device index beyond the no-allocation form's table");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_of[dev]) {
        uint32_t *p = nullptr;
        hipError_t e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(RNS_EDEVICE, "hipGetSymbolAddress(scratch) returned a null address");
        g_scratch_of[dev] = p;
    }
    *out = g_scratch_of[dev];
    return RNS_OK;
}

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

extern "C" {

int rsa_decrypt_noalloc(const rsa_key *key, const uint32_t *c, uint32_t *m, size_t batch, int use_crt,
                        void *hip_stream) {
    if (!key) return fail(RNS_EINVAL, "null key");
    if (batch == 0) return ok();
    if (!c || !m) return fail(RNS_EINVAL, "null buffer");
    if (batch > (size_t)INT32_MAX - 64) return fail(RNS_EINVAL, "batch too large");
    hipStream_t s = (hipStream_t)hip_stream;
    const rns_ctx *x = nullptr;
    size_t mpq_bytes = 0, table_bytes = 0;
    // a small batch is spread over extra workgroups (as rsa_decrypt does)
    // only while their window tables still fit the array
    bool spread = true;
    if (use_crt) {
        if (!key->has_crt) return fail(RNS_EINVAL, "key has no CRT parts");
        mpq_bytes = round_up(batch * 2 * key->half * sizeof(uint32_t), 256);
        table_bytes = modexp_scratch_bytes(key->p, 2, batch, spread);
        if (mpq_bytes + table_bytes > kNoallocScratchBytes) {
            spread = false;
            table_bytes = modexp_scratch_bytes(key->p, 2, batch, spread);
        }
    } else {
        if (!key->d_d) return fail(RNS_EINVAL, "key has no private exponent");
        if (!key->n) return fail(RNS_EUNSUPPORTED, "CRT-only key: no context for the full modulus");
        x = key->n;
        table_bytes = modexp_scratch_bytes(x, 1, batch, spread);
        if (table_bytes > kNoallocScratchBytes) {
            spread = false;
            table_bytes = modexp_scratch_bytes(x, 1, batch, spread);
        }
    }
    if (mpq_bytes + table_bytes > kNoallocScratchBytes)
        return fail(RNS_EINVAL, "batch of " + std::to_string(batch) + " needs " +
                                    std::to_string(mpq_bytes + table_bytes) +
                                    " bytes of scratch; the no-allocation form holds " +
                                    std::to_string(kNoallocScratchBytes) + " (use a smaller batch or window)");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    const rns_ctx *owner = use_crt ? key->p : x;
    if (dev != owner->device) return fail(RNS_EINVAL, "key belongs to another device");
    uint32_t *base = nullptr;
    int rc = scratch_address(dev, &base);
    if (rc) return rc;
    if ((rc = check_inputs(key, c, batch, s))) return rc;
    if (!use_crt) {
        rc = run_modexp(x, nullptr, entry_of(x), nullptr, c, x->plan.L, key->d_d, nullptr, (int)key->n_limbs, 0, m,
                        nullptr, x->plan.L, batch, s, base, spread);
        return rc ? rc : ok();
    }
    uint32_t *mpq = base;
    uint32_t *table = base + mpq_bytes / sizeof(uint32_t);
    if ((rc = crt_halves(key, c, mpq, batch, s, table, spread))) return rc;
    if ((rc = crt_combine(key, mpq, m, batch, s))) return rc;
    return ok();
}

}  // extern "C"
