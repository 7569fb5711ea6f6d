// Device check that the inputs of RSA operations lie below n (range.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "capi_internal.hpp"

namespace rnsrsa {

// Elements [elem0, elem0 + count) of a launch: `count` inputs of `limbs`
// limbs (rows `stride` limbs apart) compared with the limbs of n; each input
// >= n adds one to *status.
struct RangeJob {
    const uint32_t *in;
    const uint32_t *n;
    unsigned long long *status;
    int limbs, stride, count, elem0;
};

// One launch over `total` elements: one job inline, or a device table of
// njobs jobs ordered by elem0.
struct RangeLaunch {
    RangeJob inl;
    const RangeJob *jobs;
    int njobs;
    int total;
};

hipError_t launch_range_check(const RangeLaunch &a, hipStream_t s);

namespace api {

// The check of `count` inputs of `key` (its device limbs of n and status word).
RangeJob range_job(const rsa_key *key, const uint32_t *in, size_t count);
// Enqueue the check of one operation's inputs on s.
int check_inputs(const rsa_key *key, const uint32_t *in, size_t count, hipStream_t s);
// Host check of one input row (n_limbs limbs): x < n.
bool host_below_n(const rsa_key *key, const uint32_t *x);

}  // namespace api
}  // namespace rnsrsa
