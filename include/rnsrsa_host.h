/*
 * rnsrsa_host.h -- host-side planning and a host model of the kernels.
 *
 * These entry points let a machine without a GPU inspect the RNS bases and
 * constants librnsrsa would install on the device, and run a sequential host
 * model of exactly the kernels' arithmetic (same constant tables, same
 * channel reductions, same exponent schedule).  They exist for testing and
 * tooling.  The device entry points of rnsrsa.h never call them: a context
 * without a working GPU fails with RNS_EDEVICE instead.
 *
 * All pointers here are HOST pointers.  Status codes and conventions are
 * those of rnsrsa.h.
 */
#ifndef RNSRSA_HOST_H
#define RNSRSA_HOST_H

#include "rnsrsa.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rns_plan rns_plan;

/* Choose the bases for modulus N exactly as rns_setup would, without touching
 * a device.  Release with rns_plan_free. */
int rns_plan_create(const uint32_t *mod, size_t mod_limbs, const rns_opts *opts, rns_plan **out);
void rns_plan_free(rns_plan *plan);
int rns_plan_info(const rns_plan *plan, rns_info *info);
/* The 2k channel primes, B then B'. */
int rns_plan_primes(const rns_plan *plan, uint32_t *primes, size_t n);

/* Host model of rns_modexp_batch (same argument meaning, host memory). */
int rns_emul_modexp(const rns_plan *plan, const uint32_t *base, const uint32_t *exp, size_t exp_limbs,
                    size_t exp_stride, uint32_t *out, size_t batch);

/* Host model of rns_mont_mul_batch (same layout, host memory). */
int rns_emul_mont_mul(const rns_plan *plan, const uint32_t *x, const uint32_t *y, uint32_t *out, size_t batch);

#ifdef __cplusplus
}
#endif

#endif /* RNSRSA_HOST_H */
