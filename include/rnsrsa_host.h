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

/*
 * Host model of one base extension of the matrix-core kernel (which = 1: the
 * first, q^ into B' and 2^32; which = 2: the second, into B), on raw digits
 * xi ([batch][k], any 32-bit words; the kernel's digits are residues below
 * their channel prime).  *rows receives the number of slot rows (waves * 4 *
 * tiles of the plan's shape); with partials and value both NULL nothing else
 * is done.  partials: [batch][rows][4] the exact byte partials P_b of every
 * slot row, in the kernel's slot order: the int32 sums the matrix cores
 * accumulate; value: [batch][rows] S = sum_b 2^(8b) P_b formed as the kernel
 * forms it.  Returns RNS_EVERIFY when a partial leaves int32 or the kernel's
 * way of combining them would wrap (every output is still written),
 * RNS_EUNSUPPORTED for a plan on the channel engine.
 */
int rns_emul_mfma_extension(const rns_plan *plan, int which, const uint32_t *xi, size_t batch, size_t *rows,
                            int64_t *partials, int64_t *value);

/*
 * The constant matrix of one extension of the matrix-core kernel (which as
 * above), read back from the plan's tables through the matrix cores' operand
 * layout: A[rows][4][kdim] signed bytes, byte b of slot row r at K index
 * kappa (4 per input channel digit, then the offset column, then zero
 * padding).  *rows and *kdim receive the sizes; with A NULL nothing else is
 * done.  RNS_EUNSUPPORTED for a plan on the channel engine.
 */
int rns_emul_mfma_matrix(const rns_plan *plan, int which, size_t *rows, size_t *kdim, int8_t *A);

#ifdef __cplusplus
}
#endif

#endif /* RNSRSA_HOST_H */
