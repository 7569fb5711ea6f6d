/*
 * rnsrsa.h -- C ABI of librnsrsa: RSA modular exponentiation over bignums held
 * in the Residue Number System, on AMD MI355X (gfx950).
 *
 * The library implements the modular-arithmetic and RSA layers of Chauvet &
 * Mahe, "Secrets from the GPU" (arXiv:1305.3699):
 *   - RNS representation and binary <-> RNS conversion (Sec. 3.1),
 *   - the RNS Montgomery product with R = M = prod(m_i) and its two base
 *     extensions, constants precomputed and kept on the device (Sec. 3.1),
 *   - exponentiation by square-and-multiply chaining Montgomery products in
 *     the Montgomery domain (Sec. 3.1), here with a fixed window,
 *   - RSA encryption c = m^e mod n and decryption m = c^d mod n with d the
 *     inverse of e modulo (p-1)(q-1) (Sec. 3.3), and CRT-split decryption
 *     with p- and q-halves run side by side (the related-work split of
 *     Sec. 4.1) recombined by Garner's formula.
 * Every result is exact and canonical: outputs lie in [0, N).
 *
 * Conventions
 *   Bignums are little-endian arrays of uint32 limbs.  A batch of B numbers of
 *   L limbs is B*L contiguous limbs, number i at limbs [i*L, (i+1)*L).
 *   Set-up inputs (moduli, keys, options) are HOST pointers, copied during the
 *   call.  Batch inputs and outputs are DEVICE pointers owned by the caller.
 *   Batch calls validate on the host, enqueue on hip_stream (NULL = the null
 *   stream) and return; results are valid once the stream reaches the point of
 *   the call.  Contexts and keys are immutable after creation and may be used
 *   from several streams at once; the caller synchronises those streams before
 *   freeing them.
 *   Every function returns RNS_OK (0) or a negative status.  On any status
 *   other than RNS_EDEVICE nothing was enqueued.  rns_last_error() describes
 *   the last failure of the calling thread.  No exception or abort crosses
 *   this boundary.
 *   Exponentiation follows Python's pow: e = 0 gives 1 mod N (0^0 = 1), bases
 *   of any value representable in L limbs are accepted and reduced mod N.
 */
#ifndef RNSRSA_H
#define RNSRSA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum rns_status {
    RNS_OK = 0,
    RNS_EINVAL = -1,        /* bad argument (null pointer, bad size, bad option) */
    RNS_ERANGE = -2,        /* modulus < 2, or too large for any supported base; an RSA input not
                               below n (rsa_key_status, rsa_server_replay) */
    RNS_EFACTOR = -3,       /* a channel prime of an explicit base divides N */
    RNS_ENOMEM = -4,        /* host or device allocation failed */
    RNS_EDEVICE = -5,       /* HIP runtime error */
    RNS_EVERIFY = -6,       /* a result failed its self-check (key generation's d e = 1 mod f;
                               the host model's one-step reduction range check) */
    RNS_EBUSY = -7,         /* the request server's admission limits refuse a request (device-memory
                               budget below one request, or the pending queue full) */
    RNS_EUNSUPPORTED = -8   /* no kernel is built for the requested shape */
};

/* Exponentiation engines (the same results; different hardware paths). */
enum rns_engine {
    RNS_ENGINE_AUTO = 0,     /* matrix cores when a kernel exists for k, else channel */
    RNS_ENGINE_CHANNEL = 1,  /* base extensions as 32x32->64 multiply-adds on the vector ALUs */
    RNS_ENGINE_MATRIX = 2    /* base extensions as int8 matrix products (MFMA), exact int32 sums */
};

/* Prime ranges for the channel moduli. */
enum rns_prime_range {
    RNS_PRIMES_HIGH = 0,    /* primes = 3 mod 4 in [2^32 - 2^24, 2^32) */
    RNS_PRIMES_FULL = 1     /* primes = 3 mod 4 in (2^31, 2^32) */
};

/*
 * Options for context / key creation.  Pass NULL for defaults; a zeroed struct
 * means defaults too.
 *   k           channels per RNS base (0 = the smallest built base size that
 *               meets the bounds below).  Built sizes: 2, 3, 5, 9, 17, 33, 49,
 *               65, 66, 97, 129, 257 (moduli up to 8192 bits) and 513 (up to
 *               16384 bits; matrix-core engine only).
 *   window      exponent window width w in 1..6 (0 = 5).  The exponent loop
 *               precomputes 2^w table entries and does w squarings plus one
 *               multiplication per w-bit digit.
 *   waves       wavefronts per workgroup, which split the channels of 64
 *               messages (0 = default for k; needs an explicit k).
 *   prime_range rns_prime_range; prime_seed seeds the deterministic draw.
 *   primes      optional explicit bases: n_primes = 2k distinct primes in
 *               (2^31, 2^32), B first then B'.  Overrides k and prime_range.
 *               The matrix-core engine reduces each base-extension output
 *               in one step, which needs every B' prime <= 2^32 - 2^18 and
 *               every prime m with m 2^s > 4k*0x80808080*128 + 0x80808080
 *               (s = 17 up to k = 257, 18 beyond; B' also below the REDC
 *               limit, checked exactly per prime); a base that fails takes
 *               the channel engine (or RNS_EUNSUPPORTED if the matrix engine
 *               was requested or k = 513, which has no channel kernel).
 *               Full-range draws at k = 257 usually fail it.
 *   engine      rns_engine (0 = auto).  The Garner step of CRT decryption
 *               always uses the channel kernels; k = 513 runs on the matrix
 *               engine only (the channel engine returns RNS_EUNSUPPORTED
 *               there).
 *   group       matrix-core engine: preferred elements per workgroup, 16 or
 *               32, used by every launch (a k without a kernel of that size
 *               uses its default).  0: the default for k, except that a
 *               launch too small to give the GPU 1.5 resident waves per SIMD
 *               with 32-element workgroups takes 16-element ones.
 *               rns_info.group reports the requested or default size.
 *   unscaled    matrix-core engine, k <= 66: 1 keeps the B residues in the
 *               plain Montgomery form x 2^32 mod m_i.  0 (default): they
 *               are kept as x 2^32 s_i mod m_i with s_i^2 = +-c_i 2^-32
 *               (c_i = -N^-1 M_i^-1 mod m_i), which makes each product's
 *               quotient digit one modular reduction of the two operands
 *               instead of two; a key gets that form when such an s_i
 *               exists for every B prime (always for the drawn bases, whose
 *               primes are 3 mod 4), and rns_info.scaled reports it.  The
 *               results are the same either way.
 * Both bases hold k primes; with the redundant channel 2^32 an operand has
 * 2k+1 residues.  A base pair is accepted for modulus N of L limbs when
 *   M >= (k+1)^2 N,  M >= 2^(32L+1),  M' >= (k+1) N,  gcd(N, M) = 1,
 * which keeps every Montgomery product below (k+1) N and makes the second
 * base extension exact (the redundant residue fixes its multiple of M').
 */
typedef struct rns_opts {
    int k;
    int window;
    int waves;
    int prime_range;
    uint64_t prime_seed;
    const uint32_t *primes;
    size_t n_primes;
    int engine;
    int group;
    int unscaled;
} rns_opts;

typedef struct rns_info {
    int k;              /* channels per base */
    int waves;          /* wavefronts per workgroup */
    int window;         /* exponent window width */
    int mod_limbs;      /* L */
    int mod_bits;       /* bit length of N */
    int engine;         /* RNS_ENGINE_CHANNEL or RNS_ENGINE_MATRIX */
    int group;          /* elements served by one workgroup */
    int scaled;         /* 1: the matrix engine keeps this key's B residues scaled */
} rns_info;

typedef struct rns_ctx rns_ctx;
typedef struct rsa_key rsa_key;

/* Status text of the calling thread's last failure ("" if none).  The pointer
 * is valid until the next library call on this thread. */
const char *rns_last_error(void);

/* ABI version of this header (currently 6). */
int rns_abi_version(void);

/*
 * rns_setup -- precompute and upload the constants for modulus N (Sec. 3.1:
 * constants of base extension and of the Montgomery product are computed at
 * initialisation and installed in GPU memory).
 *   mod        host, mod_limbs limbs, N >= 2 (top limbs may be zero; L =
 *              mod_limbs is the operand width of every batch call)
 *   opts       host or NULL
 *   out        receives the context; release it with rns_free.
 * Errors: RNS_EINVAL, RNS_ERANGE, RNS_EFACTOR, RNS_EUNSUPPORTED, RNS_ENOMEM,
 * RNS_EDEVICE.  Uses the current HIP device.
 */
int rns_setup(const uint32_t *mod, size_t mod_limbs, const rns_opts *opts, rns_ctx **out);
void rns_free(rns_ctx *ctx);
int rns_get_info(const rns_ctx *ctx, rns_info *info);
/* Copies the 2k channel primes (B then B') to host memory primes[0..2k). */
int rns_get_primes(const rns_ctx *ctx, uint32_t *primes, size_t n);

/*
 * rns_modexp_batch -- out[i] = base[i]^e_i mod N for i < batch (Sec. 3.1:
 * square-and-multiply chaining RNS Montgomery products, entered and left
 * once per exponentiation).
 *   base       device, batch x L limbs (any value below 2^(32L))
 *   exp        device, exponent limbs (exp_limbs >= 1 each)
 *   exp_stride 0: one exponent exp[0..exp_limbs) shared by the batch;
 *              otherwise element i's exponent starts at exp + i*exp_stride
 *              (exp_stride >= exp_limbs)
 *   out        device, batch x L limbs, canonical; may alias base
 *   batch      0 is allowed (nothing is enqueued)
 * Scratch: 2^w * (2k+1) * 4 bytes per element, allocated stream-ordered.
 */
int rns_modexp_batch(rns_ctx *ctx, const uint32_t *base, const uint32_t *exp, size_t exp_limbs,
                     size_t exp_stride, uint32_t *out, size_t batch, void *hip_stream);

/*
 * rns_modexp_jobs -- several exponentiation batches, each on its own context
 * (modulus), in as few launches as possible: the paper runs a batch of
 * independent exponentiations side by side (Sec. 3.3), and Miller-Rabin
 * takes one modulus per candidate (Sec. 3.2).  Jobs on matrix-core contexts
 * of one kernel shape (and requested tile) share one grouped launch whatever
 * their moduli; jobs on channel-engine contexts take one launch each.
 *   jobs[i].ctx        context of job i (modulus, window, engine, tile)
 *   jobs[i].base, exp, exp_limbs, exp_stride, out, count
 *                      as the arguments of rns_modexp_batch on that context
 *                      (device buffers; L = the context's mod_limbs); a job
 *                      of count 0 is skipped
 * A job's out may alias its own base; it must not overlap another job's
 * base or out (the jobs of a launch run concurrently).  Every context must
 * belong to the current device.  Every job is validated before anything is
 * enqueued (RNS_EINVAL names the job); RNS_ENOMEM or RNS_EDEVICE after that
 * may leave earlier launches enqueued.  Asynchronous on hip_stream; the
 * library's host copy of a launch's job table is released by the stream
 * once copied.  Scratch as rns_modexp_batch, per launch.
 */
typedef struct rns_job {
    const rns_ctx *ctx;
    const uint32_t *base;
    const uint32_t *exp;
    size_t exp_limbs;
    size_t exp_stride;
    uint32_t *out;
    size_t count;
} rns_job;

int rns_modexp_jobs(const rns_job *jobs, size_t njobs, void *hip_stream);

/*
 * rns_mont_mul_batch -- one RNS Montgomery product per element in the residue
 * domain (Sec. 3.1, the operation the paper times in its Fig. 1):
 *   r = (X*Y + q^*N) / M,   q^ = sum_i |x_i y_i (-N^-1) M_i^-1|_{m_i} M_i,
 * so r == X*Y*M^-1 (mod N) and r < (k+1)N when X, Y < (k+1)N.
 *   x, y, out  device, (2k+1) x batch residues, channel-major ("structure of
 *              arrays"): channel c of element i at [c*batch + i]; channels
 *              0..k-1 are B, k..2k-1 are B', 2k is the redundant 2^32 channel.
 *              Each input must be the residue vector of one integer below
 *              (k+1)N; out may alias x or y.
 * Runs on the context's engine: the matrix cores by default (each element
 * converted into the kernel's kept representation and back around one
 * product), the channel kernels when the context asked for them (no channel
 * kernel for k = 513: RNS_EUNSUPPORTED).  Both give the same residues.
 */
int rns_mont_mul_batch(rns_ctx *ctx, const uint32_t *x, const uint32_t *y, uint32_t *out,
                       size_t batch, void *hip_stream);

/*
 * rsa_key_load -- load an RSA key and build its contexts (Sec. 3.3).
 *   n          host, n_limbs limbs; e host, e_limbs limbs
 *   d          host, n_limbs limbs, or NULL (public-only key)
 *   p, q, dp, dq, qinv   host, half_limbs limbs each, or all NULL (no CRT);
 *              qinv = q^-1 mod p, dp = d mod (p-1), dq = d mod (q-1), n = p*q
 *   opts       host or NULL; applied to every context of the key, except that
 *              an explicit k too small for n (one sized for the CRT halves)
 *              leaves the full-modulus context sized automatically
 * A key with CRT parts whose full modulus no base covers, or that no kernel
 * of the requested engine runs (the channel engine on a 16384-bit modulus,
 * k = 513), loads as a CRT-only key: CRT decryption works; encryption,
 * decryption with use_crt = 0 and rsa_key_info(key, 0) return
 * RNS_EUNSUPPORTED, as do batched operations and served requests that need
 * the full modulus.  With default options keys up to 16384 bits get a
 * full-modulus context (k = 513 above 8192 bits) and CRT halves on bases of
 * up to 257 channels.
 * The private parts stay in library-owned memory (the paper keeps private keys
 * on the GPU, Sec. 4.3).  Release with rsa_key_free.
 */
int rsa_key_load(const uint32_t *n, size_t n_limbs, const uint32_t *e, size_t e_limbs,
                 const uint32_t *d, const uint32_t *p, const uint32_t *q, const uint32_t *dp,
                 const uint32_t *dq, const uint32_t *qinv, size_t half_limbs, const rns_opts *opts,
                 rsa_key **out);
void rsa_key_free(rsa_key *key);
int rsa_key_info(const rsa_key *key, int which /* 0 n, 1 p, 2 q */, rns_info *info);

/*
 * rsa_encrypt -- c[i] = m[i]^e mod n (Sec. 3.3).  m, c: device, batch x n_limbs.
 * Raw RSA works on integers below n: an input >= n is still reduced mod n and
 * exponentiated, and it is counted on the device in the key's status word
 * (rsa_key_status reports RNS_ERANGE).  The same holds for the inputs of
 * rsa_decrypt, rsa_crt_halves and the batched form.
 */
int rsa_encrypt(const rsa_key *key, const uint32_t *m, uint32_t *c, size_t batch, void *hip_stream);

/*
 * rsa_decrypt -- m[i] = c[i]^d mod n.  use_crt = 0: one full-size
 * exponentiation with d (Sec. 3.3).  use_crt = 1: m_p = c^dp mod p and
 * m_q = c^dq mod q as two half-size exponentiations in one launch, then
 * h = (m_p - m_q) qinv mod p and m = m_q + h q (Garner).  c, m: device,
 * batch x n_limbs, c < n.  RNS_EINVAL if the key lacks the needed parts.
 */
int rsa_decrypt(const rsa_key *key, const uint32_t *c, uint32_t *m, size_t batch, int use_crt,
                void *hip_stream);

/*
 * rsa_decrypt_noalloc -- rsa_decrypt for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same kernels and results as rsa_decrypt with the
 * same arguments (a batch too small to fill the GPU is spread over extra
 * workgroups only while their window tables fit), but the window tables and
 * the CRT intermediates live in a
 * fixed array of RSA_NOALLOC_SCRATCH_BYTES bytes that the library holds on
 * each device it runs on (one copy per device, from first use until the
 * process ends).  The call makes no device allocation.
 *   Limit: a batch whose scratch exceeds the array returns RNS_EINVAL with
 *   the bytes it needs, before anything is enqueued.  Scratch per element:
 *   the window table of each exponentiation (2^w entries of the kernel's
 *   residue slots, a little over 2k+1 words, rounded up to whole workgroup
 *   tiles), two of them for CRT, plus 8 * half_limbs bytes of CRT
 *   intermediates.  RSA-2048 CRT (k = 33): about 43 KB per ciphertext at
 *   window 6 and 22 KB at window 5, i.e. up to about 1,500 and 3,000
 *   ciphertexts per call.
 *   Sharing: every call on one device uses the same array, which keeps the
 *   last call's contents; calls that overlap on one device (two streams,
 *   two threads) race and give wrong results.  Serialise them.
 * Errors as rsa_decrypt.
 */
#define RSA_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int rsa_decrypt_noalloc(const rsa_key *key, const uint32_t *c, uint32_t *m, size_t batch, int use_crt,
                        void *hip_stream);

/*
 * rsa_key_status -- the input range status of a key (Sec. 3.3: raw RSA on
 * integers below n).  Synchronises hip_stream, then reads and clears the
 * key's device count of inputs >= n enqueued by rsa_encrypt, rsa_decrypt,
 * rsa_crt_halves and rsa_batch_run on this key since the last read (work on
 * other streams is counted once it has run).  *n_out_of_range (optional,
 * host) receives that count.  Returns RNS_OK when it is zero, RNS_ERANGE
 * otherwise; RNS_EINVAL for a null key, RNS_EDEVICE.
 */
int rsa_key_status(const rsa_key *key, size_t *n_out_of_range, void *hip_stream);

/*
 * The two launches of a CRT decryption, exposed separately (rsa_decrypt with
 * use_crt = 1 is exactly rsa_crt_halves followed by rsa_crt_combine):
 *   rsa_crt_halves   mpq[i] = (c[i]^dp mod p, c[i]^dq mod q): both half-size
 *                    exponentiations in one launch.  c: device, batch x
 *                    n_limbs; mpq: device, batch x (2 * half_limbs), m_p in
 *                    the first half_limbs limbs of a row, m_q in the rest.
 *   rsa_crt_combine  m[i] = m_q + q ((m_p - m_q) qinv mod p) (Garner), from
 *                    an mpq buffer laid out as above; m: batch x n_limbs.
 * RNS_EINVAL if the key has no CRT parts.
 */
int rsa_crt_halves(const rsa_key *key, const uint32_t *c, uint32_t *mpq, size_t batch, void *hip_stream);
int rsa_crt_combine(const rsa_key *key, const uint32_t *mpq, uint32_t *m, size_t batch, void *hip_stream);

/*
 * rns_probe_alu -- measured throughput of one vector-ALU wide multiply form
 * on the current device: the denominator of the roofline of the per-channel
 * steps of an RNS product (32 x 32 -> 64-bit multiply-adds).  Each lane runs
 * 8 independent chains of 4096 dependent instructions; 32 workgroups of 256
 * lanes per compute unit; the second of two launches is timed with HIP
 * events on hip_stream (synchronised).  *lane_ops_per_s = instructions x
 * lanes per second.  RNS_EINVAL for an unknown op or a null output.
 */
enum rns_probe_op {
    RNS_PROBE_MAD_U64_U32 = 0,   /* v_mad_u64_u32: the REDC and residue products */
    RNS_PROBE_MAD_I64_I32 = 1    /* v_mad_i64_i32: recombination of the matrix cores' byte partials */
};
int rns_probe_alu(int op, double *lane_ops_per_s, void *hip_stream);

/*
 * rsa_crt_verify -- check of CRT decryption results against fault attacks
 * (a fault in one half of a CRT decryption gives an m whose gcd with n
 * reveals a factor; the paper keeps the private key on the GPU, Sec. 4.3):
 * m[i]^e mod n is recomputed on the full-modulus context and compared with
 * c[i]; every m[i] that fails is overwritten with zeros.
 *   c      device, batch x n_limbs: the ciphertexts (< n), not aliasing m
 *   m      device, batch x n_limbs: the results of rsa_decrypt (CRT)
 *   n_bad  host or NULL: number of failing elements
 * Synchronises hip_stream.  RNS_OK if every element passes, RNS_EVERIFY if
 * any fails (outputs zeroed, count in n_bad); RNS_EINVAL (null buffers,
 * c == m), RNS_EUNSUPPORTED for a CRT-only key.  Cost: one exponentiation by
 * e per element on the full modulus (17 products for e = 65537).
 */
int rsa_crt_verify(const rsa_key *key, const uint32_t *c, uint32_t *m, size_t batch, size_t *n_bad,
                   void *hip_stream);

/*
 * Batched form: many RSA operations over keys of different sizes in a fixed
 * set of launches (Sec. 3.3 operations, batched as in Sec. 4.3's throughput
 * use of many messages).  rsa_batch_create plans a list of operations once;
 * rsa_batch_run enqueues all of them.  Exponentiations of every key whose
 * half- or full-size k share a matrix-core kernel shape run in ONE launch per
 * shape (one workgroup per tile of 16 or 32 elements, longest jobs first),
 * the launches of different shapes run concurrently on internal streams, and
 * the Garner steps of CRT decryptions follow, grouped the same way: one
 * launch per base shape of the halves (on the stream of the exponentiation
 * group that produced the halves when that group alone did).  With
 * use_graph the whole set is captured once into a hipGraph and each run is
 * one graph launch.
 *
 *   rsa_op.kind  RSA_OP_ENCRYPT: out = in^e mod n;
 *                RSA_OP_DECRYPT: out = in^d mod n, by CRT when the key has
 *                its CRT parts.
 *   in, out      device, count x n_limbs(key); they may not overlap other
 *                operations' buffers; out may equal in.
 * The buffers, keys and counts are bound at creation: a batch is re-run on
 * new data by writing into the same buffers.  Keys must outlive the batch.
 *
 * Tuning (rsa_batch_opts, NULL = defaults):
 *   autotune     1: at creation, for each kernel shape class, time the whole
 *                group launch (outputs to scratch) with each candidate tile
 *                (16 or 32 elements per workgroup) and keep the fastest; then,
 *                for each exponent length in the class, time the window
 *                offsets -1 and +1 from every job's product-minimising window
 *                and keep one that is at least 1% faster.  The choices are
 *                cached per process and also used by later batches and by
 *                the request server.  The base size k is not a tuning
 *                dimension: every job runs on the smallest base its modulus
 *                fits (see rsa_batch_classes for what was chosen).  0: each
 *                launch's tile chosen as for rns_opts.group = 0 (keys set up
 *                with an explicit group keep it), windows minimise products.
 *   use_graph    1: capture into a hipGraph at creation (default 1; not
 *                used when some key runs on the channel engine).
 *   window       0: per job, the window width minimising the number of
 *                Montgomery products for its exponent; 1..6: fixed.
 * Errors: RNS_EINVAL (bad op, null buffer), RNS_ENOMEM, RNS_EDEVICE.
 * rsa_batch_create synchronises `hip_stream` (autotuning runs on an internal
 * stream) and returns when the batch is ready to run.
 */
enum rsa_op_kind { RSA_OP_ENCRYPT = 0, RSA_OP_DECRYPT = 1 };

typedef struct rsa_op {
    const rsa_key *key;
    int kind;
    const uint32_t *in;
    uint32_t *out;
    size_t count;
} rsa_op;

typedef struct rsa_batch_opts {
    int autotune;
    int use_graph;
    int window;
} rsa_batch_opts;

typedef struct rsa_batch_info {
    int launches;            /* exponentiation launches per run */
    int jobs;                /* exponentiation jobs (a CRT decryption is 2) */
    int garner_launches;     /* grouped Garner launches per run (one per base shape of CRT halves) */
    size_t workspace_bytes;  /* device memory held by the batch */
    size_t modmuls;          /* RNS Montgomery products per element, summed over elements */
    int tuning_launches;     /* group launches the autotuner timed at creation */
} rsa_batch_info;


typedef struct rsa_batch rsa_batch;

int rsa_batch_create(const rsa_op *ops, size_t n_ops, const rsa_batch_opts *opts, void *hip_stream,
                     rsa_batch **out);
int rsa_batch_run(rsa_batch *b, void *hip_stream);
int rsa_batch_info_get(const rsa_batch *b, rsa_batch_info *info);
/*
 * What the batch runs, per (kernel shape class, exponent length): one entry
 * per class in launch order.  out: host array of cap entries (may be NULL
 * with cap = 0 to count); *n receives the number of classes.
 */
typedef struct rsa_batch_class {
    int k;               /* channels per base */
    int waves;           /* wavefronts per workgroup */
    int group;           /* elements per workgroup (the tile) */
    int exp_bits;        /* exponent length of the class's jobs (32 x limbs) */
    int window;          /* window width of the class's most expensive job */
    int window_offset;   /* offset from each job's product-minimising window */
    int jobs;            /* exponentiation jobs of this exponent length */
    int tuned;           /* 1 when the autotuner chose tile and window offset */
    double launch_ms;    /* autotune: measured time of the whole group launch */
} rsa_batch_class;

int rsa_batch_classes(const rsa_batch *b, rsa_batch_class *out, size_t cap, size_t *n);
/* Waits for the batch's device work, then releases it. */
void rsa_batch_free(rsa_batch *b);

/*
 * Request server: the served form of the batched path (Sec. 3.3 operations
 * on resident keys).  Keys stay resident; requests are admitted as dispatch
 * slots and device memory free up (continuous batching: requests that arrive
 * while others run on the GPU join the next dispatch), each dispatch plans
 * grouped launches as rsa_batch does, and up to max_inflight dispatches run
 * concurrently on their own streams.
 *
 *   rsa_server_opts  hbm_budget: device bytes in-flight dispatches may use
 *                    (0 = 64 GiB; each dispatch slot also keeps its device
 *                    arena, up to 1.25 x the largest dispatch it ran, until
 *                    rsa_server_free); max_inflight: concurrent dispatches
 *                    (0 = 4, the hardware queues HIP gives a process by
 *                    default; streams beyond them share queues and
 *                    serialise); max_dispatch_ops: requests per dispatch
 *                    (0 = 16384); max_pending: requests waiting for
 *                    admission at most (0 = no limit): a request arriving
 *                    while that many wait is refused (load shedding).
 * A dispatch holds requests of one kernel-shape class (the base size k of
 * their exponentiations), so short requests never wait for long ones in the
 * same dispatch; a free slot goes to the class whose oldest pending request
 * arrived first.
 *   rsa_request      one RSA operation on key `key` (an index into the
 *                    server's key list): in and out are HOST buffers of
 *                    n_limbs(key) limbs; out is written when it completes.
 *                    arrival: seconds after the start of the replay.
 * rsa_server_replay runs an open-loop trace: request i is admitted no earlier
 * than its arrival time on the host's monotonic clock (arrivals must be
 * non-decreasing); it returns when all have completed.  latency (optional,
 * n entries) receives completion - arrival in seconds; the completion time is
 * when the host sees the dispatch's results copied back.  A refused request
 * keeps its output untouched, gets latency -1 and is counted in
 * stats.rejected; the others complete, and the call then returns RNS_EBUSY.
 * Errors, before anything runs: RNS_EINVAL (bad key index or kind, null
 * buffer, decreasing arrivals), RNS_ERANGE (an input not below its key's n),
 * RNS_EBUSY (a request that alone exceeds the device-memory budget); while
 * running: RNS_ENOMEM, RNS_EDEVICE.  The keys must outlive the server.
 */
typedef struct rsa_server_opts {
    size_t hbm_budget;
    int max_inflight;
    size_t max_dispatch_ops;
    size_t max_pending;
} rsa_server_opts;

typedef struct rsa_request {
    int key;
    int kind;
    const uint32_t *in;
    uint32_t *out;
    double arrival;
} rsa_request;

typedef struct rsa_server_stats {
    size_t completed;
    size_t rejected;             /* refused by the pending-queue limit */
    size_t dispatches;
    double elapsed;              /* first arrival to last completion, seconds */
    double p50_latency, p99_latency, max_latency;   /* seconds */
    double mean_dispatch_ops;
    size_t peak_inflight_bytes;  /* device bytes held by dispatches at once */
    int peak_inflight;           /* dispatches in flight at once */
} rsa_server_stats;

typedef struct rsa_server rsa_server;

int rsa_server_create(const rsa_key *const *keys, size_t n_keys, const rsa_server_opts *opts, rsa_server **out);
int rsa_server_replay(rsa_server *srv, const rsa_request *reqs, size_t n, double *latency, rsa_server_stats *stats);
void rsa_server_free(rsa_server *srv);

/* ------------------------------------------------------------------------ */
/* Primality steps of key generation                                         */
/* ------------------------------------------------------------------------ */

/*
 * rsa_trial_division -- the small-primes step of key generation (Sec. 4.3:
 * testing candidates against the first 10,000 primes): flags[i] = 0 when one
 * of the first n_primes primes divides candidate i and differs from it (i is
 * then composite), else 1.
 *   cand       device, count x limbs little-endian 32-bit limbs
 *   n_primes   1..10000
 *   flags      device, count bytes
 * Asynchronous on hip_stream.  Errors: RNS_EINVAL (null buffer, limbs
 * outside 1..4096, n_primes outside 1..10000), RNS_EDEVICE.
 */
int rsa_trial_division(const uint32_t *cand, size_t count, int limbs, int n_primes, uint8_t *flags,
                       void *hip_stream);

/*
 * rsa_miller_rabin -- the Miller-Rabin test of key generation (Sec. 3.2, with
 * the number of rounds the caller chooses, e.g. FIPS 186's, Sec. 4.3): with
 * N - 1 = 2^s d, d odd, base a passes when a^d = 1 or a^(2^j d) = N - 1 for
 * some j < s (mod N); verdict[i] = 1 when every base of candidate i passes
 * (a probable prime), 0 when one fails (N composite).  The exponentiations
 * run in RNS in the Montgomery domain: one context per candidate (constants
 * computed on the host from the candidate), all candidates of a kernel
 * shape in one grouped launch per step (a^d, then squarings until every
 * base is decided); the comparisons with 1 and N - 1 run on the host.
 *   cand       host, count x limbs, odd candidates > 3
 *   bases      host, count x rounds x limbs, each in [2, N - 2]
 *   rounds     1..64
 *   verdict    host, count bytes
 * Synchronises hip_stream.  Errors: RNS_EINVAL (null buffer, limbs outside
 * 1..4096, rounds outside 1..64, an even or small candidate, a base out of
 * range), RNS_ERANGE (no base size for the candidates), RNS_ENOMEM,
 * RNS_EDEVICE.
 */
int rsa_miller_rabin(const uint32_t *cand, size_t count, int limbs, const uint32_t *bases, int rounds,
                     uint8_t *verdict, void *hip_stream);

/*
 * rsa_keygen -- RSA key generation (Sec. 3.3 and Sec. 4.3): p is the first
 * candidate of cand_p, in stream order, that passes rsa_trial_division
 * (first 10,000 primes), has gcd(e, p - 1) = 1 and passes rsa_miller_rabin
 * with its bases; q likewise from cand_q (q != p).  n = p q;
 * d = e^-1 mod (p-1)(q-1) by Arazi's formula d = (1 + f (-f^-1 mod e)) / e
 * with f = (p-1)(q-1), in RNS channel by channel on the GPU (Sec. 3.1; the
 * scalar -f^-1 mod e from f mod e on the host), back to binary through the
 * base's exit, and checked (d e = 1 mod f, else RNS_EVERIFY);
 * dp = d mod (p-1), dq = d mod (q-1), qinv = q^-1 mod p (host).  The key is loaded
 * as by rsa_key_load with opts; only n (n_out) and the handle come back, p,
 * q and d stay in library memory.
 *   cand_p, cand_q    host, count x half_limbs limbs each
 *   bases_p, bases_q  host, count x rounds x half_limbs (the Miller-Rabin
 *                     bases of each candidate, each in [2, c - 2])
 *   e                 odd, >= 3
 *   n_out             host, 2 * half_limbs limbs
 * Synchronises hip_stream.  Errors: RNS_EINVAL (bad argument, a base out of
 * range), RNS_ERANGE (a stream holds no probable prime), RNS_EUNSUPPORTED
 * (e equal to a channel prime; keys above 8192 bits, half_limbs > 128, whose
 * (p-1)(q-1) needs a base without a channel kernel for Arazi's step),
 * RNS_EVERIFY, as rsa_key_load.
 */
int rsa_keygen(const uint32_t *cand_p, const uint32_t *bases_p, const uint32_t *cand_q, const uint32_t *bases_q,
               size_t count, int half_limbs, int rounds, uint32_t e, const rns_opts *opts, uint32_t *n_out,
               rsa_key **out, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* RNSRSA_H */
