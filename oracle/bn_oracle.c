/*
 * bn_oracle.c -- plain CPU oracle for RSA modular exponentiation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library; the GPU library never
 * does, and this file shares no code with it.
 *
 * What it computes is the plain definition of the paper's hot path:
 *   modexp(b, e, N) = b^e mod N, canonical in [0, N)          (Sec. 3.1)
 *   RSA encryption  c = m^e mod n, decryption m = c^d mod n  (Sec. 3.3)
 * The paper does the arithmetic in the Residue Number System with RNS
 * Montgomery multiplication; the method is exact, so the oracle uses plain
 * positional ("schoolbook") bignums instead, the traditional arithmetic that
 * Sec. 3 contrasts with RNS:
 *   - limbs of ORACLE_LIMB_BITS bits (32 for the product build; an 8-bit
 *     build exists only so that tests reach the rare correction paths of
 *     the division often);
 *   - schoolbook multiplication;
 *   - remainder by Knuth's Algorithm D (TAOCP vol. 2, Sec. 4.3.1);
 *   - left-to-right binary square-and-multiply, the "traditional
 *     square-and-multiply" exponentiation of Sec. 3.1.
 * A Garner-style CRT decryption is provided for timing a fair CPU baseline;
 * its result is, by definition, the same c^d mod n.
 *
 * Conventions (Python pow): e = 0 gives 1 mod N (so 0^0 = 1), bases >= N are
 * reduced first, N must be >= 1 (N = 1 gives 0).  All arrays are little-endian
 * limb vectors.  Functions return 0 on success, -1 on invalid arguments.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef ORACLE_LIMB_BITS
#define ORACLE_LIMB_BITS 32
#endif

#if ORACLE_LIMB_BITS == 32
typedef uint32_t limb_t;
typedef uint64_t dlimb_t;
#define ORACLE_SYM(name) oracle_##name
#elif ORACLE_LIMB_BITS == 8
typedef uint8_t limb_t;
typedef uint32_t dlimb_t;
#define ORACLE_SYM(name) oracle8_##name
#else
#error "ORACLE_LIMB_BITS must be 8 or 32"
#endif

#define LB ORACLE_LIMB_BITS
#define LIMB_BASE ((dlimb_t)1 << LB)
#define LIMB_MASK (LIMB_BASE - 1)

/* Number of times Algorithm D's final add-back step (D6) ran, per thread. */
static _Thread_local long long g_addback = 0;
/* Number of times the D3 test lowered the trial quotient, per thread. */
static _Thread_local long long g_qhat_fix = 0;

/* Significant length of x (at least 1). */
static size_t bn_len(const limb_t *x, size_t n) {
    while (n > 1 && x[n - 1] == 0) n--;
    return n;
}

/* w[0 .. la+lb) = a * b, schoolbook (TAOCP Algorithm 4.3.1 M). */
static void bn_mul(const limb_t *a, size_t la, const limb_t *b, size_t lb, limb_t *w) {
    memset(w, 0, (la + lb) * sizeof(limb_t));
    for (size_t j = 0; j < lb; j++) {
        dlimb_t carry = 0;
        for (size_t i = 0; i < la; i++) {
            dlimb_t t = (dlimb_t)a[i] * b[j] + w[i + j] + carry;
            w[i + j] = (limb_t)(t & LIMB_MASK);
            carry = t >> LB;
        }
        w[j + la] = (limb_t)carry;
    }
}

/* Number of leading zero bits of a nonzero limb. */
static int limb_clz(limb_t x) {
    int s = 0;
    while (!(x & ((limb_t)1 << (LB - 1)))) { x = (limb_t)(x << 1); s++; }
    return s;
}

/*
 * Knuth's Algorithm D: u (m+n limbs) divided by v (n limbs, v[n-1] != 0).
 * q receives m+1 limbs (may be NULL), r receives n limbs.  Scratch is
 * allocated here.  Returns 0, or -1 on allocation failure.
 */
static int bn_divmod_knuth(const limb_t *u, size_t lu, const limb_t *v, size_t n,
                           limb_t *q, limb_t *r) {
    if (lu < n) {                    /* quotient 0, remainder u */
        memset(r, 0, n * sizeof(limb_t));
        memcpy(r, u, lu * sizeof(limb_t));
        return 0;
    }
    size_t m = lu - n;
    if (n == 1) {                    /* short division */
        dlimb_t rem = 0;
        for (size_t j = lu; j-- > 0;) {
            dlimb_t cur = (rem << LB) | u[j];
            if (q) q[j] = (limb_t)(cur / v[0]);
            rem = cur % v[0];
        }
        r[0] = (limb_t)rem;
        return 0;
    }
    limb_t *un = (limb_t *)calloc(lu + 1, sizeof(limb_t));
    limb_t *vn = (limb_t *)calloc(n, sizeof(limb_t));
    if (!un || !vn) { free(un); free(vn); return -1; }
    /* D1: normalise so that the top limb of v has its top bit set. */
    int s = limb_clz(v[n - 1]);
    for (size_t i = n; i-- > 0;) {
        dlimb_t hi = (dlimb_t)v[i] << s;
        dlimb_t lo = (s && i) ? ((dlimb_t)v[i - 1] >> (LB - s)) : 0;
        vn[i] = (limb_t)((hi | lo) & LIMB_MASK);
    }
    un[lu] = s ? (limb_t)((dlimb_t)u[lu - 1] >> (LB - s)) : 0;
    for (size_t i = lu; i-- > 0;) {
        dlimb_t hi = (dlimb_t)u[i] << s;
        dlimb_t lo = (s && i) ? ((dlimb_t)u[i - 1] >> (LB - s)) : 0;
        un[i] = (limb_t)((hi | lo) & LIMB_MASK);
    }
    /* D2 .. D7: one quotient limb per step, most significant first. */
    for (size_t j = m + 1; j-- > 0;) {
        /* D3: trial quotient from the top two limbs, then Knuth's test. */
        dlimb_t num = ((dlimb_t)un[j + n] << LB) | un[j + n - 1];
        dlimb_t qhat = num / vn[n - 1];
        dlimb_t rhat = num % vn[n - 1];
        while (qhat >= LIMB_BASE ||
               qhat * vn[n - 2] > ((rhat << LB) | un[j + n - 2])) {
            qhat--;
            rhat += vn[n - 1];
            g_qhat_fix++;
            if (rhat >= LIMB_BASE) break;
        }
        /* D4: multiply and subtract qhat * v from un[j .. j+n]. */
        dlimb_t borrow = 0, carry = 0;
        for (size_t i = 0; i < n; i++) {
            dlimb_t p = qhat * vn[i] + carry;
            carry = p >> LB;
            dlimb_t sub = (dlimb_t)un[i + j] - (p & LIMB_MASK) - borrow;
            un[i + j] = (limb_t)(sub & LIMB_MASK);
            borrow = (sub >> LB) ? 1 : 0;   /* wrapped below zero */
        }
        dlimb_t sub = (dlimb_t)un[j + n] - carry - borrow;
        un[j + n] = (limb_t)(sub & LIMB_MASK);
        int negative = (sub >> LB) ? 1 : 0;
        /* D5/D6: if the subtraction went negative, add v back once. */
        if (negative) {
            qhat--;
            g_addback++;
            dlimb_t c = 0;
            for (size_t i = 0; i < n; i++) {
                dlimb_t t = (dlimb_t)un[i + j] + vn[i] + c;
                un[i + j] = (limb_t)(t & LIMB_MASK);
                c = t >> LB;
            }
            un[j + n] = (limb_t)(((dlimb_t)un[j + n] + c) & LIMB_MASK);
        }
        if (q) q[j] = (limb_t)qhat;
    }
    /* D8: unnormalise the remainder. */
    for (size_t i = 0; i < n; i++) {
        dlimb_t lo = (dlimb_t)un[i] >> s;
        dlimb_t hi = s ? ((dlimb_t)un[i + 1] << (LB - s)) & LIMB_MASK : 0;
        r[i] = (limb_t)(lo | hi);
    }
    free(un);
    free(vn);
    return 0;
}

/* r (ln limbs) = x mod N, where N has ln limbs and its top limb may be 0. */
static int bn_mod(const limb_t *x, size_t lx, const limb_t *N, size_t ln, limb_t *r) {
    size_t n = bn_len(N, ln);
    size_t l = bn_len(x, lx);
    memset(r, 0, ln * sizeof(limb_t));
    return bn_divmod_knuth(x, l, N, n, NULL, r);
}

/* out (ln limbs) = a*b mod N, with a, b < N of ln limbs.  tmp: 2*ln limbs. */
static int bn_mulmod(const limb_t *a, const limb_t *b, const limb_t *N, size_t ln,
                     limb_t *tmp, limb_t *out) {
    bn_mul(a, ln, b, ln, tmp);
    return bn_mod(tmp, 2 * ln, N, ln, out);
}

/*
 * out = base^exp mod N by left-to-right binary square-and-multiply
 * (Sec. 3.1's traditional square-and-multiply): scan the exponent bits from
 * the most significant one, square at every bit and multiply by the base at
 * every set bit.
 */
static int bn_modexp(const limb_t *base, size_t lb, const limb_t *exp, size_t le,
                     const limb_t *N, size_t ln, limb_t *out) {
    if (bn_len(N, ln) == 1 && N[0] == 0) return -1;
    limb_t *b = (limb_t *)calloc(ln, sizeof(limb_t));
    limb_t *acc = (limb_t *)calloc(ln, sizeof(limb_t));
    limb_t *t = (limb_t *)calloc(ln, sizeof(limb_t));
    limb_t *tmp = (limb_t *)calloc(2 * ln, sizeof(limb_t));
    limb_t *one = (limb_t *)calloc(ln, sizeof(limb_t));
    int rc = -1;
    if (!b || !acc || !t || !tmp || !one) goto done;
    if (bn_mod(base, lb, N, ln, b)) goto done;
    one[0] = 1;
    if (bn_mod(one, 1, N, ln, acc)) goto done;          /* 1 mod N */
    for (size_t w = le; w-- > 0;) {
        for (int bit = LB - 1; bit >= 0; bit--) {
            if (bn_mulmod(acc, acc, N, ln, tmp, t)) goto done;
            memcpy(acc, t, ln * sizeof(limb_t));
            if ((exp[w] >> bit) & 1) {
                if (bn_mulmod(acc, b, N, ln, tmp, t)) goto done;
                memcpy(acc, t, ln * sizeof(limb_t));
            }
        }
    }
    memcpy(out, acc, ln * sizeof(limb_t));
    rc = 0;
done:
    free(b); free(acc); free(t); free(tmp); free(one);
    return rc;
}

/* ----------------------------------------------------------------------- */
/* Exported entry points                                                   */
/* ----------------------------------------------------------------------- */

/* q (lu limbs) = floor(u / v), r (lv limbs) = u mod v.  v must be nonzero. */
int ORACLE_SYM(divmod)(const limb_t *u, size_t lu, const limb_t *v, size_t lv,
                       limb_t *q, limb_t *r) {
    if (!u || !v || !r || lu == 0 || lv == 0) return -1;
    size_t n = bn_len(v, lv);
    if (n == 1 && v[0] == 0) return -1;
    size_t l = bn_len(u, lu);
    limb_t *qq = (limb_t *)calloc(l + 2, sizeof(limb_t));
    limb_t *rr = (limb_t *)calloc(n, sizeof(limb_t));
    if (!qq || !rr) { free(qq); free(rr); return -1; }
    int rc = bn_divmod_knuth(u, l, v, n, qq, rr);
    if (rc == 0) {
        if (q) {
            memset(q, 0, lu * sizeof(limb_t));
            size_t nq = l >= n ? l - n + 1 : 0;
            memcpy(q, qq, (nq < lu ? nq : lu) * sizeof(limb_t));
        }
        memset(r, 0, lv * sizeof(limb_t));
        memcpy(r, rr, n * sizeof(limb_t));
    }
    free(qq); free(rr);
    return rc;
}

/* w (la + lb limbs) = a * b. */
int ORACLE_SYM(mul)(const limb_t *a, size_t la, const limb_t *b, size_t lb, limb_t *w) {
    if (!a || !b || !w || la == 0 || lb == 0) return -1;
    bn_mul(a, la, b, lb, w);
    return 0;
}

long long ORACLE_SYM(addback_count)(void) { return g_addback; }
long long ORACLE_SYM(qhat_fix_count)(void) { return g_qhat_fix; }
void ORACLE_SYM(reset_counters)(void) { g_addback = 0; g_qhat_fix = 0; }

/*
 * out[i] = base[i]^exp_i mod N for i < batch.
 *   base:  batch x lb limbs;   N: ln limbs;   out: batch x ln limbs
 *   exp:   le limbs each; exp_stride = 0 means one exponent for the batch,
 *          otherwise element i's exponent starts at exp + i*exp_stride.
 *   nthreads: OpenMP threads (<= 0: the runtime's default).
 */
int ORACLE_SYM(modexp_batch)(const limb_t *base, size_t lb, const limb_t *exp,
                             size_t le, size_t exp_stride, const limb_t *N, size_t ln,
                             limb_t *out, size_t batch, int nthreads) {
    if (!base || !exp || !N || !out || lb == 0 || le == 0 || ln == 0) return -1;
    if (bn_len(N, ln) == 1 && N[0] == 0) return -1;
    int bad = 0;
    long long nb = (long long)batch;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) reduction(|:bad) num_threads(nthreads > 0 ? nthreads : omp_get_max_threads())
#endif
    for (long long i = 0; i < nb; i++) {
        const limb_t *e = exp + (size_t)i * exp_stride;
        if (bn_modexp(base + (size_t)i * lb, lb, e, le, N, ln, out + (size_t)i * ln)) bad |= 1;
    }
    return bad ? -1 : 0;
}

/*
 * CRT decryption by Garner's recombination (a CPU baseline; its result is
 * c^d mod n):  m_p = c^dp mod p, m_q = c^dq mod q,
 *              h = (m_p - m_q) * qinv mod p,  m = m_q + h*q.
 *   c: batch x ln limbs (c < n);  p, q, dp, dq, qinv: lh limbs each;
 *   out: batch x ln limbs, ln >= 2*lh.
 */
int ORACLE_SYM(rsa_crt_batch)(const limb_t *c, size_t ln, const limb_t *p, const limb_t *q,
                              const limb_t *dp, const limb_t *dq, const limb_t *qinv,
                              size_t lh, limb_t *out, size_t batch, int nthreads) {
    if (!c || !p || !q || !dp || !dq || !qinv || !out || lh == 0 || ln < 2 * lh) return -1;
    int bad = 0;
    long long nb = (long long)batch;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) reduction(|:bad) num_threads(nthreads > 0 ? nthreads : omp_get_max_threads())
#endif
    for (long long i = 0; i < nb; i++) {
        limb_t *mp = (limb_t *)calloc(lh, sizeof(limb_t));
        limb_t *mq = (limb_t *)calloc(lh, sizeof(limb_t));
        limb_t *mqp = (limb_t *)calloc(lh, sizeof(limb_t));
        limb_t *d = (limb_t *)calloc(lh + 1, sizeof(limb_t));
        limb_t *h = (limb_t *)calloc(lh, sizeof(limb_t));
        limb_t *tmp = (limb_t *)calloc(2 * lh + 2, sizeof(limb_t));
        limb_t *hq = (limb_t *)calloc(2 * lh, sizeof(limb_t));
        if (!mp || !mq || !mqp || !d || !h || !tmp || !hq) { bad |= 1; goto next; }
        {
            const limb_t *ci = c + (size_t)i * ln;
            limb_t *o = out + (size_t)i * ln;
            if (bn_modexp(ci, ln, dp, lh, p, lh, mp)) { bad |= 1; goto next; }
            if (bn_modexp(ci, ln, dq, lh, q, lh, mq)) { bad |= 1; goto next; }
            /* d = m_p + p - (m_q mod p), in [1, 2p), then reduced mod p. */
            if (bn_mod(mq, lh, p, lh, mqp)) { bad |= 1; goto next; }
            dlimb_t carry = 0;
            for (size_t k = 0; k < lh; k++) {
                dlimb_t t = (dlimb_t)mp[k] + p[k] + carry;
                d[k] = (limb_t)(t & LIMB_MASK);
                carry = t >> LB;
            }
            d[lh] = (limb_t)carry;
            dlimb_t borrow = 0;
            for (size_t k = 0; k <= lh; k++) {
                dlimb_t sub = (dlimb_t)d[k] - (k < lh ? mqp[k] : 0) - borrow;
                d[k] = (limb_t)(sub & LIMB_MASK);
                borrow = (sub >> LB) ? 1 : 0;
            }
            if (bn_mod(d, lh + 1, p, lh, h)) { bad |= 1; goto next; }
            /* h = h * qinv mod p */
            bn_mul(h, lh, qinv, lh, tmp);
            if (bn_mod(tmp, 2 * lh, p, lh, h)) { bad |= 1; goto next; }
            /* m = m_q + h*q */
            bn_mul(h, lh, q, lh, hq);
            memset(o, 0, ln * sizeof(limb_t));
            carry = 0;
            for (size_t k = 0; k < ln; k++) {
                dlimb_t t = (dlimb_t)(k < 2 * lh ? hq[k] : 0) + (k < lh ? mq[k] : 0) + carry;
                o[k] = (limb_t)(t & LIMB_MASK);
                carry = t >> LB;
            }
        }
    next:
        free(mp); free(mq); free(mqp); free(d); free(h); free(tmp); free(hq);
    }
    return bad ? -1 : 0;
}

int ORACLE_SYM(limb_bits)(void) { return LB; }
