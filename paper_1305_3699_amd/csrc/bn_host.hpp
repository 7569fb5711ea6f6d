// Minimal host-side unsigned bignum used only to precompute RNS constants at
// set-up time (Sec. 3.1: the constants of base extension and of the RNS
// Montgomery product are computed once and kept resident on the device).
// Nothing here runs per message; simplicity beats speed.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <vector>

namespace rnsrsa {

using Limbs = std::vector<uint32_t>;  // little-endian 32-bit limbs

inline void bn_trim(Limbs &a) {
    while (!a.empty() && a.back() == 0) a.pop_back();
}

inline Limbs bn_from_u64(uint64_t v) {
    Limbs r{(uint32_t)v, (uint32_t)(v >> 32)};
    bn_trim(r);
    return r;
}

inline Limbs bn_from_ptr(const uint32_t *p, size_t n) {
    Limbs r(p, p + n);
    bn_trim(r);
    return r;
}

inline bool bn_is_zero(const Limbs &a) {
    for (uint32_t x : a)
        if (x) return false;
    return true;
}

inline unsigned bn_bits(const Limbs &a) {
    for (size_t i = a.size(); i-- > 0;)
        if (a[i]) return (unsigned)(32 * i + 32 - __builtin_clz(a[i]));
    return 0;
}

inline int bn_cmp(const Limbs &a, const Limbs &b) {
    size_t n = std::max(a.size(), b.size());
    for (size_t i = n; i-- > 0;) {
        uint32_t x = i < a.size() ? a[i] : 0, y = i < b.size() ? b[i] : 0;
        if (x != y) return x < y ? -1 : 1;
    }
    return 0;
}

inline Limbs bn_add(const Limbs &a, const Limbs &b) {
    size_t n = std::max(a.size(), b.size());
    Limbs r(n + 1);
    uint64_t c = 0;
    for (size_t i = 0; i < n; i++) {
        c += (uint64_t)(i < a.size() ? a[i] : 0) + (i < b.size() ? b[i] : 0);
        r[i] = (uint32_t)c;
        c >>= 32;
    }
    r[n] = (uint32_t)c;
    bn_trim(r);
    return r;
}

// a - b, requires a >= b
inline Limbs bn_sub(const Limbs &a, const Limbs &b) {
    Limbs r(a.size());
    int64_t br = 0;
    for (size_t i = 0; i < a.size(); i++) {
        int64_t t = (int64_t)a[i] - (i < b.size() ? b[i] : 0) - br;
        br = t < 0;
        r[i] = (uint32_t)(t + (br ? ((int64_t)1 << 32) : 0));
    }
    bn_trim(r);
    return r;
}

inline Limbs bn_mul(const Limbs &a, const Limbs &b) {
    if (a.empty() || b.empty()) return Limbs{};
    Limbs r(a.size() + b.size(), 0);
    for (size_t i = 0; i < a.size(); i++) {
        uint64_t c = 0;
        for (size_t j = 0; j < b.size(); j++) {
            c += (uint64_t)a[i] * b[j] + r[i + j];
            r[i + j] = (uint32_t)c;
            c >>= 32;
        }
        r[i + b.size()] = (uint32_t)c;
    }
    bn_trim(r);
    return r;
}

inline Limbs bn_mul_word(const Limbs &a, uint32_t w) { return bn_mul(a, bn_from_u64(w)); }

inline Limbs bn_shl(const Limbs &a, unsigned bits) {
    if (a.empty()) return a;
    unsigned w = bits / 32, s = bits % 32;
    Limbs r(a.size() + w + 1, 0);
    for (size_t i = 0; i < a.size(); i++) {
        r[i + w] |= a[i] << s;
        if (s) r[i + w + 1] |= a[i] >> (32 - s);
    }
    bn_trim(r);
    return r;
}

inline Limbs bn_shr1(const Limbs &a) {
    Limbs r(a.size(), 0);
    for (size_t i = 0; i < a.size(); i++) r[i] = (a[i] >> 1) | (i + 1 < a.size() ? a[i + 1] << 31 : 0u);
    bn_trim(r);
    return r;
}

// x mod n by bit-serial shift-and-subtract (n > 0), in place on a buffer of
// n's length plus one limb (the running remainder stays below 2n).
inline Limbs bn_mod(const Limbs &x, const Limbs &n_in) {
    Limbs n = n_in;
    bn_trim(n);
    const size_t L = n.size();
    Limbs r(L + 1, 0);
    for (unsigned b = bn_bits(x); b-- > 0;) {
        uint32_t carry = (x[b / 32] >> (b % 32)) & 1u;
        for (size_t i = 0; i <= L; i++) {
            const uint32_t t = r[i];
            r[i] = (t << 1) | carry;
            carry = t >> 31;
        }
        bool ge = r[L] != 0;
        if (!ge) {
            ge = true;
            for (size_t i = L; i-- > 0;)
                if (r[i] != n[i]) {
                    ge = r[i] > n[i];
                    break;
                }
        }
        if (ge) {
            int64_t br = 0;
            for (size_t i = 0; i <= L; i++) {
                const int64_t t = (int64_t)r[i] - (i < L ? n[i] : 0u) - br;
                br = t < 0;
                r[i] = (uint32_t)t;
            }
        }
    }
    bn_trim(r);
    return r;
}

inline uint32_t bn_mod_word(const Limbs &x, uint32_t m) {
    uint64_t r = 0;
    for (size_t i = x.size(); i-- > 0;) r = ((r << 32) | x[i]) % m;
    return (uint32_t)r;
}

inline uint32_t bn_low(const Limbs &x) { return x.empty() ? 0u : x[0]; }

inline uint32_t mulmod32(uint32_t a, uint32_t b, uint32_t m) { return (uint32_t)((uint64_t)a * b % m); }

inline uint32_t powmod32(uint32_t a, uint64_t e, uint32_t m) {
    uint64_t r = 1 % m, b = a % m;
    while (e) {
        if (e & 1) r = r * b % m;
        b = b * b % m;
        e >>= 1;
    }
    return (uint32_t)r;
}

// prod(ms) mod m
inline uint32_t prod_mod32(const std::vector<uint32_t> &ms, uint32_t m) {
    uint64_t r = 1 % m;
    for (uint32_t x : ms) r = r * (x % m) % m;
    return (uint32_t)r;
}

inline uint32_t pow2_32_mod(uint32_t m) { return (uint32_t)(((uint64_t)1 << 32) % m); }

inline uint32_t pow2_64_mod(uint32_t m) {
    uint64_t r = ((uint64_t)1 << 32) % m;
    return (uint32_t)(r * r % m);
}

// a^-1 mod m by the extended Euclidean algorithm; 0 when gcd(a, m) != 1.
inline uint32_t invmod32(uint32_t a, uint32_t m) {
    int64_t t = 0, nt = 1, r = m, nr = a % m;
    while (nr) {
        int64_t q = r / nr, tmp;
        tmp = t - q * nt; t = nt; nt = tmp;
        tmp = r - q * nr; r = nr; nr = tmp;
    }
    if (r != 1) return 0;
    if (t < 0) t += m;
    return (uint32_t)t;
}

// a^-1 mod 2^32 for odd a (Newton iteration).
inline uint32_t inv2_32(uint32_t a) {
    uint32_t x = a;  // correct to 3 bits for odd a
    for (int i = 0; i < 5; i++) x *= 2u - a * x;
    return x;
}

// Deterministic primality for 32-bit n: Miller-Rabin with bases 2, 7, 61.
inline bool is_prime32(uint32_t n) {
    if (n < 2) return false;
    for (uint32_t p : {2u, 3u, 5u, 7u, 11u, 13u, 17u, 19u, 23u, 29u, 31u, 37u, 41u, 43u, 47u, 53u, 59u, 61u})
        if (n % p == 0) return n == p;
    uint32_t d = n - 1;
    int s = 0;
    while (!(d & 1)) { d >>= 1; s++; }
    for (uint32_t a : {2u, 7u, 61u}) {
        uint64_t x = powmod32(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int i = 1; i < s; i++) {
            x = x * x % n;
            if (x == n - 1) { comp = false; break; }
        }
        if (comp) return false;
    }
    return true;
}

}  // namespace rnsrsa
