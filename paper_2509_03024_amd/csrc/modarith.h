// Modular arithmetic on 64-bit residues for primes q < 2^61.
//
// Two reductions are used, both exact:
//  * Shoup multiplication by a precomputed constant w (twiddles, CRT
//    constants): with w' = floor(w * 2^64 / q),
//        h = floor(a * w' / 2^64),  r = a*w - h*q  (mod 2^64),  r in [0, 2q)
//    for any a < 2^64, followed by one conditional subtraction.
//  * Montgomery multiplication for two variable operands: with
//    q' = -q^-1 mod 2^64 and R = 2^64,
//        z = a*b,  m = (z mod R) * q' mod R,  t = (z + m*q) / R  in [0, 2q)
//    so mont(a, b) = a*b*R^-1 mod q.  Stored operands that are multiplied
//    often (switching keys, the public key, plaintext masks) are kept as
//    x*R mod q so that mont(a, xR) = a*x.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define CSRMF_HD __host__ __device__ __forceinline__
#else
#define CSRMF_HD inline
#endif

namespace csrmf {

CSRMF_HD uint64_t mulhi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul64hi(a, b);
#else
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

CSRMF_HD uint64_t add_mod(uint64_t a, uint64_t b, uint64_t q) {
    uint64_t s = a + b;
    return s >= q ? s - q : s;
}

CSRMF_HD uint64_t sub_mod(uint64_t a, uint64_t b, uint64_t q) {
    return a >= b ? a - b : a + q - b;
}

CSRMF_HD uint64_t neg_mod(uint64_t a, uint64_t q) { return a ? q - a : 0; }

// a * w mod q, w < q, wp = floor(w * 2^64 / q); a may be any 64-bit value.
CSRMF_HD uint64_t mul_shoup(uint64_t a, uint64_t w, uint64_t wp, uint64_t q) {
    uint64_t h = mulhi64(a, wp);
    uint64_t r = a * w - h * q;
    return r >= q ? r - q : r;
}

// Same, result left in [0, 2q).
CSRMF_HD uint64_t mul_shoup_lazy(uint64_t a, uint64_t w, uint64_t wp, uint64_t q) {
    uint64_t h = mulhi64(a, wp);
    return a * w - h * q;
}

// a * b * 2^-64 mod q for a, b < q (or a*b < q*2^64).
CSRMF_HD uint64_t mul_mont(uint64_t a, uint64_t b, uint64_t q, uint64_t qneg_inv) {
    uint64_t lo = a * b;
    uint64_t hi = mulhi64(a, b);
    uint64_t m = lo * qneg_inv;
    uint64_t mh = mulhi64(m, q);
    uint64_t t = hi + mh + (lo != 0 ? 1u : 0u);
    return t >= q ? t - q : t;
}

// Signed integer -> residue.
CSRMF_HD uint64_t from_signed(int64_t x, uint64_t q) {
    if (x >= 0) return (uint64_t)x % q;
    uint64_t r = (uint64_t)(-(x + 1)) % q;   // avoids overflow at INT64_MIN
    return q - 1 - r;
}

// Per-prime constants, shared by host and device.
struct Modulus {
    uint64_t q;
    uint64_t qneg_inv;     // -q^-1 mod 2^64
    uint64_t r_mod;        // 2^64 mod q
    uint64_t r_mod_shoup;
    uint64_t r2_mod;       // 2^128 mod q
    uint64_t n_inv;        // N^-1 mod q
    uint64_t n_inv_shoup;
    uint64_t psi;          // smallest primitive 2N-th root of unity
};

inline uint64_t shoup_pre(uint64_t w, uint64_t q) {
    return (uint64_t)(((unsigned __int128)w << 64) / q);
}

}  // namespace csrmf
