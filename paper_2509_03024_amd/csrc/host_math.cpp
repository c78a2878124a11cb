// Host-side number theory, ChaCha20 sampling and the FP64 CKKS encoder.
#include "host_math.h"

#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

namespace csrmf {

typedef unsigned __int128 u128;

uint64_t mul_mod_host(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((u128)a * b % q); }

uint64_t pow_mod(uint64_t b, uint64_t e, uint64_t q) {
    uint64_t r = 1 % q;
    b %= q;
    while (e) {
        if (e & 1) r = mul_mod_host(r, b, q);
        b = mul_mod_host(b, b, q);
        e >>= 1;
    }
    return r;
}

uint64_t inv_mod(uint64_t a, uint64_t q) { return pow_mod(a, q - 2, q); }  // q prime

bool is_prime_u64(uint64_t n) {
    if (n < 2) return false;
    static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (uint64_t p : bases) {
        if (n % p == 0) return n == p;
    }
    uint64_t d = n - 1;
    int s = 0;
    while ((d & 1) == 0) { d >>= 1; ++s; }
    for (uint64_t a : bases) {
        uint64_t x = pow_mod(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int r = 1; r < s; ++r) {
            x = mul_mod_host(x, x, n);
            if (x == n - 1) { comp = false; break; }
        }
        if (comp) return false;
    }
    return true;
}

bool ntt_primes(int bits, uint64_t N, int count, std::vector<uint64_t>& out) {
    out.clear();
    if (bits < 20 || bits > 61) return false;
    const uint64_t top = 1ull << bits, low = 1ull << (bits - 1), step = 2 * N;
    for (uint64_t j = 1; (int)out.size() < count; ++j) {
        if (j * step >= top - low) return false;
        uint64_t q = top - j * step + 1;
        if (is_prime_u64(q)) out.push_back(q);
    }
    return true;
}

static uint64_t gcd_u64(uint64_t a, uint64_t b) {
    while (b) { uint64_t t = a % b; a = b; b = t; }
    return a;
}

static void factor_rec(uint64_t n, std::vector<uint64_t>& f) {
    if (n == 1) return;
    if (is_prime_u64(n)) { f.push_back(n); return; }
    for (uint64_t c = 1;; ++c) {   // Pollard rho, Floyd cycle detection
        uint64_t x = 2, y = 2, d = 1;
        while (d == 1) {
            x = (mul_mod_host(x, x, n) + c) % n;
            y = (mul_mod_host(y, y, n) + c) % n;
            y = (mul_mod_host(y, y, n) + c) % n;
            d = gcd_u64(x > y ? x - y : y - x, n);
        }
        if (d != n) { factor_rec(d, f); factor_rec(n / d, f); return; }
    }
}

static std::vector<uint64_t> distinct_factors(uint64_t n) {
    std::vector<uint64_t> f;
    for (uint64_t p = 2; p < 1000; ++p) {
        if (n % p == 0) { f.push_back(p); while (n % p == 0) n /= p; }
    }
    factor_rec(n, f);
    std::vector<uint64_t> u;
    for (uint64_t p : f) {
        bool seen = false;
        for (uint64_t v : u) seen |= (v == p);
        if (!seen) u.push_back(p);
    }
    return u;
}

uint64_t smallest_primitive_root_2n(uint64_t q, uint64_t N) {
    const uint64_t order = 2 * N;
    std::vector<uint64_t> fac = distinct_factors(q - 1);
    uint64_t g = 2;
    for (;; ++g) {
        bool gen = true;
        for (uint64_t p : fac) gen &= pow_mod(g, (q - 1) / p, q) != 1;
        if (gen) break;
    }
    // The primitive 2N-th roots are base^k, k odd; take the smallest.
    const uint64_t base = pow_mod(g, (q - 1) / order, q);
    const uint64_t base2 = mul_mod_host(base, base, q);
    uint64_t x = base, best = base;
    for (uint64_t k = 0; k < N; ++k) {
        if (x < best) best = x;
        x = mul_mod_host(x, base2, q);
    }
    return best;
}

// ----------------------------------------------------------------- ChaCha20
static inline uint32_t rotl32(uint32_t x, int n) { return (x << n) | (x >> (32 - n)); }

#define CSRMF_QR(a, b, c, d)                 \
    a += b; d ^= a; d = rotl32(d, 16);        \
    c += d; b ^= c; b = rotl32(b, 12);        \
    a += b; d ^= a; d = rotl32(d, 8);         \
    c += d; b ^= c; b = rotl32(b, 7);

static void chacha20_block(const uint32_t in[16], uint32_t out[16]) {
    uint32_t x[16];
    std::memcpy(x, in, sizeof(x));
    for (int i = 0; i < 10; ++i) {
        CSRMF_QR(x[0], x[4], x[8], x[12]);
        CSRMF_QR(x[1], x[5], x[9], x[13]);
        CSRMF_QR(x[2], x[6], x[10], x[14]);
        CSRMF_QR(x[3], x[7], x[11], x[15]);
        CSRMF_QR(x[0], x[5], x[10], x[15]);
        CSRMF_QR(x[1], x[6], x[11], x[12]);
        CSRMF_QR(x[2], x[7], x[8], x[13]);
        CSRMF_QR(x[3], x[4], x[9], x[14]);
    }
    for (int i = 0; i < 16; ++i) out[i] = x[i] + in[i];
}

void chacha20_words(const uint8_t key[32], uint32_t purpose, uint32_t object, uint32_t limb,
                    uint64_t n_words, uint64_t* out) {
    uint32_t st[16];
    st[0] = 0x61707865u; st[1] = 0x3320646eu; st[2] = 0x79622d32u; st[3] = 0x6b206574u;
    for (int i = 0; i < 8; ++i) {
        st[4 + i] = (uint32_t)key[4 * i] | ((uint32_t)key[4 * i + 1] << 8) |
                    ((uint32_t)key[4 * i + 2] << 16) | ((uint32_t)key[4 * i + 3] << 24);
    }
    st[13] = purpose; st[14] = object; st[15] = limb;
    uint32_t blk[16];
    for (uint64_t w = 0, ctr = 0; w < n_words; ++ctr) {
        st[12] = (uint32_t)ctr;
        chacha20_block(st, blk);
        for (int i = 0; i < 8 && w < n_words; ++i, ++w) {
            out[w] = (uint64_t)blk[2 * i] | ((uint64_t)blk[2 * i + 1] << 32);
        }
    }
}

void sample_uniform(const uint8_t key[32], uint32_t purpose, uint32_t object, uint32_t limb,
                    uint64_t N, uint64_t q, uint64_t* out) {
    std::vector<uint64_t> w(2 * N);
    chacha20_words(key, purpose, object, limb, 2 * N, w.data());
    for (uint64_t n = 0; n < N; ++n) out[n] = (uint64_t)((((u128)w[2 * n]) << 64 | w[2 * n + 1]) % q);
}

void sample_ternary(const uint8_t key[32], uint32_t purpose, uint32_t object, uint64_t N,
                    int64_t* out) {
    std::vector<uint64_t> w(N);
    chacha20_words(key, purpose, object, 0, N, w.data());
    for (uint64_t n = 0; n < N; ++n) out[n] = (int64_t)(w[n] % 3) - 1;
}

void sample_cbd21(const uint8_t key[32], uint32_t purpose, uint32_t object, uint64_t N,
                  int64_t* out) {
    std::vector<uint64_t> w(N);
    chacha20_words(key, purpose, object, 0, N, w.data());
    const uint64_t mask = (1ull << 21) - 1;
    for (uint64_t n = 0; n < N; ++n) {
        out[n] = (int64_t)__builtin_popcountll(w[n] & mask) -
                 (int64_t)__builtin_popcountll((w[n] >> 21) & mask);
    }
}

// ------------------------------------------------------------------ encoder
// In-place radix-2 FFT of length M (power of two), sign = -1 forward
// (sum x_k e^{-2 pi i k n / M}), +1 for the conjugate transform.
static void fft_inplace(std::vector<std::complex<double>>& a, int sign) {
    const size_t M = a.size();
    for (size_t i = 1, j = 0; i < M; ++i) {
        size_t bit = M >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    for (size_t len = 2; len <= M; len <<= 1) {
        const double ang = sign * 2.0 * M_PI / (double)len;
        for (size_t i = 0; i < M; i += len) {
            for (size_t k = 0; k < len / 2; ++k) {
                const std::complex<double> w(std::cos(ang * (double)k), std::sin(ang * (double)k));
                const std::complex<double> u = a[i + k], v = a[i + k + len / 2] * w;
                a[i + k] = u + v;
                a[i + k + len / 2] = u - v;
            }
        }
    }
}

bool ckks_encode(const double* z, int n, int logN, double scale, int64_t* m) {
    const uint64_t N = 1ull << logN, M = 2 * N;
    std::vector<std::complex<double>> A(M, 0.0);
    uint64_t pos = 1;
    for (int j = 0; j < n && (uint64_t)j < N / 2; ++j) {
        A[pos] = z[j];
        pos = pos * 5 % M;
    }
    fft_inplace(A, -1);
    const double f = scale * 2.0 / (double)N;
    for (uint64_t i = 0; i < N; ++i) {
        const double v = std::nearbyint(f * A[i].real());   // default rounding: half to even
        if (!(std::fabs(v) < 9.2e18)) return false;
        m[i] = (int64_t)v;
    }
    return true;
}

void ckks_decode(const int64_t* m, int logN, double scale, double* z, int n) {
    const uint64_t N = 1ull << logN, M = 2 * N;
    std::vector<std::complex<double>> B(M, 0.0);
    for (uint64_t i = 0; i < N; ++i) B[i] = (double)m[i];
    fft_inplace(B, +1);
    uint64_t pos = 1;
    for (int j = 0; j < n && (uint64_t)j < N / 2; ++j) {
        z[j] = B[pos].real() / scale;
        pos = pos * 5 % M;
    }
}

}  // namespace csrmf
