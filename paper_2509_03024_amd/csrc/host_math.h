// Host-side number theory, randomness and the CKKS encoder.
#pragma once
#include <stdint.h>

#include <vector>

namespace csrmf {

bool is_prime_u64(uint64_t n);

// The `count` largest primes q < 2^bits with q = 1 (mod 2N), descending.
// Returns false if fewer exist above 2^(bits-1).
bool ntt_primes(int bits, uint64_t N, int count, std::vector<uint64_t>& out);

// Smallest primitive 2N-th root of unity modulo the prime q.
uint64_t smallest_primitive_root_2n(uint64_t q, uint64_t N);

uint64_t pow_mod(uint64_t b, uint64_t e, uint64_t q);
uint64_t inv_mod(uint64_t a, uint64_t q);
uint64_t mul_mod_host(uint64_t a, uint64_t b, uint64_t q);

// ChaCha20 (RFC 8439) keystream read as little-endian u64 words.  The nonce
// is (purpose, object, limb) as three little-endian u32, counter from 0.
void chacha20_words(const uint8_t key[32], uint32_t purpose, uint32_t object, uint32_t limb,
                    uint64_t n_words, uint64_t* out);

// Stream purposes.
enum : uint32_t {
    kSecret = 1, kPkA = 2, kPkE = 3, kKskA = 4, kKskE = 5,
    kEncV = 6, kEncE0 = 7, kEncE1 = 8, kRefreshMask = 9, kRefreshEnc = 10,
};

// coefficient n = (w[2n]*2^64 + w[2n+1]) mod q
void sample_uniform(const uint8_t key[32], uint32_t purpose, uint32_t object, uint32_t limb,
                    uint64_t N, uint64_t q, uint64_t* out);
// coefficient n = (w[n] mod 3) - 1     (limb field 0)
void sample_ternary(const uint8_t key[32], uint32_t purpose, uint32_t object, uint64_t N,
                    int64_t* out);
// coefficient n = popcount(w & (2^21-1)) - popcount((w >> 21) & (2^21-1))   (limb field 0)
void sample_cbd21(const uint8_t key[32], uint32_t purpose, uint32_t object, uint64_t N,
                  int64_t* out);

// CKKS canonical-embedding encoder for real slot values:
//   m_n = round_half_even(scale * (2/N) * Re sum_j z_j zeta_j^-n),
//   zeta_j = exp(i pi 5^j / N), j < N/2 (missing slots are 0).
// Returns false if a coefficient does not fit in int64.
bool ckks_encode(const double* z, int n, int logN, double scale, int64_t* m);
//   z_j = Re sum_n m_n zeta_j^n / scale, for j < n.
void ckks_decode(const int64_t* m, int logN, double scale, double* z, int n);

}  // namespace csrmf
