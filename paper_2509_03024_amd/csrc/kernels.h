// Launch wrappers of the gfx950 kernels (implemented in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <stdexcept>

#include "modarith.h"

namespace csrmf {

constexpr int kMaxMapRows = 64;

// A set of polynomial rows (each N uint64 residues) addressed as `batch`
// groups of `n` rows.  Row (b, k) starts at
//     P(b) + off(k) * N,   P(b) = ptrs ? ptrs[b] : base + b * batch_stride
// and is reduced modulo chain modulus mod(k); entry k packs (off << 8) | mod.
// Kernels that touch both polynomials of a ciphertext find c1's row at
// c0's row + poly_stride words.
struct RowMap {
    uint64_t* base = nullptr;
    uint64_t* const* ptrs = nullptr;   // device array of `batch` pointers, or null
    int64_t batch_stride = 0;          // words
    int64_t poly_stride = 0;           // words
    int32_t n = 0;
    int32_t batch = 1;
    uint32_t e[kMaxMapRows];

    void push(uint32_t off, uint32_t mod) {
        if (n >= kMaxMapRows || mod > 0xffu || off > 0xffffffu) throw std::length_error("RowMap capacity exceeded");
        e[n++] = (off << 8) | mod;
    }
    int rows() const { return n * batch; }
};

// Primes below this bound use the exact FP64 transform; their twiddle tables
// hold doubles: w and fl(w/q) in place of w and shoup(w).
constexpr uint64_t kFp64PrimeBound = 1ull << 44;
// Basis-conversion targets below this bound sum their products in exact FP64
// (the 40-bit scale primes); see launch_basis_convert for their constants.
constexpr uint64_t kBcFp64Bound = 1ull << 40;
// Words of a basis-conversion target's constant record for ns sources.
constexpr int kBcRecordWords(int ns) { return 2 * ns + 8; }

// Device-resident tables of the modulus chain.
struct DevTables {
    int logN;
    int L1;                      // stages done by the column pass (NTT schedule; ntt_split_valid)
    const Modulus* mods;         // [n_mod]
    const uint64_t* tw;          // [n_mod][4][N]: psi^brev, shoup, psi^-brev, shoup
                                 // (FP64 primes: as doubles, w then fl(w/q))
    int ntt_chunk_rows = 0;      // NTT schedule (host side): rows per pair of passes, 0 = the whole batch
    int ntt_cached_mid = 0;      // NTT schedule: the intermediate between the passes goes through the caches
};

// A pass holds 2^6 to 2^9-point sub-transforms (a rows sub-transform within
// one wave), so the column pass may take L1 stages when both L1 and
// logN - L1 lie in 6..9.  The transform's output does not depend on L1.
inline bool ntt_split_valid(int logN, int L1) { return L1 >= 6 && L1 <= 9 && logN - L1 >= 6 && logN - L1 <= 9; }

void launch_ntt(const DevTables& t, const RowMap& rows, bool inverse, hipStream_t s);
// The same transform of rows that are read from `src` (same shape; its first
// pass reads src, writes rows) and left in `rows`; src is not modified.
void launch_ntt_from(const DevTables& t, const RowMap& rows, const RowMap& src, bool inverse, hipStream_t s);


// out row (b, k) = from_signed(src + b*src_batch_stride + (k % n_src)*N), int64
// coefficients (n_src = 1 broadcasts one signed polynomial to every limb).
void launch_expand_signed(const DevTables& t, const RowMap& out, const int64_t* src, int n_src,
                          int64_t src_batch_stride, hipStream_t s);

// out row (b, k) = the residue mod the row's prime of the centred integer of
// src[b*src_batch_stride + i] (residues mod q0, coefficient form): ModRaise.
void launch_lift_centred(const DevTables& t, const RowMap& out, const uint64_t* src, int64_t src_batch_stride,
                         uint64_t q0, hipStream_t s);

enum EwOp { EW_ADD = 0, EW_SUB = 1, EW_NEG = 2, EW_COPY = 3, EW_F64C = 4, EW_F64U = 5 };
// out = a (op) b (EW_NEG: out = -a; EW_COPY: out = a; EW_F64C: rows of primes
// below 2^44 become their centred values as raw doubles, the others are
// copied; EW_F64U: the inverse of EW_F64C); maps share (n, batch).
void launch_ew(const DevTables& t, EwOp op, const RowMap& out, const RowMap& a, const RowMap& b,
               hipStream_t s);

// out = mont(a, b) = a*b*2^-64 mod q; with b stored as x*2^64 this is a*x.
// If acc != 0, out += mont(a, b) instead.
void launch_mul_mont(const DevTables& t, const RowMap& out, const RowMap& a, const RowMap& b,
                     bool acc, hipStream_t s);

// out = a * c(k), one constant per map entry k: consts[2k] = c, consts[2k+1] = shoup(c)
// (device array).  With both_polys, rows at +poly_stride are treated too.
void launch_mul_const(const DevTables& t, const RowMap& out, const RowMap& a,
                      const uint64_t* consts, bool both_polys, hipStream_t s);

// Tensor product per limb of ciphertexts a and b (evaluation form):
// d0 = a0 b0, d1 = a0 b1 + a1 b0, d2 = a1 b1.  Maps describe the c0 rows; c1
// rows at +poly_stride; d has three polys at +poly_stride steps.
void launch_tensor(const DevTables& t, const RowMap& d, const RowMap& a, const RowMap& b,
                   hipStream_t s);

// Automorphism tau_g in evaluation form: out[k] = in[perm_g(k)] with
// perm_g(k) = brev(((2 brev(k) + 1) g mod 2N - 1) / 2).  both_polys: also rows at +poly_stride.
void launch_automorphism(const DevTables& t, uint32_t g, const RowMap& out, const RowMap& in,
                         bool both_polys, hipStream_t s);

// Fast basis conversion (coefficient form), per batch element:
//   y_i = x_i * [Qhat_i^-1]_{q_i},   out_t = sum_i y_i * [Qhat_i]_t  (mod t)
// src map: n_src (1..16) rows; dst map: n_tgt rows.  Device constants:
//   yc[4i .. 4i+3]              = source i: w = Qhat_i^-1 mod q_i, then
//     q_i below kFp64PrimeBound: doubles (bit patterns) w, fl(w/q_i), q_i, 1/q_i;
//     other sources: w, shoup(w), q_i, 0
//   cc[t*R .. t*R + R-1]        = target t's record, R = kBcRecordWords(n_src) words:
//     target below kBcFp64Bound (with n_src <= 16 centred, <= 8 otherwise):
//       doubles (bit patterns) c_0, d_0, .., c_{n-1}, d_{n-1}
//       (Qhat_i mod t = c_i + d_i 2^20, c_i in [-2^19, 2^19)), then t, 1/t,
//       2^20 mod t, (2^20 mod t)/t, 2^30 mod t, (2^30 mod t)/t, 2^50 mod t, (2^50 mod t)/t;
//     other targets: Qhat_i * 2^64 mod t (Montgomery form) for i < n_src, zeros up
//       to word 2 n_src, which stays 0 (the kind of the record), then t, -t^-1 mod 2^64
// centered: y_i taken in (-q_i/2, q_i/2] (ModUp of key-switching digits), so
// the result is the centred representative mod Q plus a small multiple of Q.
void launch_basis_convert(const DevTables& t, const RowMap& dst, const RowMap& src,
                          const uint64_t* yc, const uint64_t* cc, bool centered, hipStream_t s);

// Key-switching inner product over the extended basis Q_l u P (n_rows = l+1+alpha
// rows): u0[t] = sum_j mont(ext_j[t][perm(k)], kb_j[row(t)]), u1 likewise with
// the key's a part.  ext row (j, t) = ext + b*ext_batch_stride + j*ext_digit_stride
// + t*N; key row (j, t) = key + j*key_digit_stride + row(t)*N with
// row(t) = t for t < n_q and t + key_shift otherwise (special primes); the a
// part is at +key_poly_stride.  Keys are stored times 2^64 (Montgomery form).
// u: map with n = n_rows (u0 rows), u1 rows at +poly_stride.  g != 1 applies
// tau_g to the ext rows on the fly (hoisted rotation).
struct KsArgs {
    const uint64_t* ext;       // ModUp output [batch][digit][limb][N]; a digit's own Q limbs are not stored there
    int64_t ext_batch_stride;
    int64_t ext_digit_stride;
    const uint64_t* key;
    int64_t key_digit_stride;
    int64_t key_poly_stride;
    int32_t n_q;
    int32_t key_shift;
    int32_t n_digits;
    int32_t digit_of[kMaxMapRows];   // Q limb -> the digit that holds it
    RowMap own;                      // the key-switched polynomial itself (evaluation form), rows = Q limbs
    int32_t row0;                    // limb of the first output row (the map's rows are limbs row0, row0+1, ...)
};
void launch_ks_inner(const DevTables& t, const RowMap& u, const KsArgs& a, uint32_t g, hipStream_t s);

// Key-switch tail over the Q limbs q_0..q_l, fused: u = sum_j ext_j * key_j
// (the inner product of launch_ks_inner, Galois element g applied to the ext
// reads), then the ModDown combine out_i = (u_i - conv_i) * P^-1 (mod q_i)
// [+ tau_g_add(addend_i) if addend.n > 0, on both polynomials when
// addend_both, else on poly 0]; consts[2i], +1 = P^-1 mod q_i and its shoup.
// With acc.n > 0 the accumulator acc (both polynomials) is added as well.
// The Q limbs' inner product is never stored.  a.row0 must be 0; out, conv,
// addend and acc have n = l + 1 rows (the Q limbs in order).
void launch_ks_combine(const DevTables& t, const RowMap& out, const KsArgs& a, uint32_t g, const RowMap& conv,
                       const RowMap& addend, uint32_t g_add, bool addend_both, const uint64_t* consts,
                       const RowMap& acc, hipStream_t s);

// Multi-task masked MAC (the inner sums of block permutations): task t
// accumulates into acc[t] (both polynomials, limbs 0..n_limbs-1) its groups
// [grp_begin[t], grp_begin[t+1]), each src[g] (.) M_g with
// M_g = sum_m W_m tau_{gs[m]}(I0) over the group's terms
// [term_begin[g], term_begin[g+1]) (a term with gs[m] = 0 adds the constant W_m),
// formed on the fly from the evaluation-form plaintext I0 (limb k at i0 + k*N);
// cw[2*(wi[m]*cw_stride + k)], +1 = W_m * 2^64 mod q_k and its shoup, or, for
// a prime below 2^44, the centred W_m mod q_k and fl(W_m / q_k) as raw doubles
// (the I0 rows of those limbs hold centred doubles too).
// first[t] != 0: the accumulator starts at zero.  All pointers are device arrays.
struct MaskTasks {
    uint64_t* const* acc;       // [n_tasks] ciphertext base pointers
    const int32_t* grp_begin;   // [n_tasks + 1]
    const int32_t* first;       // [n_tasks]
    const uint64_t* const* src; // [n_groups]
    const int32_t* term_begin;  // [n_groups + 1]
    const uint32_t* gs;         // [n_terms] Galois element of I_p, or 0 for a constant term
    const int32_t* wi;          // [n_terms] row of the term's weight in cw
    const uint64_t* cw;         // [n_weights][cw_stride][2]
    int32_t n_tasks, n_limbs, cw_stride;
    int64_t poly_stride;
};
void launch_mask_mac_tasks(const DevTables& t, const MaskTasks& T, const uint64_t* i0, double bytes, hipStream_t s);

// Kernel arguments are these structs by value: the host and device passes
// must agree on their layout, and the largest argument list (k_ks_combine:
// DevTables, KsArgs, four RowMaps and scalars, about 2 KiB) must stay under
// the 4 KiB kernel-argument limit.
static_assert(sizeof(RowMap) == 296 && alignof(RowMap) == 8, "RowMap layout");
static_assert(sizeof(KsArgs) == 624 && offsetof(KsArgs, own) == 320, "KsArgs layout");
static_assert(sizeof(DevTables) == 32, "DevTables layout");   // two ints share the last 8 bytes
static_assert(sizeof(MaskTasks) == 88, "MaskTasks layout");
static_assert(sizeof(DevTables) + sizeof(KsArgs) + 4 * sizeof(RowMap) + 32 < 4096, "kernel arguments");

// Rescale step 1 (coefficient form top limb, one row per batch element and
// poly): t = (c_l + h) mod q_l with h = floor(q_l/2), then dst row k =
// (t - h) mod q_{mod(k)}; rounding adds h to every coefficient, so it is
// folded in here, in coefficient form.
// top: map with n = 1 (poly 0 row; poly 1 at +poly_stride); dst: n = l rows
// for poly 0 (poly 1 at +poly_stride).
void launch_rescale_spread(const DevTables& t, const RowMap& dst, const RowMap& top,
                           uint32_t top_mod, hipStream_t s);
// Rescale step 2 (evaluation form): out_i = (c_i - T_i) * q_l^-1 mod q_i with
// T_i the transform of step 1's output; consts[4i+1], [4i+2] = q_l^-1 mod q_i
// and its shoup.  Both polys.
void launch_rescale_combine(const DevTables& t, const RowMap& out, const RowMap& c,
                            const RowMap& T, const uint64_t* consts, hipStream_t s);

}  // namespace csrmf
