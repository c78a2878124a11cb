/*
 * csrmf.h -- C ABI of libcsrmf: CKKS arithmetic for encrypted CSR matrix
 * factorisation on one AMD Instinct MI355X (gfx950).
 *
 * The calls follow the problem statement of the paper "Efficient
 * Privacy-Preserving Recommendation on Sparse Data using Fully Homomorphic
 * Encryption" (arXiv 2509.03024):
 *   - the crypto service provider generates the key pair (Sec. III-B,
 *     initialisation phase)                                  -> csrmf_keygen
 *   - non-zero ratings are extracted in CSR order and encrypted
 *     (Alg. 1, EncryptCsrMatrix; CSR layout of Sec. II-A.3)  -> csrmf_encrypt_csr_rows
 *   - the server initialises and encrypts U and V (Alg. 1)   -> csrmf_init_factors
 *   - gradient-descent epochs on encrypted data (Alg. 1 evaluated as a
 *     synchronous epoch, with the per-entity accumulator of Alg. 2)
 *                                                            -> csrmf_mf_epochs
 *   - predicted ratings R_hat = U V^T on the observed set    -> csrmf_predict
 *   - the crypto service provider decrypts (recommendation phase)
 *                                                            -> csrmf_decrypt_*
 * plus the homomorphic primitives of Sec. II-A.2 (Eq. 6-9: ct+ct, ct*ct,
 * ct+pt, ct*pt), the rotations and rescale a leveled CKKS evaluation needs,
 * and import/export hooks that let an independent implementation check the
 * ciphertexts bit for bit.
 *
 * Conventions
 *   - Every call returns 0 on success or a negative CSRMF_E_* code; the
 *     message of the calling thread's last failure is csrmf_last_error().
 *   - The caller owns every host array passed in or out.  Inputs are copied;
 *     outputs are written into caller buffers of the documented size.
 *   - The library owns all device memory and every ciphertext.  A ciphertext is
 *     named by an opaque non-zero uint64_t handle, valid until csrmf_free_ct()
 *     or csrmf_destroy().
 *   - Ciphertexts are kept in HBM in the library's own evaluation (NTT) form.
 *     The external form of a ciphertext (import/export) is coefficient form:
 *     uint64 residues in [0, q_i), laid out [2][level+1][N] (polynomial c0 then
 *     c1, limb q_0 first).
 *   - Calls on one context are serialised by a lock (the serving worker
 *     shares it).  All device work of a context runs in order on its stream;
 *     evaluation calls return once their work is enqueued, calls that return
 *     host data (decrypt, export) or touch caller device memory wait for it.
 *   - A ciphertext at level l has limbs q_0..q_l; q_0 is the base prime and
 *     q_1 > ... > q_L are the scale primes dropped by rescale, smallest first.
 */
#ifndef CSRMF_H
#define CSRMF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CSRMF_OK         0
#define CSRMF_E_INVAL   -1   /* invalid argument or parameter set             */
#define CSRMF_E_NOMEM   -2   /* device or host allocation failed / budget hit  */
#define CSRMF_E_LEVEL   -3   /* not enough levels left for the operation       */
#define CSRMF_E_SCALE   -4   /* operand scales differ by more than 2^-30       */
#define CSRMF_E_STATE   -5   /* call out of order (e.g. no keys yet)           */
#define CSRMF_E_DEVICE  -6   /* HIP runtime error                              */
#define CSRMF_E_KEY     -7   /* the rotation key the operation needs is absent */

typedef struct csrmf_ctx csrmf_ctx;

/* CKKS and matrix-factorisation parameters.
 * Primes: the largest primes q < 2^bits with q = 1 (mod 2N), descending.  The
 * base_bits list gives q_0 and, when special_bits == base_bits, the special
 * primes after it; the scale_bits list gives q_1 > q_2 > ... > q_L.
 * Key-switching digits: D_j = [j*g, min((j+1)*g, L+1)), g = ceil((L+1)/dnum). */
typedef struct csrmf_params {
    int32_t log2N;          /* ring degree N = 2^log2N, 12..16                  */
    int32_t base_bits;      /* bits of q_0 (<= 60)                              */
    int32_t n_scale_primes; /* L, number of scale primes                        */
    int32_t scale_bits;     /* bits of q_1..q_L (<= 60)                         */
    int32_t n_special;      /* alpha, number of special primes (>= 1)           */
    int32_t special_bits;   /* bits of the special primes (<= 60)               */
    int32_t dnum;           /* number of key-switching digits (>= 1)            */
    int32_t log2_scale;     /* default encoding scale Delta = 2^log2_scale      */
    /* matrix factorisation (Alg. 1 / Alg. 2) */
    int32_t k;              /* latent factors per user / item                   */
    double  lr;             /* learning rate alpha                              */
    double  lambda;         /* regularisation lambda (= mu)                     */
    double  damp;           /* dampening: alpha_t = alpha / (1 + damp * t)      */
    int32_t rule;           /* 1 = R1 (Alg. 1 summed), 2 = R2 (degree-normalised)*/
    int32_t refresh_mode;   /* 0 = fail with CSRMF_E_LEVEL when levels run out;  */
                            /* 1 = refresh the factor tables (csrmf_mf_epochs) */
    int32_t batch_pairs;    /* 0 = CSR rows packed greedily, synchronous epochs  */
                            /* (Alg. 1 with the accumulator of Alg. 2);          */
                            /* 1 = user-item batch pairs (Alg. 2, Sec. III-D)   */
} csrmf_params;

/* Create a context (the "encryption context" Alg. 1 takes as input; the CKKS
 * scheme of Sec. II-A.2): derives the prime chain and roots, uploads the
 * transform tables to the current HIP device.  seed is the 32-byte ChaCha20
 * master key from which every random polynomial is drawn.
 * Errors: INVAL (N out of range, not enough primes, k' = 2^ceil(log2 k) too
 * large for the slots), NOMEM, DEVICE. */
int csrmf_create(const csrmf_params* p, const uint8_t seed[32], csrmf_ctx** out);

/* Free every device and host resource of the context.  NULL is ignored. */
void csrmf_destroy(csrmf_ctx* ctx);

/* Message of the calling thread's last failed call, csrmf_create included
 * (empty if that thread's last call succeeded; never NULL).  The pointer
 * stays valid until the thread's next call into the library.  ctx is not
 * used and may be NULL. */
const char* csrmf_last_error(const csrmf_ctx* ctx);

/* Run all further device work of ctx on this hipStream_t (NULL = the null
 * stream).  The stream must outlive its use by the context. */
int csrmf_set_stream(csrmf_ctx* ctx, void* hip_stream);

/* Wait until all device work of the context has finished. */
int csrmf_sync(csrmf_ctx* ctx);

/* Query the modulus chain: q[0..L] then p[0..alpha-1] into moduli (caller
 * array of L+1+alpha entries); any pointer may be NULL. */
int csrmf_get_chain(const csrmf_ctx* ctx, int32_t* L, int32_t* alpha, uint64_t* moduli);

/* Work counters of the context since its creation: key switches enqueued
 * (relinearisations and rotations, each ciphertext of a batch counted once).
 * Errors: INVAL (null pointer). */
int csrmf_counters(const csrmf_ctx* ctx, int64_t* key_switches);

/* Key generation (Sec. III-B: the crypto service provider creates the keys).
 * Creates the secret key s, the public key, the relinearisation key (s^2 -> s)
 * and one rotation key per entry of rot_steps (left rotation by r slots,
 * Galois element 5^(r mod N/2) mod 2N) plus the conjugation key if conj != 0.
 * May be called again to add rotation keys; existing keys are kept.
 * Errors: NOMEM, DEVICE. */
int csrmf_keygen(csrmf_ctx* ctx, const int32_t* rot_steps, int32_t n_steps, int32_t conj);

/* ------------------------------------------------------------------------ */
/* Ciphertexts and the homomorphic primitives (Sec. II-A.2, Eq. 6-9).        */
/* ------------------------------------------------------------------------ */

/* Encode a real vector (n <= N/2 slots, the rest 0) at the given scale and
 * encrypt it at `level` with the public key.  The integer plaintext is
 * m_n = round_half_even(scale * (2/N) * Re sum_j z_j zeta_j^-n),
 * zeta_j = exp(i*pi*5^j/N).  Errors: INVAL, STATE (no keys). */
int csrmf_encrypt(csrmf_ctx* ctx, const double* z, int32_t n, int32_t level, double scale,
                  uint64_t* handle);

/* Encrypt an integer plaintext polynomial m[N] (signed coefficients) at
 * `level`; `scale` is recorded as metadata only. */
int csrmf_encrypt_int(csrmf_ctx* ctx, const int64_t* m, int32_t level, double scale,
                      uint64_t* handle);

/* Decrypt: m = c0 + c1*s kept mod q_0 and centred, into m[N] (int64). */
int csrmf_decrypt_int(csrmf_ctx* ctx, uint64_t handle, int64_t* m);

/* Decrypt and decode the first n slots into z[n] (real parts). */
int csrmf_decrypt(csrmf_ctx* ctx, uint64_t handle, double* z, int32_t n);

/* The host encoder/decoder on their own (FP64). */
int csrmf_encode(const csrmf_ctx* ctx, const double* z, int32_t n, double scale, int64_t* m);
int csrmf_decode(const csrmf_ctx* ctx, const int64_t* m, double scale, double* z, int32_t n);

/* Import / export a ciphertext in coefficient form ([2][level+1][N] uint64). */
int csrmf_import_ct(csrmf_ctx* ctx, const uint64_t* coeffs, int32_t level, double scale,
                    uint64_t* handle);
int csrmf_export_ct(csrmf_ctx* ctx, uint64_t handle, uint64_t* coeffs, int32_t* level,
                    double* scale);
int csrmf_ct_info(const csrmf_ctx* ctx, uint64_t handle, int32_t* level, double* scale);
int csrmf_free_ct(csrmf_ctx* ctx, uint64_t handle);

/* Export the key material in coefficient form (test hook):
 * which = 0: secret key s over all limbs, [L+1+alpha][N];
 * which = 1: public key (b, a), [2][L+1][N];
 * which = 2: relinearisation key, [dnum][2][L+1+alpha][N] (digit, b/a, limb);
 * which = 3: rotation key of Galois element `galois`, same layout as 2.
 * Residues in [0, q). */
int csrmf_export_key(csrmf_ctx* ctx, int32_t which, uint32_t galois, uint64_t* out);

/* Eq. 6 and its inverse.  Operands at different levels are aligned by
 * dropping the higher one's top limbs; scales must agree to 2^-30 (SCALE);
 * the result takes a's scale.  out receives a new handle. */
int csrmf_add(csrmf_ctx* ctx, uint64_t a, uint64_t b, uint64_t* out);
int csrmf_sub(csrmf_ctx* ctx, uint64_t a, uint64_t b, uint64_t* out);

/* Batched Eq. 6: out[i] = a[i] + b[i] (or a[i] - b[i] if subtract != 0) in
 * one launch; all operands at one level after alignment. */
int csrmf_add_batch(csrmf_ctx* ctx, const uint64_t* a, const uint64_t* b, int32_t n, int32_t subtract,
                    uint64_t* out);

/* Eq. 8: add the integer plaintext polynomial m[N]. */
int csrmf_add_plain(csrmf_ctx* ctx, uint64_t a, const int64_t* m, uint64_t* out);

/* Eq. 9: multiply by the integer plaintext polynomial m[N] whose scale is
 * pt_scale (result scale = scale * pt_scale; no rescale). */
int csrmf_mul_plain(csrmf_ctx* ctx, uint64_t a, const int64_t* m, double pt_scale, uint64_t* out);

/* Multiply by the integer constant w (result scale = scale * w). */
int csrmf_mul_int(csrmf_ctx* ctx, uint64_t a, int64_t w, uint64_t* out);

/* Eq. 7: tensor product, relinearisation (s^2 -> s key switch) and rescale,
 * in that order.  Result level = min(level) - 1.  Errors: LEVEL, STATE. */
int csrmf_hmult(csrmf_ctx* ctx, uint64_t a, uint64_t b, uint64_t* out);

/* Tensor product + relinearisation without rescale. */
int csrmf_mul_relin(csrmf_ctx* ctx, uint64_t a, uint64_t b, uint64_t* out);

/* Rescale: divide by q_l with rounding half up, drop limb l, scale /= q_l. */
int csrmf_rescale(csrmf_ctx* ctx, uint64_t a, uint64_t* out);

/* Drop the top limbs down to `level` (scale unchanged). */
int csrmf_mod_drop(csrmf_ctx* ctx, uint64_t a, int32_t level, uint64_t* out);

/* Left rotation by r slots (slot j takes old slot j + r), non-hoisted key
 * switch: (tau_g(c0) + u0, u1), (u0, u1) = KS_{tau_g(s) -> s}(tau_g(c1)).
 * Errors: KEY (no key for this step). */
int csrmf_rotate(csrmf_ctx* ctx, uint64_t a, int32_t r, uint64_t* out);

/* Allocation-free variant of csrmf_rotate, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the rotation by r of ciphertext a is written into
 * the existing ciphertext `out` (any handle of this context other than a; its
 * level and scale become a's), and every temporary lives in one static
 * 128 MiB device buffer of the library (one per device, held until the
 * process ends).  The call allocates nothing: no hipMalloc, no pool block, no
 * staging.  Same bits as csrmf_rotate.
 * Limit: the rotation's scratch, 8 N ((l+1) * 3 + dnum_l * (l+1+alpha) +
 * 2 (l+1+alpha)) bytes at level l (dnum_l = digits present at that level),
 * must fit in 128 MiB: every level of the N <= 2^15 chains and of the
 * N = 2^16 chain with 3 digits does; with 4-limb digits at N = 2^16, levels
 * up to 20 do.
 * Calls on one device share the buffer; they are ordered on one context's
 * stream, but calls on two contexts (or streams) of one device that overlap
 * in time race.  Errors: INVAL (a == out, unknown handle, scratch too
 * large), KEY. */
int csrmf_rotate_noalloc(csrmf_ctx* ctx, uint64_t a, int32_t r, uint64_t out);

/* Complex conjugation of the slots (Galois element 2N-1). */
int csrmf_conjugate(csrmf_ctx* ctx, uint64_t a, uint64_t* out);

/* Several rotations of one ciphertext sharing one ModUp of c1 (hoisting);
 * tau_g is applied to the extended digits.  out[n] receives n handles. */
int csrmf_rotate_hoisted(csrmf_ctx* ctx, uint64_t a, const int32_t* r, int32_t n, uint64_t* out);

/* Batched forms: the same operation over n ciphertexts in as few launches as
 * possible (all operands must share level and scale).  out[n] receives new
 * handles; out may alias nothing. */
int csrmf_hmult_batch(csrmf_ctx* ctx, const uint64_t* a, const uint64_t* b, int32_t n,
                      uint64_t* out);
int csrmf_rotate_batch(csrmf_ctx* ctx, const uint64_t* a, int32_t n, int32_t r, uint64_t* out);
/* out[i] = acc[i] + Rot(a[i], r), the step of a rotate-and-sum (Sec. III-C:
 * the dot products over a block are summed by rotations), with the addition
 * fused into the key switch's last kernel.  acc[i] must have a[i]'s scale and
 * at least its level; the result has a[i]'s level.  acc may equal a. */
int csrmf_rotate_add_batch(csrmf_ctx* ctx, const uint64_t* a, const uint64_t* acc, int32_t n, int32_t r,
                           uint64_t* out);
int csrmf_conjugate_batch(csrmf_ctx* ctx, const uint64_t* a, int32_t n, uint64_t* out);

/* ------------------------------------------------------------------------ */
/* Bootstrapping (renews the levels of a ciphertext without decrypting it).   */
/* ------------------------------------------------------------------------ */

/* Sec. IV-C claims that the factorisation runs without communication; the
 * epochs use levels the paper gives no way to renew.  Bootstrapping renews
 * them on the device by the published method for approximate homomorphic
 * encryption (Cheon, Han, Kim, Kim, Song, EUROCRYPT 2018), sparse packing:
 * ModRaise, SubSum (the trace onto Z[X^(N/2n)]), CoeffToSlot, EvalMod
 * (exp(i theta) by a Taylor series of degree `degree`, squared `squarings`
 * times, minus its conjugate) and SlotToCoeff.
 *   n_slots    n: the message's slots repeat with period n (power of two,
 *              1..N/4: the linear maps use 2n-periodic vectors); the
 *              output's slots repeat with the same period;
 *   squarings  r: the series' argument is 2 pi (m/q_0 + I) / 2^r, where
 *              |I| (about sqrt(N/18) for the dense ternary secret) must stay
 *              below K with 2 pi (K + 1/2) / 2^r below about 0.8;
 *   degree     d (1..18): the series' degree (11 keeps its error below 2^-32
 *              for arguments up to 0.8);
 *   pre_bits   the level-0 input is multiplied by 2^pre_bits before ModRaise,
 *              so that the message uses about 2^-8 of q_0 (2^-6 with arcsine;
 *              precision against the linearisation sin x ~ x);
 *   arcsine    1: after EvalMod, D - D^3/24 (D = 2 i sin), the cubic term of
 *              arcsin, two more levels; 0: none. */
typedef struct csrmf_boot_config {
    int32_t n_slots;
    int32_t squarings;
    int32_t degree;
    int32_t pre_bits;
    int32_t arcsine;
} csrmf_boot_config;

/* Levels one bootstrap consumes: 2 + ceil(log2 degree) + 1 + squarings
 * (+ 2 with arcsine) + 1.
 * Errors: INVAL (null arguments). */
int csrmf_boot_levels(const csrmf_boot_config* cfg, int32_t* levels);

/* The rotation steps whose keys csrmf_bootstrap needs (1 .. 2n-1 and n 2^j
 * below N/2), ascending, into steps[cap]; *count receives their number (also
 * when cap is too small, then with CSRMF_E_INVAL).  Relinearisation and
 * conjugation keys are needed too (csrmf_keygen with conj = 1). */
int csrmf_boot_rotation_steps(csrmf_ctx* ctx, const csrmf_boot_config* cfg, int32_t* steps, int32_t cap,
                              int32_t* count);

/* Bootstrap the ciphertexts in[0..n) (one scale shared by all, any level; the
 * top limbs above level 0 are ignored) into new handles out[0..n), at level
 * L - csrmf_boot_levels(cfg) and a scale of about 2^log2_scale, every step on
 * the whole batch in the library's kernels.  The outputs decrypt to the
 * inputs' slot values up to the method's error, for |values| <= 1: about
 * 4e-4 on the N = 2^12 test chain (r = 9, pre_bits 12), 3e-5 there with the
 * arcsine term (r = 8, pre_bits 15), about 5e-3 at N = 2^16 (r = 10,
 * pre_bits 15, arcsine term).  Errors: INVAL (configuration, handles),
 * LEVEL (chain too short), SCALE (scales differ), STATE (no keys), KEY (a
 * needed key is absent: nothing is enqueued). */
int csrmf_bootstrap(csrmf_ctx* ctx, const csrmf_boot_config* cfg, const uint64_t* in, int32_t n,
                    uint64_t* out);

/* ------------------------------------------------------------------------ */
/* Raw transforms on caller device memory (test and benchmark hooks).        */
/* ------------------------------------------------------------------------ */

/* In-place negacyclic NTT (inverse != 0: inverse NTT) of n_rows rows of N
 * uint64 residues at device pointer `data` (row r at data + r*N), row r
 * reduced modulo chain limb limb_idx[r % n_idx] (0..L for q_i, L+1+k for
 * p_k).  Forward output position t holds a(psi^(2*brev(t)+1)), with brev the
 * log2N-bit reversal and psi the smallest primitive 2N-th root mod the limb's
 * prime.  Inputs must be reduced.  limb_idx is a host array.  The context's
 * stream does not wait for other streams: writes to `data` must be complete
 * when the call is made; the transform is complete when it returns. */
int csrmf_ntt_rows(csrmf_ctx* ctx, uint64_t* data, int32_t n_rows, const int32_t* limb_idx,
                   int32_t n_idx, int32_t inverse);

/* ------------------------------------------------------------------------ */
/* Serving: encrypted per-user requests against resident factor tables.     */
/* ------------------------------------------------------------------------ */

typedef struct csrmf_server csrmf_server;

/* Create a request server on ctx (keys must exist).  The factor tables U[n_users*k]
 * and V[n_items*k] (row-major) are encrypted once and stay resident in HBM with
 * the baby-step rotations of the gathers; the rotation keys the requests need
 * are generated if missing.  A worker thread admits queued requests while
 * their ciphertext footprint (about 16 ciphertexts per row chunk) fits in
 * what hbm_budget_bytes leaves beside the batches still on the device,
 * enqueues each batch (at most max_batch requests) without waiting for it,
 * and pipelines up to four batches on the context's stream (continuous
 * batching); a request is done, and its footprint returned, when its batch's
 * completion event has fired.
 * Errors: INVAL, STATE, NOMEM, DEVICE, LEVEL (a chain of fewer than 2 levels). */
int csrmf_server_create(csrmf_ctx* ctx, int32_t n_users, int32_t n_items, const double* U, const double* V,
                        double hbm_budget_bytes, int32_t max_batch, csrmf_server** out);

/* csrmf_server_create with the tables given as integer plaintexts (the
 * caller's encodings, so that an independent implementation can check the
 * results bit for bit): utab[ceil(n_users/D)][N], vtab[ceil(n_items/D)][N]
 * (entity a*D + b at block b, k factors in slots bB..bB+k-1, scale
 * 2^log2_scale) and mask_gather[N], the indicator of slots 0..k-1 encoded at
 * 2^(log2_scale - 10).  The tables are encrypted at the top level with the context's running
 * serial numbers, the U tables first.  Errors as csrmf_server_create. */
int csrmf_server_create_int(csrmf_ctx* ctx, int32_t n_users, int32_t n_items, const int64_t* utab,
                            const int64_t* vtab, const int64_t* mask_gather, double hbm_budget_bytes,
                            int32_t max_batch, csrmf_server** out);

/* Queue a request: op 0 = PREDICT (r_hat = <u_user, v_j> for the row's items),
 * op 1 = UPDATE (one R2 gradient step of u_user on the row:
 * u' = (1 - lr*lambda) u + (lr/d) sum_j (r_j - <u, v_j>) v_j; items stay fixed).
 * items[n]: the row's item ids, increasing; ratings[n]: the row's ratings
 * (UPDATE only; chunk c of the row is encoded in slots tB..tB+k-1 of block t
 * and encrypted on admission at the top level with encryption serial
 * 0x40000000 + 8 * client_serial + c, so equal requests give equal
 * ciphertexts).  client_serial < 2^27; an UPDATE may not reuse the serial of
 * an earlier UPDATE on the same server (the randomness would repeat).  Rows
 * longer than D blocks are cut into up to 8 chunks.  id receives the request
 * id.  A PREDICT uses 2 levels of the chain, an UPDATE 4.
 * Errors: INVAL (also a reused UPDATE serial), NOMEM (the request alone
 * exceeds the budget), LEVEL (an UPDATE on a chain of fewer than 4 levels). */
int csrmf_server_submit(csrmf_server* s, int32_t op, int32_t user, int32_t n, const int32_t* items,
                        const double* ratings, uint32_t client_serial, uint64_t* id);

/* csrmf_server_submit with an UPDATE's rating chunks already encoded by the
 * client: plain[ceil(n/D)][N] (int64), NULL for a PREDICT. */
int csrmf_server_submit_int(csrmf_server* s, int32_t op, int32_t user, int32_t n, const int32_t* items,
                            const int64_t* plain, uint32_t client_serial, uint64_t* id);

/* Status of a request (wait != 0: block until it finishes): 0 queued,
 * 1 running, 2 done, or a negative error code (also returned).  When done,
 * the result handles (owned by the caller, freed with csrmf_free_ct) go to
 * results[cap]: PREDICT one ciphertext per row chunk, slot t*B holding
 * r_hat of the chunk's t-th item; UPDATE one ciphertext with u' in slots
 * 0..k-1.  latency_s = completion - submission time. */
int csrmf_server_poll(csrmf_server* s, uint64_t id, int32_t wait, int32_t* status, uint64_t* results,
                      int32_t cap, int32_t* n_results, double* latency_s);

/* JSON counters (batches, processed, largest batch, queue length, bytes in
 * flight, budget) into buf (NUL-terminated, truncated to cap); returns the
 * full length. */
int csrmf_server_stats(csrmf_server* s, char* buf, int32_t cap);

/* Stop the worker (finishing the batch on the device) and free the server. */
void csrmf_server_destroy(csrmf_server* s);

/* ------------------------------------------------------------------------ */
/* Schedule autotuning.                                                      */
/* ------------------------------------------------------------------------ */

/* Time the candidate NTT schedules (rows transformed per pair of passes, the
 * intermediate cached or streamed, the split of the stages between the two
 * passes) on `rows` limbs of this context's ring
 * (0: 64 ciphertexts x 2 x (L+1) limbs, the batched key-switching shape) and,
 * if the context has a rotation key, rank the four fastest of them again and
 * then the ModUp sub-batch sizes on batched rotations of up to 64 zero
 * ciphertexts, with HIP events, and keep the fastest for all later work of
 * this context.  Writes a JSON report of the timings into
 * report (NUL-terminated, truncated to cap bytes; may be NULL).
 * Errors: NOMEM, DEVICE. */
int csrmf_autotune(csrmf_ctx* ctx, int32_t rows, char* report, int32_t cap);

/* Fix this context's NTT schedule instead of tuning it: transform chunk_rows
 * rows per pair of passes (0: the whole batch at once).  For repeatable
 * profiles.  Results do not depend on the schedule.  Errors: INVAL (negative). */
int csrmf_set_ntt_schedule(csrmf_ctx* ctx, int32_t chunk_rows);

/* The whole schedule of this context: NTT rows per pair of passes (0: the
 * whole batch), whether the intermediate between the two passes goes through
 * the caches (1) or is streamed past them (0), and ciphertexts per ModUp
 * sub-batch of a key switch (0: the whole batch; a sub-batch runs its inverse
 * transform, conversions and forward transforms before the next, so a small
 * one keeps each stage's output in the last-level cache), and the split of
 * the transform into its two passes: ntt_split of the log2 N butterfly
 * stages in the column pass, the rest in the row pass, each pass taking 6 to
 * 9 (0: log2 N / 2; a column pass of s stages reads runs of 2^(12-s)
 * consecutive residues).  Results do not depend on the schedule.
 * csrmf_autotune chooses all four (the ModUp sub-batch only when the context
 * has a rotation key).  Errors: INVAL (a negative value, a split outside
 * that range). */
int csrmf_set_schedule(csrmf_ctx* ctx, int32_t ntt_chunk_rows, int32_t ntt_cached_mid, int32_t modup_chunk,
                       int32_t ntt_split);
int csrmf_get_schedule(const csrmf_ctx* ctx, int32_t* ntt_chunk_rows, int32_t* ntt_cached_mid, int32_t* modup_chunk,
                       int32_t* ntt_split);

/* ------------------------------------------------------------------------ */
/* HIP graphs of evaluation sequences.                                       */
/* ------------------------------------------------------------------------ */

/* Record instead of run: after csrmf_graph_begin the context's evaluation
 * calls (add, mul_int, hmult, relinearise, rescale, rotations, their batched
 * forms, free_ct) are captured from the context's stream into a HIP graph
 * until csrmf_graph_end, which instantiates it and returns its id; nothing
 * runs until csrmf_graph_launch, which replays the whole sequence on the
 * stream.  Calls that wait for the device (encryption, decryption, export,
 * keys, csrmf_ntt_rows, csrmf_sync) fail with STATE while capturing.  The
 * ciphertexts the captured calls create are the graph's buffers: every launch
 * writes them again, from the inputs as they are at launch time; handles
 * freed during the capture may be reused only within it; all of the graph's
 * memory (its buffers and a 32 MiB pinned argument arena) is freed by
 * csrmf_graph_destroy, after which handles created during the capture must
 * not be used.  Per-kernel profiling must be off while capturing.
 * Errors: STATE (capture open or not open, profiling on), NOMEM, DEVICE,
 * INVAL (unknown graph). */
int csrmf_graph_begin(csrmf_ctx* ctx);
int csrmf_graph_end(csrmf_ctx* ctx, uint64_t* graph);
int csrmf_graph_launch(csrmf_ctx* ctx, uint64_t graph);
int csrmf_graph_destroy(csrmf_ctx* ctx, uint64_t graph);

/* ------------------------------------------------------------------------ */
/* Per-kernel timing (benchmark hook; process-wide).                         */
/* ------------------------------------------------------------------------ */

/* enable != 0: clear the records and bracket every later kernel launch of the
 * library with two HIP events on the launch stream; 0: stop recording. */
int csrmf_profile_enable(int32_t enable);

/* Write {"kernel": [launches, total_ms], ...} for the recorded launches into
 * buf (NUL-terminated, truncated to cap bytes).  Synchronises on the recorded
 * events.  Returns the length of the full report. */
int csrmf_profile_report(char* buf, int32_t cap);

/* ------------------------------------------------------------------------ */
/* Encrypted CSR matrix factorisation (Alg. 1 / Alg. 2).                     */
/* ------------------------------------------------------------------------ */

/* With params.batch_pairs = 1 the ratings are grouped by user-item batch
 * pair instead (Sec. III-D, Alg. 2): a batch is one factor-table ciphertext
 * (D profiles: user i is local index i mod D of batch i div D, items
 * likewise), the pairs come in the order of their first rating in CSR order,
 * and each pair's ratings (CSR order) fill rating ciphertexts of their own.
 *
 * Pack the CSR rating matrix (n_rows users x n_cols items; row_ptr[n_rows+1],
 * col_idx[nnz] sorted within a row, values[nnz]) into block layout and encrypt
 * it (Alg. 1 EncryptCsrMatrix).  With k' = 2^ceil(log2 k), block width B = 2k'
 * and D = N/(2B) blocks per ciphertext, rows are packed greedily in CSR order;
 * a row that does not fit in the current ciphertext starts a new one and a
 * row longer than D is split into chunks of D.  Block t of a rating
 * ciphertext holds r_ij in slots tB..tB+k-1.  n_ct receives the number of
 * rating ciphertexts.  The rotation keys the program needs (windowed sum:
 * 1, 2, .., B/2 and -k'; block permutations: beta*B and gamma*G*B with
 * G = 2^ceil(log2(D)/2)) are generated here if missing.  Errors: INVAL
 * (row_ptr not monotone, columns unsorted, duplicated or out of range, NaN),
 * STATE (no keys). */
int csrmf_encrypt_csr_rows(csrmf_ctx* ctx, int32_t n_rows, int32_t n_cols, const int64_t* row_ptr,
                           const int32_t* col_idx, const double* values, int32_t* n_ct);

/* Same as csrmf_encrypt_csr_rows but each rating ciphertext's plaintext is
 * supplied already encoded: plain[n_ct][N] (int64).  Used to check the
 * evaluation bit for bit independently of floating-point encoding. */
int csrmf_encrypt_csr_rows_int(csrmf_ctx* ctx, int32_t n_rows, int32_t n_cols,
                               const int64_t* row_ptr, const int32_t* col_idx,
                               const int64_t* plain, int32_t n_plain, int32_t* n_ct);

/* Encrypt the initial factors (Alg. 1: the server draws and encrypts U and V):
 * U0[n_rows*k], V0[n_cols*k] row-major.  Creates the factor tables (user a*D+b
 * at block b of table ciphertext a, likewise items) and the gathered copies
 * in the rating layout (u_i and v_j in the slots of every rating (i, j)).
 * Errors: STATE (no ratings encrypted yet). */
int csrmf_init_factors(csrmf_ctx* ctx, const double* U0, const double* V0);

/* Integer-plaintext form of csrmf_init_factors plus the block indicator masks:
 * utab[n_utab][N], vtab[n_vtab][N], ug[n_ct][N], vg[n_ct][N];
 * mask_scatter[N] and mask_gather[N] = encodings of the indicator of slots
 * 0..k-1 at scales 2^(log2_scale - 16) (scatters) and 2^(log2_scale - 10)
 * (gathers, whose weights are all 1): 2^24 and 2^30 at log2_scale = 40.
 * Counts are reported by csrmf_mf_layout.  Errors: INVAL (null pointer), STATE. */
int csrmf_init_factors_int(csrmf_ctx* ctx, const int64_t* utab, const int64_t* vtab,
                           const int64_t* ug, const int64_t* vg, const int64_t* mask_scatter,
                           const int64_t* mask_gather);

/* Layout counts: rating ciphertexts, user-table and item-table ciphertexts,
 * blocks per ciphertext D and block width B. */
int csrmf_mf_layout(const csrmf_ctx* ctx, int32_t* n_ct, int32_t* n_utab, int32_t* n_vtab,
                    int32_t* D, int32_t* B);

/* With params.batch_pairs = 1 an epoch is Alg. 2: the batch pairs in turn,
 * each from the tables as they are when it starts: gather of its user table
 * and item table into its rating ciphertexts, dot products, errors, gradient
 * terms, and the scatter into those two tables with weight a_t per rating
 * and self term (1 - a_t*lambda*c) (c = the entity's ratings in the pair; 1
 * for entities without one); a pair costs 4 levels of its tables, and all
 * tables are refreshed (refresh_mode = 1) before a pair whose tables are
 * below level 4.  Forward predictions are those at the start of each
 * rating's pair.
 *
 * Run n_epochs synchronous encrypted gradient-descent epochs.  Each epoch
 * computes for every rating ciphertext P = Ug*Vg, the block dot products by a
 * windowed rotate-and-sum, E = R - <u,v>, the gradient terms E*Vg and E*Ug,
 * scatters them into the factor tables (held at scale 2^(log2_scale + 10)) with the
 * learning-rate weights and the (1 - alpha*lambda*...) self term; every
 * further epoch first gathers the factors back into the rating layout.  The
 * first epoch on gathered factors costs 3 levels, each further one 4.
 * Rule 1: weights alpha_t and self term 1 - alpha_t*lambda*d; rule 2: alpha_t/d
 * and 1 - alpha_t*lambda (entities without ratings are left unchanged).
 * alpha_t = lr / (1 + damp * t), t = epochs run so far.
 * With params.refresh_mode = 1, tables below level 4 are refreshed before a
 * gather, following the masking step of the protocol (Sec. III-B): a mask
 * polynomial (ChaCha20 purpose 9, object round*1024 + table, coefficients
 * (w mod 2^51) - 2^50) is added, the key holder decrypts to integers mod q_0
 * and encrypts them anew at the top level and the same scale (serial
 * 0x20000000 + round*1024 + table), and the mask is subtracted.
 * Errors: LEVEL (not enough levels, refresh off or chain shorter than 4),
 * STATE, DEVICE. */
int csrmf_mf_epochs(csrmf_ctx* ctx, int32_t n_epochs);

/* Memory bound of the block permutations (scatters and gathers): at most
 * max_babies baby-step rotations of the sources (ciphertexts of the source's
 * size) are alive at once; sources are processed in chunks that respect it
 * (default 1024).  Every baby is built the same way in any chunk and the
 * sums are exact, so results do not depend on it.  Errors: INVAL (< 1). */
int csrmf_set_baby_budget(csrmf_ctx* ctx, int32_t max_babies);

/* Encrypted predictions r_hat = <u_i, v_j> on the observed ratings from the
 * current factor tables (gather + product + windowed sum): Alg. 1's encrypted
 * R_hat = U V^T restricted to the rated cells, the set Eq. 10 is evaluated on.
 * Errors: LEVEL. */
int csrmf_predict(csrmf_ctx* ctx);

/* Decrypt the factor tables (the key holder's decryption, Sec. III-B,
 * recommendation phase): U[n_rows*k], V[n_cols*k] row-major.  Errors: STATE. */
int csrmf_decrypt_factors(csrmf_ctx* ctx, double* U, double* V);

/* Decrypt predictions on the observed ratings (Sec. III-B, recommendation
 * phase; the r_hat of Eq. 10), in CSR order, into rhat[nnz]:
 * which = 0: the forward predictions of the last epoch (epoch-start factors);
 * which = 1: the output of csrmf_predict.  Errors: STATE, INVAL. */
int csrmf_decrypt_predictions(csrmf_ctx* ctx, double* rhat, int32_t which);

/* Progress of the MF program since csrmf_init_factors: epochs run, table
 * refreshes done, and the wall time spent in refreshes (seconds, device work
 * included).  Any pointer may be NULL.  Errors: STATE. */
int csrmf_mf_stats(const csrmf_ctx* ctx, int32_t* epochs_done, int32_t* refreshes, double* refresh_seconds);

/* Work of the masked multiply-accumulate (the BlockPermute MAC of the MF
 * program) since csrmf_init_factors, into counts[7]: accumulators (tasks),
 * source ciphertexts (groups), mask terms, constant terms, and tasks, groups
 * and mask terms each multiplied by the limbs of their launch (one limb row
 * is N residues).  Errors: INVAL (counts NULL), STATE. */
int csrmf_mf_mac_counts(const csrmf_ctx* ctx, int64_t* counts);

/* Handles of the program's ciphertexts (test hook; owned by the program, do
 * not free): which = 0 rating ciphertexts, 1 user tables, 2 item tables,
 * 3 gathered users, 4 gathered items, 5 forward dot products of the last
 * epoch, 6 the output of csrmf_predict.  Writes up to `cap` handles into out
 * and the count into n. */
int csrmf_mf_handles(const csrmf_ctx* ctx, int32_t which, uint64_t* out, int32_t cap, int32_t* n);

/* ------------------------------------------------------------------------ */
/* The three-party protocol (Sec. III-B) with message accounting.            */
/* ------------------------------------------------------------------------ */

/* Initialization phase of the protocol between the users, the recommendation
 * server (RS) and the crypto service provider (CSP, the key holder; keys from
 * csrmf_keygen), played on one context with every message serialised and
 * counted: each user encrypts its CSR row with pk (one rating per slot,
 * encryption serial 0x50000000 + 64 * user + chunk) and sends it to the RS;
 * the RS adds a mask per rating (ChaCha20 purpose 12, object = rating index:
 * ((w mod 2^21) - 2^20) / 2^10) and sends the result to the CSP; the CSP
 * decrypts the masked ratings, packs them in the CSR block layout of
 * csrmf_encrypt_csr_rows and encrypts them (serial 0x58000000 + ciphertext
 * index) for the RS, which removes its masks.  The result replaces the MF
 * program's rating ciphertexts, as csrmf_encrypt_csr_rows does; n_ct receives
 * their count.  Errors as csrmf_encrypt_csr_rows. */
int csrmf_protocol_ingest(csrmf_ctx* ctx, int32_t n_rows, int32_t n_cols, const int64_t* row_ptr,
                          const int32_t* col_idx, const double* values, int32_t* n_ct);

/* Recommendation phase: the RS masks the encrypted predictions (which = 0:
 * the last epoch's forward predictions, 1: csrmf_predict's; masks from
 * ChaCha20 purpose 13 as above) and sends them to the CSP, which decrypts
 * them and sends the masked plaintext predictions to the users; the RS sends
 * the users the masks, and the users remove them.  rhat[nnz] receives the
 * users' predictions in CSR order.  Errors: STATE, INVAL. */
int csrmf_protocol_recommend(csrmf_ctx* ctx, int32_t which, double* rhat);

/* Messages and bytes per channel since the last csrmf_protocol_ingest,
 * msgs[8] and bytes[8]: 0 CSP->users (public key), 1 CSP->RS (public and
 * evaluation keys), 2 users->RS (encrypted rows), 3 RS->CSP (masked rows),
 * 4 CSP->RS (re-packed rating ciphertexts), 5 RS->CSP (masked encrypted
 * predictions), 6 CSP->users (masked plaintext predictions, 8 bytes each),
 * 7 RS->users (prediction masks, 8 bytes each).  A ciphertext message is
 * 2 (level+1) N 8 bytes.  Errors: INVAL (null pointer). */
int csrmf_protocol_counters(const csrmf_ctx* ctx, int64_t* msgs, int64_t* bytes);

#ifdef __cplusplus
}
#endif
#endif /* CSRMF_H */
