// Internal pieces of the encrypted MF program shared with the serving loop.
#pragma once
#include <cmath>
#include <map>
#include <utility>
#include <vector>

#include "context.h"

namespace csrmf {

struct MfState {
    int k = 0, kp = 0, B = 0, D = 0, G = 0;
    int n_users = 0, n_items = 0, nnz = 0;
    int n_ct = 0, n_utab = 0, n_vtab = 0;
    std::vector<int64_t> row_ptr;
    std::vector<int32_t> col_idx;
    std::vector<int32_t> rows, ct_of, blk_of;
    std::vector<double> deg_u, deg_v;
    std::vector<uint64_t> R, Utab, Vtab, Ug, Vg, Sdot, Pred;   // handles
    // I0 in evaluation form [L+1][N]: canonical residues, or centred raw
    // doubles in the rows of primes below 2^44 (the masked MAC's FP64 form)
    uint64_t* mask0 = nullptr;      // at the scatter mask scale
    uint64_t* maskg = nullptr;      // at the gather mask scale
    // Alg. 2 (params.batch_pairs): the user-item batch pairs in order, each
    // with its user table ub, item table vb, rating ciphertexts [ct0, ct1)
    // and ratings (CSR indices, in CSR order)
    struct Pair {
        int ub = 0, vb = 0, ct0 = 0, ct1 = 0;
        std::vector<int32_t> ratings;
    };
    bool pairs = false;
    std::vector<Pair> pair_list;
    int epochs_done = 0;
    int refresh_round = 0;
    double refresh_seconds = 0;     // wall time spent in refreshes (host + device)
    // masked-MAC work since initialisation: tasks (accumulators), groups
    // (source ciphertexts), mask terms (constant terms apart), and the same
    // counts weighted by the limbs each launch covers
    int64_t mac_tasks = 0, mac_groups = 0, mac_terms = 0, mac_const_terms = 0;
    int64_t mac_task_rows = 0, mac_group_rows = 0, mac_term_rows = 0;
    bool factors = false;
};

namespace mfp {

// Scales of the program, relative to the chain's scale Delta = 2^log2_scale
// (the values in brackets are those at Delta = 2^40).  Rounding the block
// indicator I0's coefficients puts an error of about sqrt(N/24)/S_I on every
// slot of every mask; a gather (all weights 1) sums D masks, so it takes the
// larger mask scale Delta / 2^10 [2^30] and declares the exact scale of its
// terms instead of rounding a weight; a scatter needs room for small integer
// weights (learning rate over degree): masks at Delta / 2^16 [2^24] with the
// factor tables held at Delta 2^10 [2^50], and the self term's common weight
// applied as a constant so only corrections are masked.  The scatter weights
// alpha/d are ~1e-5; their integers are W ~ w 2^26 at any Delta (a target of
// Delta with masks at Delta / 2^20 would give W ~ 10, rounded by up to 5
// percent the same way every epoch).  Gathered factors are at Delta.
inline double mask_scale(const Context* c) { return std::ldexp(1.0, c->prm.log2_scale - 16); }
inline double gather_mask_scale(const Context* c) { return std::ldexp(1.0, c->prm.log2_scale - 10); }
inline double target_scale(const Context* c) { return std::ldexp(1.0, c->prm.log2_scale); }
inline double table_scale(const Context* c) { return std::ldexp(1.0, c->prm.log2_scale + 10); }
// Refresh of level-exhausted tables: tables below this level are refreshed
// before the next gather; masks have integer coefficients in [-2^50, 2^50);
// refreshed table j of round r is encrypted with serial kRefreshSerial + r*1024 + j.
constexpr int kRefreshLevel = 4;
constexpr int kRefreshMaskBits = 50;
constexpr uint32_t kRefreshSerial = 0x20000000u;

// A block move: source ciphertext `src`, block a -> destination block b, weight w.
struct Move {
    int src, a, b;
    double w;
};

// Self term of a scatter destination: T (.) (c + sum_b (w_b - c) I_b).
struct SelfTerm {
    Ct* t = nullptr;
    double c = 1.0;
    std::vector<std::pair<int, double>> corr;   // (block, w_b - c), w_b != c
};

// (source index, baby step beta) -> HRot_{beta B}(source) at the permutation's level
typedef std::map<std::pair<int, int>, Ct> BabyCache;

MfState& state(Context* c);   // the context's MF state (STATE error if none)
void free_handles(Context* c, std::vector<uint64_t>& v);
void release(Context* c, std::vector<Ct>& v);
std::vector<Ct*> ptrs(std::vector<Ct>& v);
std::vector<Ct> dropped(const std::vector<Ct*>& v, int level);
std::vector<Ct> hmult_all(Context* c, const std::vector<Ct*>& a, const std::vector<Ct*>& b);
std::vector<Ct> rotate_all(Context* c, const std::vector<Ct*>& a, int64_t r);
std::vector<Ct> rotate_add_all(Context* c, const std::vector<Ct*>& a, int64_t r);   // a + Rot(a, r), fused
std::vector<Ct> add_all(Context* c, const std::vector<Ct*>& a, const std::vector<Ct*>& b, bool sub);
int64_t weight_int(double w, double s_src, double q_acc, double mask_scale, double target);
std::vector<int64_t> encode_all(Context* c, const std::vector<std::vector<double>>& zs, double scale);
std::vector<uint64_t> put_all(Context* c, std::vector<Ct>& v);
void upload_masks(Context* c, MfState& m, const int64_t* mask_scatter, const int64_t* mask_gather);
void encode_masks(Context* c, int k, std::vector<int64_t>& mask_scatter, std::vector<int64_t>& mask_gather);
void free_masks(Context* c, MfState& m);
// unit: every move has weight 1 (a gather): I0 at the gather scale, target
// 2^40 and the accumulator declared at the exact scale of its terms;
// otherwise (a scatter) I0 at the scatter scale and target kTableScale.
// block_permute: the MF program's schedule (baby-step size per call, baby and
// giant trees); block_permute_cached: serving's (layout G, cached or hoisted
// babies, direct giant rotations).
std::vector<Ct> block_permute(Context* c, MfState& m, const std::vector<Ct*>& srcs,
                              const std::vector<std::vector<Move>>& dests, const std::vector<SelfTerm>* selfs,
                              int level, bool unit);
std::vector<Ct> block_permute_cached(Context* c, MfState& m, const std::vector<Ct*>& srcs,
                                     const std::vector<std::vector<Move>>& dests,
                                     const std::vector<SelfTerm>* selfs, int level, const BabyCache* cache,
                                     bool unit);
int choose_G(const std::vector<std::vector<Move>>& dests, int D);
std::vector<Ct> dot_products(Context* c, MfState& m, const std::vector<Ct*>& ug, const std::vector<Ct*>& vg,
                             double* sp_out);
// Validate the CSR arrays, compute the layout, generate the program's
// rotation keys and install it as the context's MF state (replacing one).
void install_layout(Context* c, int32_t n_rows, int32_t n_cols, const int64_t* row_ptr, const int32_t* col_idx);
// Slot vectors of the rating-layout ciphertexts (which: 0 ratings, 1 users, 2 items).
void fill_rating_slots(const MfState& m, int which, const double* values, const double* U, const double* V,
                       std::vector<std::vector<double>>& zs);
// Encrypt count integer plaintexts at the top level (running serials).
std::vector<uint64_t> encrypt_list(Context* c, const int64_t* m, int count, double scale);

}  // namespace mfp
}  // namespace csrmf
