// Encrypted CSR matrix-factorisation program: Alg. 1 of the paper evaluated
// as a synchronous epoch (every rating's error uses the epoch-start factors,
// the per-entity gradient terms are accumulated and applied once, as the
// accumulator of Alg. 2 does), over block-packed CSR rating ciphertexts.
//
// Layout (k' = 2^ceil(log2 k), B = 2k', D = N/(2B) blocks per ciphertext):
//   rating ciphertexts: rows packed greedily in CSR order (a row that does not
//   fit starts a new ciphertext, a row longer than D is cut into chunks of D);
//   block t holding rating (i, j) carries r_ij / u_i / v_j in slots tB..tB+k-1.
//   factor tables: table ciphertext a holds entity a*D + b at block b.
// Epoch (gathered factors at level l):
//   P = HMult(Ug, Vg); T_{s+1} = T_s + Rot(T_s, 2^s), s < log2 B;
//   Sdot = Rot(T, -k') (slot tB+f holds <u_i, v_j>);
//   E = drop(Rescale(R * W_R)) - Sdot, W_R = rint((S_P * q_L) / S_R);
//   G_U = HMult(E, Vg), G_V = HMult(E, Ug);
//   tables <- BlockPermute(G -> tables, learning-rate weights) + self term;
//   gathered factors <- BlockPermute(tables -> rating layout, weight 1).
// BlockPermute (move: source c, block a -> destination block b, weight w;
// (a - b) mod D = gamma*G + beta with the baby-step size G of the call chosen
// by choose_G, babies built in blocks of kBabyBlock by rotation trees):
//   acc_d = sum_gamma Rot_{gamma G B}( sum_{c,beta} Rot_{beta B}(src_c) (.) M_{d,c,gamma,beta} )
//   M = sum_moves W * tau_{g_p}(I0), p = (b + gamma G) mod D, g_p = 5^((-pB) mod N/2),
//   W = rint((w * S_t * q_ell) / (S_src * S_I)); one rescale per destination.
//   With Delta the chain's scale: scatter S_I = Delta / 2^16, S_t = Delta 2^10
//   (the tables' scale), self term as a constant plus masked corrections;
//   gather S_I = Delta / 2^10, S_t = Delta, the accumulator declared at the
//   exact scale of its terms (all weights are 1).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>
#include <unordered_map>

#include "mf_internal.h"
#include "host_math.h"

namespace csrmf {

void destroy_mf(MfState* m) { delete m; }

namespace mfp {

void free_handles(Context* c, std::vector<uint64_t>& v) {
    for (uint64_t h : v) c->free_ct(h);
    v.clear();
}

std::vector<Ct*> cts_of(Context* c, const std::vector<uint64_t>& v) {
    std::vector<Ct*> out;
    for (uint64_t h : v) out.push_back(&c->get(h));
    return out;
}

MfState& state(Context* c) {
    if (!c->mf) throw Error(CSRMF_E_STATE, "no rating matrix has been encrypted");
    return *c->mf;
}

// Validate the CSR arrays and compute the block layout.
MfState* make_layout(Context* c, int32_t n_rows, int32_t n_cols, const int64_t* row_ptr, const int32_t* col_idx) {
    if (n_rows <= 0 || n_cols <= 0 || !row_ptr || !col_idx) throw Error(CSRMF_E_INVAL, "empty or null CSR matrix");
    const int k = c->prm.k;
    if (k <= 0) throw Error(CSRMF_E_INVAL, "params.k must be positive for the MF program");
    if (row_ptr[0] != 0) throw Error(CSRMF_E_INVAL, "row_ptr[0] must be 0");
    for (int i = 0; i < n_rows; ++i) {
        if (row_ptr[i + 1] < row_ptr[i]) throw Error(CSRMF_E_INVAL, "row_ptr is not monotone");
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            if (col_idx[p] < 0 || col_idx[p] >= n_cols) throw Error(CSRMF_E_INVAL, "column index out of range");
            if (p > row_ptr[i] && col_idx[p] <= col_idx[p - 1])
                throw Error(CSRMF_E_INVAL, "column indices unsorted or duplicated within a row");
        }
    }
    const int64_t nnz = row_ptr[n_rows];
    if (nnz <= 0 || nnz > (int64_t)1 << 30) throw Error(CSRMF_E_INVAL, "bad number of ratings");
    MfState* m = new MfState();
    m->k = k;
    m->kp = 1;
    while (m->kp < k) m->kp *= 2;
    m->B = 2 * m->kp;
    m->D = (int)(c->N / (2 * (uint64_t)m->B));
    int logD = 0;
    while ((1 << (logD + 1)) <= m->D) ++logD;
    m->G = 1 << ((logD + 1) / 2);
    m->n_users = n_rows;
    m->n_items = n_cols;
    m->nnz = (int)nnz;
    m->row_ptr.assign(row_ptr, row_ptr + n_rows + 1);
    m->col_idx.assign(col_idx, col_idx + nnz);
    m->rows.resize(nnz);
    m->ct_of.resize(nnz);
    m->blk_of.resize(nnz);
    m->deg_u.assign(n_rows, 0.0);
    m->deg_v.assign(n_cols, 0.0);
    int ct = 0, used = 0;
    bool started = false;
    for (int i = 0; i < n_rows; ++i) {
        int64_t pos = row_ptr[i];
        const int64_t e = row_ptr[i + 1];
        while (pos < e) {
            const int chunk = (int)std::min<int64_t>(m->D, e - pos);
            if (!started) started = true;
            else if (used + chunk > m->D) { ++ct; used = 0; }
            for (int q = 0; q < chunk; ++q) {
                m->ct_of[pos + q] = ct;
                m->blk_of[pos + q] = used + q;
                m->rows[pos + q] = i;
            }
            used += chunk;
            pos += chunk;
        }
        m->deg_u[i] = (double)(e - row_ptr[i]);
    }
    for (int64_t p = 0; p < nnz; ++p) m->deg_v[col_idx[p]] += 1.0;
    m->n_ct = ct + 1;
    m->n_utab = (n_rows + m->D - 1) / m->D;
    m->n_vtab = (n_cols + m->D - 1) / m->D;
    if (c->prm.batch_pairs) {
        // Alg. 2: group by (user batch, item batch) with a batch of D profiles,
        // pairs in the order of their first rating; each pair's ratings (CSR
        // order) fill rating ciphertexts of their own
        std::map<std::pair<int, int>, int> index;
        for (int64_t p = 0; p < nnz; ++p) {
            const std::pair<int, int> key{m->rows[p] / m->D, col_idx[p] / m->D};
            auto it = index.find(key);
            if (it == index.end()) {
                it = index.emplace(key, (int)m->pair_list.size()).first;
                m->pair_list.emplace_back();
                m->pair_list.back().ub = key.first;
                m->pair_list.back().vb = key.second;
            }
            m->pair_list[it->second].ratings.push_back((int32_t)p);
        }
        int c0 = 0;
        for (auto& pr : m->pair_list) {
            const int n = (int)pr.ratings.size();
            pr.ct0 = c0;
            pr.ct1 = c0 + (n + m->D - 1) / m->D;
            for (int q = 0; q < n; ++q) {
                m->ct_of[pr.ratings[q]] = c0 + q / m->D;
                m->blk_of[pr.ratings[q]] = q % m->D;
            }
            c0 = pr.ct1;
        }
        m->n_ct = c0;
        m->pairs = true;
    }
    return m;
}

// slot vectors of all rating-layout ciphertexts in one pass over the ratings
// (which: 0 ratings, 1 users, 2 items)
void fill_rating_slots(const MfState& m, int which, const double* values, const double* U, const double* V,
                       std::vector<std::vector<double>>& zs) {
    for (auto& z : zs) std::fill(z.begin(), z.end(), 0.0);
    for (int r = 0; r < m.nnz; ++r) {
        double* dst = zs[m.ct_of[r]].data() + (size_t)m.blk_of[r] * m.B;
        for (int f = 0; f < m.k; ++f) {
            if (which == 0) dst[f] = values[r];
            else if (which == 1) dst[f] = U[(size_t)m.rows[r] * m.k + f];
            else dst[f] = V[(size_t)m.col_idx[r] * m.k + f];
        }
    }
}

void fill_table_slots(const MfState& m, int a, int n_ent, const double* F, std::vector<double>& z) {
    std::fill(z.begin(), z.end(), 0.0);
    for (int b = 0; b < m.D; ++b) {
        const int e = a * m.D + b;
        if (e >= n_ent) break;
        for (int f = 0; f < m.k; ++f) z[(size_t)b * m.B + f] = F[(size_t)e * m.k + f];
    }
}

std::vector<int64_t> encode_all(Context* c, const std::vector<std::vector<double>>& zs, double scale) {
    std::vector<int64_t> out(zs.size() * c->N);
    for (size_t i = 0; i < zs.size(); ++i)
        if (!ckks_encode(zs[i].data(), (int)zs[i].size(), c->logN, scale, out.data() + i * c->N))
            throw Error(CSRMF_E_INVAL, "value too large to encode");
    return out;
}

std::vector<uint64_t> encrypt_list(Context* c, const int64_t* m, int count, double scale) {
    std::vector<Ct> cts;
    c->encrypt_int_batch(m, count, c->L, scale, cts);
    std::vector<uint64_t> h;
    for (auto& x : cts) h.push_back(c->put(x));
    return h;
}

static void upload_one(Context* c, uint64_t*& dst, const int64_t* mask) {
    if (!dst) dst = (uint64_t*)c->pool.get((size_t)(c->L + 1) * c->N * 8);
    Scratch src(c->pool, c->N);
    CSRMF_HIP(hipMemcpyAsync(src.p, mask, c->N * 8, hipMemcpyHostToDevice, c->stream));
    RowMap mm;
    mm.base = dst;
    for (int i = 0; i <= c->L; ++i) mm.push(i, i);
    launch_expand_signed(c->tabs, mm, (const int64_t*)src.p, 1, 0, c->stream);
    launch_ntt(c->tabs, mm, false, c->stream);
    launch_ew(c->tabs, EW_F64C, mm, mm, mm, c->stream);   // the MAC's FP64 limbs read centred doubles
    c->sync();
}

void upload_masks(Context* c, MfState& m, const int64_t* mask_scatter, const int64_t* mask_gather) {
    upload_one(c, m.mask0, mask_scatter);
    upload_one(c, m.maskg, mask_gather);
}

void encode_masks(Context* c, int k, std::vector<int64_t>& mask_scatter, std::vector<int64_t>& mask_gather) {
    std::vector<double> ind(c->N / 2, 0.0);
    for (int f = 0; f < k; ++f) ind[f] = 1.0;
    mask_scatter.assign(c->N, 0);
    mask_gather.assign(c->N, 0);
    ckks_encode(ind.data(), (int)ind.size(), c->logN, mask_scale(c), mask_scatter.data());
    ckks_encode(ind.data(), (int)ind.size(), c->logN, gather_mask_scale(c), mask_gather.data());
}

void free_masks(Context* c, MfState& m) {
    if (m.mask0) c->pool.put(m.mask0);
    if (m.maskg) c->pool.put(m.maskg);
    m.mask0 = m.maskg = nullptr;
}

// Ct views at a lower level (same device buffer)
std::vector<Ct> dropped(const std::vector<Ct*>& v, int level) {
    std::vector<Ct> out;
    for (Ct* x : v) {
        if (x->level < level) throw Error(CSRMF_E_LEVEL, "cannot raise a level");
        Ct y = *x;
        y.level = level;
        out.push_back(y);
    }
    return out;
}

std::vector<Ct*> ptrs(std::vector<Ct>& v) {
    std::vector<Ct*> out;
    for (auto& x : v) out.push_back(&x);
    return out;
}

void release(Context* c, std::vector<Ct>& v) {
    for (auto& x : v) c->pool.put(x.d);
    v.clear();
}

std::vector<Ct> hmult_all(Context* c, const std::vector<Ct*>& a, const std::vector<Ct*>& b) {
    std::vector<Ct> out(a.size());
    std::vector<Ct*> po = ptrs(out);
    c->mul_relin(a, b, po);
    c->rescale(po);
    return out;
}

std::vector<Ct> rotate_all(Context* c, const std::vector<Ct*>& a, int64_t r) {
    std::vector<Ct> out(a.size());
    std::vector<Ct*> po = ptrs(out);
    c->rotate(a, c->galois_for_step(r), po);
    return out;
}

// a[i] + Rot(a[i], r), the addition fused into the key switch
std::vector<Ct> rotate_add_all(Context* c, const std::vector<Ct*>& a, int64_t r) {
    std::vector<Ct> out(a.size());
    std::vector<Ct*> po = ptrs(out);
    c->rotate(a, c->galois_for_step(r), po, &a);
    return out;
}

std::vector<Ct> add_all(Context* c, const std::vector<Ct*>& a, const std::vector<Ct*>& b, bool sub) {
    std::vector<Ct> out(a.size());
    std::vector<Ct*> po = ptrs(out);
    c->add_batch(a, b, po, sub);
    return out;
}

int64_t weight_int(double w, double s_src, double q_acc, double mask_scale, double target) {
    return (int64_t)std::nearbyint((w * target * q_acc) / (s_src * mask_scale));
}

// Per-limb constants of an integer weight W, computed once per distinct W:
// for a prime below 2^44 (the MAC's FP64 form) the centred W mod q_i and
// fl(W/q_i) as raw doubles, otherwise W * 2^64 mod q_i and its Shoup factor.
class WeightRows {
public:
    WeightRows(Context* c, int nl) : c_(c), nl_(nl) {}
    const std::vector<uint64_t>& row(int64_t W) {
        auto it = rows_.find(W);
        if (it != rows_.end()) return it->second;
        std::vector<uint64_t> r;
        r.reserve(2 * (size_t)nl_);
        for (int i = 0; i < nl_; ++i) {
            const uint64_t q = c_->moduli[i];
            const uint64_t w = from_signed(W, q);
            if (q < kFp64PrimeBound) {
                const double wd = w > q / 2 ? -(double)(q - w) : (double)w, wq = wd / (double)q;
                uint64_t b0, b1;
                std::memcpy(&b0, &wd, 8);
                std::memcpy(&b1, &wq, 8);
                r.push_back(b0);
                r.push_back(b1);
            } else {
                const uint64_t x = mul_mod_host(w, c_->mh[i].r_mod, q);
                r.push_back(x);
                r.push_back(shoup_pre(x, q));
            }
        }
        return rows_.emplace(W, std::move(r)).first->second;
    }

private:
    Context* c_;
    int nl_;
    std::unordered_map<int64_t, std::vector<uint64_t>> rows_;
};

// One multi-task masked MAC launch being assembled on the host.
struct MacLaunch {
    std::vector<uint64_t*> acc, src;
    std::vector<int32_t> grp_begin, first, term_begin, wi;
    std::vector<uint32_t> gs;
    std::vector<uint64_t> cw;
    std::unordered_map<int64_t, int32_t> widx;

    // Algorithmic HBM bytes of the launch: every distinct source read once
    // (both polynomials), every accumulator written (and read unless it
    // starts at zero); the mask values come from the resident I_0 rows.
    double hbm_bytes(int nl, uint64_t N) const {
        std::vector<uint64_t*> u(src);
        std::sort(u.begin(), u.end());
        const size_t n_src = (size_t)(std::unique(u.begin(), u.end()) - u.begin());
        size_t acc_rows = 0;
        for (int32_t f : first) acc_rows += f ? 2 : 4;
        return (double)N * 8.0 * nl * (2.0 * (double)n_src + (double)acc_rows);
    }

    void task(uint64_t* a, bool is_first) {
        acc.push_back(a);
        first.push_back(is_first ? 1 : 0);
        grp_begin.push_back((int32_t)src.size());
    }
    void group(const uint64_t* s) {
        src.push_back(const_cast<uint64_t*>(s));
        term_begin.push_back((int32_t)gs.size());
    }
    void term(uint32_t g, int64_t W, WeightRows& rows) {
        auto it = widx.find(W);
        int32_t w;
        if (it == widx.end()) {
            w = (int32_t)widx.size();
            widx.emplace(W, w);
            const std::vector<uint64_t>& r = rows.row(W);
            cw.insert(cw.end(), r.begin(), r.end());
        } else {
            w = it->second;
        }
        gs.push_back(g);
        wi.push_back(w);
    }
    // Stage the arguments, launch, and fence the staging ring behind the launch.
    void run(Context* c, int nl, const uint64_t* mask, double bytes) {
        if (acc.empty()) return;
        grp_begin.push_back((int32_t)src.size());
        term_begin.push_back((int32_t)gs.size());
        MaskTasks T;
        T.acc = (uint64_t* const*)c->stage(acc.data(), acc.size() * sizeof(uint64_t*));
        T.grp_begin = (const int32_t*)c->stage(grp_begin.data(), grp_begin.size() * 4);
        T.first = (const int32_t*)c->stage(first.data(), first.size() * 4);
        T.src = (const uint64_t* const*)c->stage(src.data(), src.size() * sizeof(uint64_t*));
        T.term_begin = (const int32_t*)c->stage(term_begin.data(), term_begin.size() * 4);
        T.gs = (const uint32_t*)c->stage(gs.data(), gs.size() * 4);
        T.wi = (const int32_t*)c->stage(wi.data(), wi.size() * 4);
        T.cw = (const uint64_t*)c->stage(cw.data(), cw.size() * 8);
        T.n_tasks = (int32_t)acc.size();
        T.n_limbs = nl;
        if (c->mf) {   // the MF program's counters (a server's launches are not counted)
            MfState& st = *c->mf;
            const int64_t n_const = std::count(gs.begin(), gs.end(), 0u);
            st.mac_tasks += (int64_t)acc.size();
            st.mac_groups += (int64_t)src.size();
            st.mac_terms += (int64_t)gs.size() - n_const;
            st.mac_const_terms += n_const;
            st.mac_task_rows += (int64_t)acc.size() * nl;
            st.mac_group_rows += (int64_t)src.size() * nl;
            st.mac_term_rows += ((int64_t)gs.size() - n_const) * nl;
        }
        T.cw_stride = nl;
        T.poly_stride = c->poly_stride();
        launch_mask_mac_tasks(c->tabs, T, mask, bytes, c->stream);
        c->fence();
    }
};

constexpr int kHoistChunk = 128;   // sources whose digits are extended together

// Serving's permutation (tables are read-only, so their baby rotations are
// cached): baby-step size m.G, babies HRot_{beta B} hoisted (or taken from
// `cache`), one direct giant rotation per (destination, gamma).
// srcs: source ciphertexts (viewed at `level`); dests[d]: moves into destination d;
// selfs[d]: optional self term (constant plus masked corrections).  Schedule: the sources
// are extended (ModUp) once per chunk; for every baby step beta one batched
// inner product + ModDown gives HRot_beta of all sources of the chunk, and one
// multi-task launch accumulates every (destination, gamma) inner sum that uses
// them; then one batched giant rotation per gamma, the self terms, and one
// batched rescale.  Sums are exact, so this order gives the defined result.
std::vector<Ct> block_permute_cached(Context* c, MfState& m, const std::vector<Ct*>& srcs,
                                     const std::vector<std::vector<Move>>& dests,
                                     const std::vector<SelfTerm>* selfs, int level, const BabyCache* cache,
                                     bool unit) {
    const int D = m.D, G = m.G, B = m.B;
    const int nl = level + 1;
    const double s_src = srcs.empty() ? 1.0 : srcs[0]->scale;
    const double q_acc = (double)c->moduli[level];
    const double mask_scale = unit ? gather_mask_scale(c) : csrmf::mfp::mask_scale(c);
    const double target = unit ? target_scale(c) : table_scale(c);
    const uint64_t* mask = unit ? m.maskg : m.mask0;
    if (!mask) throw Error(CSRMF_E_STATE, "block masks not uploaded");
    double acc_scale = target * q_acc;
    if (unit) {
        for (const auto& dv : dests)
            for (const Move& x : dv)
                if (x.w != 1.0) throw Error(CSRMF_E_INVAL, "unit permutation with a weight other than 1");
        if (selfs) throw Error(CSRMF_E_INVAL, "unit permutation with self terms");
        acc_scale = s_src * mask_scale * (double)weight_int(1.0, s_src, q_acc, mask_scale, target);
    }
    const int n_dest = (int)dests.size();
    const int n_gamma = D / G;
    WeightRows wrows(c, nl);
    auto gal = [&](int p) { return c->galois_for_step(-(int64_t)p * B); };

    // groups keyed by (beta, source, destination, gamma) -> terms (p, W)
    std::map<std::tuple<int, int, int, int>, std::vector<std::pair<int, int64_t>>> groups;
    std::map<int, std::vector<int>> betas_of_src;
    for (int d = 0; d < n_dest; ++d)
        for (const Move& x : dests[d]) {
            const int delta = ((x.a - x.b) % D + D) % D;
            const int gamma = delta / G, beta = delta % G;
            groups[{beta, x.src, d, gamma}].push_back({(x.b + gamma * G) % D, weight_int(x.w, s_src, q_acc, mask_scale, target)});
            auto& v = betas_of_src[x.src];
            if (std::find(v.begin(), v.end(), beta) == v.end()) v.push_back(beta);
        }
    // accumulators: gamma 0 sums go straight into acc[d]; inner[d][gamma] otherwise
    std::vector<Ct> acc(n_dest);
    std::vector<char> acc_init(n_dest, 0);
    for (int d = 0; d < n_dest; ++d) acc[d] = c->new_ct(level, acc_scale);
    std::vector<std::vector<Ct>> inner(n_dest, std::vector<Ct>(n_gamma));
    std::vector<std::vector<char>> inner_init(n_dest, std::vector<char>(n_gamma, 0));
    for (auto& kv : groups) {
        const int d = std::get<2>(kv.first), gamma = std::get<3>(kv.first);
        if (gamma && !inner[d][gamma].d) inner[d][gamma] = c->new_ct(level, acc_scale);
    }
    std::vector<int> src_list;
    for (auto& kv : betas_of_src) src_list.push_back(kv.first);

    for (size_t c0 = 0; c0 < src_list.size(); c0 += kHoistChunk) {
        const size_t c1 = std::min(src_list.size(), c0 + kHoistChunk);
        std::vector<Ct> views;
        std::vector<int> ids;
        std::vector<int> betas;
        for (size_t i = c0; i < c1; ++i) {
            Ct v = *srcs[src_list[i]];
            v.level = level;
            views.push_back(v);
            ids.push_back(src_list[i]);
            for (int b : betas_of_src[src_list[i]])
                if (std::find(betas.begin(), betas.end(), b) == betas.end()) betas.push_back(b);
        }
        std::sort(betas.begin(), betas.end());
        std::map<int, int> pos;   // source id -> index in the chunk
        for (size_t i = 0; i < ids.size(); ++i) pos[ids[i]] = (int)i;
        std::vector<Ct*> pviews = ptrs(views);
        Context::Hoist hs;
        const bool any_rot = betas.size() > 1 || (betas.size() == 1 && betas[0] != 0);
        if (any_rot && !cache) c->hoist_begin(hs, pviews);
        for (int beta : betas) {
            std::vector<Ct> babies;
            std::vector<uint64_t*> baby_ptr(views.size());
            for (size_t i = 0; i < views.size(); ++i) baby_ptr[i] = views[i].d;
            if (beta && cache) {
                for (size_t i = 0; i < views.size(); ++i) {
                    auto it = cache->find({ids[i], beta});
                    baby_ptr[i] = it == cache->end() ? nullptr : it->second.d;
                }
            } else if (beta) {
                babies.resize(views.size());
                std::vector<Ct*> pb = ptrs(babies);
                c->hoist_rotate(hs, c->galois_for_step((int64_t)beta * B), pb);
                for (size_t i = 0; i < views.size(); ++i) baby_ptr[i] = babies[i].d;
            }
            // tasks: one per (destination, gamma) receiving groups of this beta from this chunk
            std::map<std::pair<int, int>, std::vector<std::pair<int, const std::vector<std::pair<int, int64_t>>*>>> tasks;
            auto lo = groups.lower_bound({beta, ids.front(), -1, -1});
            for (auto it = lo; it != groups.end() && std::get<0>(it->first) == beta; ++it) {
                const int src = std::get<1>(it->first);
                auto pit = pos.find(src);
                if (pit == pos.end()) continue;
                tasks[{std::get<2>(it->first), std::get<3>(it->first)}].push_back({pit->second, &it->second});
            }
            if (tasks.empty()) continue;
            MacLaunch ml;
            for (auto& tk : tasks) {
                const int d = tk.first.first, gamma = tk.first.second;
                Ct& tgt = gamma ? inner[d][gamma] : acc[d];
                char& init = gamma ? inner_init[d][gamma] : acc_init[d];
                ml.task(tgt.d, !init);
                init = 1;
                for (auto& gr : tk.second) {
                    if (!baby_ptr[gr.first]) throw Error(CSRMF_E_STATE, "missing cached baby-step rotation");
                    ml.group(baby_ptr[gr.first]);
                    for (auto& tm : *gr.second) ml.term(gal(tm.first), tm.second, wrows);
                }
            }
            const double bytes = ml.hbm_bytes(nl, c->N);
            ml.run(c, nl, mask, bytes);
            release(c, babies);
        }
    }
    // giant steps: one batched rotation per gamma over the destinations that use it
    for (int gamma = 1; gamma < n_gamma; ++gamma) {
        std::vector<int> ds;
        for (int d = 0; d < n_dest; ++d)
            if (inner[d][gamma].d) ds.push_back(d);
        if (ds.empty()) continue;
        // destinations with a running sum take acc + Rot(inner) in one fused
        // key switch; the others start their sum with the rotation
        const uint32_t gg = c->galois_for_step((int64_t)gamma * G * B);
        std::vector<int> part[2];   // [0]: no running sum yet, [1]: acc + rotation
        for (int d : ds) part[acc_init[d] ? 1 : 0].push_back(d);
        for (int with_acc = 0; with_acc < 2; ++with_acc) {
            const std::vector<int>& dd = part[with_acc];
            if (dd.empty()) continue;
            std::vector<Ct*> in, accs;
            for (int d : dd) {
                in.push_back(&inner[d][gamma]);
                accs.push_back(&acc[d]);
            }
            std::vector<Ct> rot(dd.size());
            std::vector<Ct*> prot = ptrs(rot);
            c->rotate(in, gg, prot, with_acc ? &accs : nullptr);
            for (size_t i = 0; i < dd.size(); ++i) {
                const int d = dd[i];
                c->pool.put(inner[d][gamma].d);
                inner[d][gamma].d = nullptr;
                if (acc[d].d) c->pool.put(acc[d].d);
                acc[d] = rot[i];
                acc_init[d] = 1;
            }
        }
    }
    // self terms: one task per destination; the constant c is a term with
    // Galois element 0 (no mask), the corrections are masked terms
    if (selfs) {
        MacLaunch ml;
        for (int d = 0; d < n_dest; ++d) {
            const SelfTerm& st = (*selfs)[d];
            if (!st.t) continue;
            const double s_self = st.t->scale;
            ml.task(acc[d].d, !acc_init[d]);
            acc_init[d] = 1;
            ml.group(st.t->d);
            ml.term(0, weight_int(st.c, s_self, q_acc, 1.0, target), wrows);
            for (auto& bw : st.corr)
                ml.term(gal(bw.first), weight_int(bw.second, s_self, q_acc, mask_scale, target), wrows);
        }
        const double bytes = ml.hbm_bytes(nl, c->N);
        ml.run(c, nl, mask, bytes);
    }
    for (int d = 0; d < n_dest; ++d)
        if (!acc_init[d]) throw Error(CSRMF_E_INVAL, "block permutation with an empty destination");
    for (auto& a : acc) a.scale = acc_scale;
    std::vector<Ct*> pacc = ptrs(acc);
    c->rescale(pacc);
    return acc;
}

// ---------------------------------------------------------------- the MF program's permutation schedule
constexpr int kBabyBlock = 64;          // babies are built in blocks of this many steps
constexpr int kMaxAccumulators = 1024;  // bound on destinations * D/G inner sums alive at once
constexpr int kRotateBatch = 128;       // ciphertexts per batched rotation call (ModUp scratch)

int giant_rotations(std::vector<char> nodes, int width) {
    int count = 0;
    while (width > 1) {
        std::vector<char> nxt(width / 2, 0);
        for (int t = 0; t < width / 2; ++t) {
            if (nodes[2 * t + 1]) ++count;
            nxt[t] = nodes[2 * t] || nodes[2 * t + 1];
        }
        nodes.swap(nxt);
        width /= 2;
    }
    return count;
}

// Baby-step size: the power of two G <= D with the fewest rotations (a source
// needing baby steps up to beta costs beta rotations; a destination costs the
// rotations of the pairwise giant tree over its D/G positions), among those
// with n_dest * D/G <= kMaxAccumulators; ties go to the smaller G; D if none.
int choose_G(const std::vector<std::vector<Move>>& dests, int D) {
    long best = -1;
    int best_G = D;
    for (int G = 1; G <= D; G *= 2) {
        const int ng = D / G;
        if ((long)dests.size() * ng > kMaxAccumulators) continue;
        std::map<int, int> top;
        long cost = 0;
        for (const auto& dv : dests) {
            if (dv.empty()) continue;
            std::vector<char> present(ng, 0);
            for (const Move& x : dv) {
                const int delta = ((x.a - x.b) % D + D) % D;
                const int gamma = delta / G, beta = delta % G;
                auto it = top.find(x.src);
                if (it == top.end()) top[x.src] = beta;
                else if (beta > it->second) it->second = beta;
                present[gamma] = 1;
            }
            cost += giant_rotations(present, ng);
        }
        for (auto& kv : top) cost += kv.second;
        if (best < 0 || cost < best) {
            best = cost;
            best_G = G;
        }
    }
    return best_G;
}

// out[i] = Rot_g(in[i]) (+ acc[i], fused, when acc is given)
static void rotate_chunked(Context* c, std::vector<Ct*>& in, uint32_t g, std::vector<Ct*>& out,
                           const std::vector<Ct*>* acc = nullptr) {
    for (size_t i = 0; i < in.size(); i += kRotateBatch) {
        const size_t j = std::min(in.size(), i + kRotateBatch);
        std::vector<Ct*> a(in.begin() + (long)i, in.begin() + (long)j), o(out.begin() + (long)i, out.begin() + (long)j);
        if (acc) {
            std::vector<Ct*> s(acc->begin() + (long)i, acc->begin() + (long)j);
            c->rotate(a, g, o, &s);
        } else {
            c->rotate(a, g, o);
        }
    }
}

// The MF program's BlockPermute (same order of rotations as the definition):
// baby-step size G = choose_G; per source, babies Rot_{beta B}(src) for beta
// up to the largest one it needs, in blocks of kBabyBlock (block base
// Rot_{k B}(src), inside a block baby k+s+j = Rot_{s B}(baby k+j) for s = 1, 2,
// 4, ..; next base = Rot_{kBabyBlock B}(base)); inner sums per (destination,
// gamma) by multi-task masked MAC launches, one per baby step; giant steps as
// a pairwise tree (level j: node t = node 2t + Rot_{2^j G B}(node 2t+1));
// then the self terms and one batched rescale.  Rotations of one level are
// batched; modular sums are exact, so batching does not change the result.
std::vector<Ct> block_permute(Context* c, MfState& m, const std::vector<Ct*>& srcs,
                              const std::vector<std::vector<Move>>& dests, const std::vector<SelfTerm>* selfs,
                              int level, bool unit) {
    const int D = m.D, B = m.B;
    const int G = choose_G(dests, D);
    const int n_gamma = D / G;
    const int nl = level + 1;
    const double s_src = srcs.empty() ? 1.0 : srcs[0]->scale;
    const double q_acc = (double)c->moduli[level];
    const double mask_scale = unit ? gather_mask_scale(c) : csrmf::mfp::mask_scale(c);
    const double target = unit ? target_scale(c) : table_scale(c);
    const uint64_t* mask = unit ? m.maskg : m.mask0;
    if (!mask) throw Error(CSRMF_E_STATE, "block masks not uploaded");
    double acc_scale = target * q_acc;
    if (unit) {
        for (const auto& dv : dests)
            for (const Move& x : dv)
                if (x.w != 1.0) throw Error(CSRMF_E_INVAL, "unit permutation with a weight other than 1");
        if (selfs) throw Error(CSRMF_E_INVAL, "unit permutation with self terms");
        acc_scale = s_src * mask_scale * (double)weight_int(1.0, s_src, q_acc, mask_scale, target);
    }
    const int n_dest = (int)dests.size();
    WeightRows wrows(c, nl);
    auto gal = [&](int p) { return c->galois_for_step(-(int64_t)p * B); };

    // groups keyed by (beta, source, destination, gamma) -> terms (p, W); top baby step per source
    std::map<std::tuple<int, int, int, int>, std::vector<std::pair<int, int64_t>>> groups;
    std::map<int, int> top;
    for (int d = 0; d < n_dest; ++d)
        for (const Move& x : dests[d]) {
            const int delta = ((x.a - x.b) % D + D) % D;
            const int gamma = delta / G, beta = delta % G;
            groups[{beta, x.src, d, gamma}].push_back(
                {(x.b + gamma * G) % D, weight_int(x.w, s_src, q_acc, mask_scale, target)});
            auto it = top.find(x.src);
            if (it == top.end()) top[x.src] = beta;
            else if (beta > it->second) it->second = beta;
        }
    // leaves of the giant tree (d == nullptr: no moves with that gamma)
    std::vector<std::vector<Ct>> nodes(n_dest, std::vector<Ct>(n_gamma));
    std::vector<int> src_list;
    int max_n = 1;
    for (auto& kv : top) {
        src_list.push_back(kv.first);
        max_n = std::max(max_n, kv.second + 1);
    }
    // sources whose babies are built together: at most c->max_babies babies alive
    // (a memory bound only: every baby is built the same way in any chunk)
    const int chunk = std::max(1, std::min(kHoistChunk, c->max_babies / std::min(kBabyBlock, max_n)));
    for (size_t c0 = 0; c0 < src_list.size(); c0 += (size_t)chunk) {
        const size_t c1 = std::min(src_list.size(), c0 + (size_t)chunk);
        const int ns = (int)(c1 - c0);
        std::vector<Ct> base(ns);
        std::vector<char> base_owned(ns, 0);
        std::vector<int> n_of(ns);
        int kmax = 0;
        for (int i = 0; i < ns; ++i) {
            base[i] = *srcs[src_list[c0 + i]];
            base[i].level = level;
            n_of[i] = top[src_list[c0 + i]] + 1;
            kmax = std::max(kmax, n_of[i]);
        }
        for (int k = 0; k < kmax; k += kBabyBlock) {
            // babies of this block: bab[i][j] = Rot_{(k+j) B}(source i)
            std::vector<std::vector<Ct>> bab(ns);
            std::vector<int> width(ns, 0);
            for (int i = 0; i < ns; ++i) {
                width[i] = std::max(0, std::min(kBabyBlock, n_of[i] - k));
                bab[i].resize(width[i]);
                if (width[i] > 0) bab[i][0] = base[i];
            }
            for (int s = 1; s < kBabyBlock; s *= 2) {
                std::vector<Ct*> in, out;
                for (int i = 0; i < ns; ++i)
                    for (int j = 0; j < s && s + j < width[i]; ++j) {
                        in.push_back(&bab[i][j]);
                        out.push_back(&bab[i][s + j]);
                    }
                if (in.empty()) break;
                rotate_chunked(c, in, c->galois_for_step((int64_t)s * B), out);
            }
            // one multi-task MAC launch for every baby step of the block: each
            // (destination, gamma) accumulator is read and written once per block
            std::map<std::pair<int, int>, std::vector<std::pair<const Ct*, const std::vector<std::pair<int, int64_t>>*>>> tasks;
            for (int j = 0; j < kBabyBlock && k + j < kmax; ++j) {
                const int beta = k + j;
                for (int i = 0; i < ns; ++i) {
                    if (j >= width[i]) continue;
                    auto lo = groups.lower_bound({beta, src_list[c0 + i], -1, -1});
                    for (auto it = lo; it != groups.end() && std::get<0>(it->first) == beta &&
                                       std::get<1>(it->first) == src_list[c0 + i]; ++it)
                        tasks[{std::get<2>(it->first), std::get<3>(it->first)}].push_back({&bab[i][j], &it->second});
                }
            }
            if (!tasks.empty()) {
                MacLaunch ml;
                for (auto& tk : tasks) {
                    Ct& tgt = nodes[tk.first.first][tk.first.second];
                    const bool first = tgt.d == nullptr;
                    if (first) tgt = c->new_ct(level, acc_scale);
                    ml.task(tgt.d, first);
                    for (auto& gr : tk.second) {
                        ml.group(gr.first->d);
                        for (auto& tm : *gr.second) ml.term(gal(tm.first), tm.second, wrows);
                    }
                }
                const double bytes = ml.hbm_bytes(nl, c->N);
                ml.run(c, nl, mask, bytes);
            }
            // next block's base; then drop this block's babies
            std::vector<Ct> nb(ns);
            std::vector<Ct*> bin, bout;
            for (int i = 0; i < ns; ++i)
                if (n_of[i] > k + kBabyBlock) {
                    bin.push_back(&base[i]);
                    bout.push_back(&nb[i]);
                }
            if (!bin.empty()) rotate_chunked(c, bin, c->galois_for_step((int64_t)kBabyBlock * B), bout);
            for (int i = 0; i < ns; ++i) {
                for (int jj = 1; jj < width[i]; ++jj) c->pool.put(bab[i][jj].d);
                if (nb[i].d) {
                    if (base_owned[i]) c->pool.put(base[i].d);
                    base[i] = nb[i];
                    base_owned[i] = 1;
                }
            }
        }
        for (int i = 0; i < ns; ++i)
            if (base_owned[i]) c->pool.put(base[i].d);
    }
    // giant steps: pairwise tree, one batched rotation per level (the addition
    // of the left node fused into the key switch where both nodes exist)
    int width = n_gamma;
    int64_t step = (int64_t)G * B;
    while (width > 1) {
        const int half = width / 2;
        std::vector<std::vector<Ct>> nxt(n_dest, std::vector<Ct>(half));
        std::vector<Ct*> in_f, acc_f, out_f, in_p, out_p;
        for (int d = 0; d < n_dest; ++d)
            for (int t2 = 0; t2 < half; ++t2) {
                Ct& left = nodes[d][2 * t2];
                Ct& right = nodes[d][2 * t2 + 1];
                if (left.d && right.d) {
                    in_f.push_back(&right);
                    acc_f.push_back(&left);
                    out_f.push_back(&nxt[d][t2]);
                } else if (right.d) {
                    in_p.push_back(&right);
                    out_p.push_back(&nxt[d][t2]);
                } else if (left.d) {
                    nxt[d][t2] = left;
                }
            }
        const uint32_t gs = c->galois_for_step(step);
        if (!in_f.empty()) rotate_chunked(c, in_f, gs, out_f, &acc_f);
        if (!in_p.empty()) rotate_chunked(c, in_p, gs, out_p);
        for (Ct* x : in_f) c->pool.put(x->d);
        for (Ct* x : acc_f) c->pool.put(x->d);
        for (Ct* x : in_p) c->pool.put(x->d);
        nodes.swap(nxt);
        width = half;
        step *= 2;
    }
    std::vector<Ct> acc(n_dest);
    std::vector<char> acc_init(n_dest, 0);
    for (int d = 0; d < n_dest; ++d) {
        if (nodes[d][0].d) {
            acc[d] = nodes[d][0];
            acc_init[d] = 1;
        } else {
            acc[d] = c->new_ct(level, acc_scale);
        }
    }
    if (selfs) {
        MacLaunch ml;
        for (int d = 0; d < n_dest; ++d) {
            const SelfTerm& st = (*selfs)[d];
            if (!st.t) continue;
            const double s_self = st.t->scale;
            ml.task(acc[d].d, !acc_init[d]);
            acc_init[d] = 1;
            ml.group(st.t->d);
            ml.term(0, weight_int(st.c, s_self, q_acc, 1.0, target), wrows);
            for (auto& bw : st.corr)
                ml.term(gal(bw.first), weight_int(bw.second, s_self, q_acc, mask_scale, target), wrows);
        }
        const double bytes = ml.hbm_bytes(nl, c->N);
        ml.run(c, nl, mask, bytes);
    }
    for (int d = 0; d < n_dest; ++d)
        if (!acc_init[d]) throw Error(CSRMF_E_INVAL, "block permutation with an empty destination");
    for (auto& x : acc) x.scale = acc_scale;
    std::vector<Ct*> pacc = ptrs(acc);
    c->rescale(pacc);
    return acc;
}

std::vector<Ct> scatter(Context* c, MfState& m, const std::vector<Ct*>& Gs, const std::vector<uint64_t>& tabs,
                        bool users, double a_t, int level) {
    const double lam = c->prm.lambda;
    const int n_ent = users ? m.n_users : m.n_items;
    const std::vector<double>& deg = users ? m.deg_u : m.deg_v;
    std::vector<std::vector<Move>> moves(tabs.size());
    for (int r = 0; r < m.nnz; ++r) {
        const int e = users ? m.rows[r] : m.col_idx[r];
        const double w = c->prm.rule == 2 ? a_t / deg[e] : a_t;
        moves[e / m.D].push_back({m.ct_of[r], m.blk_of[r], e % m.D, w});
    }
    std::vector<SelfTerm> selfs(tabs.size());
    for (size_t d = 0; d < tabs.size(); ++d) {
        selfs[d].t = &c->get(tabs[d]);
        std::vector<std::pair<int, double>> ws;
        for (int b = 0; b < m.D; ++b) {
            const int e = (int)d * m.D + b;
            if (e >= n_ent) break;
            double w;
            if (c->prm.rule == 2) w = deg[e] > 0 ? (1.0 - a_t * lam) : 1.0;
            else w = 1.0 - a_t * lam * deg[e];
            ws.push_back({b, w});
        }
        // c: the lower median of the entries' weights
        std::vector<double> srt;
        for (auto& bw : ws) srt.push_back(bw.second);
        std::sort(srt.begin(), srt.end());
        selfs[d].c = srt[(srt.size() - 1) / 2];
        for (auto& bw : ws)
            if (bw.second != selfs[d].c) selfs[d].corr.push_back({bw.first, bw.second - selfs[d].c});
    }
    return block_permute(c, m, Gs, moves, &selfs, level, false);
}

std::vector<Ct> gather(Context* c, MfState& m, const std::vector<uint64_t>& tabs, bool users) {
    std::vector<std::vector<Move>> moves(m.n_ct);
    for (int r = 0; r < m.nnz; ++r) {
        const int e = users ? m.rows[r] : m.col_idx[r];
        moves[m.ct_of[r]].push_back({e / m.D, e % m.D, m.blk_of[r], 1.0});
    }
    std::vector<Ct*> srcs = cts_of(c, tabs);
    return block_permute(c, m, srcs, moves, nullptr, srcs[0]->level, true);
}

std::vector<uint64_t> put_all(Context* c, std::vector<Ct>& v) {
    std::vector<uint64_t> h;
    for (auto& x : v) h.push_back(c->put(x));
    v.clear();
    return h;
}

// Forward dot products of gathered factors: HMult + windowed block sum.
std::vector<Ct> dot_products(Context* c, MfState& m, const std::vector<Ct*>& ug, const std::vector<Ct*>& vg,
                             double* sp_out) {
    std::vector<Ct> T = hmult_all(c, ug, vg);
    if (sp_out) *sp_out = T[0].scale;
    for (int s = 1; s < m.B; s *= 2) {
        std::vector<Ct> sum = rotate_add_all(c, ptrs(T), s);
        release(c, T);
        T = std::move(sum);
    }
    std::vector<Ct*> pt = ptrs(T);
    std::vector<Ct> S = rotate_all(c, pt, -(int64_t)m.kp);
    release(c, T);
    return S;
}

// Refresh of the tables (see kRefreshLevel): mask, decrypt to integers mod q_0,
// encrypt the same integers at the top level and scale, unmask.
void refresh_tables(Context* c, MfState& m) {
    c->sync();
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<uint64_t> all;
    for (uint64_t h : m.Utab) all.push_back(h);
    for (uint64_t h : m.Vtab) all.push_back(h);
    std::vector<uint64_t> w(c->N);
    std::vector<int64_t> mask(c->N), neg(c->N), plain(c->N);
    std::vector<uint64_t> fresh;
    for (size_t j = 0; j < all.size(); ++j) {
        const uint32_t obj = (uint32_t)m.refresh_round * 1024u + (uint32_t)j;
        chacha20_words(c->seed, kRefreshMask, obj, 0, c->N, w.data());
        for (uint64_t n = 0; n < c->N; ++n) {
            mask[n] = (int64_t)(w[n] % (1ull << (kRefreshMaskBits + 1))) - (int64_t)(1ull << kRefreshMaskBits);
            neg[n] = -mask[n];
        }
        const Ct& t = c->get(all[j]);
        Ct masked;
        c->add_plain(t, mask.data(), masked);
        c->decrypt_int(masked, plain.data());
        c->pool.put(masked.d);
        std::vector<Ct> out;
        const uint32_t serial = kRefreshSerial + obj;
        c->encrypt_int_batch(plain.data(), 1, c->L, t.scale, out, &serial);
        Ct un;
        c->add_plain(out[0], neg.data(), un);
        c->pool.put(out[0].d);
        fresh.push_back(c->put(un));
    }
    const size_t nu = m.Utab.size();
    free_handles(c, m.Utab);
    free_handles(c, m.Vtab);
    m.Utab.assign(fresh.begin(), fresh.begin() + (long)nu);
    m.Vtab.assign(fresh.begin() + (long)nu, fresh.end());
    m.refresh_round++;
    c->sync();
    m.refresh_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// Gather the factors for an epoch, refreshing the tables first if their level
// is below kRefreshLevel (only when the parameters allow refresh).
void prepare_epoch(Context* c, MfState& m) {
    if (c->get(m.Utab[0]).level < kRefreshLevel) {
        if (!c->prm.refresh_mode) throw Error(CSRMF_E_LEVEL, "level budget exhausted (refresh_mode = 0)");
        refresh_tables(c, m);
    }
    std::vector<Ct> gu = gather(c, m, m.Utab, true);
    std::vector<Ct> gv = gather(c, m, m.Vtab, false);
    free_handles(c, m.Ug);
    free_handles(c, m.Vg);
    m.Ug = put_all(c, gu);
    m.Vg = put_all(c, gv);
}

// One epoch from the gathered factors m.Ug, m.Vg: dot products, errors,
// gradient terms, scatter into the tables.
void run_epoch(Context* c, MfState& m) {
    const double a_t = c->prm.lr / (1.0 + c->prm.damp * (double)m.epochs_done);
    std::vector<Ct*> ug = cts_of(c, m.Ug), vg = cts_of(c, m.Vg), R = cts_of(c, m.R);
    const int lvl = ug[0]->level;
    if (lvl < 3) throw Error(CSRMF_E_LEVEL, "not enough levels left for an epoch");
    double sp = 0;
    std::vector<Ct> S = dot_products(c, m, ug, vg, &sp);
    const int slv = S[0].level;
    // R_e = drop(Rescale(R * W_R)); E = R_e - Sdot
    const double q_R = (double)c->moduli[R[0]->level];
    const int64_t WR = (int64_t)std::nearbyint((sp * q_R) / R[0]->scale);
    std::vector<Ct> Re(m.n_ct);
    for (int i = 0; i < m.n_ct; ++i) c->mul_int(*R[i], WR, Re[i]);
    std::vector<Ct*> pre = ptrs(Re);
    c->rescale(pre);
    for (auto& x : Re) x.level = slv;
    std::vector<Ct*> ps = ptrs(S);
    std::vector<Ct> E = add_all(c, pre, ps, true);
    release(c, Re);
    const int elv = E[0].level;
    std::vector<Ct*> pe = ptrs(E);
    std::vector<Ct> vgd = dropped(vg, elv), ugd = dropped(ug, elv);
    std::vector<Ct*> pvgd = ptrs(vgd), pugd = ptrs(ugd);
    std::vector<Ct> GU = hmult_all(c, pe, pvgd);
    std::vector<Ct> GV = hmult_all(c, pe, pugd);
    release(c, E);
    // the gathered factors are not needed any more (the next epoch gathers anew)
    free_handles(c, m.Ug);
    free_handles(c, m.Vg);
    const int glv = GU[0].level;
    std::vector<Ct*> pgu = ptrs(GU), pgv = ptrs(GV);
    std::vector<Ct> nu = scatter(c, m, pgu, m.Utab, true, a_t, glv);
    std::vector<Ct> nv = scatter(c, m, pgv, m.Vtab, false, a_t, glv);
    release(c, GU);
    release(c, GV);
    free_handles(c, m.Utab);
    free_handles(c, m.Vtab);
    m.Utab = put_all(c, nu);
    m.Vtab = put_all(c, nv);
    free_handles(c, m.Sdot);
    m.Sdot = put_all(c, S);
    m.epochs_done++;
}

// One Alg. 2 epoch: the batch pairs in turn (see csrmf_mf_epochs).
void run_pair_epoch(Context* c, MfState& m) {
    const double a_t = c->prm.lr / (1.0 + c->prm.damp * (double)m.epochs_done);
    const double lam = c->prm.lambda;
    if (m.Sdot.size() != (size_t)m.n_ct) {
        free_handles(c, m.Sdot);
        m.Sdot.assign(m.n_ct, 0);
    }
    // the initial gathered copies are not used: every pair gathers from the tables
    free_handles(c, m.Ug);
    free_handles(c, m.Vg);
    std::vector<Ct*> R = cts_of(c, m.R);
    for (const MfState::Pair& pr : m.pair_list) {
        if (std::min(c->get(m.Utab[pr.ub]).level, c->get(m.Vtab[pr.vb]).level) < kRefreshLevel) {
            if (!c->prm.refresh_mode) throw Error(CSRMF_E_LEVEL, "level budget exhausted (refresh_mode = 0)");
            refresh_tables(c, m);
        }
        const int nct = pr.ct1 - pr.ct0;
        // gathers from one user table and one item table into the pair's ciphertexts
        std::vector<std::vector<Move>> mu(nct), mv(nct);
        for (int32_t r : pr.ratings) {
            const int t = m.ct_of[r] - pr.ct0;
            mu[t].push_back({0, m.rows[r] % m.D, m.blk_of[r], 1.0});
            mv[t].push_back({0, m.col_idx[r] % m.D, m.blk_of[r], 1.0});
        }
        std::vector<Ct*> su{&c->get(m.Utab[pr.ub])}, sv{&c->get(m.Vtab[pr.vb])};
        std::vector<Ct> ug = block_permute(c, m, su, mu, nullptr, su[0]->level, true);
        std::vector<Ct> vg = block_permute(c, m, sv, mv, nullptr, sv[0]->level, true);
        std::vector<Ct*> pu = ptrs(ug), pv = ptrs(vg);
        double sp = 0;
        std::vector<Ct> S = dot_products(c, m, pu, pv, &sp);
        const int slv = S[0].level;
        std::vector<Ct*> Rp(R.begin() + pr.ct0, R.begin() + pr.ct1);
        const double q_R = (double)c->moduli[Rp[0]->level];
        const int64_t WR = (int64_t)std::nearbyint((sp * q_R) / Rp[0]->scale);
        std::vector<Ct> Re(nct);
        for (int i = 0; i < nct; ++i) c->mul_int(*Rp[i], WR, Re[i]);
        std::vector<Ct*> pre = ptrs(Re);
        c->rescale(pre);
        for (auto& x : Re) x.level = slv;
        std::vector<Ct*> ps = ptrs(S);
        std::vector<Ct> E = add_all(c, pre, ps, true);
        release(c, Re);
        const int elv = E[0].level;
        std::vector<Ct*> pe = ptrs(E);
        std::vector<Ct> vgd = dropped(pv, elv), ugd = dropped(pu, elv);
        std::vector<Ct*> pvgd = ptrs(vgd), pugd = ptrs(ugd);
        std::vector<Ct> GU = hmult_all(c, pe, pvgd);
        std::vector<Ct> GV = hmult_all(c, pe, pugd);
        release(c, E);
        release(c, ug);
        release(c, vg);
        const int glv = GU[0].level;
        // scatter into the pair's two tables: weight a_t per rating, self term
        // 1 - a_t lambda c_e (c_e = the entity's ratings in this pair)
        for (int side = 0; side < 2; ++side) {
            const bool users = side == 0;
            const int tab = users ? pr.ub : pr.vb;
            const int n_ent = users ? m.n_users : m.n_items;
            std::vector<uint64_t>& tabs = users ? m.Utab : m.Vtab;
            std::vector<std::vector<Move>> mvs(1);
            std::map<int, double> cnt;
            for (int32_t r : pr.ratings) {
                const int e = users ? m.rows[r] : m.col_idx[r];
                mvs[0].push_back({m.ct_of[r] - pr.ct0, m.blk_of[r], e % m.D, a_t});
                cnt[e] += 1.0;
            }
            std::vector<SelfTerm> selfs(1);
            selfs[0].t = &c->get(tabs[tab]);
            std::vector<std::pair<int, double>> ws;
            for (int b = 0; b < m.D; ++b) {
                const int e = tab * m.D + b;
                if (e >= n_ent) break;
                auto it = cnt.find(e);
                ws.push_back({b, 1.0 - a_t * lam * (it == cnt.end() ? 0.0 : it->second)});
            }
            std::vector<double> srt;
            for (auto& bw : ws) srt.push_back(bw.second);
            std::sort(srt.begin(), srt.end());
            selfs[0].c = srt[(srt.size() - 1) / 2];
            for (auto& bw : ws)
                if (bw.second != selfs[0].c) selfs[0].corr.push_back({bw.first, bw.second - selfs[0].c});
            std::vector<Ct*> pg = ptrs(users ? GU : GV);
            std::vector<Ct> nt = block_permute(c, m, pg, mvs, &selfs, glv, false);
            c->free_ct(tabs[tab]);
            tabs[tab] = c->put(nt[0]);
        }
        release(c, GU);
        release(c, GV);
        for (int i = 0; i < nct; ++i) {
            if (m.Sdot[pr.ct0 + i]) c->free_ct(m.Sdot[pr.ct0 + i]);
            m.Sdot[pr.ct0 + i] = c->put(S[i]);
        }
    }
    m.epochs_done++;
}

void decrypt_slots(Context* c, uint64_t h, std::vector<double>& z) {
    const Ct& ct = c->get(h);
    std::vector<int64_t> mm(c->N);
    c->decrypt_int(ct, mm.data());
    z.assign(c->N / 2, 0.0);
    ckks_decode(mm.data(), c->logN, ct.scale, z.data(), (int)(c->N / 2));
}

}  // namespace mfp

}  // namespace csrmf

using csrmf::Context;
using csrmf::Error;
using csrmf::MfState;

#define API_BEGIN(ctx)                 \
    if (!(ctx)) { csrmf::last_error() = "null context"; return CSRMF_E_INVAL; } \
    std::lock_guard<std::recursive_mutex> lk_((ctx)->mu); \
    try {
#define API_END_EARLY                  \
    { csrmf::last_error().clear(); return CSRMF_OK; }
#define API_END(ctx)                   \
        csrmf::last_error().clear();            \
        return CSRMF_OK;               \
    } catch (const Error& e) {         \
        csrmf::last_error() = e.what();         \
        return e.code;                 \
    } catch (const std::bad_alloc&) {  \
        csrmf::last_error() = "host allocation failed"; \
        return CSRMF_E_NOMEM;          \
    } catch (const std::exception& e) { \
        csrmf::last_error() = e.what();         \
        return CSRMF_E_DEVICE;         \
    }

void csrmf::mfp::install_layout(Context* c, int32_t n_rows, int32_t n_cols, const int64_t* row_ptr,
                                const int32_t* col_idx) {
    if (!c->have_keys) throw Error(CSRMF_E_STATE, "keygen first");
    MfState* m = csrmf::mfp::make_layout(c, n_rows, n_cols, row_ptr, col_idx);
    // rotation keys the program uses: windowed sum 1, 2, .., B/2 and -k'; the
    // block steps 2^j B (j < log2 D) of the baby and giant trees
    std::vector<int32_t> steps;
    for (int s = 1; s < m->B; s *= 2) steps.push_back(s);
    steps.push_back(-m->kp);
    for (int s = 1; s < m->D; s *= 2) steps.push_back(s * m->B);
    try {
        c->keygen(steps.data(), (int)steps.size(), false);
    } catch (...) {
        delete m;
        throw;
    }
    if (c->mf) {
        csrmf::mfp::free_handles(c, c->mf->R);
        csrmf::mfp::free_handles(c, c->mf->Utab);
        csrmf::mfp::free_handles(c, c->mf->Vtab);
        csrmf::mfp::free_handles(c, c->mf->Ug);
        csrmf::mfp::free_handles(c, c->mf->Vg);
        csrmf::mfp::free_handles(c, c->mf->Sdot);
        csrmf::mfp::free_handles(c, c->mf->Pred);
        csrmf::mfp::free_masks(c, *c->mf);
        delete c->mf;
    }
    c->mf = m;
}

extern "C" {

int csrmf_encrypt_csr_rows(csrmf_ctx* cx, int32_t n_rows, int32_t n_cols, const int64_t* row_ptr,
                           const int32_t* col_idx, const double* values, int32_t* n_ct) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    if (!values) throw Error(CSRMF_E_INVAL, "values");
    for (int64_t p = 0; row_ptr && n_rows > 0 && p < row_ptr[n_rows]; ++p)
        if (!std::isfinite(values[p])) throw Error(CSRMF_E_INVAL, "non-finite rating");
    csrmf::mfp::install_layout(c, n_rows, n_cols, row_ptr, col_idx);
    MfState& m = *c->mf;
    std::vector<std::vector<double>> zs(m.n_ct, std::vector<double>(c->N / 2));
    csrmf::mfp::fill_rating_slots(m, 0, values, nullptr, nullptr, zs);
    const double scale = std::ldexp(1.0, c->prm.log2_scale);
    std::vector<int64_t> pt = csrmf::mfp::encode_all(c, zs, scale);
    m.R = csrmf::mfp::encrypt_list(c, pt.data(), m.n_ct, scale);
    if (n_ct) *n_ct = m.n_ct;
    API_END(c)
}

int csrmf_encrypt_csr_rows_int(csrmf_ctx* cx, int32_t n_rows, int32_t n_cols, const int64_t* row_ptr,
                               const int32_t* col_idx, const int64_t* plain, int32_t n_plain, int32_t* n_ct) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    if (!plain) throw Error(CSRMF_E_INVAL, "plaintexts");
    csrmf::mfp::install_layout(c, n_rows, n_cols, row_ptr, col_idx);
    MfState& m = *c->mf;
    if (n_plain != m.n_ct) throw Error(CSRMF_E_INVAL, "number of plaintexts differs from the layout's ciphertexts");
    m.R = csrmf::mfp::encrypt_list(c, plain, m.n_ct, std::ldexp(1.0, c->prm.log2_scale));
    if (n_ct) *n_ct = m.n_ct;
    API_END(c)
}

int csrmf_mf_layout(const csrmf_ctx* cx, int32_t* n_ct, int32_t* n_utab, int32_t* n_vtab, int32_t* D, int32_t* B) {
    Context* c = const_cast<Context*>(reinterpret_cast<const Context*>(cx));
    API_BEGIN(c)
    MfState& m = csrmf::mfp::state(c);
    if (n_ct) *n_ct = m.n_ct;
    if (n_utab) *n_utab = m.n_utab;
    if (n_vtab) *n_vtab = m.n_vtab;
    if (D) *D = m.D;
    if (B) *B = m.B;
    API_END(c)
}

int csrmf_mf_stats(const csrmf_ctx* cx, int32_t* epochs_done, int32_t* refreshes, double* refresh_seconds) {
    Context* c = const_cast<Context*>(reinterpret_cast<const Context*>(cx));
    API_BEGIN(c)
    MfState& m = csrmf::mfp::state(c);
    if (epochs_done) *epochs_done = m.epochs_done;
    if (refreshes) *refreshes = m.refresh_round;
    if (refresh_seconds) *refresh_seconds = m.refresh_seconds;
    API_END(c)
}

int csrmf_mf_mac_counts(const csrmf_ctx* cx, int64_t* counts) {
    Context* c = const_cast<Context*>(reinterpret_cast<const Context*>(cx));
    API_BEGIN(c)
    if (!counts) throw Error(CSRMF_E_INVAL, "counts");
    const MfState& m = csrmf::mfp::state(c);
    const int64_t v[7] = {m.mac_tasks, m.mac_groups, m.mac_terms, m.mac_const_terms,
                          m.mac_task_rows, m.mac_group_rows, m.mac_term_rows};
    std::memcpy(counts, v, sizeof(v));
    API_END(c)
}

int csrmf_init_factors(csrmf_ctx* cx, const double* U0, const double* V0) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    MfState& m = csrmf::mfp::state(c);
    if (!U0 || !V0) throw Error(CSRMF_E_INVAL, "factors");
    const double scale = std::ldexp(1.0, c->prm.log2_scale);
    std::vector<std::vector<double>> zu(m.n_utab, std::vector<double>(c->N / 2)), zv(m.n_vtab, std::vector<double>(c->N / 2));
    std::vector<std::vector<double>> gu(m.n_ct, std::vector<double>(c->N / 2)), gv(m.n_ct, std::vector<double>(c->N / 2));
    for (int a = 0; a < m.n_utab; ++a) csrmf::mfp::fill_table_slots(m, a, m.n_users, U0, zu[a]);
    for (int a = 0; a < m.n_vtab; ++a) csrmf::mfp::fill_table_slots(m, a, m.n_items, V0, zv[a]);
    csrmf::mfp::fill_rating_slots(m, 1, nullptr, U0, V0, gu);
    csrmf::mfp::fill_rating_slots(m, 2, nullptr, U0, V0, gv);
    std::vector<int64_t> pu = csrmf::mfp::encode_all(c, zu, scale), pv = csrmf::mfp::encode_all(c, zv, scale);
    std::vector<int64_t> pgu = csrmf::mfp::encode_all(c, gu, scale), pgv = csrmf::mfp::encode_all(c, gv, scale);
    std::vector<int64_t> mask_s, mask_g;
    csrmf::mfp::encode_masks(c, m.k, mask_s, mask_g);
    for (auto* v : {&m.Utab, &m.Vtab, &m.Ug, &m.Vg}) csrmf::mfp::free_handles(c, *v);
    m.Utab = csrmf::mfp::encrypt_list(c, pu.data(), m.n_utab, scale);
    m.Vtab = csrmf::mfp::encrypt_list(c, pv.data(), m.n_vtab, scale);
    m.Ug = csrmf::mfp::encrypt_list(c, pgu.data(), m.n_ct, scale);
    m.Vg = csrmf::mfp::encrypt_list(c, pgv.data(), m.n_ct, scale);
    csrmf::mfp::upload_masks(c, m, mask_s.data(), mask_g.data());
    m.factors = true;
    m.epochs_done = 0;
    m.refresh_round = 0;
    m.refresh_seconds = 0;
    API_END(c)
}

int csrmf_init_factors_int(csrmf_ctx* cx, const int64_t* utab, const int64_t* vtab, const int64_t* ug,
                           const int64_t* vg, const int64_t* mask_scatter, const int64_t* mask_gather) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    MfState& m = csrmf::mfp::state(c);
    if (!utab || !vtab || !ug || !vg || !mask_scatter || !mask_gather) throw Error(CSRMF_E_INVAL, "plaintexts");
    const double scale = std::ldexp(1.0, c->prm.log2_scale);
    for (auto* v : {&m.Utab, &m.Vtab, &m.Ug, &m.Vg}) csrmf::mfp::free_handles(c, *v);
    m.Utab = csrmf::mfp::encrypt_list(c, utab, m.n_utab, scale);
    m.Vtab = csrmf::mfp::encrypt_list(c, vtab, m.n_vtab, scale);
    m.Ug = csrmf::mfp::encrypt_list(c, ug, m.n_ct, scale);
    m.Vg = csrmf::mfp::encrypt_list(c, vg, m.n_ct, scale);
    csrmf::mfp::upload_masks(c, m, mask_scatter, mask_gather);
    m.factors = true;
    m.epochs_done = 0;
    m.refresh_round = 0;
    m.refresh_seconds = 0;
    API_END(c)
}

int csrmf_mf_epochs(csrmf_ctx* cx, int32_t n_epochs) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    MfState& m = csrmf::mfp::state(c);
    if (!m.factors) throw Error(CSRMF_E_STATE, "init_factors first");
    if (n_epochs < 0) throw Error(CSRMF_E_INVAL, "n_epochs");
    if (n_epochs == 0) API_END_EARLY;
    if (m.pairs) {
        if (c->L < csrmf::mfp::kRefreshLevel) throw Error(CSRMF_E_LEVEL, "a batch pair needs 4 levels");
        for (int t = 0; t < n_epochs; ++t) csrmf::mfp::run_pair_epoch(c, m);
        if (!c->capturing) c->sync();
        API_END_EARLY;
    }
    // Level budget: an epoch on gathered factors uses 3 levels, every further
    // one 4 (its gather included).  Without refresh the whole request must fit;
    // with refresh, tables below kRefreshLevel are refreshed before a gather.
    const bool have_g = !m.Ug.empty();
    const int lvl = have_g ? c->get(m.Ug[0]).level : c->get(m.Utab[0]).level - 1;
    if (!c->prm.refresh_mode) {
        if (lvl < 3 + 4 * (n_epochs - 1)) throw Error(CSRMF_E_LEVEL, "not enough levels for the requested epochs");
    } else if (c->L < csrmf::mfp::kRefreshLevel) {
        if (lvl < 3 + 4 * (n_epochs - 1)) throw Error(CSRMF_E_LEVEL, "chain too short to refresh");
    }
    for (int t = 0; t < n_epochs; ++t) {
        if (t > 0 || !have_g) csrmf::mfp::prepare_epoch(c, m);
        csrmf::mfp::run_epoch(c, m);
    }
    if (!c->capturing) c->sync();   // a captured epoch runs when its graph is launched
    API_END(c)
}

int csrmf_set_baby_budget(csrmf_ctx* cx, int32_t max_babies) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    if (max_babies < 1) throw Error(CSRMF_E_INVAL, "baby budget must be at least 1");
    c->max_babies = max_babies;
    API_END(c)
}

int csrmf_predict(csrmf_ctx* cx) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    MfState& m = csrmf::mfp::state(c);
    if (!m.factors) throw Error(CSRMF_E_STATE, "init_factors first");
    if (c->get(m.Utab[0]).level < 2) throw Error(CSRMF_E_LEVEL, "predict needs 2 levels (gather + product)");
    std::vector<csrmf::Ct> gu = csrmf::mfp::gather(c, m, m.Utab, true);
    std::vector<csrmf::Ct> gv = csrmf::mfp::gather(c, m, m.Vtab, false);
    std::vector<csrmf::Ct*> pu = csrmf::mfp::ptrs(gu), pv = csrmf::mfp::ptrs(gv);
    std::vector<csrmf::Ct> S = csrmf::mfp::dot_products(c, m, pu, pv, nullptr);
    csrmf::mfp::release(c, gu);
    csrmf::mfp::release(c, gv);
    csrmf::mfp::free_handles(c, m.Pred);
    m.Pred = csrmf::mfp::put_all(c, S);
    API_END(c)
}

int csrmf_decrypt_factors(csrmf_ctx* cx, double* U, double* V) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    MfState& m = csrmf::mfp::state(c);
    if (!m.factors) throw Error(CSRMF_E_STATE, "init_factors first");
    if (!U || !V) throw Error(CSRMF_E_INVAL, "outputs");
    std::vector<double> z;
    for (int a = 0; a < m.n_utab; ++a) {
        csrmf::mfp::decrypt_slots(c, m.Utab[a], z);
        for (int b = 0; b < m.D && a * m.D + b < m.n_users; ++b)
            for (int f = 0; f < m.k; ++f) U[(size_t)(a * m.D + b) * m.k + f] = z[(size_t)b * m.B + f];
    }
    for (int a = 0; a < m.n_vtab; ++a) {
        csrmf::mfp::decrypt_slots(c, m.Vtab[a], z);
        for (int b = 0; b < m.D && a * m.D + b < m.n_items; ++b)
            for (int f = 0; f < m.k; ++f) V[(size_t)(a * m.D + b) * m.k + f] = z[(size_t)b * m.B + f];
    }
    API_END(c)
}

int csrmf_decrypt_predictions(csrmf_ctx* cx, double* rhat, int32_t which) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    MfState& m = csrmf::mfp::state(c);
    if (!rhat) throw Error(CSRMF_E_INVAL, "output");
    const std::vector<uint64_t>& src = which == 0 ? m.Sdot : m.Pred;
    if (which != 0 && which != 1) throw Error(CSRMF_E_INVAL, "which must be 0 or 1");
    if (src.empty()) throw Error(CSRMF_E_STATE, which == 0 ? "no epoch has run" : "csrmf_predict has not run");
    std::vector<double> z;
    int cur = -1;
    for (int r = 0; r < m.nnz; ++r) {
        if (m.ct_of[r] != cur) {
            cur = m.ct_of[r];
            csrmf::mfp::decrypt_slots(c, src[cur], z);
        }
        rhat[r] = z[(size_t)m.blk_of[r] * m.B];
    }
    API_END(c)
}

int csrmf_mf_handles(const csrmf_ctx* cx, int32_t which, uint64_t* out, int32_t cap, int32_t* n) {
    Context* c = const_cast<Context*>(reinterpret_cast<const Context*>(cx));
    API_BEGIN(c)
    MfState& m = csrmf::mfp::state(c);
    const std::vector<uint64_t>* v;
    switch (which) {
        case 0: v = &m.R; break;
        case 1: v = &m.Utab; break;
        case 2: v = &m.Vtab; break;
        case 3: v = &m.Ug; break;
        case 4: v = &m.Vg; break;
        case 5: v = &m.Sdot; break;
        case 6: v = &m.Pred; break;
        default: throw Error(CSRMF_E_INVAL, "which");
    }
    if (n) *n = (int32_t)v->size();
    for (int32_t i = 0; out && i < cap && i < (int32_t)v->size(); ++i) out[i] = (*v)[i];
    API_END(c)
}

}  // extern "C"
