// Serving loop: per-user encrypted PREDICT / UPDATE requests against resident
// encrypted factor tables, with continuous batching and admission by
// ciphertext memory footprint.
//
// A request carries a user i, its items j_1..j_d (and, for UPDATE, the
// ratings r_ij, encrypted on admission with randomness derived from the
// client's serial, so a request's ciphertexts do not depend on its batch).
// The row is cut into chunks of at most D blocks.  For each chunk:
//   gather Ug (u_i in every used block) and Vg (v_j in block t) from the
//   tables (block permutation with the tables' baby-step rotations cached at
//   server creation, since the tables are read-only while serving);
//   Sdot = windowed block sum of HMult(Ug, Vg)         (slot tB holds <u_i, v_j>)
// PREDICT returns Sdot per chunk.  UPDATE (rule R2 of the epoch, one user):
//   E = drop(Rescale(R * W_R)) - Sdot;  G = HMult(E, Vg);
//   T = sum over all D blocks (rotate-and-sum by B*2^a) of G, added over chunks;
//   u_i' = (1 - a*lambda) * Ug + (a/d) * T     (integer weights at a declared
//   scale 2^40 * q, one rescale), returned in broadcast layout (block 0 read).
// Every step is a deterministic function of the request and the resident
// state, and batching only groups launches, so a result is the same alone
// and in any mix.
//
// Continuous batching: the worker admits queued requests while their
// ciphertext footprint fits the budget left by every batch still on the
// device, enqueues the batch's launches on the context's stream and records
// a completion event, without waiting; up to max_inflight batches are
// pipelined, so the host prepares (encodes, encrypts, plans) the next batch
// while earlier ones run and the device never idles between batches.  A
// request is done, and its footprint returned, when its batch's event has
// completed.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>
#include <unordered_set>

#include "host_math.h"
#include "mf_internal.h"

namespace csrmf {

namespace {
double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
}  // namespace

struct ServeRequest {
    uint64_t id = 0;
    int op = 0;                 // 0 PREDICT, 1 UPDATE
    int user = 0;
    uint32_t client_serial = 0;
    std::vector<int32_t> items;
    std::vector<double> ratings;
    std::vector<int64_t> plain;     // UPDATE: encoded rating chunks [n_chunks][N] (else empty: encode ratings)
    int status = 0;             // 0 queued, 1 running, 2 done, < 0 error code
    std::string error;
    std::vector<uint64_t> result;
    double t_submit = 0, t_start = 0, t_done = 0;
    size_t footprint = 0;
    int n_chunks = 0;
};

struct Server {
    Context* c = nullptr;
    MfState lay;                           // k, k', B, D, G and the indicator I0
    std::vector<uint64_t> Utab, Vtab;      // resident tables (handles)
    mfp::BabyCache ucache, vcache;
    double lr = 0, lam = 0;
    size_t budget = 0, in_flight = 0;
    int max_batch = 64;
    int max_inflight = 4;                  // batches enqueued and not yet complete
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv, done_cv;
    bool stop = false;
    std::deque<ServeRequest*> pending;
    std::map<uint64_t, ServeRequest*> reqs;
    std::unordered_set<uint32_t> update_serials;   // client serials of admitted UPDATEs (encryption randomness)
    uint64_t next_id = 1;
    long batches = 0, processed = 0, max_seen_batch = 0, overlapped = 0, max_seen_inflight = 0;
    std::string fatal;

    struct InFlight {
        std::vector<ServeRequest*> batch;
        hipEvent_t done = nullptr;
    };
    std::deque<InFlight> inflight;         // worker thread only (under mu)
    std::vector<hipEvent_t> spare_events;

    ~Server();
    void run();
    void process(std::vector<ServeRequest*>& batch);
    void retire_locked(bool wait_all);
};

namespace {

uint32_t chunk_serial(uint32_t client_serial, int chunk) { return 0x40000000u + client_serial * 8u + (uint32_t)chunk; }

void encrypt_tables(Context* c, MfState& m, int n_ent, const double* F, std::vector<uint64_t>& out) {
    const int n_tab = (n_ent + m.D - 1) / m.D;
    std::vector<std::vector<double>> zs(n_tab, std::vector<double>(c->N / 2, 0.0));
    for (int e = 0; e < n_ent; ++e)
        for (int f = 0; f < m.k; ++f) zs[e / m.D][(size_t)(e % m.D) * m.B + f] = F[(size_t)e * m.k + f];
    const double scale = std::ldexp(1.0, c->prm.log2_scale);
    std::vector<int64_t> pt = mfp::encode_all(c, zs, scale);
    std::vector<Ct> cts;
    c->encrypt_int_batch(pt.data(), n_tab, c->L, scale, cts);
    out = mfp::put_all(c, cts);
}

void cache_babies(Context* c, MfState& m, const std::vector<uint64_t>& tabs, mfp::BabyCache& cache) {
    std::vector<Ct*> src;
    for (uint64_t h : tabs) src.push_back(&c->get(h));
    Context::Hoist hs;
    c->hoist_begin(hs, src);
    for (int beta = 1; beta < m.G; ++beta) {
        std::vector<Ct> out(src.size());
        std::vector<Ct*> po = mfp::ptrs(out);
        c->hoist_rotate(hs, c->galois_for_step((int64_t)beta * m.B), po);
        for (size_t i = 0; i < src.size(); ++i) cache[{(int)i, beta}] = out[i];
    }
}

size_t request_footprint(const Context* c, int n_chunks) {
    // rating, two gathered factors, product, window sums, error, gradient,
    // block sums and the combine: about 16 ciphertexts per chunk
    return (size_t)n_chunks * 16 * c->ct_words() * 8;
}

}  // namespace

void destroy_server(Server* s) { delete s; }

Server::~Server() {
    {
        std::lock_guard<std::mutex> lk(mu);
        stop = true;
    }
    cv.notify_all();
    if (worker.joinable()) worker.join();
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    for (hipEvent_t e : spare_events) (void)hipEventDestroy(e);
    for (size_t i = 0; i < c->servers.size(); ++i)
        if (c->servers[i] == this) {
            c->servers.erase(c->servers.begin() + (long)i);
            break;
        }
    for (auto& kv : reqs) delete kv.second;
    for (auto& kv : ucache) c->pool.put(kv.second.d);
    for (auto& kv : vcache) c->pool.put(kv.second.d);
    mfp::free_handles(c, Utab);
    mfp::free_handles(c, Vtab);
    mfp::free_masks(c, lay);
}

// Batches whose completion event has fired are done (oldest first; one
// stream, so they complete in order).  wait_all: wait for every batch.
void Server::retire_locked(bool wait_all) {
    while (!inflight.empty()) {
        InFlight& f = inflight.front();
        if (wait_all) {
            (void)hipEventSynchronize(f.done);
        } else {
            const hipError_t q = hipEventQuery(f.done);
            if (q == hipErrorNotReady) break;
            if (q != hipSuccess)
                for (ServeRequest* r : f.batch)
                    if (r->status == 1) { r->status = CSRMF_E_DEVICE; r->error = hipGetErrorString(q); }
        }
        const double t = now_s();
        for (ServeRequest* r : f.batch) {
            if (r->status == 1) r->status = 2;
            r->t_done = t;
            in_flight -= r->footprint;
        }
        spare_events.push_back(f.done);
        inflight.pop_front();
        done_cv.notify_all();
    }
}

void Server::run() {
    for (;;) {
        std::vector<ServeRequest*> batch;
        {
            std::unique_lock<std::mutex> lk(mu);
            retire_locked(false);
            if (stop) {
                retire_locked(true);
                return;
            }
            // admit while the footprint fits the budget left by the batches in flight
            if ((int)inflight.size() < max_inflight) {
                while (!pending.empty() && (int)batch.size() < max_batch &&
                       in_flight + pending.front()->footprint <= budget) {
                    ServeRequest* r = pending.front();
                    pending.pop_front();
                    in_flight += r->footprint;
                    r->status = 1;
                    r->t_start = now_s();
                    batch.push_back(r);
                }
            }
            if (batch.empty()) {
                if (inflight.empty()) cv.wait(lk, [&] { return stop || !pending.empty(); });
                else cv.wait_for(lk, std::chrono::microseconds(200));   // poll the device
                continue;
            }
            if (!inflight.empty()) overlapped++;
        }
        hipEvent_t ev = nullptr;
        bool failed = false;
        try {
            std::lock_guard<std::recursive_mutex> lk(c->mu);
            process(batch);
            {
                std::lock_guard<std::mutex> lk2(mu);
                if (!spare_events.empty()) {
                    ev = spare_events.back();
                    spare_events.pop_back();
                }
            }
            if (!ev) CSRMF_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
            CSRMF_HIP(hipEventRecord(ev, c->stream));
        } catch (const Error& e) {
            failed = true;
            std::lock_guard<std::mutex> lk(mu);
            for (ServeRequest* r : batch) { r->status = e.code; r->error = e.what(); }
        } catch (const std::exception& e) {
            failed = true;
            std::lock_guard<std::mutex> lk(mu);
            for (ServeRequest* r : batch) { r->status = CSRMF_E_DEVICE; r->error = e.what(); }
        }
        if (failed) {
            // let queued work drain before the footprint is given back
            try {
                std::lock_guard<std::recursive_mutex> lk(c->mu);
                c->sync();
            } catch (...) {
            }
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            if (failed || !ev) {
                const double t = now_s();
                for (ServeRequest* r : batch) {
                    r->t_done = t;
                    in_flight -= r->footprint;
                }
                if (ev) spare_events.push_back(ev);
                done_cv.notify_all();
            } else {
                inflight.push_back({batch, ev});
                if ((long)inflight.size() > max_seen_inflight) max_seen_inflight = (long)inflight.size();
            }
            batches++;
            processed += (long)batch.size();
            if ((long)batch.size() > max_seen_batch) max_seen_batch = (long)batch.size();
        }
    }
}

void Server::process(std::vector<ServeRequest*>& batch) {
    const int D = lay.D, B = lay.B, k = lay.k, L = c->L;
    struct Chunk { int req; int s, e; };
    std::vector<Chunk> chunks;
    for (int r = 0; r < (int)batch.size(); ++r) {
        const int d = (int)batch[r]->items.size();
        for (int s = 0; s < d; s += D) chunks.push_back({r, s, std::min(d, s + D)});
    }
    const int nc = (int)chunks.size();
    // gather u_i and the v_j of every chunk
    std::vector<std::vector<mfp::Move>> mu_(nc), mv_(nc);
    for (int i = 0; i < nc; ++i) {
        const ServeRequest* r = batch[chunks[i].req];
        for (int t = chunks[i].s; t < chunks[i].e; ++t) {
            mu_[i].push_back({r->user / D, r->user % D, t - chunks[i].s, 1.0});
            const int j = r->items[t];
            mv_[i].push_back({j / D, j % D, t - chunks[i].s, 1.0});
        }
    }
    std::vector<Ct*> us, vs;
    for (uint64_t h : Utab) us.push_back(&c->get(h));
    for (uint64_t h : Vtab) vs.push_back(&c->get(h));
    std::vector<Ct> Ug = mfp::block_permute_cached(c, lay, us, mu_, nullptr, L, &ucache, true);
    std::vector<Ct> Vg = mfp::block_permute_cached(c, lay, vs, mv_, nullptr, L, &vcache, true);
    std::vector<Ct*> pu = mfp::ptrs(Ug), pv = mfp::ptrs(Vg);
    double sp = 0;
    std::vector<Ct> S = mfp::dot_products(c, lay, pu, pv, &sp);
    // PREDICT: the dot products are the result
    std::vector<int> upd;
    for (int i = 0; i < nc; ++i) {
        ServeRequest* r = batch[chunks[i].req];
        if (r->op == 0) {
            r->result.push_back(c->put(S[i]));
            S[i].d = nullptr;
        } else {
            upd.push_back(i);
        }
    }
    if (!upd.empty()) {
        // encrypt the rating chunks (client side; randomness from the client
        // serial): the client's encoded plaintexts, or the ratings encoded here
        const int nu = (int)upd.size();
        const size_t N = c->N;
        std::vector<int64_t> pt((size_t)nu * N);
        std::vector<uint32_t> serials;
        for (int u = 0; u < nu; ++u) {
            const Chunk& ch = chunks[upd[u]];
            const ServeRequest* r = batch[ch.req];
            int idx = 0;
            for (int i = 0; i < upd[u]; ++i) idx += chunks[i].req == ch.req;
            serials.push_back(chunk_serial(r->client_serial, idx));
            if (!r->plain.empty()) {
                std::memcpy(pt.data() + (size_t)u * N, r->plain.data() + (size_t)idx * N, N * 8);
            } else {
                std::vector<std::vector<double>> zs(1, std::vector<double>(N / 2, 0.0));
                for (int t = ch.s; t < ch.e; ++t)
                    for (int f = 0; f < k; ++f) zs[0][(size_t)(t - ch.s) * B + f] = r->ratings[t];
                std::vector<int64_t> one = mfp::encode_all(c, zs, std::ldexp(1.0, c->prm.log2_scale));
                std::memcpy(pt.data() + (size_t)u * N, one.data(), N * 8);
            }
        }
        const double scale = std::ldexp(1.0, c->prm.log2_scale);
        std::vector<Ct> R;
        c->encrypt_int_batch(pt.data(), nu, L, scale, R, serials.data());
        // E = drop(Rescale(R * W_R)) - Sdot
        const int64_t WR = (int64_t)std::nearbyint((sp * (double)c->moduli[L]) / R[0].scale);
        std::vector<Ct> Re(nu);
        for (int u = 0; u < nu; ++u) c->mul_int(R[u], WR, Re[u]);
        std::vector<Ct*> pre = mfp::ptrs(Re);
        c->rescale(pre);
        std::vector<Ct*> ps, pvg, pug;
        for (int u = 0; u < nu; ++u) {
            Re[u].level = S[upd[u]].level;
            ps.push_back(&S[upd[u]]);
        }
        std::vector<Ct> E = mfp::add_all(c, pre, ps, true);
        std::vector<Ct> vgd, ugd;
        for (int u = 0; u < nu; ++u) {
            Ct a = Vg[upd[u]];
            a.level = E[0].level;
            vgd.push_back(a);
        }
        std::vector<Ct*> pe = mfp::ptrs(E), pvd = mfp::ptrs(vgd);
        std::vector<Ct> T = mfp::hmult_all(c, pe, pvd);
        // sum over all blocks
        for (int s = B; s < B * D; s *= 2) {
            std::vector<Ct> sum = mfp::rotate_add_all(c, mfp::ptrs(T), s);
            mfp::release(c, T);
            T = std::move(sum);
        }
        // per request: add chunk sums, then combine with the self term
        std::map<int, std::vector<int>> by_req;
        for (int u = 0; u < nu; ++u) by_req[chunks[upd[u]].req].push_back(u);
        for (auto& kv : by_req) {
            ServeRequest* r = batch[kv.first];
            Ct tot = T[kv.second[0]];
            T[kv.second[0]].d = nullptr;
            for (size_t q = 1; q < kv.second.size(); ++q) {
                Ct sum;
                c->add(tot, T[kv.second[q]], sum, false);
                c->pool.put(tot.d);
                tot = sum;
            }
            const int lvl = tot.level;
            const double q_acc = (double)c->moduli[lvl];
            const double target = mfp::target_scale(c) * q_acc;
            const double d = (double)r->items.size();
            Ct self = Ug[upd[kv.second[0]]];
            self.level = lvl;
            const int64_t Ws = (int64_t)std::nearbyint(((1.0 - lr * lam) * mfp::target_scale(c) * q_acc) / self.scale);
            const int64_t Wg = (int64_t)std::nearbyint(((lr / d) * mfp::target_scale(c) * q_acc) / tot.scale);
            Ct a, b, out;
            c->mul_int(self, Ws, a, target);
            c->mul_int(tot, Wg, b, target);
            c->add(a, b, out, false);
            c->pool.put(a.d);
            c->pool.put(b.d);
            c->pool.put(tot.d);
            std::vector<Ct*> po{&out};
            c->rescale(po);
            r->result.push_back(c->put(out));
        }
        mfp::release(c, R);
        mfp::release(c, Re);
        mfp::release(c, E);
        for (auto& t : T)
            if (t.d) c->pool.put(t.d);
    }
    for (auto& s : S)
        if (s.d) c->pool.put(s.d);
    mfp::release(c, Ug);
    mfp::release(c, Vg);
}

}  // namespace csrmf

using csrmf::Context;
using csrmf::Error;
using csrmf::Server;
using csrmf::ServeRequest;

namespace {

// Shared by the float and the integer-plaintext forms: tables from U, V
// (encoded here) or from the caller's encodings utab/vtab with the gather
// indicator mask_g (I_0 at 2^30); table encryptions take the context's
// running serials, U tables first.
int create_server(Context* c, int32_t n_users, int32_t n_items, const double* U, const double* V,
                  const int64_t* utab, const int64_t* vtab, const int64_t* mask_g_in, double hbm_budget_bytes,
                  int32_t max_batch, csrmf_server** out) {
    if (!c || !out) {
        csrmf::last_error() = "server: null argument";
        return CSRMF_E_INVAL;
    }
    *out = nullptr;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    Server* s = nullptr;
    try {
        if (!c->have_keys) throw Error(CSRMF_E_STATE, "keygen first");
        const bool from_int = utab != nullptr;
        if (n_users <= 0 || n_items <= 0 || !(hbm_budget_bytes > 0) || max_batch <= 0 ||
            (from_int ? (!vtab || !mask_g_in) : (!U || !V)))
            throw Error(CSRMF_E_INVAL, "server arguments");
        const int k = c->prm.k;
        if (k <= 0) throw Error(CSRMF_E_INVAL, "params.k must be positive");
        // a PREDICT uses 2 levels (gather, product), an UPDATE 4 (and its gradient and combine)
        if (c->L < 2) throw Error(CSRMF_E_LEVEL, "serving needs at least 2 levels (4 for updates)");
        s = new Server();
        s->c = c;
        csrmf::MfState& m = s->lay;
        m.k = k;
        m.kp = 1;
        while (m.kp < k) m.kp *= 2;
        m.B = 2 * m.kp;
        m.D = (int)(c->N / (2 * (uint64_t)m.B));
        int logD = 0;
        while ((1 << (logD + 1)) <= m.D) ++logD;
        m.G = 1 << ((logD + 1) / 2);
        m.n_users = n_users;
        m.n_items = n_items;
        s->lr = c->prm.lr;
        s->lam = c->prm.lambda;
        s->budget = (size_t)hbm_budget_bytes;
        s->max_batch = max_batch;
        std::vector<int32_t> steps;
        for (int q = 1; q < m.B; q *= 2) steps.push_back(q);
        steps.push_back(-m.kp);
        for (int b = 1; b < m.G; ++b) steps.push_back(b * m.B);
        for (int g = 1; g < m.D / m.G; ++g) steps.push_back(g * m.G * m.B);
        for (int q = m.B; q < m.B * m.D; q *= 2) steps.push_back(q);
        c->keygen(steps.data(), (int)steps.size(), false);
        std::vector<int64_t> mask_s, mask_g;
        if (from_int) {
            mask_g.assign(mask_g_in, mask_g_in + c->N);
            mask_s = mask_g;   // serving gathers only; the scatter mask is not used
        } else {
            csrmf::mfp::encode_masks(c, k, mask_s, mask_g);
        }
        csrmf::mfp::upload_masks(c, m, mask_s.data(), mask_g.data());
        if (from_int) {
            const double scale = std::ldexp(1.0, c->prm.log2_scale);
            const int nu = (n_users + m.D - 1) / m.D, nv = (n_items + m.D - 1) / m.D;
            std::vector<csrmf::Ct> cu, cv;
            c->encrypt_int_batch(utab, nu, c->L, scale, cu);
            c->encrypt_int_batch(vtab, nv, c->L, scale, cv);
            s->Utab = csrmf::mfp::put_all(c, cu);
            s->Vtab = csrmf::mfp::put_all(c, cv);
        } else {
            csrmf::encrypt_tables(c, m, n_users, U, s->Utab);
            csrmf::encrypt_tables(c, m, n_items, V, s->Vtab);
        }
        csrmf::cache_babies(c, m, s->Utab, s->ucache);
        csrmf::cache_babies(c, m, s->Vtab, s->vcache);
        c->sync();
        c->servers.push_back(s);
        s->worker = std::thread([s] { s->run(); });
    } catch (const Error& e) {
        csrmf::last_error() = e.what();
        delete s;
        return e.code;
    } catch (const std::exception& e) {
        csrmf::last_error() = e.what();
        delete s;
        return CSRMF_E_DEVICE;
    }
    csrmf::last_error().clear();
    *out = reinterpret_cast<csrmf_server*>(s);
    return CSRMF_OK;
}

int submit(Server* s, int32_t op, int32_t user, int32_t n, const int32_t* items, const double* ratings,
           const int64_t* plain, uint32_t client_serial, uint64_t* id) {
    auto fail = [](int code, const char* msg) {
        csrmf::last_error() = msg;
        return code;
    };
    if (!s || !id || n <= 0 || !items || (op != 0 && op != 1)) return fail(CSRMF_E_INVAL, "submit: bad arguments");
    if (op == 1 && !ratings && !plain) return fail(CSRMF_E_INVAL, "submit: an UPDATE needs its ratings");
    if (user < 0 || user >= s->lay.n_users) return fail(CSRMF_E_INVAL, "submit: user out of range");
    if (client_serial >= (1u << 27)) return fail(CSRMF_E_INVAL, "submit: client serial must be below 2^27");
    if (op == 1 && s->c->L < 4) return fail(CSRMF_E_LEVEL, "an UPDATE needs 4 levels");
    for (int32_t i = 0; i < n; ++i) {
        if (items[i] < 0 || items[i] >= s->lay.n_items) return fail(CSRMF_E_INVAL, "submit: item out of range");
        if (i > 0 && items[i] <= items[i - 1]) return fail(CSRMF_E_INVAL, "submit: items must increase (a CSR row)");
        if (op == 1 && ratings && !std::isfinite(ratings[i])) return fail(CSRMF_E_INVAL, "submit: rating not finite");
    }
    const int n_chunks = (n + s->lay.D - 1) / s->lay.D;
    if (n_chunks > 8) return fail(CSRMF_E_INVAL, "submit: a row may span at most 8 chunks of D items");
    const size_t fp = csrmf::request_footprint(s->c, n_chunks);
    if (fp > s->budget) return fail(CSRMF_E_NOMEM, "submit: the request alone exceeds the memory budget");
    ServeRequest* r = new ServeRequest();
    r->op = op;
    r->user = user;
    r->client_serial = client_serial;
    r->items.assign(items, items + n);
    if (op == 1) {
        if (plain) r->plain.assign(plain, plain + (size_t)n_chunks * s->c->N);
        else r->ratings.assign(ratings, ratings + n);
    }
    r->n_chunks = n_chunks;
    r->footprint = fp;
    r->t_submit = csrmf::now_s();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        // an UPDATE's encryption randomness derives from its serial: a reused
        // serial would encrypt different ratings with the same randomness
        if (op == 1 && !s->update_serials.insert(client_serial).second) {
            delete r;
            return fail(CSRMF_E_INVAL, "submit: client serial already used by an UPDATE on this server");
        }
        r->id = s->next_id++;
        s->reqs[r->id] = r;
        s->pending.push_back(r);
        *id = r->id;
    }
    s->cv.notify_all();
    csrmf::last_error().clear();
    return CSRMF_OK;
}

}  // namespace

extern "C" {

int csrmf_server_create(csrmf_ctx* cx, int32_t n_users, int32_t n_items, const double* U, const double* V,
                        double hbm_budget_bytes, int32_t max_batch, csrmf_server** out) {
    return create_server(reinterpret_cast<Context*>(cx), n_users, n_items, U, V, nullptr, nullptr, nullptr,
                         hbm_budget_bytes, max_batch, out);
}

int csrmf_server_create_int(csrmf_ctx* cx, int32_t n_users, int32_t n_items, const int64_t* utab,
                            const int64_t* vtab, const int64_t* mask_gather, double hbm_budget_bytes,
                            int32_t max_batch, csrmf_server** out) {
    if (!utab) {
        csrmf::last_error() = "server: null table plaintexts";
        return CSRMF_E_INVAL;
    }
    return create_server(reinterpret_cast<Context*>(cx), n_users, n_items, nullptr, nullptr, utab, vtab,
                         mask_gather, hbm_budget_bytes, max_batch, out);
}

int csrmf_server_submit(csrmf_server* sv, int32_t op, int32_t user, int32_t n, const int32_t* items,
                        const double* ratings, uint32_t client_serial, uint64_t* id) {
    return submit(reinterpret_cast<Server*>(sv), op, user, n, items, ratings, nullptr, client_serial, id);
}

int csrmf_server_submit_int(csrmf_server* sv, int32_t op, int32_t user, int32_t n, const int32_t* items,
                            const int64_t* plain, uint32_t client_serial, uint64_t* id) {
    if (op == 1 && !plain) {
        csrmf::last_error() = "submit: an UPDATE needs its encoded rating chunks";
        return CSRMF_E_INVAL;
    }
    return submit(reinterpret_cast<Server*>(sv), op, user, n, items, nullptr, plain, client_serial, id);
}

int csrmf_server_poll(csrmf_server* sv, uint64_t id, int32_t wait, int32_t* status, uint64_t* results, int32_t cap,
                      int32_t* n_results, double* latency_s) {
    Server* s = reinterpret_cast<Server*>(sv);
    if (!s) return CSRMF_E_INVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return CSRMF_E_INVAL;
    ServeRequest* r = it->second;
    if (wait) s->done_cv.wait(lk, [&] { return r->status == 2 || r->status < 0; });
    if (status) *status = r->status;
    if (r->status == 2) {
        if (n_results) *n_results = (int32_t)r->result.size();
        for (int32_t i = 0; results && i < cap && i < (int32_t)r->result.size(); ++i) results[i] = r->result[i];
        if (latency_s) *latency_s = r->t_done - r->t_submit;
    }
    return r->status < 0 ? r->status : CSRMF_OK;
}

int csrmf_server_stats(csrmf_server* sv, char* buf, int32_t cap) {
    Server* s = reinterpret_cast<Server*>(sv);
    if (!s) return CSRMF_E_INVAL;
    std::string o;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        o = "{\"batches\": " + std::to_string(s->batches) + ", \"processed\": " + std::to_string(s->processed) +
            ", \"max_batch\": " + std::to_string(s->max_seen_batch) + ", \"queued\": " +
            std::to_string(s->pending.size()) + ", \"in_flight_bytes\": " + std::to_string(s->in_flight) +
            ", \"budget_bytes\": " + std::to_string(s->budget) +
            ", \"overlapped_batches\": " + std::to_string(s->overlapped) +
            ", \"max_batches_in_flight\": " + std::to_string(s->max_seen_inflight) +
            ", \"batches_in_flight\": " + std::to_string(s->inflight.size()) + "}";
    }
    if (buf && cap > 0) {
        const size_t n = std::min<size_t>(o.size(), (size_t)cap - 1);
        std::memcpy(buf, o.data(), n);
        buf[n] = 0;
    }
    return (int)o.size();
}

void csrmf_server_destroy(csrmf_server* sv) { delete reinterpret_cast<Server*>(sv); }

}  // extern "C"
