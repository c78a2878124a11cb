// Context set-up, keys, encryption and the evaluation primitives.
#include "context.h"

#include <algorithm>
#include <cmath>
#include <cstring>

#include "host_math.h"
#include "prof.h"

namespace csrmf {

typedef unsigned __int128 u128;

// ------------------------------------------------------------------ pool
Pool::~Pool() { release_all(); }

size_t Pool::size_class(size_t bytes) {
    if (bytes <= 4096) return 4096;
    int e = 63 - __builtin_clzll((unsigned long long)(bytes - 1));   // 2^e < bytes <= 2^(e+1)
    const size_t step = (size_t)1 << (e - 2);                          // eight classes per octave
    return (bytes + step - 1) / step * step;
}

void* Pool::get(size_t bytes) {
    bytes = size_class(bytes);
    if (capture_) {
        auto ci = cap_free_.find(bytes);
        if (ci != cap_free_.end()) {   // a block the capture freed earlier
            void* p = ci->second;
            cap_free_.erase(ci);
            in_use_ += bytes;
            return p;
        }
    }
    auto it = free_.find(bytes);
    void* p = nullptr;
    if (it != free_.end()) {
        p = it->second;
        free_.erase(it);
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            // give cached blocks back (after the device is idle: queued work may
            // still use them) and retry once
            (void)hipDeviceSynchronize();
            for (auto& kv : free_) { (void)hipFree(kv.second); sizes_.erase(kv.second); }
            free_.clear();
            (void)hipGetLastError();
            e = hipMalloc(&p, bytes);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                throw Error(CSRMF_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
            }
        }
        sizes_[p] = bytes;
    }
    in_use_ += bytes;
    if (capture_) cap_blocks_[p] = bytes;
    return p;
}

void Pool::put(void* p) {
    if (!p) return;
    if (graph_owned_.count(p)) return;   // a graph's block: freed with the graph
    auto it = sizes_.find(p);
    if (it == sizes_.end()) return;
    in_use_ -= it->second;
    if (capture_) {
        cap_blocks_[p] = it->second;
        cap_free_.emplace(it->second, p);
        return;
    }
    free_.emplace(it->second, p);
}

void Pool::begin_capture() {
    capture_ = true;
    cap_blocks_.clear();
    cap_free_.clear();
}

std::vector<void*> Pool::end_capture() {
    capture_ = false;
    std::vector<void*> out;
    for (auto& kv : cap_blocks_) {
        out.push_back(kv.first);
        graph_owned_[kv.first] = kv.second;
    }
    // blocks freed during the capture stay out of the free list: the graph uses them
    for (auto& kv : cap_free_) in_use_ += kv.first;
    cap_blocks_.clear();
    cap_free_.clear();
    return out;
}

void Pool::free_blocks(const std::vector<void*>& v) {
    for (void* p : v) {
        auto g = graph_owned_.find(p);
        if (g == graph_owned_.end()) continue;
        in_use_ -= g->second;
        graph_owned_.erase(g);
        sizes_.erase(p);
        (void)hipFree(p);
    }
}

void Pool::release_all() {
    graph_owned_.clear();
    cap_blocks_.clear();
    cap_free_.clear();
    for (auto& kv : sizes_) (void)hipFree(kv.first);
    sizes_.clear();
    free_.clear();
    in_use_ = 0;
}

// Batched calls process at most this many ciphertexts per launch sequence, so
// that their scratch (ModUp digits: n_digits * (l+1+alpha) limbs per
// ciphertext, ~140 MB at N = 2^16 and 28 limbs) stays bounded; each
// ciphertext's arithmetic is independent of the batch it is in.
constexpr int kMaxBatch = 128;

template <typename F>
static bool split_batch(size_t n, F&& f) {
    if (n <= (size_t)kMaxBatch) return false;
    for (size_t i = 0; i < n; i += kMaxBatch) f(i, std::min(n, i + kMaxBatch));
    return true;
}

static std::vector<Ct*> slice(const std::vector<Ct*>& v, size_t i, size_t j) {
    return std::vector<Ct*>(v.begin() + (long)i, v.begin() + (long)j);
}

std::string& last_error() {
    static thread_local std::string msg;
    return msg;
}

// ------------------------------------------------------------------ staging ring
hipEvent_t HipMarkers::record() {
    hipEvent_t e;
    if (!spare.empty()) {
        e = spare.back();
        spare.pop_back();
    } else {
        CSRMF_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    CSRMF_HIP(hipEventRecord(e, stream));
    return e;
}

void HipMarkers::wait(hipEvent_t e) { CSRMF_HIP(hipEventSynchronize(e)); }

HipMarkers::~HipMarkers() {
    for (hipEvent_t e : spare) (void)hipEventDestroy(e);
}

void Staging::init(hipStream_t s) {
    ops_.stream = s;
    CSRMF_HIP(hipHostMalloc((void**)&host_, kBytes, hipHostMallocDefault));
    CSRMF_HIP(hipMalloc((void**)&dev_, kBytes));
}

void Staging::release() {
    if (ops_.stream) (void)hipStreamSynchronize(ops_.stream);
    ring_.drained(ops_);
    if (host_) (void)hipHostFree(host_);
    if (dev_) (void)hipFree(dev_);
    host_ = dev_ = nullptr;
    ops_.stream = nullptr;
}

void* Staging::put(const void* src, size_t bytes) {
    if (arena_host_) {   // graph capture: the graph's own arena
        const size_t need = (bytes + 255) / 256 * 256;
        if (arena_used_ + need > arena_cap_) throw Error(CSRMF_E_NOMEM, "graph argument arena full");
        uint8_t* h = arena_host_ + arena_used_;
        uint8_t* d = arena_dev_ + arena_used_;
        arena_used_ += need;
        if (bytes) {
            std::memcpy(h, src, bytes);
            CSRMF_HIP(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, ops_.stream));
        }
        return d;
    }
    if (!host_) throw Error(CSRMF_E_STATE, "staging ring not initialised");
    const size_t off = ring_.reserve(bytes, ops_);
    if (bytes) {
        std::memcpy(host_ + off, src, bytes);
        CSRMF_HIP(hipMemcpyAsync(dev_ + off, host_ + off, bytes, hipMemcpyHostToDevice, ops_.stream));
    }
    return dev_ + off;
}

void Context::sync(const char* caller) {
    if (capturing)
        throw Error(CSRMF_E_STATE, std::string(caller) + " waits for the device and cannot be captured in a graph");
    CSRMF_HIP(hipStreamSynchronize(stream));
    staging.drained();
}

// ------------------------------------------------------------------ graphs
void Context::graph_begin() {
    if (capturing) throw Error(CSRMF_E_STATE, "a capture is already open");
    if (prof_enabled()) throw Error(CSRMF_E_STATE, "per-kernel profiling records events: disable it to capture");
    if (!stream) throw Error(CSRMF_E_STATE, "capture needs the context's own stream, not the null stream");
    sync();
    CapturedGraph g;
    CSRMF_HIP(hipHostMalloc((void**)&g.arena_host, kGraphArenaBytes, hipHostMallocDefault));
    hipError_t e = hipMalloc((void**)&g.arena_dev, kGraphArenaBytes);
    if (e != hipSuccess) {
        (void)hipHostFree(g.arena_host);
        throw Error(CSRMF_E_NOMEM, "graph argument arena");
    }
    e = hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
        (void)hipHostFree(g.arena_host);
        (void)hipFree(g.arena_dev);
        throw Error(CSRMF_E_DEVICE, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
    }
    staging.begin_arena(g.arena_host, g.arena_dev, kGraphArenaBytes);
    pool.begin_capture();
    capturing = true;
    graphs[0] = g;   // slot 0: the capture in progress
}

uint64_t Context::graph_end() {
    if (!capturing) throw Error(CSRMF_E_STATE, "no capture is open");
    capturing = false;
    staging.end_arena();
    CapturedGraph g = graphs[0];
    graphs.erase(0);
    g.blocks = pool.end_capture();
    hipError_t e = hipStreamEndCapture(stream, &g.graph);
    if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
    const uint64_t id = next_graph++;
    graphs[id] = g;
    if (e != hipSuccess) {
        graph_destroy(id);
        throw Error(CSRMF_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
    return id;
}

void Context::graph_launch(uint64_t id) {
    auto it = graphs.find(id);
    if (id == 0 || it == graphs.end()) throw Error(CSRMF_E_INVAL, "unknown graph");
    if (capturing) throw Error(CSRMF_E_STATE, "cannot launch a graph while capturing");
    CSRMF_HIP(hipGraphLaunch(it->second.exec, stream));
}

void Context::graph_destroy(uint64_t id) {
    auto it = graphs.find(id);
    if (id == 0 || it == graphs.end()) throw Error(CSRMF_E_INVAL, "unknown graph");
    (void)hipStreamSynchronize(stream);
    CapturedGraph& g = it->second;
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    pool.free_blocks(g.blocks);
    if (g.arena_host) (void)hipHostFree(g.arena_host);
    if (g.arena_dev) (void)hipFree(g.arena_dev);
    graphs.erase(it);
}

// ------------------------------------------------------------------ helpers
static uint64_t mm(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((u128)a * b % q); }

// Constant records of a basis conversion (layout: launch_basis_convert):
// hats[i * targets.size() + t] = Qhat_i mod targets[t]; r_mod[t] = 2^64 mod
// targets[t], qneg_inv[t] = -targets[t]^-1 mod 2^64.  The FP64 form serves the
// targets below kBcFp64Bound when the sums of the sources fit it (centred:
// up to 16 sources, canonical: up to 8).
static std::vector<uint64_t> bc_records(const std::vector<uint64_t>& hats, int ns, bool centered,
                                        const std::vector<uint64_t>& targets, const std::vector<uint64_t>& r_mod,
                                        const std::vector<uint64_t>& qneg_inv) {
    const int R = kBcRecordWords(ns), nt = (int)targets.size();
    const bool fp64_sum = centered ? ns <= 16 : ns <= 8;
    std::vector<uint64_t> rec((size_t)nt * R, 0);
    auto put = [&](size_t at, double v) { std::memcpy(&rec[at], &v, 8); };
    for (int t = 0; t < nt; ++t) {
        const uint64_t q = targets[t];
        const bool f64 = fp64_sum && q < kBcFp64Bound;
        const size_t base = (size_t)t * R;
        for (int i = 0; i < ns; ++i) {
            const uint64_t h = hats[(size_t)i * nt + t];
            if (f64) {
                const int64_t lo = (int64_t)((h + (1u << 19)) & ((1u << 20) - 1)) - (1 << 19);
                put(base + 2 * i, (double)lo);
                put(base + 2 * i + 1, (double)(((int64_t)h - lo) >> 20));
            } else {
                rec[base + i] = mm(h, r_mod[t], q);
            }
        }
        if (!f64) {
            rec[base + 2 * ns + 1] = q;
            rec[base + 2 * ns + 2] = qneg_inv[t];
        } else {
            const double qd = (double)q;
            put(base + 2 * ns, qd);
            put(base + 2 * ns + 1, 1.0 / qd);
            const int sh[3] = {20, 30, 50};
            for (int k = 0; k < 3; ++k) {
                const uint64_t w = (1ull << sh[k]) % q;
                put(base + 2 * ns + 2 + 2 * k, (double)w);
                put(base + 2 * ns + 3 + 2 * k, (double)w / qd);
            }
        }
    }
    return rec;
}

// Per-source constants of a basis conversion (layout: launch_basis_convert):
// w = (Qhat_i)^-1 mod q_i with what the source's product needs.
static void push_source_consts(std::vector<uint64_t>& v, uint64_t w, uint64_t q) {
    auto bits = [](double d) { uint64_t u; std::memcpy(&u, &d, 8); return u; };
    if (q < kFp64PrimeBound) {
        const double wd = (double)w, qd = (double)q;
        v.insert(v.end(), {bits(wd), bits(wd / qd), bits(qd), bits(1.0 / qd)});
    } else {
        v.insert(v.end(), {w, shoup_pre(w, q), q, 0});
    }
}

static void upload(void* dst, const void* src, size_t bytes, hipStream_t s) {
    CSRMF_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
    CSRMF_HIP(hipStreamSynchronize(s));   // the host buffer may be reused on return
}

static uint64_t* upload_consts(Pool& pool, const std::vector<uint64_t>& v, hipStream_t s) {
    uint64_t* d = (uint64_t*)pool.get(std::max<size_t>(8, v.size() * 8));
    if (!v.empty()) upload(d, v.data(), v.size() * 8, s);
    return d;
}

Context::~Context() {
    while (!servers.empty()) destroy_server(servers.back());   // joins the worker threads
    if (capturing) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(stream, &g);
        if (g) (void)hipGraphDestroy(g);
        capturing = false;
        staging.end_arena();
        graphs[0].blocks = pool.end_capture();
    }
    while (!graphs.empty()) {
        const uint64_t id = graphs.begin()->first;
        CapturedGraph& g = graphs.begin()->second;
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
        if (g.arena_host) (void)hipHostFree(g.arena_host);
        if (g.arena_dev) (void)hipFree(g.arena_dev);
        graphs.erase(id);   // the blocks go with release_all below
    }
    if (stream) (void)hipStreamSynchronize(stream);
    else (void)hipDeviceSynchronize();
    destroy_mf(mf);
    mf = nullptr;
    staging.release();
    pool.release_all();
    if (own_stream) (void)hipStreamDestroy(own_stream);
    stream = own_stream = nullptr;
}

// ------------------------------------------------------------------ init
void Context::init(const csrmf_params& p, const uint8_t s[32]) {
    prm = p;
    std::memcpy(seed, s, 32);
    if (p.log2N < 12 || p.log2N > 16) throw Error(CSRMF_E_INVAL, "log2N must be in [12, 16]");
    if (p.n_scale_primes < 0 || p.n_scale_primes > 40 || p.n_special < 1 || p.n_special > 8 || p.dnum < 1)
        throw Error(CSRMF_E_INVAL, "bad prime counts");
    if (p.base_bits > 60 || p.scale_bits > 60 || p.special_bits > 60)
        throw Error(CSRMF_E_INVAL, "primes must be below 2^60");
    logN = p.log2N;
    N = 1ull << logN;
    L = p.n_scale_primes;
    alpha = p.n_special;
    dnum = p.dnum;
    gsize = (L + 1 + dnum - 1) / dnum;
    if (gsize > 16 || alpha > 16) throw Error(CSRMF_E_INVAL, "key-switching digits hold at most 16 limbs");
    if (L + 1 + alpha > 64) throw Error(CSRMF_E_INVAL, "too many limbs");
    if (p.k < 0 || (p.k > 0 && 4 * (uint64_t)p.k > N / 2)) throw Error(CSRMF_E_INVAL, "k too large for the slots");

    std::vector<uint64_t> big, sc, sp;
    const bool shared = p.special_bits == p.base_bits;
    if (!ntt_primes(p.base_bits, N, 1 + (shared ? alpha : 0), big)) throw Error(CSRMF_E_INVAL, "not enough base primes");
    if (!ntt_primes(p.scale_bits, N, L, sc) && L > 0) throw Error(CSRMF_E_INVAL, "not enough scale primes");
    if (shared) sp.assign(big.begin() + 1, big.end());
    else if (!ntt_primes(p.special_bits, N, alpha, sp)) throw Error(CSRMF_E_INVAL, "not enough special primes");
    moduli.clear();
    moduli.push_back(big[0]);
    for (uint64_t q : sc) moduli.push_back(q);
    for (uint64_t q : sp) moduli.push_back(q);
    for (size_t i = 0; i < moduli.size(); ++i)
        for (size_t j = 0; j < i; ++j)
            if (moduli[i] == moduli[j]) throw Error(CSRMF_E_INVAL, "prime chain has a repeated prime");

    CSRMF_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
    own_stream = stream;
    staging.init(stream);
    noalloc_scratch = noalloc_scratch_for_current_device();

    const int nm = (int)moduli.size();
    mh.resize(nm);
    std::vector<uint64_t> tw((size_t)nm * 4 * N);
    for (int mi = 0; mi < nm; ++mi) {
        const uint64_t q = moduli[mi];
        Modulus& m = mh[mi];
        m.q = q;
        uint64_t inv = 1;                     // q^-1 mod 2^64 by Newton iteration
        for (int it = 0; it < 7; ++it) inv *= 2 - q * inv;
        m.qneg_inv = (uint64_t)0 - inv;
        m.r_mod = (uint64_t)(((u128)1 << 64) % q);
        m.r_mod_shoup = shoup_pre(m.r_mod, q);
        m.r2_mod = mm(m.r_mod, m.r_mod, q);
        m.n_inv = inv_mod(N % q, q);
        m.n_inv_shoup = shoup_pre(m.n_inv, q);
        m.psi = smallest_primitive_root_2n(q, N);
        const uint64_t psi_inv = inv_mod(m.psi, q);
        uint64_t* T = tw.data() + (size_t)mi * 4 * N;
        // powers in natural order, then scatter to bit-reversed positions
        uint64_t x = 1, y = 1;
        for (uint64_t k = 0; k < N; ++k) {
            uint64_t r = 0;
            for (int b = 0; b < logN; ++b) r |= ((k >> b) & 1) << (logN - 1 - b);
            T[r] = x;
            T[2 * N + r] = y;
            x = mm(x, m.psi, q);
            y = mm(y, psi_inv, q);
        }
        if (q < kFp64PrimeBound) {
            // exact FP64 transform: w and fl(w/q) as doubles
            for (uint64_t k = 0; k < N; ++k) {
                for (int part = 0; part < 2; ++part) {
                    const double w = (double)T[2 * part * N + k];
                    const double wq = w / (double)q;
                    std::memcpy(&T[2 * part * N + k], &w, 8);
                    std::memcpy(&T[(2 * part + 1) * N + k], &wq, 8);
                }
            }
        } else {
            for (uint64_t k = 0; k < N; ++k) {
                T[N + k] = shoup_pre(T[k], q);
                T[3 * N + k] = shoup_pre(T[2 * N + k], q);
            }
        }
    }
    d_mods = (Modulus*)pool.get(sizeof(Modulus) * nm);
    upload(d_mods, mh.data(), sizeof(Modulus) * nm, stream);
    d_tw = (uint64_t*)pool.get(tw.size() * 8);
    upload(d_tw, tw.data(), tw.size() * 8, stream);
    tabs.logN = logN;
    tabs.L1 = logN / 2;
    tabs.mods = d_mods;
    tabs.tw = d_tw;

    // per-level constants
    lv.resize(L + 1);
    for (int l = 0; l <= L; ++l) {
        LevelConsts& c = lv[l];
        const int nr = n_ext(l);
        for (int j = 0; j < dnum; ++j) {
            const int lo = j * gsize, hi = std::min(std::min((j + 1) * gsize, L + 1), l + 1);
            if (lo >= hi) break;
            DigitConsts dc;
            dc.lo = lo;
            dc.hi = hi;
            std::vector<uint64_t> yc, cc;
            std::vector<int> tg;
            for (int t = 0; t < nr; ++t)
                if (!(t >= lo && t < hi)) tg.push_back(gmod_ext(l, t));
            for (int i = lo; i < hi; ++i) {
                const uint64_t qi = moduli[i];
                uint64_t hat = 1;
                for (int k = lo; k < hi; ++k) if (k != i) hat = mm(hat, moduli[k] % qi, qi);
                push_source_consts(yc, inv_mod(hat, qi), qi);
            }
            std::vector<uint64_t> hats, tq, trm, tni;
            for (int tm : tg) { tq.push_back(moduli[tm]); trm.push_back(mh[tm].r_mod); tni.push_back(mh[tm].qneg_inv); }
            for (int i = lo; i < hi; ++i) {
                for (int tm : tg) {
                    const uint64_t qt = moduli[tm];
                    uint64_t hat = 1;
                    for (int k = lo; k < hi; ++k) if (k != i) hat = mm(hat, moduli[k] % qt, qt);
                    hats.push_back(hat);
                }
            }
            cc = bc_records(hats, hi - lo, true, tq, trm, tni);
            dc.yc = upload_consts(pool, yc, stream);
            dc.cc = upload_consts(pool, cc, stream);
            c.digits.push_back(dc);
        }
        std::vector<uint64_t> y, cv, pinv, rs;
        for (int k = 0; k < alpha; ++k) {
            const uint64_t pk_ = moduli[L + 1 + k];
            uint64_t hat = 1;
            for (int kk = 0; kk < alpha; ++kk) if (kk != k) hat = mm(hat, moduli[L + 1 + kk] % pk_, pk_);
            push_source_consts(y, inv_mod(hat, pk_), pk_);
        }
        std::vector<uint64_t> md_hats, md_tq, md_trm, md_tni;
        for (int i = 0; i <= l; ++i) {
            md_tq.push_back(moduli[i]);
            md_trm.push_back(mh[i].r_mod);
            md_tni.push_back(mh[i].qneg_inv);
        }
        for (int k = 0; k < alpha; ++k) {
            for (int i = 0; i <= l; ++i) {
                const uint64_t qi = moduli[i];
                uint64_t hat = 1;
                for (int kk = 0; kk < alpha; ++kk) if (kk != k) hat = mm(hat, moduli[L + 1 + kk] % qi, qi);
                md_hats.push_back(hat);
            }
        }
        cv = bc_records(md_hats, alpha, false, md_tq, md_trm, md_tni);
        for (int i = 0; i <= l; ++i) {
            const uint64_t qi = moduli[i];
            uint64_t P = 1;
            for (int k = 0; k < alpha; ++k) P = mm(P, moduli[L + 1 + k] % qi, qi);
            const uint64_t w = inv_mod(P, qi);
            pinv.push_back(w);
            pinv.push_back(shoup_pre(w, qi));
        }
        if (l >= 1) {
            const uint64_t ql = moduli[l];
            for (int i = 0; i < l; ++i) {
                const uint64_t qi = moduli[i];
                const uint64_t w = inv_mod(ql % qi, qi);
                rs.push_back((ql / 2) % qi);
                rs.push_back(w);
                rs.push_back(shoup_pre(w, qi));
                rs.push_back(0);
            }
        }
        c.md_y = upload_consts(pool, y, stream);
        c.md_c = upload_consts(pool, cv, stream);
        c.md_pinv = upload_consts(pool, pinv, stream);
        c.rs = upload_consts(pool, rs, stream);
    }
}

// ------------------------------------------------------------------ store
Ct Context::new_ct(int level, double scale) {
    Ct c;
    c.d = (uint64_t*)pool.get(ct_words() * 8);
    c.level = level;
    c.scale = scale;
    return c;
}

uint64_t Context::put(const Ct& c) {
    const uint64_t h = next_handle++;
    cts[h] = c;
    return h;
}

Ct& Context::get(uint64_t h) {
    auto it = cts.find(h);
    if (it == cts.end()) throw Error(CSRMF_E_INVAL, "unknown ciphertext handle " + std::to_string(h));
    return it->second;
}

void Context::free_ct(uint64_t h) {
    auto it = cts.find(h);
    if (it == cts.end()) throw Error(CSRMF_E_INVAL, "unknown ciphertext handle");
    pool.put(it->second.d);   // later users of the block are ordered after this on the stream
    cts.erase(it);
}

uint64_t** Context::ptr_table(const std::vector<uint64_t*>& v) {
    return (uint64_t**)stage(v.data(), v.size() * sizeof(uint64_t*));
}

RowMap Context::map_ct(uint64_t* d, int nlimbs, int first) const {
    RowMap m;
    m.base = d;
    m.poly_stride = poly_stride();
    m.batch_stride = 2 * poly_stride();
    for (int i = 0; i < nlimbs; ++i) m.push(first + i, first + i);
    return m;
}

RowMap Context::map_cts(const std::vector<Ct*>& v, int nlimbs, int first) {
    RowMap m = map_ct(v.empty() ? nullptr : v[0]->d, nlimbs, first);
    m.batch = (int)v.size();
    if (v.size() > 1) {
        std::vector<uint64_t*> ps;
        for (Ct* c : v) ps.push_back(c->d);
        m.ptrs = ptr_table(ps);
    }
    return m;
}

// ------------------------------------------------------------------ keys
uint32_t Context::galois_for_step(int64_t r) const {
    const int64_t half = (int64_t)(N / 2);
    int64_t e = r % half;
    if (e < 0) e += half;
    return (uint32_t)pow_mod(5, (uint64_t)e, 2 * N);
}

const Key& Context::key_for(uint32_t g) const {
    auto it = rot.find(g);
    if (it == rot.end()) throw Error(CSRMF_E_KEY, "no rotation key for Galois element " + std::to_string(g));
    return it->second;
}

void Context::keygen(const int32_t* steps, int n, bool conj) {
    const int nall = L + 1 + alpha;
    if (!have_keys) {
        std::vector<int64_t> sv(N);
        sample_ternary(seed, kSecret, 0, N, sv.data());
        Scratch ss(pool, N);
        upload(ss.p, sv.data(), N * 8, stream);
        s_ntt = (uint64_t*)pool.get((size_t)nall * N * 8);
        s_mont = (uint64_t*)pool.get((size_t)nall * N * 8);
        RowMap ms;
        ms.base = s_ntt;
        for (int i = 0; i < nall; ++i) ms.push(i, i);
        launch_expand_signed(tabs, ms, (const int64_t*)ss.p, 1, 0, stream);
        launch_ntt(tabs, ms, false, stream);
        RowMap mm_ = ms;
        mm_.base = s_mont;
        std::vector<uint64_t> rc;
        for (int i = 0; i < nall; ++i) { rc.push_back(mh[i].r_mod); rc.push_back(mh[i].r_mod_shoup); }
        Scratch rcd(pool, rc.size());
        upload(rcd.p, rc.data(), rc.size() * 8, stream);
        launch_mul_const(tabs, mm_, ms, rcd.p, false, stream);

        // public key: b = -a*s + e over Q_L
        pk = (uint64_t*)pool.get(2 * (size_t)(L + 1) * N * 8);
        std::vector<uint64_t> av((size_t)(L + 1) * N);
        for (int i = 0; i <= L; ++i) sample_uniform(seed, kPkA, 0, i, N, moduli[i], av.data() + (size_t)i * N);
        std::vector<int64_t> ev(N);
        sample_cbd21(seed, kPkE, 0, N, ev.data());
        uint64_t* pb = pk;
        uint64_t* pa = pk + (size_t)(L + 1) * N;
        upload(pa, av.data(), av.size() * 8, stream);
        Scratch es(pool, N);
        upload(es.p, ev.data(), N * 8, stream);
        RowMap ma, mb, msm;
        ma.base = pa; mb.base = pb; msm.base = s_mont;
        for (int i = 0; i <= L; ++i) { ma.push(i, i); mb.push(i, i); msm.push(i, i); }
        launch_ntt(tabs, ma, false, stream);
        launch_expand_signed(tabs, mb, (const int64_t*)es.p, 1, 0, stream);
        launch_ntt(tabs, mb, false, stream);
        Scratch as(pool, (size_t)(L + 1) * N);
        RowMap mas = ma;
        mas.base = as.p;
        launch_mul_mont(tabs, mas, ma, msm, false, stream);          // a*s
        launch_ew(tabs, EW_SUB, mb, mb, mas, stream);                // e - a*s
        // store pk times 2^64
        RowMap mpk;
        mpk.base = pk;
        mpk.poly_stride = (int64_t)(L + 1) * N;
        for (int i = 0; i <= L; ++i) mpk.push(i, i);
        launch_mul_const(tabs, mpk, mpk, rcd.p, true, stream);

        // relinearisation key: s' = s^2
        Scratch s2(pool, (size_t)(L + 1) * N);
        RowMap m2 = msm;
        m2.base = s2.p;
        RowMap msq = msm;
        msq.base = s_ntt;
        launch_mul_mont(tabs, m2, msq, msm, false, stream);
        make_switching_key(relin, s2.p, 0);
        have_keys = true;
    }
    for (int i = 0; i < n; ++i) add_rotation_key(galois_for_step(steps[i]));
    if (conj) add_rotation_key((uint32_t)(2 * N - 1));
    sync();
}

void Context::add_rotation_key(uint32_t g) {
    if (g == 1 || rot.count(g)) return;
    Scratch sg(pool, (size_t)(L + 1) * N);
    RowMap mi, mo;
    mi.base = s_ntt;
    mo.base = sg.p;
    for (int i = 0; i <= L; ++i) { mi.push(i, i); mo.push(i, i); }
    launch_automorphism(tabs, g, mo, mi, false, stream);
    Key k;
    make_switching_key(k, sg.p, g);
    rot[g] = k;
}

void Context::make_switching_key(Key& key, const uint64_t* sprime, uint32_t key_index) {
    const int nall = L + 1 + alpha;
    const size_t rows_words = (size_t)nall * N;
    key.n_digits = 0;
    for (int j = 0; j < dnum; ++j) if (j * gsize < L + 1) key.n_digits++;
    key.d = (uint64_t*)pool.get((size_t)key.n_digits * 2 * rows_words * 8);
    // P mod q_i
    std::vector<uint64_t> pc;
    for (int i = 0; i <= L; ++i) {
        uint64_t P = 1;
        for (int k = 0; k < alpha; ++k) P = mm(P, moduli[L + 1 + k] % moduli[i], moduli[i]);
        pc.push_back(P);
        pc.push_back(shoup_pre(P, moduli[i]));
    }
    Scratch pcd(pool, pc.size());
    upload(pcd.p, pc.data(), pc.size() * 8, stream);
    std::vector<uint64_t> rc;
    RowMap mk_int, mk_f64;   // key rows by form (both polynomials of mk_int through poly_stride)
    mk_int.base = key.d;
    mk_int.poly_stride = (int64_t)rows_words;
    for (int i = 0; i < nall; ++i) {
        if (moduli[i] < kFp64PrimeBound) {
            mk_f64.push(i, i);
        } else {
            mk_int.push(i, i);
            rc.push_back(mh[i].r_mod);
            rc.push_back(mh[i].r_mod_shoup);
        }
    }
    Scratch rci(pool, std::max<size_t>(1, rc.size()));
    if (!rc.empty()) upload(rci.p, rc.data(), rc.size() * 8, stream);
    std::vector<uint64_t> av(rows_words);
    std::vector<int64_t> ev(N);
    Scratch es(pool, N), tmp(pool, rows_words);
    for (int j = 0; j < key.n_digits; ++j) {
        const uint32_t obj = key_index * (uint32_t)dnum + (uint32_t)j;
        for (int t = 0; t < nall; ++t) sample_uniform(seed, kKskA, obj, t, N, moduli[t], av.data() + (size_t)t * N);
        sample_cbd21(seed, kKskE, obj, N, ev.data());
        uint64_t* kb = key.d + (size_t)j * 2 * rows_words;
        uint64_t* ka = kb + rows_words;
        upload(ka, av.data(), rows_words * 8, stream);
        upload(es.p, ev.data(), N * 8, stream);
        RowMap ma, mb, ms, mt;
        ma.base = ka; mb.base = kb; ms.base = s_mont; mt.base = tmp.p;
        for (int t = 0; t < nall; ++t) { ma.push(t, t); mb.push(t, t); ms.push(t, t); mt.push(t, t); }
        launch_ntt(tabs, ma, false, stream);
        launch_expand_signed(tabs, mb, (const int64_t*)es.p, 1, 0, stream);
        launch_ntt(tabs, mb, false, stream);
        launch_mul_mont(tabs, mt, ma, ms, false, stream);   // a*s
        launch_ew(tabs, EW_SUB, mb, mb, mt, stream);        // e - a*s
        const int lo = j * gsize, hi = std::min((j + 1) * gsize, L + 1);
        RowMap dq, sq, tq;
        dq.base = kb; sq.base = (uint64_t*)sprime; tq.base = tmp.p;
        for (int i = lo; i < hi; ++i) { dq.push(i, i); sq.push(i, i); tq.push(i, i); }
        launch_mul_const(tabs, tq, sq, pcd.p + 2 * lo, false, stream);   // P * s'
        launch_ew(tabs, EW_ADD, dq, dq, tq, stream);
        mk_int.base = kb;
        // store the 60-bit rows times 2^64 (Montgomery form), the rows of
        // primes below 2^44 as centred doubles (the inner products' FP64 form)
        if (mk_int.n) launch_mul_const(tabs, mk_int, mk_int, rci.p, true, stream);
        for (uint64_t* base : {kb, ka}) {
            RowMap mf = mk_f64;
            mf.base = base;
            if (mf.n) launch_ew(tabs, EW_F64C, mf, mf, mf, stream);
        }
    }
    sync();
}

// ------------------------------------------------------------------ encrypt
void Context::encrypt_int_batch(const int64_t* m, int count, int level, double scale, std::vector<Ct>& out,
                                const uint32_t* serials) {
    if (count > kMaxBatch) {   // in order, so running serial numbers are unchanged
        out.clear();
        for (int i = 0; i < count; i += kMaxBatch) {
            std::vector<Ct> part;
            encrypt_int_batch(m + (size_t)i * N, std::min(kMaxBatch, count - i), level, scale, part,
                              serials ? serials + i : nullptr);
            out.insert(out.end(), part.begin(), part.end());
        }
        return;
    }
    if (!have_keys) throw Error(CSRMF_E_STATE, "keygen first");
    if (level < 0 || level > L) throw Error(CSRMF_E_INVAL, "level out of range");
    // signed inputs: [count][4][N] = v, e0, e1, m
    std::vector<int64_t> host((size_t)count * 4 * N);
    for (int c = 0; c < count; ++c) {
        const uint64_t ser = serials ? serials[c] : serial++;
        int64_t* h = host.data() + (size_t)c * 4 * N;
        sample_ternary(seed, kEncV, (uint32_t)ser, N, h);
        sample_cbd21(seed, kEncE0, (uint32_t)ser, N, h + N);
        sample_cbd21(seed, kEncE1, (uint32_t)ser, N, h + 2 * N);
        std::memcpy(h + 3 * N, m + (size_t)c * N, N * 8);
    }
    Scratch src(pool, host.size());
    upload(src.p, host.data(), host.size() * 8, stream);
    const int nl = level + 1;
    Scratch ex(pool, (size_t)count * 4 * nl * N);
    // expand: rows [c][poly p][limb i] at off p*nl + i
    for (int p = 0; p < 4; ++p) {
        RowMap me;
        me.base = ex.p + (size_t)p * nl * N;
        me.batch = count;
        me.batch_stride = (int64_t)4 * nl * N;
        for (int i = 0; i < nl; ++i) me.push(i, i);
        launch_expand_signed(tabs, me, (const int64_t*)src.p + (size_t)p * N, 1, (int64_t)4 * N, stream);
    }
    out.clear();
    for (int c = 0; c < count; ++c) out.push_back(new_ct(level, scale));
    // NTT all expanded rows: count*4 polynomials of nl limbs, contiguous
    RowMap all;
    all.base = ex.p;
    all.batch = count * 4;
    all.batch_stride = (int64_t)nl * N;
    for (int i = 0; i < nl; ++i) all.push(i, i);
    launch_ntt(tabs, all, false, stream);
    std::vector<Ct*> po;
    for (auto& c : out) po.push_back(&c);
    RowMap o0 = map_cts(po, nl);
    RowMap o1 = o0;
    for (int i = 0; i < nl; ++i) o1.e[i] = ((uint32_t)(L + 1 + i) << 8) | (uint32_t)i;
    auto vmap = [&](int p) {
        RowMap r;
        r.base = ex.p + (size_t)p * nl * N;
        r.batch = count;
        r.batch_stride = (int64_t)4 * nl * N;
        for (int i = 0; i < nl; ++i) r.push(i, i);
        return r;
    };
    RowMap pb, pa;
    pb.base = pk;
    pa.base = pk + (size_t)(L + 1) * N;
    for (int i = 0; i < nl; ++i) { pb.push(i, i); pa.push(i, i); }
    pb.batch = pa.batch = count;   // batch stride 0: the same key rows for every ciphertext
    launch_mul_mont(tabs, o0, vmap(0), pb, false, stream);
    launch_mul_mont(tabs, o1, vmap(0), pa, false, stream);
    launch_ew(tabs, EW_ADD, o0, o0, vmap(3), stream);
    launch_ew(tabs, EW_ADD, o0, o0, vmap(1), stream);
    launch_ew(tabs, EW_ADD, o1, o1, vmap(2), stream);
    sync();
}

Ct Context::encrypt_int(const int64_t* m, int level, double scale) {
    std::vector<Ct> out;
    encrypt_int_batch(m, 1, level, scale, out);
    return out[0];
}

void Context::decrypt_int(const Ct& c, int64_t* m) {
    if (!have_keys) throw Error(CSRMF_E_STATE, "keygen first");
    Scratch x(pool, N);
    RowMap mx, m0, m1, ms;
    mx.base = x.p;
    mx.push(0, 0);
    m0.base = c.d;
    m0.push(0, 0);
    m1.base = c.d;
    m1.push(L + 1, 0);
    ms.base = s_mont;
    ms.push(0, 0);
    launch_mul_mont(tabs, mx, m1, ms, false, stream);
    launch_ew(tabs, EW_ADD, mx, mx, m0, stream);
    launch_ntt(tabs, mx, true, stream);
    std::vector<uint64_t> h(N);
    CSRMF_HIP(hipMemcpyAsync(h.data(), x.p, N * 8, hipMemcpyDeviceToHost, stream));
    sync();
    const uint64_t q0 = moduli[0];
    for (uint64_t i = 0; i < N; ++i) m[i] = h[i] > q0 / 2 ? -(int64_t)(q0 - h[i]) : (int64_t)h[i];
}

void Context::export_ct(const Ct& c, uint64_t* coeffs) {
    const int nl = c.level + 1;
    Scratch x(pool, 2 * (size_t)nl * N);
    RowMap src = map_ct(c.d, nl), dst;
    dst.base = x.p;
    dst.poly_stride = (int64_t)nl * N;
    for (int i = 0; i < nl; ++i) dst.push(i, i);
    RowMap src1 = src, dst1 = dst;
    for (int i = 0; i < nl; ++i) {
        src1.e[i] = ((uint32_t)(L + 1 + i) << 8) | (uint32_t)i;
        dst1.e[i] = ((uint32_t)(nl + i) << 8) | (uint32_t)i;
    }
    launch_ew(tabs, EW_COPY, dst, src, src, stream);
    launch_ew(tabs, EW_COPY, dst1, src1, src1, stream);
    RowMap both = dst;
    for (int i = 0; i < nl; ++i) both.push(nl + i, i);
    launch_ntt(tabs, both, true, stream);
    CSRMF_HIP(hipMemcpyAsync(coeffs, x.p, 2 * (size_t)nl * N * 8, hipMemcpyDeviceToHost, stream));
    sync();
}

Ct Context::import_ct(const uint64_t* coeffs, int level, double scale) {
    if (level < 0 || level > L) throw Error(CSRMF_E_INVAL, "level out of range");
    const int nl = level + 1;
    for (int p = 0; p < 2; ++p)
        for (int i = 0; i < nl; ++i)
            for (uint64_t n = 0; n < N; ++n)
                if (coeffs[((size_t)p * nl + i) * N + n] >= moduli[i]) throw Error(CSRMF_E_INVAL, "residue not reduced");
    Ct c = new_ct(level, scale);
    for (int p = 0; p < 2; ++p)
        CSRMF_HIP(hipMemcpyAsync(c.d + (size_t)p * poly_stride(), coeffs + (size_t)p * nl * N, (size_t)nl * N * 8,
                                 hipMemcpyHostToDevice, stream));
    RowMap m = map_ct(c.d, nl);
    for (int i = 0; i < nl; ++i) m.push(L + 1 + i, i);
    launch_ntt(tabs, m, false, stream);
    sync();
    return c;
}

void Context::export_key(int which, uint32_t g, uint64_t* out) {
    if (!have_keys) throw Error(CSRMF_E_STATE, "keygen first");
    const int nall = L + 1 + alpha;
    std::vector<uint64_t> h;
    // mont: rows stored times 2^64; f64: rows of primes below 2^44 stored as
    // centred doubles (switching keys)
    auto pull = [&](const uint64_t* d, int rows, const std::vector<int>& mods, bool mont, bool f64 = false) {
        Scratch x(pool, (size_t)rows * N);
        CSRMF_HIP(hipMemcpyAsync(x.p, d, (size_t)rows * N * 8, hipMemcpyDeviceToDevice, stream));
        RowMap m;
        m.base = x.p;
        for (int r = 0; r < rows; ++r) m.push(r, mods[r]);
        if (f64) launch_ew(tabs, EW_F64U, m, m, m, stream);
        launch_ntt(tabs, m, true, stream);
        std::vector<uint64_t> v((size_t)rows * N);
        CSRMF_HIP(hipMemcpyAsync(v.data(), x.p, v.size() * 8, hipMemcpyDeviceToHost, stream));
        sync();
        if (mont) {
            for (int r = 0; r < rows; ++r) {
                const uint64_t q = moduli[mods[r]];
                if (f64 && q < kFp64PrimeBound) continue;
                const uint64_t rinv = inv_mod(mh[mods[r]].r_mod, q);
                for (uint64_t n = 0; n < N; ++n) v[(size_t)r * N + n] = mm(v[(size_t)r * N + n], rinv, q);
            }
        }
        h.insert(h.end(), v.begin(), v.end());
    };
    std::vector<int> all_mods, q_mods;
    for (int i = 0; i < nall; ++i) all_mods.push_back(i);
    for (int i = 0; i <= L; ++i) q_mods.push_back(i);
    if (which == 0) {
        pull(s_ntt, nall, all_mods, false);
    } else if (which == 1) {
        std::vector<int> m2 = q_mods;
        m2.insert(m2.end(), q_mods.begin(), q_mods.end());
        pull(pk, 2 * (L + 1), m2, true);
    } else if (which == 2 || which == 3) {
        const Key& k = which == 2 ? relin : key_for(g);
        for (int j = 0; j < k.n_digits; ++j) {
            pull(k.d + (size_t)j * 2 * nall * N, nall, all_mods, true, true);
            pull(k.d + (size_t)j * 2 * nall * N + (size_t)nall * N, nall, all_mods, true, true);
        }
    } else {
        throw Error(CSRMF_E_INVAL, "unknown key selector");
    }
    std::memcpy(out, h.data(), h.size() * 8);
}

// ------------------------------------------------------------------ evaluation
// Operands of an addition must carry the same scale up to the rounding of the
// integer weights that produced them: 2^-30 relative, or 2^-(log2_scale - 4)
// on chains with a smaller scale (their weights are integers of about
// log2_scale bits).
void Context::check_scales(double a, double b) const {
    if (std::fabs(a / b - 1.0) > std::ldexp(1.0, std::max(-30, 4 - prm.log2_scale)))
        throw Error(CSRMF_E_SCALE, "operand scales differ: " + std::to_string(a) + " vs " + std::to_string(b));
}

void Context::add(const Ct& a, const Ct& b, Ct& out, bool sub) {
    check_scales(a.scale, b.scale);
    const int lvl = std::min(a.level, b.level);
    out = new_ct(lvl, a.scale);
    RowMap ma = map_ct(a.d, lvl + 1), mb = map_ct(b.d, lvl + 1), mo = map_ct(out.d, lvl + 1);
    for (int i = 0; i <= lvl; ++i) {
        ma.push(L + 1 + i, i);
        mb.push(L + 1 + i, i);
        mo.push(L + 1 + i, i);
    }
    launch_ew(tabs, sub ? EW_SUB : EW_ADD, mo, ma, mb, stream);
}

void Context::add_batch(const std::vector<Ct*>& a, const std::vector<Ct*>& b, std::vector<Ct*>& out, bool sub) {
    const int B = (int)a.size();
    if (B == 0) return;
    const int lvl = std::min(a[0]->level, b[0]->level);
    for (int i = 0; i < B; ++i) {
        check_scales(a[i]->scale, b[i]->scale);
        if (std::min(a[i]->level, b[i]->level) != lvl) throw Error(CSRMF_E_INVAL, "batch operands must share a level");
    }
    for (int i = 0; i < B; ++i) *out[i] = new_ct(lvl, a[i]->scale);
    RowMap ma = map_cts(a, lvl + 1), mb = map_cts(b, lvl + 1), mo = map_cts(out, lvl + 1);
    for (int i = 0; i <= lvl; ++i) {
        ma.push(L + 1 + i, i);
        mb.push(L + 1 + i, i);
        mo.push(L + 1 + i, i);
    }
    launch_ew(tabs, sub ? EW_SUB : EW_ADD, mo, ma, mb, stream);
    fence();
}

void Context::add_plain(const Ct& a, const int64_t* m, Ct& out) {
    const int nl = a.level + 1;
    Scratch ex(pool, (size_t)nl * N);
    const int64_t* src = (const int64_t*)stage(m, N * 8);
    RowMap me;
    me.base = ex.p;
    for (int i = 0; i < nl; ++i) me.push(i, i);
    launch_expand_signed(tabs, me, src, 1, 0, stream);
    launch_ntt(tabs, me, false, stream);
    out = new_ct(a.level, a.scale);
    RowMap ma = map_ct(a.d, nl), mo = map_ct(out.d, nl);
    launch_ew(tabs, EW_ADD, mo, ma, me, stream);
    RowMap ma1 = ma, mo1 = mo;
    for (int i = 0; i < nl; ++i) {
        ma1.e[i] = ((uint32_t)(L + 1 + i) << 8) | (uint32_t)i;
        mo1.e[i] = ((uint32_t)(L + 1 + i) << 8) | (uint32_t)i;
    }
    launch_ew(tabs, EW_COPY, mo1, ma1, ma1, stream);
    fence();
}

void Context::mul_plain(const Ct& a, const int64_t* m, double pt_scale, Ct& out) {
    const int nl = a.level + 1;
    Scratch ex(pool, (size_t)nl * N);
    const int64_t* src = (const int64_t*)stage(m, N * 8);
    RowMap me;
    me.base = ex.p;
    for (int i = 0; i < nl; ++i) me.push(i, i);
    launch_expand_signed(tabs, me, src, 1, 0, stream);
    launch_ntt(tabs, me, false, stream);
    std::vector<uint64_t> rc;
    for (int i = 0; i < nl; ++i) { rc.push_back(mh[i].r_mod); rc.push_back(mh[i].r_mod_shoup); }
    const uint64_t* rcd = (const uint64_t*)stage(rc.data(), rc.size() * 8);
    launch_mul_const(tabs, me, me, rcd, false, stream);   // plaintext times 2^64
    out = new_ct(a.level, a.scale * pt_scale);
    RowMap ma = map_ct(a.d, nl), mo = map_ct(out.d, nl);
    launch_mul_mont(tabs, mo, ma, me, false, stream);
    for (int i = 0; i < nl; ++i) {
        ma.e[i] = ((uint32_t)(L + 1 + i) << 8) | (uint32_t)i;
        mo.e[i] = ((uint32_t)(L + 1 + i) << 8) | (uint32_t)i;
    }
    launch_mul_mont(tabs, mo, ma, me, false, stream);
    fence();
}

void Context::mul_int(const Ct& a, int64_t w, Ct& out, double declared) {
    const int nl = a.level + 1;
    std::vector<uint64_t> c;
    for (int i = 0; i < nl; ++i) {
        const uint64_t r = from_signed(w, moduli[i]);
        c.push_back(r);
        c.push_back(shoup_pre(r, moduli[i]));
    }
    const uint64_t* cd = (const uint64_t*)stage(c.data(), c.size() * 8);
    out = new_ct(a.level, declared != 0.0 ? declared : a.scale * (double)w);
    launch_mul_const(tabs, map_ct(out.d, nl), map_ct(a.d, nl), cd, true, stream);
    fence();
}

void Context::mul_plain_batch(const std::vector<Ct*>& a, const int64_t* m, double pt_scale, std::vector<Ct*>& out,
                              bool accumulate) {
    const int B = (int)a.size();
    if (B == 0) return;
    const int lvl = a[0]->level;
    for (Ct* c : a)
        if (c->level != lvl) throw Error(CSRMF_E_INVAL, "batch operands must share a level");
    if (accumulate)
        for (int i = 0; i < B; ++i) {
            if (out[i]->level != lvl) throw Error(CSRMF_E_INVAL, "accumulator must have the operand's level");
            check_scales(out[i]->scale, a[i]->scale * pt_scale);
        }
    const int nl = lvl + 1;
    Scratch ex(pool, (size_t)nl * N);
    const int64_t* src = (const int64_t*)stage(m, N * 8);
    RowMap me;
    me.base = ex.p;
    for (int i = 0; i < nl; ++i) me.push(i, i);
    launch_expand_signed(tabs, me, src, 1, 0, stream);
    launch_ntt(tabs, me, false, stream);
    std::vector<uint64_t> rc;
    for (int i = 0; i < nl; ++i) { rc.push_back(mh[i].r_mod); rc.push_back(mh[i].r_mod_shoup); }
    const uint64_t* rcd = (const uint64_t*)stage(rc.data(), rc.size() * 8);
    launch_mul_const(tabs, me, me, rcd, false, stream);   // plaintext times 2^64
    if (!accumulate)
        for (int i = 0; i < B; ++i) *out[i] = new_ct(lvl, a[i]->scale * pt_scale);
    RowMap ma = map_cts(a, nl), mo = map_cts(out, nl);
    RowMap mb = me;                                        // one plaintext for every batch element
    mb.batch = B;
    mb.batch_stride = 0;
    launch_mul_mont(tabs, mo, ma, mb, accumulate, stream);
    for (int i = 0; i < nl; ++i) {
        ma.e[i] = ((uint32_t)(L + 1 + i) << 8) | (uint32_t)i;
        mo.e[i] = ((uint32_t)(L + 1 + i) << 8) | (uint32_t)i;
    }
    launch_mul_mont(tabs, mo, ma, mb, accumulate, stream);
    fence();
}

void Context::mod_raise(const std::vector<Ct*>& in, double scale, std::vector<Ct*>& out) {
    const int B = (int)in.size();
    if (B == 0) return;
    for (Ct* c : in)
        if (c->level != 0) throw Error(CSRMF_E_INVAL, "ModRaise takes ciphertexts at level 0");
    // limb 0 of c0 and c1 back to coefficient form: [B][2][N]
    Scratch coef(pool, 2 * (size_t)B * N);
    RowMap src = map_cts(in, 1, 0);
    src.push(L + 1, 0);
    RowMap mc;
    mc.base = coef.p;
    mc.batch = B;
    mc.batch_stride = 2 * (int64_t)N;
    mc.poly_stride = (int64_t)N;
    mc.push(0, 0);
    mc.push(1, 0);
    launch_ntt_from(tabs, mc, src, true, stream);
    for (int i = 0; i < B; ++i) *out[i] = new_ct(L, scale);
    RowMap o0 = map_cts(out, L + 1), o1 = o0;
    for (int i = 0; i <= L; ++i) o1.e[i] = ((uint32_t)(L + 1 + i) << 8) | (uint32_t)i;
    launch_lift_centred(tabs, o0, coef.p, 2 * (int64_t)N, moduli[0], stream);
    launch_lift_centred(tabs, o1, coef.p + N, 2 * (int64_t)N, moduli[0], stream);
    launch_ntt(tabs, o0, false, stream);
    launch_ntt(tabs, o1, false, stream);
    fence();
}

void Context::mod_drop(Ct& c, int level) {
    if (level > c.level) throw Error(CSRMF_E_LEVEL, "cannot raise the level");
    c.level = level;
}

// ModUp of every digit of d (evaluation form, B ciphertext rows of level+1
// limbs) into ext [B][n_digits][l+1+alpha][N] (evaluation form).
// Rows of batch elements [b0, b0 + n) of a map.
static RowMap sub_batch(const RowMap& m, int b0, int n) {
    RowMap r = m;
    r.batch = n;
    if (m.ptrs) r.ptrs = m.ptrs + b0;
    else r.base = m.base + (int64_t)b0 * m.batch_stride;
    return r;
}

// The ModUp runs over sub-batches of `modup_chunk` ciphertexts (0: the whole
// batch): inverse transform, then per digit the conversion and the forward
// transform, so that a sub-batch small enough for the last-level cache hands
// each stage's output to the next from there.
void Context::ks_modup(const RowMap& d_in, int level, int B, uint64_t* ext, uint64_t* coef) {
    const int nl = level + 1, nr = n_ext(level);
    const LevelConsts& c = lv[level];
    const int nd = (int)c.digits.size();
    const int mcb = modup_chunk > 0 ? std::min(modup_chunk, B) : B;
    for (int b0 = 0; b0 < B; b0 += mcb) {
        const int nb = std::min(mcb, B - b0);
        RowMap mc;
        mc.base = coef + (size_t)b0 * nl * N;
        mc.batch = nb;
        mc.batch_stride = (int64_t)nl * N;
        for (int i = 0; i < nl; ++i) mc.push(i, i);
        launch_ntt_from(tabs, mc, sub_batch(d_in, b0, nb), true, stream);   // coefficient form of d_in, unchanged
        for (int jj = 0; jj < nd; ++jj) {
            const DigitConsts& dc = c.digits[jj];
            RowMap src, dst;
            src.base = mc.base;
            src.batch = nb;
            src.batch_stride = (int64_t)nl * N;
            for (int i = dc.lo; i < dc.hi; ++i) src.push(i, i);
            dst.base = ext + (size_t)b0 * nd * nr * N;
            dst.batch = nb;
            dst.batch_stride = (int64_t)nd * nr * N;
            for (int t = 0; t < nr; ++t)
                if (!(t >= dc.lo && t < dc.hi)) dst.push(jj * nr + t, gmod_ext(level, t));
            launch_basis_convert(tabs, dst, src, dc.yc, dc.cc, true, stream);   // centred digits
            launch_ntt(tabs, dst, false, stream);
            // the digit's own limbs are d_in's: ks_inner reads them there
        }
    }
}

KsArgs Context::ks_args(const uint64_t* ext, const RowMap& d_in, int level, int B, const Key& key) const {
    const int nr = n_ext(level);
    const int nd = (int)lv[level].digits.size();
    const int nall = L + 1 + alpha;
    KsArgs a;
    a.ext = ext;
    a.ext_batch_stride = (int64_t)nd * nr * N;
    a.ext_digit_stride = (int64_t)nr * N;
    a.key = key.d;
    a.key_digit_stride = 2 * (int64_t)nall * N;
    a.key_poly_stride = (int64_t)nall * N;
    a.n_q = level + 1;
    a.key_shift = L - level;
    a.n_digits = nd;
    if (d_in.n != level + 1 || d_in.batch != B) throw Error(CSRMF_E_INVAL, "key-switch input map does not match the level or batch");
    for (int j = 0; j < nd; ++j)
        for (int i = lv[level].digits[j].lo; i < lv[level].digits[j].hi; ++i) a.digit_of[i] = j;
    a.own = d_in;
    a.row0 = 0;
    return a;
}

// The inner product of the special limbs (the P part of u, which ModDown
// converts); the Q limbs' inner product is formed inside the ModDown combine.
void Context::ks_inner(const KsArgs& a, int level, int B, uint32_t g, uint64_t* u) {
    const int nl = level + 1, nr = n_ext(level);
    RowMap mu;
    mu.base = u;
    mu.batch = B;
    mu.batch_stride = 2 * (int64_t)nr * N;
    mu.poly_stride = (int64_t)nr * N;
    for (int t = nl; t < nr; ++t) mu.push(t, gmod_ext(level, t));
    KsArgs ap = a;
    ap.row0 = nl;
    launch_ks_inner(tabs, mu, ap, g, stream);
}

void Context::ks_moddown(const KsArgs& a, uint32_t g, uint64_t* u, int level, int B, const RowMap& out,
                         const RowMap& addend, uint32_t g_add, bool addend_both, const RowMap& acc,
                         uint64_t* conv_buf) {
    const int nl = level + 1, nr = n_ext(level);
    const LevelConsts& c = lv[level];
    RowMap mp;   // P rows of u0 and u1: 2B groups of alpha rows
    mp.base = u;
    mp.batch = 2 * B;
    mp.batch_stride = (int64_t)nr * N;
    for (int k = 0; k < alpha; ++k) mp.push(nl + k, L + 1 + k);
    launch_ntt(tabs, mp, true, stream);
    std::unique_ptr<Scratch> own;
    if (!conv_buf) {
        own.reset(new Scratch(pool, 2 * (size_t)B * nl * N));
        conv_buf = own->p;
    }
    RowMap mcv;
    mcv.base = conv_buf;
    mcv.batch = 2 * B;
    mcv.batch_stride = (int64_t)nl * N;
    for (int i = 0; i < nl; ++i) mcv.push(i, i);
    launch_basis_convert(tabs, mcv, mp, c.md_y, c.md_c, false, stream);
    launch_ntt(tabs, mcv, false, stream);
    RowMap mc2;
    mc2.base = conv_buf;
    mc2.batch = B;
    mc2.batch_stride = 2 * (int64_t)nl * N;
    mc2.poly_stride = (int64_t)nl * N;
    for (int i = 0; i < nl; ++i) mc2.push(i, i);
    launch_ks_combine(tabs, out, a, g, mc2, addend, g_add, addend_both, c.md_pinv, acc, stream);
}

void Context::mul_relin(const std::vector<Ct*>& a, const std::vector<Ct*>& b, std::vector<Ct*>& out) {
    if (split_batch(a.size(), [&](size_t i, size_t j) {
            std::vector<Ct*> sa = slice(a, i, j), sb = slice(b, i, j), so = slice(out, i, j);
            mul_relin(sa, sb, so);
        }))
        return;
    const int B = (int)a.size();
    if (B == 0) return;
    if (!have_keys) throw Error(CSRMF_E_STATE, "keygen first");
    const int lvl = std::min(a[0]->level, b[0]->level);
    for (int i = 0; i < B; ++i)
        if (std::min(a[i]->level, b[i]->level) != lvl) throw Error(CSRMF_E_INVAL, "batch operands must share a level");
    const int nl = lvl + 1, nr = n_ext(lvl);
    const int nd = (int)lv[lvl].digits.size();
    Scratch d(pool, (size_t)B * 3 * nl * N);
    RowMap md;
    md.base = d.p;
    md.batch = B;
    md.batch_stride = 3 * (int64_t)nl * N;
    md.poly_stride = (int64_t)nl * N;
    for (int i = 0; i < nl; ++i) md.push(i, i);
    launch_tensor(tabs, md, map_cts(a, nl), map_cts(b, nl), stream);
    RowMap d2 = md;
    for (int i = 0; i < nl; ++i) d2.e[i] = ((uint32_t)(2 * nl + i) << 8) | (uint32_t)i;
    Scratch ext(pool, (size_t)B * nd * nr * N), coef(pool, (size_t)B * nl * N), u(pool, (size_t)B * 2 * nr * N);
    ks_modup(d2, lvl, B, ext.p, coef.p);
    n_key_switches += B;
    const KsArgs ka = ks_args(ext.p, d2, lvl, B, relin);
    ks_inner(ka, lvl, B, 1, u.p);
    for (int i = 0; i < B; ++i) *out[i] = new_ct(lvl, a[i]->scale * b[i]->scale);
    ks_moddown(ka, 1, u.p, lvl, B, map_cts(out, nl), md, 1, true);
    fence();
}

void Context::rescale(const std::vector<Ct*>& v) {
    if (split_batch(v.size(), [&](size_t i, size_t j) { rescale(slice(v, i, j)); })) return;
    const int B = (int)v.size();
    if (B == 0) return;
    const int l = v[0]->level;
    for (Ct* c : v)
        if (c->level != l) throw Error(CSRMF_E_INVAL, "batch operands must share a level");
    if (l < 1) throw Error(CSRMF_E_LEVEL, "no level left to rescale");
    Scratch top(pool, 2 * (size_t)B * N), T(pool, 2 * (size_t)B * l * N);
    RowMap src = map_cts(v, 1, l);
    src.push(L + 1 + l, l);
    RowMap mt;
    mt.base = top.p;
    mt.batch = B;
    mt.batch_stride = 2 * (int64_t)N;
    mt.poly_stride = (int64_t)N;
    mt.push(0, l);
    mt.push(1, l);
    launch_ntt_from(tabs, mt, src, true, stream);
    RowMap mt1 = mt;
    mt1.n = 1;
    RowMap mT;
    mT.base = T.p;
    mT.batch = B;
    mT.batch_stride = 2 * (int64_t)l * N;
    mT.poly_stride = (int64_t)l * N;
    for (int i = 0; i < l; ++i) mT.push(i, i);
    launch_rescale_spread(tabs, mT, mt1, (uint32_t)l, stream);
    RowMap mTall = mT;
    for (int i = 0; i < l; ++i) mTall.push(l + i, i);
    launch_ntt(tabs, mTall, false, stream);
    RowMap mc = map_cts(v, l);
    launch_rescale_combine(tabs, mc, mc, mT, lv[l].rs, stream);
    const double ql = (double)moduli[l];
    for (Ct* c : v) {
        c->level = l - 1;
        c->scale = c->scale / ql;
    }
    fence();
}

void Context::rotate(const std::vector<Ct*>& in, uint32_t g, std::vector<Ct*>& out, const std::vector<Ct*>* acc) {
    if (split_batch(in.size(), [&](size_t i, size_t j) {
            std::vector<Ct*> so = slice(out, i, j);
            if (acc) {
                std::vector<Ct*> sa = slice(*acc, i, j);
                rotate(slice(in, i, j), g, so, &sa);
            } else {
                rotate(slice(in, i, j), g, so);
            }
        }))
        return;
    const int B = (int)in.size();
    if (B == 0) return;
    const Key& key = key_for(g);
    const int lvl = in[0]->level;
    for (Ct* c : in)
        if (c->level != lvl) throw Error(CSRMF_E_INVAL, "batch operands must share a level");
    if (acc) {
        if ((int)acc->size() != B) throw Error(CSRMF_E_INVAL, "one accumulator per rotated ciphertext");
        for (int i = 0; i < B; ++i) {
            if ((*acc)[i]->level < lvl) throw Error(CSRMF_E_INVAL, "accumulator below the rotated ciphertext's level");
            check_scales(in[i]->scale, (*acc)[i]->scale);
        }
    }
    const int nl = lvl + 1, nr = n_ext(lvl);
    const int nd = (int)lv[lvl].digits.size();
    // KS(tau_g(c1)) in the hoisted form: ModUp of c1 itself, tau_g applied to
    // the extended digits as the inner product reads them.  The centred
    // extension commutes with tau_g (a negated coefficient has negated centred
    // digits), so this is bit for bit the plain rotation, without a pass that
    // writes tau_g(c1).
    RowMap c1 = map_cts(in, nl);
    for (int i = 0; i < nl; ++i) c1.e[i] = ((uint32_t)(L + 1 + i) << 8) | (uint32_t)i;
    Scratch ext(pool, (size_t)B * nd * nr * N), coef(pool, (size_t)B * nl * N), u(pool, (size_t)B * 2 * nr * N);
    ks_modup(c1, lvl, B, ext.p, coef.p);
    n_key_switches += B;
    const KsArgs ka = ks_args(ext.p, c1, lvl, B, key);
    ks_inner(ka, lvl, B, g, u.p);
    for (int i = 0; i < B; ++i) *out[i] = new_ct(lvl, in[i]->scale);
    ks_moddown(ka, g, u.p, lvl, B, map_cts(out, nl), map_cts(in, nl), g, false,
               acc ? map_cts(*acc, nl) : RowMap());
    fence();
}

void Context::rotate_hoisted(const Ct& in, const std::vector<uint32_t>& gs, std::vector<Ct*>& out) {
    const int lvl = in.level;
    const int nl = lvl + 1, nr = n_ext(lvl);
    const int nd = (int)lv[lvl].digits.size();
    for (uint32_t g : gs) if (g != 1) key_for(g);
    Scratch ext(pool, (size_t)nd * nr * N), coef(pool, (size_t)nl * N), u(pool, 2 * (size_t)nr * N);
    RowMap c1 = map_ct(in.d, nl);
    for (int i = 0; i < nl; ++i) c1.e[i] = ((uint32_t)(L + 1 + i) << 8) | (uint32_t)i;
    ks_modup(c1, lvl, 1, ext.p, coef.p);
    for (size_t k = 0; k < gs.size(); ++k) {
        const uint32_t g = gs[k];
        *out[k] = new_ct(lvl, in.scale);
        if (g == 1) {
            RowMap a = map_ct(in.d, nl), o = map_ct(out[k]->d, nl);
            for (int i = 0; i < nl; ++i) { a.push(L + 1 + i, i); o.push(L + 1 + i, i); }
            launch_ew(tabs, EW_COPY, o, a, a, stream);
            continue;
        }
        const KsArgs ka = ks_args(ext.p, c1, lvl, 1, key_for(g));
        ++n_key_switches;
        ks_inner(ka, lvl, 1, g, u.p);
        ks_moddown(ka, g, u.p, lvl, 1, map_ct(out[k]->d, nl), map_ct(in.d, nl), g, false);
    }
    fence();
}

std::string Context::autotune(int rows) {
    // Time forward + inverse transforms of `rows` limbs (a key-switching batch
    // shape) under each candidate schedule; keep the fastest.
    if (rows <= 0) rows = 64 * 2 * (L + 1);
    const int n_idx = L + 1;
    rows = (rows + n_idx - 1) / n_idx * n_idx;
    Scratch buf(pool, (size_t)rows * N);
    CSRMF_HIP(hipMemsetAsync(buf.p, 0, (size_t)rows * N * 8, stream));
    RowMap m;
    m.base = buf.p;
    m.batch = rows / n_idx;
    m.batch_stride = (int64_t)n_idx * N;
    for (int i = 0; i < n_idx; ++i) m.push(i, i);
    hipEvent_t a, b;
    CSRMF_HIP(hipEventCreate(&a));
    CSRMF_HIP(hipEventCreate(&b));
    const int cands[] = {0, 64, 128, 256, 512, 1024, 2048};
    const int half = logN / 2;
    int best = 0, best_cached = 0, best_split = half;
    float best_ms = 1e30f;
    struct Cand { float ms; int split, chunk, cached; };
    std::vector<Cand> cand;
    std::string rep = "{";
    for (int split = half - 1; split <= half + 1; ++split) {
        if (!ntt_split_valid(logN, split)) continue;
        tabs.L1 = split;
        for (int cached = 0; cached < 2; ++cached) {
            for (int cnd : cands) {
                tabs.ntt_chunk_rows = cnd;
                tabs.ntt_cached_mid = cached;
                launch_ntt(tabs, m, false, stream);     // warm
                launch_ntt(tabs, m, true, stream);
                CSRMF_HIP(hipEventRecord(a, stream));
                for (int r = 0; r < 3; ++r) {
                    launch_ntt(tabs, m, false, stream);
                    launch_ntt(tabs, m, true, stream);
                }
                CSRMF_HIP(hipEventRecord(b, stream));
                CSRMF_HIP(hipEventSynchronize(b));
                float ms = 0;
                CSRMF_HIP(hipEventElapsedTime(&ms, a, b));
                ms /= 3;
                rep += (rep.size() > 1 ? ", " : "") + std::string("\"ntt_split=") + std::to_string(split) +
                       ",ntt_chunk_rows=" + std::to_string(cnd) + (cached ? ",cached_mid" : "") + "\": " +
                       std::to_string(ms);
                cand.push_back({ms, split, cnd, cached});
                if (ms < best_ms) { best_ms = ms; best = cnd; best_cached = cached; best_split = split; }
            }
        }
    }
    tabs.ntt_chunk_rows = best;
    tabs.ntt_cached_mid = best_cached;
    tabs.L1 = best_split;
    // With a rotation key, the transform schedules are ranked again and the
    // ModUp sub-batch chosen on batched rotations of scratch ciphertexts (the
    // data does not matter)
    if (!rot.empty()) {
        const int nb = std::max(1, std::min(64, rows / (2 * (L + 1))));
        std::vector<Ct> in(nb), out(nb);
        std::vector<Ct*> pin, pout;
        for (int i = 0; i < nb; ++i) {   // zero ciphertexts: the timing does not depend on the residues
            in[i] = new_ct(L, 1.0);
            CSRMF_HIP(hipMemsetAsync(in[i].d, 0, ct_words() * 8, stream));
            pin.push_back(&in[i]);
        }
        for (Ct& x : out) pout.push_back(&x);
        const uint32_t g = rot.begin()->first;
        // one batched rotation (warm-up, then the faster of two timed runs)
        auto time_rotation = [&]() -> float {
            float best_r = 1e30f;
            for (int r = 0; r < 3; ++r) {
                CSRMF_HIP(hipEventRecord(a, stream));
                rotate(pin, g, pout);
                CSRMF_HIP(hipEventRecord(b, stream));
                CSRMF_HIP(hipEventSynchronize(b));
                for (Ct& x : out) pool.put(x.d);
                float ms = 0;
                CSRMF_HIP(hipEventElapsedTime(&ms, a, b));
                if (r > 0 && ms < best_r) best_r = ms;
            }
            return best_r;
        };
        // The transforms alone do not rank the schedules of a whole key
        // switch reliably (their launches interleave with the conversion and
        // the inner products): the four fastest transform schedules are
        // ranked again by a batched rotation.
        std::sort(cand.begin(), cand.end(), [](const Cand& x, const Cand& y) { return x.ms < y.ms; });
        if (cand.size() > 4) cand.resize(4);
        modup_chunk = 0;
        float best_rot = 1e30f;
        for (const Cand& c : cand) {
            tabs.L1 = c.split;
            tabs.ntt_chunk_rows = c.chunk;
            tabs.ntt_cached_mid = c.cached;
            const float ms = time_rotation();
            rep += ", \"rotation ntt_split=" + std::to_string(c.split) + ",ntt_chunk_rows=" + std::to_string(c.chunk) +
                   (c.cached ? ",cached_mid" : "") + "\": " + std::to_string(ms);
            if (ms < best_rot) { best_rot = ms; best = c.chunk; best_cached = c.cached; best_split = c.split; }
        }
        tabs.L1 = best_split;
        tabs.ntt_chunk_rows = best;
        tabs.ntt_cached_mid = best_cached;
        rep += ", \"chosen_by_rotation\": [" + std::to_string(best_split) + ", " + std::to_string(best) + ", " +
               std::to_string(best_cached) + "]";
        const int mcands[] = {0, 8, 16, 32};
        int best_mc = 0;
        float best_mc_ms = 1e30f;
        for (int mc : mcands) {
            if (mc >= nb) continue;
            modup_chunk = mc;
            const float ms = mc == 0 ? best_rot : time_rotation();
            rep += ", \"modup_chunk=" + std::to_string(mc) + "\": " + std::to_string(ms);
            if (ms < best_mc_ms) { best_mc_ms = ms; best_mc = mc; }
        }
        modup_chunk = best_mc;
        rep += ", \"modup_chunk\": " + std::to_string(best_mc);
        for (Ct& x : in) pool.put(x.d);
        sync();
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    rep += ", \"chosen\": " + std::to_string(tabs.ntt_chunk_rows) + ", \"cached_mid\": " +
           std::to_string(tabs.ntt_cached_mid) + ", \"ntt_split\": " + std::to_string(tabs.L1) + "}";
    return rep;
}

Context::Hoist::~Hoist() {
    if (ctx) {
        ctx->pool.put(ext);
        ctx->pool.put(coef);
    }
}

void Context::hoist_begin(Hoist& h, const std::vector<Ct*>& in) {
    const int B = (int)in.size();
    if (B == 0) throw Error(CSRMF_E_INVAL, "empty hoisting batch");
    const int lvl = in[0]->level;
    for (Ct* x : in)
        if (x->level != lvl) throw Error(CSRMF_E_INVAL, "batch operands must share a level");
    const int nl = lvl + 1, nr = n_ext(lvl), nd = (int)lv[lvl].digits.size();
    h.ctx = this;
    h.in = in;
    h.level = lvl;
    h.ext = (uint64_t*)pool.get((size_t)B * nd * nr * N * 8);
    h.coef = (uint64_t*)pool.get((size_t)B * nl * N * 8);
    RowMap c1 = map_cts(in, nl);
    for (int i = 0; i < nl; ++i) c1.e[i] = ((uint32_t)(L + 1 + i) << 8) | (uint32_t)i;
    ks_modup(c1, lvl, B, h.ext, h.coef);
    fence();
}

void Context::hoist_rotate(Hoist& h, uint32_t g, std::vector<Ct*>& out) {
    const int B = (int)h.in.size();
    const int lvl = h.level, nl = lvl + 1, nr = n_ext(lvl);
    const Key& key = key_for(g);
    Scratch u(pool, (size_t)B * 2 * nr * N);
    RowMap c1 = map_cts(h.in, nl);
    for (int i = 0; i < nl; ++i) c1.e[i] = ((uint32_t)(L + 1 + i) << 8) | (uint32_t)i;
    const KsArgs ka = ks_args(h.ext, c1, lvl, B, key);
    n_key_switches += B;
    ks_inner(ka, lvl, B, g, u.p);
    for (int i = 0; i < B; ++i) *out[i] = new_ct(lvl, h.in[i]->scale);
    ks_moddown(ka, g, u.p, lvl, B, map_cts(out, nl), map_cts(h.in, nl), g, false);
    fence();
}

void Context::ntt_rows(uint64_t* data, int n_rows, const int32_t* idx, int n_idx, bool inverse) {
    if (n_idx <= 0 || n_idx > kMaxMapRows || n_rows % n_idx) throw Error(CSRMF_E_INVAL, "bad row map");
    RowMap m;
    m.base = data;
    m.batch = n_rows / n_idx;
    m.batch_stride = (int64_t)n_idx * N;
    for (int i = 0; i < n_idx; ++i) {
        if (idx[i] < 0 || idx[i] >= (int)moduli.size()) throw Error(CSRMF_E_INVAL, "bad limb index");
        m.push(i, idx[i]);
    }
    launch_ntt(tabs, m, inverse, stream);
    sync();   // the rows are caller memory: done on return
}

}  // namespace csrmf
