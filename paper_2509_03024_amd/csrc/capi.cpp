// extern "C" entry points of libcsrmf (declared in include/csrmf.h).
#include <algorithm>
#include <cstring>
#include <new>

#include "bootstrap.h"
#include "context.h"
#include "host_math.h"
#include "prof.h"

using csrmf::Context;
using csrmf::Ct;
using csrmf::Error;

#define tl_err csrmf::last_error()

#define API_BEGIN(ctx)                                   \
    if (!(ctx)) { tl_err = "null context"; return CSRMF_E_INVAL; } \
    std::lock_guard<std::recursive_mutex> lk_((ctx)->mu); \
    try {
#define API_END(ctx)                                     \
        tl_err.clear();                                  \
        return CSRMF_OK;                                 \
    } catch (const Error& e) {                           \
        tl_err = e.what();                               \
        return e.code;                                   \
    } catch (const std::bad_alloc&) {                    \
        tl_err = "host allocation failed";               \
        return CSRMF_E_NOMEM;                            \
    } catch (const std::exception& e) {                  \
        tl_err = e.what();                               \
        return CSRMF_E_DEVICE;                           \
    }

#define NEED(cond, msg) \
    if (!(cond)) throw Error(CSRMF_E_INVAL, msg)

extern "C" {

int csrmf_create(const csrmf_params* p, const uint8_t seed[32], csrmf_ctx** out) {
    if (!p || !seed || !out) {
        tl_err = "csrmf_create: null argument";
        return CSRMF_E_INVAL;
    }
    *out = nullptr;
    Context* c = nullptr;
    try {
        c = new Context();
        c->init(*p, seed);
    } catch (const Error& e) {
        tl_err = std::string("csrmf_create: ") + e.what();
        delete c;
        return e.code;
    } catch (const std::exception& e) {
        tl_err = std::string("csrmf_create: ") + e.what();
        delete c;
        return CSRMF_E_NOMEM;
    }
    tl_err.clear();
    *out = reinterpret_cast<csrmf_ctx*>(c);
    return CSRMF_OK;
}

void csrmf_destroy(csrmf_ctx* ctx) { delete reinterpret_cast<Context*>(ctx); }

const char* csrmf_last_error(const csrmf_ctx*) { return tl_err.c_str(); }

int csrmf_set_stream(csrmf_ctx* cx, void* s) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    c->sync();
    c->stream = (hipStream_t)s;
    c->staging.set_stream(c->stream);
    API_END(c)
}

int csrmf_sync(csrmf_ctx* cx) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    c->sync();
    API_END(c)
}

int csrmf_counters(const csrmf_ctx* cx, int64_t* key_switches) {
    const Context* c = reinterpret_cast<const Context*>(cx);
    if (!c || !key_switches) {
        tl_err = "csrmf_counters: null argument";
        return CSRMF_E_INVAL;
    }
    *key_switches = c->n_key_switches;
    return CSRMF_OK;
}

int csrmf_get_chain(const csrmf_ctx* cx, int32_t* L, int32_t* alpha, uint64_t* moduli) {
    const Context* c = reinterpret_cast<const Context*>(cx);
    if (!c) return CSRMF_E_INVAL;
    if (L) *L = c->L;
    if (alpha) *alpha = c->alpha;
    if (moduli) std::memcpy(moduli, c->moduli.data(), c->moduli.size() * 8);
    return CSRMF_OK;
}

int csrmf_keygen(csrmf_ctx* cx, const int32_t* steps, int32_t n, int32_t conj) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    NEED(n >= 0 && (n == 0 || steps), "rotation steps");
    c->keygen(steps, n, conj != 0);
    API_END(c)
}

int csrmf_encode(const csrmf_ctx* cx, const double* z, int32_t n, double scale, int64_t* m) {
    const Context* c = reinterpret_cast<const Context*>(cx);
    if (!c || !m || (n > 0 && !z) || n < 0 || (uint64_t)n > c->N / 2 || !(scale > 0)) return CSRMF_E_INVAL;
    return csrmf::ckks_encode(z, n, c->logN, scale, m) ? CSRMF_OK : CSRMF_E_INVAL;
}

int csrmf_decode(const csrmf_ctx* cx, const int64_t* m, double scale, double* z, int32_t n) {
    const Context* c = reinterpret_cast<const Context*>(cx);
    if (!c || !m || !z || n < 0 || (uint64_t)n > c->N / 2 || !(scale > 0)) return CSRMF_E_INVAL;
    csrmf::ckks_decode(m, c->logN, scale, z, n);
    return CSRMF_OK;
}

int csrmf_encrypt(csrmf_ctx* cx, const double* z, int32_t n, int32_t level, double scale, uint64_t* h) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    NEED(h && (n == 0 || z) && n >= 0 && (uint64_t)n <= c->N / 2 && scale > 0, "encrypt arguments");
    std::vector<int64_t> m(c->N);
    NEED(csrmf::ckks_encode(z, n, c->logN, scale, m.data()), "value too large to encode");
    *h = c->put(c->encrypt_int(m.data(), level, scale));
    API_END(c)
}

int csrmf_encrypt_int(csrmf_ctx* cx, const int64_t* m, int32_t level, double scale, uint64_t* h) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    NEED(m && h && scale > 0, "encrypt_int arguments");
    *h = c->put(c->encrypt_int(m, level, scale));
    API_END(c)
}

int csrmf_decrypt_int(csrmf_ctx* cx, uint64_t h, int64_t* m) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    NEED(m, "output");
    c->decrypt_int(c->get(h), m);
    API_END(c)
}

int csrmf_decrypt(csrmf_ctx* cx, uint64_t h, double* z, int32_t n) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    NEED(z && n >= 0 && (uint64_t)n <= c->N / 2, "decrypt arguments");
    const Ct& ct = c->get(h);
    std::vector<int64_t> m(c->N);
    c->decrypt_int(ct, m.data());
    csrmf::ckks_decode(m.data(), c->logN, ct.scale, z, n);
    API_END(c)
}

int csrmf_import_ct(csrmf_ctx* cx, const uint64_t* coeffs, int32_t level, double scale, uint64_t* h) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    NEED(coeffs && h && scale > 0, "import arguments");
    *h = c->put(c->import_ct(coeffs, level, scale));
    API_END(c)
}

int csrmf_export_ct(csrmf_ctx* cx, uint64_t h, uint64_t* coeffs, int32_t* level, double* scale) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    const Ct& ct = c->get(h);
    if (level) *level = ct.level;
    if (scale) *scale = ct.scale;
    if (coeffs) c->export_ct(ct, coeffs);
    API_END(c)
}

int csrmf_ct_info(const csrmf_ctx* cx, uint64_t h, int32_t* level, double* scale) {
    Context* c = const_cast<Context*>(reinterpret_cast<const Context*>(cx));
    API_BEGIN(c)
    const Ct& ct = c->get(h);
    if (level) *level = ct.level;
    if (scale) *scale = ct.scale;
    API_END(c)
}

int csrmf_free_ct(csrmf_ctx* cx, uint64_t h) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    c->free_ct(h);
    API_END(c)
}

int csrmf_export_key(csrmf_ctx* cx, int32_t which, uint32_t galois, uint64_t* out) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    NEED(out, "output");
    c->export_key(which, galois, out);
    API_END(c)
}

int csrmf_add(csrmf_ctx* cx, uint64_t a, uint64_t b, uint64_t* out) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    NEED(out, "output");
    Ct r;
    c->add(c->get(a), c->get(b), r, false);
    *out = c->put(r);
    API_END(c)
}

int csrmf_sub(csrmf_ctx* cx, uint64_t a, uint64_t b, uint64_t* out) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    NEED(out, "output");
    Ct r;
    c->add(c->get(a), c->get(b), r, true);
    *out = c->put(r);
    API_END(c)
}

int csrmf_add_batch(csrmf_ctx* cx, const uint64_t* a, const uint64_t* b, int32_t n, int32_t subtract,
                    uint64_t* out) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    NEED(a && b && out && n > 0, "arguments");
    std::vector<Ct*> va, vb;
    for (int i = 0; i < n; ++i) {
        va.push_back(&c->get(a[i]));
        vb.push_back(&c->get(b[i]));
    }
    std::vector<Ct> res(n);
    std::vector<Ct*> vo;
    for (auto& r : res) vo.push_back(&r);
    c->add_batch(va, vb, vo, subtract != 0);
    for (int i = 0; i < n; ++i) out[i] = c->put(res[i]);
    API_END(c)
}

int csrmf_add_plain(csrmf_ctx* cx, uint64_t a, const int64_t* m, uint64_t* out) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    NEED(m && out, "arguments");
    Ct r;
    c->add_plain(c->get(a), m, r);
    *out = c->put(r);
    API_END(c)
}

int csrmf_mul_plain(csrmf_ctx* cx, uint64_t a, const int64_t* m, double pt_scale, uint64_t* out) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    NEED(m && out && pt_scale > 0, "arguments");
    Ct r;
    c->mul_plain(c->get(a), m, pt_scale, r);
    *out = c->put(r);
    API_END(c)
}

int csrmf_mul_int(csrmf_ctx* cx, uint64_t a, int64_t w, uint64_t* out) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    NEED(out && w != 0, "arguments");
    Ct r;
    c->mul_int(c->get(a), w, r);
    *out = c->put(r);
    API_END(c)
}

static void batch_mul(Context* c, const uint64_t* a, const uint64_t* b, int32_t n, uint64_t* out, bool rescale) {
    NEED(a && b && out && n > 0, "arguments");
    if (!c->have_keys) throw Error(CSRMF_E_STATE, "keygen first");
    std::vector<Ct*> va, vb;
    for (int i = 0; i < n; ++i) {
        va.push_back(&c->get(a[i]));
        vb.push_back(&c->get(b[i]));
        c->check_scales(va.back()->scale, va[0]->scale);
        if (rescale && std::min(va.back()->level, vb.back()->level) < 1) throw Error(CSRMF_E_LEVEL, "no level left");
    }
    std::vector<Ct> res(n);
    std::vector<Ct*> vo;
    for (auto& r : res) vo.push_back(&r);
    c->mul_relin(va, vb, vo);
    if (rescale) c->rescale(vo);
    for (int i = 0; i < n; ++i) out[i] = c->put(res[i]);
}

int csrmf_hmult(csrmf_ctx* cx, uint64_t a, uint64_t b, uint64_t* out) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    batch_mul(c, &a, &b, 1, out, true);
    API_END(c)
}

int csrmf_mul_relin(csrmf_ctx* cx, uint64_t a, uint64_t b, uint64_t* out) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    batch_mul(c, &a, &b, 1, out, false);
    API_END(c)
}

int csrmf_hmult_batch(csrmf_ctx* cx, const uint64_t* a, const uint64_t* b, int32_t n, uint64_t* out) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    batch_mul(c, a, b, n, out, true);
    API_END(c)
}

int csrmf_rescale(csrmf_ctx* cx, uint64_t a, uint64_t* out) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    NEED(out, "output");
    const Ct& src = c->get(a);
    if (src.level < 1) throw Error(CSRMF_E_LEVEL, "no level left to rescale");
    Ct r = c->new_ct(src.level, src.scale);
    CSRMF_HIP(hipMemcpyAsync(r.d, src.d, c->ct_words() * 8, hipMemcpyDeviceToDevice, c->stream));
    std::vector<Ct*> v{&r};
    c->rescale(v);
    *out = c->put(r);
    API_END(c)
}

int csrmf_mod_drop(csrmf_ctx* cx, uint64_t a, int32_t level, uint64_t* out) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    NEED(out && level >= 0, "arguments");
    const Ct& src = c->get(a);
    if (level > src.level) throw Error(CSRMF_E_LEVEL, "cannot raise the level");
    Ct r = c->new_ct(level, src.scale);
    CSRMF_HIP(hipMemcpyAsync(r.d, src.d, c->ct_words() * 8, hipMemcpyDeviceToDevice, c->stream));
    *out = c->put(r);
    API_END(c)
}

static void batch_rot(Context* c, const uint64_t* a, int32_t n, uint32_t g, uint64_t* out) {
    NEED(a && out && n > 0, "arguments");
    std::vector<Ct*> va;
    for (int i = 0; i < n; ++i) va.push_back(&c->get(a[i]));
    std::vector<Ct> res(n);
    std::vector<Ct*> vo;
    for (auto& r : res) vo.push_back(&r);
    if (g == 1) {
        for (int i = 0; i < n; ++i) {
            res[i] = c->new_ct(va[i]->level, va[i]->scale);
            CSRMF_HIP(hipMemcpyAsync(res[i].d, va[i]->d, c->ct_words() * 8, hipMemcpyDeviceToDevice, c->stream));
        }
    } else {
        c->rotate(va, g, vo);
    }
    for (int i = 0; i < n; ++i) out[i] = c->put(res[i]);
}

int csrmf_rotate(csrmf_ctx* cx, uint64_t a, int32_t r, uint64_t* out) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    batch_rot(c, &a, 1, c->galois_for_step(r), out);
    API_END(c)
}

int csrmf_rotate_batch(csrmf_ctx* cx, const uint64_t* a, int32_t n, int32_t r, uint64_t* out) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    batch_rot(c, a, n, c->galois_for_step(r), out);
    API_END(c)
}

int csrmf_rotate_add_batch(csrmf_ctx* cx, const uint64_t* a, const uint64_t* acc, int32_t n, int32_t r,
                           uint64_t* out) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    NEED(a && acc && out && n > 0, "arguments");
    const uint32_t g = c->galois_for_step(r);
    std::vector<Ct*> va, vacc;
    for (int i = 0; i < n; ++i) {
        va.push_back(&c->get(a[i]));
        vacc.push_back(&c->get(acc[i]));
    }
    std::vector<Ct> res(n);
    std::vector<Ct*> vo;
    for (auto& x : res) vo.push_back(&x);
    if (g == 1) c->add_batch(vacc, va, vo, false);
    else c->rotate(va, g, vo, &vacc);
    for (int i = 0; i < n; ++i) out[i] = c->put(res[i]);
    API_END(c)
}

int csrmf_conjugate(csrmf_ctx* cx, uint64_t a, uint64_t* out) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    batch_rot(c, &a, 1, (uint32_t)(2 * c->N - 1), out);
    API_END(c)
}

int csrmf_conjugate_batch(csrmf_ctx* cx, const uint64_t* a, int32_t n, uint64_t* out) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    batch_rot(c, a, n, (uint32_t)(2 * c->N - 1), out);
    API_END(c)
}

int csrmf_rotate_hoisted(csrmf_ctx* cx, uint64_t a, const int32_t* r, int32_t n, uint64_t* out) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    NEED(r && out && n > 0, "arguments");
    std::vector<uint32_t> gs;
    for (int i = 0; i < n; ++i) gs.push_back(c->galois_for_step(r[i]));
    std::vector<Ct> res(n);
    std::vector<Ct*> vo;
    for (auto& x : res) vo.push_back(&x);
    c->rotate_hoisted(c->get(a), gs, vo);
    for (int i = 0; i < n; ++i) out[i] = c->put(res[i]);
    API_END(c)
}

static csrmf::BootCfg boot_cfg(const csrmf_boot_config* cfg) {
    NEED(cfg, "configuration");
    csrmf::BootCfg b;
    b.n = cfg->n_slots;
    b.r = cfg->squarings;
    b.d = cfg->degree;
    b.pre_bits = cfg->pre_bits;
    NEED(cfg->arcsine == 0 || cfg->arcsine == 1, "arcsine must be 0 or 1");
    b.arcsine = cfg->arcsine != 0;
    return b;
}

int csrmf_boot_levels(const csrmf_boot_config* cfg, int32_t* levels) {
    if (!cfg || !levels || cfg->degree < 1 || (cfg->arcsine != 0 && cfg->arcsine != 1)) return CSRMF_E_INVAL;
    *levels = csrmf::boot_levels(boot_cfg(cfg));
    return CSRMF_OK;
}

int csrmf_boot_rotation_steps(csrmf_ctx* cx, const csrmf_boot_config* cfg, int32_t* steps, int32_t cap,
                              int32_t* count) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    NEED(count && (steps || cap == 0) && cap >= 0, "arguments");
    const csrmf::BootCfg b = boot_cfg(cfg);
    csrmf::boot_check(c, b);
    const std::vector<int32_t> s = csrmf::boot_rotation_steps(c->N, b.n);
    *count = (int32_t)s.size();
    NEED((int32_t)s.size() <= cap, "steps array too small");
    std::copy(s.begin(), s.end(), steps);
    API_END(c)
}

int csrmf_bootstrap(csrmf_ctx* cx, const csrmf_boot_config* cfg, const uint64_t* in, int32_t n, uint64_t* out) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    NEED(in && out && n > 0, "arguments");
    const csrmf::BootCfg b = boot_cfg(cfg);
    std::vector<Ct*> v;
    for (int i = 0; i < n; ++i) v.push_back(&c->get(in[i]));
    std::vector<Ct> res;
    csrmf::bootstrap(c, b, v, res);
    for (int i = 0; i < n; ++i) out[i] = c->put(res[i]);
    API_END(c)
}

int csrmf_ntt_rows(csrmf_ctx* cx, uint64_t* data, int32_t n_rows, const int32_t* idx, int32_t n_idx,
                   int32_t inverse) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    NEED(data && idx && n_rows > 0, "arguments");
    c->ntt_rows(data, n_rows, idx, n_idx, inverse != 0);
    API_END(c)
}

int csrmf_autotune(csrmf_ctx* cx, int32_t rows, char* report, int32_t cap) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    const std::string s = c->autotune(rows);
    if (report && cap > 0) {
        const size_t n = std::min<size_t>(s.size(), (size_t)cap - 1);
        std::memcpy(report, s.data(), n);
        report[n] = 0;
    }
    API_END(c)
}

int csrmf_set_ntt_schedule(csrmf_ctx* cx, int32_t chunk_rows) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    NEED(chunk_rows >= 0, "NTT schedule: rows per pair of passes must be >= 0");
    c->tabs.ntt_chunk_rows = chunk_rows;
    API_END(c)
}

int csrmf_set_schedule(csrmf_ctx* cx, int32_t ntt_chunk_rows, int32_t ntt_cached_mid, int32_t modup_chunk,
                       int32_t ntt_split) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    NEED(ntt_chunk_rows >= 0 && modup_chunk >= 0 && (ntt_cached_mid == 0 || ntt_cached_mid == 1), "schedule values");
    const int l1 = ntt_split ? ntt_split : c->tabs.logN / 2;
    NEED(csrmf::ntt_split_valid(c->tabs.logN, l1), "NTT split: both passes need 6 to 9 stages");
    c->tabs.ntt_chunk_rows = ntt_chunk_rows;
    c->tabs.ntt_cached_mid = ntt_cached_mid;
    c->tabs.L1 = l1;
    c->modup_chunk = modup_chunk;
    API_END(c)
}

int csrmf_get_schedule(const csrmf_ctx* cx, int32_t* ntt_chunk_rows, int32_t* ntt_cached_mid, int32_t* modup_chunk,
                       int32_t* ntt_split) {
    const Context* c = reinterpret_cast<const Context*>(cx);
    if (!c) return CSRMF_E_INVAL;
    if (ntt_chunk_rows) *ntt_chunk_rows = c->tabs.ntt_chunk_rows;
    if (ntt_cached_mid) *ntt_cached_mid = c->tabs.ntt_cached_mid;
    if (modup_chunk) *modup_chunk = c->modup_chunk;
    if (ntt_split) *ntt_split = c->tabs.L1;
    return CSRMF_OK;
}

int csrmf_graph_begin(csrmf_ctx* cx) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    c->graph_begin();
    API_END(c)
}

int csrmf_graph_end(csrmf_ctx* cx, uint64_t* graph) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    NEED(graph, "graph");
    *graph = c->graph_end();
    API_END(c)
}

int csrmf_graph_launch(csrmf_ctx* cx, uint64_t graph) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    c->graph_launch(graph);
    API_END(c)
}

int csrmf_graph_destroy(csrmf_ctx* cx, uint64_t graph) {
    Context* c = reinterpret_cast<Context*>(cx);
    API_BEGIN(c)
    c->graph_destroy(graph);
    API_END(c)
}

int csrmf_profile_enable(int32_t enable) {
    csrmf::prof_enable(enable != 0);
    return CSRMF_OK;
}

int csrmf_profile_report(char* buf, int32_t cap) {
    const std::string s = csrmf::prof_report_json();
    if (buf && cap > 0) {
        const size_t n = std::min<size_t>(s.size(), (size_t)cap - 1);
        std::memcpy(buf, s.data(), n);
        buf[n] = 0;
    }
    return (int)s.size();
}

}  // extern "C"
