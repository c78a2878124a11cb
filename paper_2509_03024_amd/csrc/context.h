// Host-side context of libcsrmf: modulus chain, device tables, keys,
// ciphertext store and the orchestration of the device kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/csrmf.h"
#include "kernels.h"
#include "staging.h"

namespace csrmf {

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define CSRMF_HIP(x)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess)                                                              \
            throw ::csrmf::Error(CSRMF_E_DEVICE, std::string(#x ": ") + hipGetErrorString(e_)); \
    } while (0)

// Device ciphertext: polynomials c0, c1 in evaluation form, each with room
// for L+1 limbs (poly stride (L+1)*N words); limbs 0..level are valid.
struct Ct {
    uint64_t* d = nullptr;
    int level = 0;
    double scale = 1.0;
};

// A switching key: [n_digits][2 (b, a)][L+1+alpha][N]; rows of 60-bit primes are
// stored times 2^64 mod q, rows of primes below 2^44 as centred doubles (bit patterns).
struct Key {
    uint64_t* d = nullptr;
    int n_digits = 0;
};

struct DigitConsts {
    int lo, hi;                 // limbs [lo, hi) of the digit at this level
    uint64_t* yc = nullptr;     // [|D|][2]
    uint64_t* cc = nullptr;     // [n_tgt][kBcRecordWords(|D|)]  conversion records (launch_basis_convert)
};

struct LevelConsts {
    std::vector<DigitConsts> digits;
    uint64_t* md_y = nullptr;       // [alpha][4]  (P/p_k)^-1 mod p_k with the constants of its product
    uint64_t* md_c = nullptr;       // [l+1][kBcRecordWords(alpha)]  records of the conversion P -> Q_l
    uint64_t* md_pinv = nullptr;    // [l+1][2]  P^-1 mod q_i
    uint64_t* rs = nullptr;         // [l][4]  h mod q_i, q_l^-1 mod q_i, shoup, 0
};

// Caching device allocator.  Requests are rounded up to size classes (eight
// per power of two), so buffers of similar size are reused instead of
// allocated.  A block handed back with put() may be handed out again at once:
// all users run on the context's single stream, so later work is ordered
// after earlier work on the block.
//
// While a HIP graph is being captured, every block the pool hands out or
// takes back is recorded: blocks freed during the capture are reused only
// within it, and at its end all recorded blocks leave the pool for the graph
// (a replay writes them again), which frees them when it is destroyed.
class Pool {
public:
    ~Pool();
    void* get(size_t bytes);
    void put(void* p);
    void release_all();
    size_t bytes_in_use() const { return in_use_; }
    static size_t size_class(size_t bytes);
    void begin_capture();
    std::vector<void*> end_capture();   // the blocks the graph now owns
    void free_blocks(const std::vector<void*>& v);

private:
    std::multimap<size_t, void*> free_;
    std::unordered_map<void*, size_t> sizes_;
    size_t in_use_ = 0;
    bool capture_ = false;
    std::unordered_map<void*, size_t> cap_blocks_;   // touched during the capture
    std::multimap<size_t, void*> cap_free_;          // freed during the capture (reusable within it)
    std::unordered_map<void*, size_t> graph_owned_;  // put() of these is ignored
};

// Markers of the staging ring: events on the context's stream.
struct HipMarkers {
    hipStream_t stream = nullptr;
    std::vector<hipEvent_t> spare;
    hipEvent_t record();
    void wait(hipEvent_t e);
    void release(hipEvent_t e) { spare.push_back(e); }
    ~HipMarkers();
};

// Pinned host ring + device ring for per-launch arguments (see staging.h).
//
// During a graph capture put() bump-allocates from the graph's own arena
// instead (pinned host + device, never reused while the graph exists): the
// captured copy node reads the host arena at every replay.
class Staging {
public:
    static constexpr size_t kBytes = (size_t)64 << 20;
    Staging() : ring_(kBytes) {}
    ~Staging() { release(); }
    void init(hipStream_t s);
    void release();   // waits for the stream, frees both rings
    void set_stream(hipStream_t s) { ops_.stream = s; }   // only after drained()
    // copy `bytes` from host memory into the device ring (asynchronously, on
    // the stream); the device pointer stays valid until work enqueued before
    // the next fence() has completed
    void* put(const void* src, size_t bytes);
    void fence() {
        if (!arena_host_) ring_.fence(ops_);
    }
    void drained() { ring_.drained(ops_); }   // after a stream synchronisation
    void begin_arena(uint8_t* host, uint8_t* dev, size_t bytes) {
        arena_host_ = host;
        arena_dev_ = dev;
        arena_cap_ = bytes;
        arena_used_ = 0;
    }
    void end_arena() { arena_host_ = arena_dev_ = nullptr; }

private:
    uint8_t* host_ = nullptr;
    uint8_t* dev_ = nullptr;
    HipMarkers ops_;
    RingPositions<HipMarkers, hipEvent_t> ring_;
    uint8_t* arena_host_ = nullptr;
    uint8_t* arena_dev_ = nullptr;
    size_t arena_cap_ = 0, arena_used_ = 0;
};

// A captured HIP graph of a context's evaluation calls and the memory it owns.
struct CapturedGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<void*> blocks;          // pool blocks the graph's kernels use
    uint8_t* arena_host = nullptr;      // staged launch arguments
    uint8_t* arena_dev = nullptr;
};

// Scratch buffer that returns itself to the pool.
struct Scratch {
    Pool* pool = nullptr;
    uint64_t* p = nullptr;
    Scratch(Pool& pl, size_t words) : pool(&pl), p((uint64_t*)pl.get(words * 8)) {}
    ~Scratch() { if (p) pool->put(p); }
    Scratch(const Scratch&) = delete;
    Scratch& operator=(const Scratch&) = delete;
};

// Message of the calling thread's last failed API call (csrmf_last_error).
std::string& last_error();

// Static device scratch of csrmf_rotate_noalloc (bytes; each device the
// library runs on holds one until the process ends).
constexpr size_t kNoAllocScratchBytes = (size_t)128 << 20;
// Device address of that buffer on the current device (looked up once per
// device with hipGetSymbolAddress, then cached).
uint64_t* noalloc_scratch_for_current_device();

// Messages and bytes per channel of the three-party protocol (protocol.cpp).
struct ProtocolCounters {
    static constexpr int kChannels = 8;
    int64_t msgs[kChannels] = {};
    int64_t bytes[kChannels] = {};
};

struct MfState;  // encrypted matrix-factorisation program (mf_program.cpp)
void destroy_mf(MfState* m);
struct Server;   // request server (serving.cpp)
void destroy_server(Server* s);

struct Context {
    csrmf_params prm{};
    uint8_t seed[32];
    int logN = 0;
    uint64_t N = 0;
    int L = 0, alpha = 0, dnum = 0, gsize = 0;
    std::vector<uint64_t> moduli;      // q_0..q_L, p_0..p_{alpha-1}
    std::vector<Modulus> mh;
    Modulus* d_mods = nullptr;
    uint64_t* d_tw = nullptr;
    DevTables tabs{};
    std::vector<LevelConsts> lv;
    hipStream_t stream = nullptr;       // stream of all device work
    hipStream_t own_stream = nullptr;   // the stream the context created (destroyed with it)
    Pool pool;
    std::recursive_mutex mu;        // serialises API calls and the serving worker

    uint64_t serial = 0;
    bool have_keys = false;
    uint64_t* s_ntt = nullptr;      // [L+1+alpha][N] plain
    uint64_t* s_mont = nullptr;     // s * 2^64
    uint64_t* pk = nullptr;         // [2][L+1][N] times 2^64
    Key relin;
    std::map<uint32_t, Key> rot;

    std::unordered_map<uint64_t, Ct> cts;
    uint64_t next_handle = 1;
    Staging staging;
    MfState* mf = nullptr;
    int max_babies = 1024;          // block permutations: baby ciphertexts alive at once
    int modup_chunk = 0;            // key switching: ciphertexts per ModUp sub-batch (0 = the whole batch)
    int64_t n_key_switches = 0;     // key switches enqueued (relinearisations and rotations)
    bool capturing = false;         // the stream is being captured into a HIP graph
    std::map<uint64_t, CapturedGraph> graphs;
    uint64_t next_graph = 1;
    static constexpr size_t kGraphArenaBytes = (size_t)32 << 20;
    void graph_begin();
    uint64_t graph_end();
    void graph_launch(uint64_t id);
    void graph_destroy(uint64_t id);
    ProtocolCounters proto;         // the last protocol run's message accounting
    std::vector<Server*> servers;   // stopped and freed before the context

    Context() = default;
    ~Context();
    void init(const csrmf_params& p, const uint8_t s[32]);

    // --- geometry
    int n_ext(int level) const { return level + 1 + alpha; }
    int gmod_ext(int level, int t) const { return t <= level ? t : L + 1 + (t - level - 1); }
    int64_t poly_stride() const { return (int64_t)(L + 1) * (int64_t)N; }
    size_t ct_words() const { return 2 * (size_t)(L + 1) * N; }

    // --- ciphertext store
    Ct new_ct(int level, double scale);
    uint64_t put(const Ct& c);
    Ct& get(uint64_t h);
    void free_ct(uint64_t h);
    // device copy of a pointer table (staging ring; valid for work enqueued before the next fence)
    uint64_t** ptr_table(const std::vector<uint64_t*>& v);
    // per-launch arguments through the staging ring; fence() after enqueueing their users
    void* stage(const void* src, size_t bytes) { return staging.put(src, bytes); }
    void fence() { staging.fence(); }
    // wait for the stream (and recycle the staging ring); `caller` names the
    // operation in the error raised while a graph is being captured
    void sync(const char* caller = __builtin_FUNCTION());

    RowMap map_ct(uint64_t* d, int nlimbs, int first = 0) const;
    RowMap map_cts(const std::vector<Ct*>& v, int nlimbs, int first = 0);

    // --- keys
    void keygen(const int32_t* steps, int n, bool conj);
    void add_rotation_key(uint32_t g);
    void make_switching_key(Key& k, const uint64_t* sprime_ntt, uint32_t key_index);
    bool has_key(uint32_t g) const { return rot.count(g) != 0; }
    const Key& key_for(uint32_t g) const;
    uint32_t galois_for_step(int64_t r) const;

    // --- encryption
    Ct encrypt_int(const int64_t* m, int level, double scale);
    void encrypt_int_batch(const int64_t* m, int count, int level, double scale, std::vector<Ct>& out,
                           const uint32_t* serials = nullptr);
    void decrypt_int(const Ct& c, int64_t* m);
    void export_ct(const Ct& c, uint64_t* coeffs);
    Ct import_ct(const uint64_t* coeffs, int level, double scale);
    void export_key(int which, uint32_t g, uint64_t* out);

    // --- evaluation (batched; every vector holds ciphertexts of equal level)
    void add(const Ct& a, const Ct& b, Ct& out, bool sub);
    void add_batch(const std::vector<Ct*>& a, const std::vector<Ct*>& b, std::vector<Ct*>& out, bool sub);
    void add_plain(const Ct& a, const int64_t* m, Ct& out);
    void mul_plain(const Ct& a, const int64_t* m, double pt_scale, Ct& out);
    // multiply by the integer w; the result's scale is scale * w, or `declared` if non-zero
    void mul_int(const Ct& a, int64_t w, Ct& out, double declared = 0.0);
    void mul_relin(const std::vector<Ct*>& a, const std::vector<Ct*>& b, std::vector<Ct*>& out);
    void rescale(const std::vector<Ct*>& v);          // in place
    void mod_drop(Ct& c, int level);                   // in place
    // ModRaise of level-0 ciphertexts: out[i] (level L, scale `scale`) holds the
    // centred residues of in[i] mod q_0 taken modulo every q_j
    void mod_raise(const std::vector<Ct*>& in, double scale, std::vector<Ct*>& out);
    // out[i] = a[i] x m for one plaintext m (signed coefficients) shared by the batch;
    // with accumulate, out[i] += a[i] x m into existing ciphertexts of a[i]'s level
    // and scale a[i].scale * pt_scale (their scale is kept)
    void mul_plain_batch(const std::vector<Ct*>& a, const int64_t* m, double pt_scale, std::vector<Ct*>& out,
                         bool accumulate = false);
    // out[i] = tau_g(in[i]) key-switched; with acc, out[i] = acc[i] + that (fused)
    void rotate(const std::vector<Ct*>& in, uint32_t g, std::vector<Ct*>& out, const std::vector<Ct*>* acc = nullptr);
    void rotate_hoisted(const Ct& in, const std::vector<uint32_t>& gs, std::vector<Ct*>& out);
    // out = tau_g(in) key-switched into the existing ciphertext `out` (not
    // `in`), all scratch in the library's static device buffer: no allocation
    void rotate_noalloc(const Ct& in, uint32_t g, Ct& out);
    uint64_t* noalloc_scratch = nullptr;   // this context's device address of that buffer
    void check_scales(double a, double b) const;

    // --- hoisted rotations of a batch: ModUp once, then any number of Galois elements
    struct Hoist {
        Context* ctx = nullptr;
        std::vector<Ct*> in;
        int level = 0;
        uint64_t* ext = nullptr;
        uint64_t* coef = nullptr;
        ~Hoist();
    };
    void hoist_begin(Hoist& h, const std::vector<Ct*>& in);
    void hoist_rotate(Hoist& h, uint32_t g, std::vector<Ct*>& out);

    // --- key-switching pieces
    void ks_modup(const RowMap& d_in, int level, int B, uint64_t* ext, uint64_t* coef);
    // Arguments of the inner product with `key`; d_in: the ModUp input
    // (evaluation form), which supplies each digit's own limbs
    KsArgs ks_args(const uint64_t* ext, const RowMap& d_in, int level, int B, const Key& key) const;
    // u's special limbs (tau_g applied to the ext reads)
    void ks_inner(const KsArgs& a, int level, int B, uint32_t g, uint64_t* u);
    // ModDown of u's special limbs, fused with the Q limbs' inner product (a, g)
    // (conv_buf: scratch of 2 B (level+1) N words for the converted P part, or
    // null to take it from the pool)
    void ks_moddown(const KsArgs& a, uint32_t g, uint64_t* u, int level, int B, const RowMap& out,
                    const RowMap& addend, uint32_t g_add, bool addend_both, const RowMap& acc = RowMap(),
                    uint64_t* conv_buf = nullptr);

    // --- schedule autotuning (returns a JSON report)
    std::string autotune(int rows);

    // --- raw NTT hook
    void ntt_rows(uint64_t* data, int n_rows, const int32_t* idx, int n_idx, bool inverse);
};

}  // namespace csrmf
