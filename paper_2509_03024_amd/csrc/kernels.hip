// gfx950 kernels for RNS-CKKS: negacyclic NTT/INTT, elementwise modular
// arithmetic, tensor product, automorphism, fast basis conversion, key
// switching inner product, ModDown and rescale.
//
// Layout: every polynomial row is N contiguous uint64 residues (limb-major);
// a launch covers a RowMap of rows.  Blocks are ordered limb-major over the
// batch (consecutive blocks share a modulus and its tables in L2).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.h"
#include "prof.h"

namespace csrmf {

namespace {

constexpr int kThreads = 256;
constexpr int kXcds = 8;          // accelerator complex dies of an MI355X (separate L2 each)
// Elements per thread of the masked MAC.  A tile is kThreads * kMacPerThread
// elements of one limb; all tasks of a tile run on one XCD, and the tiles of
// the launch's sources (babies: up to ~500 ciphertexts x 16 B per element)
// must stay within that XCD's 4 MB L2, which 2 allows (8 was measured 16 %
// slower, 4x larger tiles; 4 only 2 % faster at half the occupancy).
constexpr int kMacPerThread = 2;
constexpr int kEwPerThread = 2;

__device__ __forceinline__ uint64_t* map_row(const RowMap& m, int b, int k, int logN, int& mod) {
    const uint32_t e = m.e[k];
    mod = (int)(e & 0xffu);
    uint64_t* p = m.ptrs ? m.ptrs[b] : m.base + (int64_t)b * m.batch_stride;
    return p + ((int64_t)(e >> 8) << logN);
}

// Block -> (batch element, map entry, chunk); limb-major over the batch.
__device__ __forceinline__ void block_coords(int blk, int chunks, int batch, int& b, int& k, int& chunk) {
    chunk = blk % chunks;
    const int r = blk / chunks;
    b = r % batch;
    k = r / batch;
}

__device__ __forceinline__ uint32_t brev_n(uint32_t x, int logN) { return __brev(x) >> (32 - logN); }

// evaluation-form index permutation of tau_g
__device__ __forceinline__ uint32_t galois_perm(uint32_t k, uint32_t g, int logN) {
    const uint32_t twoN_mask = (2u << logN) - 1u;
    const uint32_t e = 2u * brev_n(k, logN) + 1u;
    const uint32_t f = (uint32_t)(((uint64_t)e * g) & twoN_mask);
    return brev_n((f - 1u) >> 1, logN);
}

// ------------------------------------------------------------------ NTT
// Forward negacyclic transform (Cooley-Tukey, psi folded into the twiddles,
// bit-reversed output).  Stage s (0-based) pairs positions j and j + N/2^(s+1)
// inside block i = j / (N/2^s) with twiddle psi^brev(2^s + i); the inverse
// runs the Gentleman-Sande butterflies in reverse with psi^-brev(...) and a
// final N^-1.  Pass A ("columns") runs stages 0..L1-1 on the 2^L1 residues
// sharing j mod 2^L2; pass B ("rows") runs stages L1..logN-1 on contiguous
// runs of 2^L2 residues.
//
// Inside a pass each sub-transform of S = 2^SL residues is held by S/8
// threads with 8 residues each.  Stages are grouped in rounds of three
// (radix-8 in registers); the first round takes SL mod 3 stages (or three),
// so every later round is a full radix-8.  Rounds exchange residues through
// LDS.  Residues stay lazily reduced (Harvey): forward values in [0, 4q),
// inverse values in [0, 2q); the pass that ends the transform reduces fully.

constexpr int kNttThreads = 512;
constexpr int kNttPerThread = 8;
constexpr int kNttBlockLog = 12;
constexpr int kNttBlockElems = kNttThreads * kNttPerThread;   // 4096 residues, 32 KiB (+2 KiB padding) of LDS
static_assert(kNttBlockElems == 1 << kNttBlockLog, "block size");

__device__ __forceinline__ void bfly_fwd(uint64_t& x, uint64_t& y, uint64_t w, uint64_t wp, uint64_t q, uint64_t q2) {
    uint64_t a = x >= q2 ? x - q2 : x;
    const uint64_t v = y * w - mulhi64(y, wp) * q;   // [0, 2q)
    x = a + v;
    y = a - v + q2;
}

__device__ __forceinline__ void bfly_inv(uint64_t& x, uint64_t& y, uint64_t w, uint64_t wp, uint64_t q, uint64_t q2) {
    uint64_t s = x + y;
    s = s >= q2 ? s - q2 : s;
    const uint64_t d = x - y + q2;
    y = d * w - mulhi64(d, wp) * q;                  // [0, 2q)
    x = s;
}

// One round of NS (<= 3) stages on the 8 registers of a thread.  The thread's
// residues sit at positions j0 + kk*2^ld; round stage s pairs kk and kk + (4>>s)
// and needs 2^s distinct twiddles: index (c0 << (a+s)) + (blk << s) + u,
// u = kk >> (3-s), with blk = j0 >> (ld+3) (c0 = 1 in the column pass,
// 2^L1 + run index in the row pass, a = first local stage of the round).
template <typename T> __device__ __forceinline__ T load_tw(const uint64_t* p);
template <> __device__ __forceinline__ uint64_t load_tw<uint64_t>(const uint64_t* p) { return *p; }
template <> __device__ __forceinline__ double load_tw<double>(const uint64_t* p) { return __longlong_as_double((long long)*p); }

// Exact FP64 arithmetic for primes q < 2^44 (the 40-bit scale primes).
// Residues are integers held in doubles, kept centred and unreduced.  For
// |y| < 2^48 and an integer twiddle w < q with wq = fl(w/q):
//   h = fl(y*w), l = fma(y, w, -h) = y*w - h exactly (integers),
//   t = rint(y*wq) is within 0.5 + 2^-4 of y*w/q,
//   r = fma(-t, q, h) + l = y*w - t*q exactly, so r = y*w (mod q), |r| <= 0.57 q.
struct ModF { double q, qinv; };

__device__ __forceinline__ double fmul_centred(double y, double w, double wq, double q) {
    const double h = y * w;
    const double l = fma(y, w, -h);
    const double t = rint(y * wq);
    return fma(-t, q, h) + l;
}

__device__ __forceinline__ void bfly_fwd(double& x, double& y, double w, double wq, const ModF& m) {
    const double v = fmul_centred(y, w, wq, m.q);   // inputs stay below ~10 q over 16 stages
    const double a = x;
    x = a + v;
    y = a - v;
}

__device__ __forceinline__ void bfly_inv(double& x, double& y, double w, double wq, const ModF& m) {
    const double s = x + y;
    const double d = x - y;
    y = fmul_centred(d, w, wq, m.q);
    x = fma(-rint(s * m.qinv), m.q, s);              // centred reduction of the sum
}

__device__ __forceinline__ void bfly_fwd(uint64_t& x, uint64_t& y, uint64_t w, uint64_t wp, const Modulus& m) {
    bfly_fwd(x, y, w, wp, m.q, 2 * m.q);
}

__device__ __forceinline__ void bfly_inv(uint64_t& x, uint64_t& y, uint64_t w, uint64_t wp, const Modulus& m) {
    bfly_inv(x, y, w, wp, m.q, 2 * m.q);
}

__device__ __forceinline__ double as_f64(uint64_t v) { return __longlong_as_double((long long)v); }
__device__ __forceinline__ uint64_t f64_bits(double v) { return (uint64_t)__double_as_longlong(v); }

// Exact conversions between integers below 2^52 and doubles through the
// bits of 2^52 + x (exponent 52, mantissa x): an add or an or and a xor
// instead of the general conversion sequences.
__device__ __forceinline__ double u52_to_f64(uint64_t x) { return as_f64(x | 0x4330000000000000ull) - 0x1p52; }
__device__ __forceinline__ uint64_t f64_to_u52(double v) { return f64_bits(v + 0x1p52) ^ 0x4330000000000000ull; }

// centred double (integer, |v| < 2^50) -> canonical residue in [0, q):
// t = rint(v/q) is within 0.5 + 2^-2/q of v/q, so r = v - t q (exact) lies
// within q/2 + 1 of zero and one correction makes it canonical.
__device__ __forceinline__ uint64_t f64_canon(double v, const ModF& m) {
    double r = fma(-rint(v * m.qinv), m.q, v);
    r = r < 0.0 ? r + m.q : r;
    return f64_to_u52(r);
}

// Streamed load / store: nontemporal (kNt) or through the caches.
template <bool kNt> __device__ __forceinline__ uint64_t ld_stream(const uint64_t* p) {
    if constexpr (kNt) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool kNt> __device__ __forceinline__ void st_stream(uint64_t v, uint64_t* p) {
    if constexpr (kNt) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <int NS, bool kInverse, typename T, typename M>
__device__ __forceinline__ void ntt_round(T (&x)[8], const uint64_t* W, const uint64_t* Wp, int c0, int a,
                                          int blk, const M& md) {
    if (!kInverse) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int h = 4 >> s;
            const int wb = (c0 << (a + s)) + (blk << s);
            T w[4], wp[4];
#pragma unroll
            for (int u = 0; u < (1 << s); ++u) { w[u] = load_tw<T>(W + wb + u); wp[u] = load_tw<T>(Wp + wb + u); }
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
                if (kk & h) continue;
                const int u = kk >> (3 - s);
                bfly_fwd(x[kk], x[kk + h], w[u], wp[u], md);
            }
        }
    } else {
#pragma unroll
        for (int s = NS - 1; s >= 0; --s) {
            const int h = 4 >> s;
            const int wb = (c0 << (a + s)) + (blk << s);
            T w[4], wp[4];
#pragma unroll
            for (int u = 0; u < (1 << s); ++u) { w[u] = load_tw<T>(W + wb + u); wp[u] = load_tw<T>(Wp + wb + u); }
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
                if (kk & h) continue;
                const int u = kk >> (3 - s);
                bfly_inv(x[kk], x[kk + h], w[u], wp[u], md);
            }
        }
    }
}

// Element access of the two representations.  The integer path keeps
// canonical uint64 residues in memory.  The FP64 path reads canonical
// residues in the first pass of a transform, keeps the centred doubles (as
// raw bits) between its two passes, and writes canonical residues at the end.
template <typename T, typename M> struct NttIo;
template <> struct NttIo<uint64_t, Modulus> {
    static __device__ __forceinline__ uint64_t in(uint64_t v, bool, const Modulus&) { return v; }
    static __device__ __forceinline__ uint64_t out_mid(uint64_t v, const Modulus&) { return v; }
    static __device__ __forceinline__ uint64_t out_fwd_end(uint64_t v, const Modulus& m) {
        const uint64_t q2 = 2 * m.q;
        v = v >= q2 ? v - q2 : v;
        return v >= m.q ? v - m.q : v;
    }
    static __device__ __forceinline__ uint64_t out_inv_end(uint64_t v, const Modulus& m) {
        return mul_shoup(v, m.n_inv, m.n_inv_shoup, m.q);
    }
};
template <> struct NttIo<double, ModF> {
    static __device__ __forceinline__ double in(uint64_t v, bool canonical, const ModF&) {
        return canonical ? u52_to_f64(v) : as_f64(v);
    }
    static __device__ __forceinline__ uint64_t out_mid(double v, const ModF&) { return f64_bits(v); }
    static __device__ __forceinline__ uint64_t out_fwd_end(double v, const ModF& m) { return f64_canon(v, m); }
    static __device__ __forceinline__ uint64_t out_inv_end(double v, const ModF& m, double ninv, double ninvq) {
        return f64_canon(fmul_centred(v, ninv, ninvq, m.q), m);
    }
};

// `in` is read once, at the start of the pass, and `data` written at its end
// (the same tile of the same limb): in == data transforms in place.  The
// transform's input and output are streamed with nontemporal loads and stores
// (each residue is touched once per pass), which leaves the cache to the
// twiddles: 5 % faster passes.  The intermediate between the two passes is
// streamed the same way if kNtMid, else written and read through the caches,
// so that a sub-batch small enough for the last-level cache can hand it from
// one pass to the next without a round trip to HBM.
// Barrier between the LDS exchanges of a pass.  A rows pass's sub-transform
// (2^SL residues, 8 per thread, SL <= 9) is held by 2^(SL-3) consecutive
// lanes of one wave and owns its own LDS range, so its exchanges only need
// that wave's LDS accesses kept in order (a wavefront-scope fence); the
// columns passes interleave their sub-transforms across the block's waves
// and need the block barrier.
template <bool kCols>
__device__ __forceinline__ void pass_sync() {
    if constexpr (kCols) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

template <int SL, bool kCols, bool kInverse, bool kNtMid, typename T, typename M>
__device__ __forceinline__ void ntt_pass_body(uint64_t* lds_raw, uint64_t* twl, const uint64_t* in, uint64_t* data,
                                              const uint64_t* W, const uint64_t* Wp, const M& md, const Modulus& mi,
                                              int L1, int L2, int chunk, int tid) {
    T* lds = reinterpret_cast<T*>(lds_raw);
    if constexpr (kCols) {
        // The columns pass uses twiddle indices below 2^SL only, the same in
        // every block: staged in LDS once per block, its rounds read them
        // there instead of issuing per-lane vector loads (the vector memory
        // path is the transform passes' busiest unit).
        for (int k = tid; k < (1 << SL); k += kNttThreads) {
            twl[k] = W[k];
            twl[(1 << SL) + k] = Wp[k];
        }
        __syncthreads();
        W = twl;
        Wp = twl + (1 << SL);
    }
    constexpr int TPS_L = SL - 3;
    static_assert(kCols || TPS_L <= 6, "a rows sub-transform is held by the lanes of one wave (pass_sync)");
    constexpr int SPB_L = kNttBlockLog - SL;        // log2(sub-transforms per block)
    constexpr int R0 = (SL % 3) ? (SL % 3) : 3;
    constexpr bool kFirstPass = kCols != kInverse;   // forward starts with columns, inverse with rows
    constexpr bool kNtLd = kFirstPass || kNtMid;     // the second pass loads the intermediate
    constexpr bool kNtSt = !kFirstPass || kNtMid;    // the first pass stores it
    int sub, tt;
    if (kCols) { sub = tid & ((1 << SPB_L) - 1); tt = tid >> SPB_L; }
    else       { sub = tid >> TPS_L;              tt = tid & ((1 << TPS_L) - 1); }
    const size_t col0 = kCols ? ((size_t)chunk << SPB_L) + sub : 0;
    const size_t run0 = kCols ? 0 : ((size_t)chunk << kNttBlockLog) + ((size_t)sub << SL);
    auto gaddr = [&](int p) -> size_t { return kCols ? col0 + ((size_t)p << L2) : run0 + p; };
    // LDS word of position p.  The rows passes pad one word after every 16:
    // their exchanges move 8 residues per thread at lane strides of 8 and 64
    // positions, which would otherwise put 4 to 8 lanes of a wave on the same
    // banks.  The columns passes interleave 2^SPB_L sub-transforms and need no
    // padding.
    // A thread's positions are a base j0 plus the bit field kk << ld, disjoint
    // from j0's bits, so the padded word splits into pad(base) + pad(offset):
    // one address register per exchange and an immediate offset per residue.
    auto pad = [](int w) -> int { return kCols ? w : w + (w >> 4); };
    auto lbase = [&](int j) -> int { return pad(kCols ? (j << SPB_L) + sub : (sub << SL) + j); };
    auto loff = [&](int kk, int l) -> int { return pad(kCols ? (kk << l) << SPB_L : kk << l); };
    const int c0 = kCols ? 1 : (1 << L1) + (chunk << SPB_L) + sub;
    typedef NttIo<T, M> Io;

    T x[8];
    int j0, ld;
    if (!kInverse) {
        ld = SL - 3;
        j0 = tt;
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) x[kk] = Io::in(ld_stream<kNtLd>(&in[gaddr(tt + (kk << ld))]), kFirstPass, md);
        ntt_round<R0, false>(x, W, Wp, c0, 0, 0, md);
#pragma unroll
        for (int a = R0; a < SL; a += 3) {
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) lds[lbase(j0) + loff(kk, ld)] = x[kk];
            pass_sync<kCols>();
            ld = SL - a - 3;
            j0 = ((tt >> ld) << (ld + 3)) | (tt & ((1 << ld) - 1));
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) x[kk] = lds[lbase(j0) + loff(kk, ld)];
            pass_sync<kCols>();
            ntt_round<3, false>(x, W, Wp, c0, a, tt >> ld, md);
        }
        if (kCols) {
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) st_stream<kNtSt>(Io::out_mid(x[kk], md), &data[gaddr(j0 + (kk << ld))]);
        } else {
            // the last round leaves each thread 8 adjacent residues; one more
            // exchange lets consecutive lanes store consecutive residues
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) lds[lbase(j0) + loff(kk, ld)] = x[kk];
            pass_sync<kCols>();
#pragma unroll
            for (int kk = 0; kk < 8; ++kk)
                st_stream<kNtSt>(Io::out_fwd_end(lds[lbase(tt) + loff(kk, SL - 3)], md), &data[gaddr(tt + (kk << (SL - 3)))]);
        }
    } else {
        ld = 0;
        j0 = tt << 3;
        if (kCols) {
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) x[kk] = Io::in(ld_stream<kNtLd>(&in[gaddr(j0 + kk)]), kFirstPass, md);
        } else {
            // consecutive lanes load consecutive residues; an exchange hands
            // each thread the 8 adjacent residues of the first round
#pragma unroll
            for (int kk = 0; kk < 8; ++kk)
                lds[lbase(tt) + loff(kk, SL - 3)] = Io::in(ld_stream<kNtLd>(&in[gaddr(tt + (kk << (SL - 3)))]), kFirstPass, md);
            pass_sync<kCols>();
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) x[kk] = lds[lbase(j0) + loff(kk, 0)];
            pass_sync<kCols>();
        }
        ntt_round<3, true>(x, W, Wp, c0, SL - 3, tt, md);
#pragma unroll
        for (int a = SL - 6; a >= R0; a -= 3) {
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) lds[lbase(j0) + loff(kk, ld)] = x[kk];
            pass_sync<kCols>();
            ld = SL - a - 3;
            j0 = ((tt >> ld) << (ld + 3)) | (tt & ((1 << ld) - 1));
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) x[kk] = lds[lbase(j0) + loff(kk, ld)];
            pass_sync<kCols>();
            ntt_round<3, true>(x, W, Wp, c0, a, tt >> ld, md);
        }
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) lds[lbase(j0) + loff(kk, ld)] = x[kk];
        pass_sync<kCols>();
        ld = SL - 3;
        j0 = tt;
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) x[kk] = lds[lbase(j0) + loff(kk, ld)];
        ntt_round<R0, true>(x, W, Wp, c0, 0, 0, md);
        if (kCols) {
            if constexpr (std::is_same<T, double>::value) {
                const double ninv = (double)mi.n_inv, ninvq = ninv / (double)mi.q;
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) st_stream<kNtSt>(Io::out_inv_end(x[kk], md, ninv, ninvq), &data[gaddr(j0 + (kk << ld))]);
            } else {
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) st_stream<kNtSt>(NttIo<uint64_t, Modulus>::out_inv_end((uint64_t)x[kk], mi), &data[gaddr(j0 + (kk << ld))]);
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) st_stream<kNtSt>(Io::out_mid(x[kk], md), &data[gaddr(j0 + (kk << ld))]);
        }
    }
}

template <int SL, bool kCols, bool kInverse, bool kNtMid>
__global__ void __launch_bounds__(kNttThreads) k_ntt_pass(DevTables t, RowMap m, RowMap src) {
    __shared__ uint64_t lds[kNttBlockElems + kNttBlockElems / 16];   // rows passes pad 1 word in 16
    __shared__ uint64_t twl[kCols ? (2 << SL) : 1];                    // columns passes: their twiddles
    constexpr int SPB_L = kNttBlockLog - SL;
    const int logN = t.logN, L1 = t.L1, L2 = logN - L1;
    const size_t N = (size_t)1 << logN;
    const int chunks = kCols ? ((1 << L2) >> SPB_L) : (int)(N >> kNttBlockLog);
    int b, k, chunk, mod;
    block_coords(blockIdx.x, chunks, m.batch, b, k, chunk);
    uint64_t* data = map_row(m, b, k, logN, mod);
    int smod;
    const uint64_t* in = src.n ? map_row(src, b, k, logN, smod) : data;
    const Modulus md = t.mods[mod];
    const uint64_t* W = t.tw + (size_t)mod * 4 * N + (kInverse ? 2 * N : 0);
    const uint64_t* Wp = W + N;
    if (md.q < kFp64PrimeBound) {
        const ModF mf{(double)md.q, 1.0 / (double)md.q};
        ntt_pass_body<SL, kCols, kInverse, kNtMid, double, ModF>(lds, twl, in, data, W, Wp, mf, md, L1, L2, chunk, threadIdx.x);
    } else {
        ntt_pass_body<SL, kCols, kInverse, kNtMid, uint64_t, Modulus>(lds, twl, in, data, W, Wp, md, md, L1, L2, chunk, threadIdx.x);
    }
}

template <int SL, bool kNtMid>
void launch_ntt_pass(const DevTables& t, const RowMap& m, const RowMap& src, bool cols, bool inverse, int blocks,
                     hipStream_t s) {
    if (cols) {
        if (inverse) hipLaunchKernelGGL((k_ntt_pass<SL, true, true, kNtMid>), dim3(blocks), dim3(kNttThreads), 0, s, t, m, src);
        else hipLaunchKernelGGL((k_ntt_pass<SL, true, false, kNtMid>), dim3(blocks), dim3(kNttThreads), 0, s, t, m, src);
    } else {
        if (inverse) hipLaunchKernelGGL((k_ntt_pass<SL, false, true, kNtMid>), dim3(blocks), dim3(kNttThreads), 0, s, t, m, src);
        else hipLaunchKernelGGL((k_ntt_pass<SL, false, false, kNtMid>), dim3(blocks), dim3(kNttThreads), 0, s, t, m, src);
    }
}

template <int SL>
void launch_ntt_pass(const DevTables& t, const RowMap& m, const RowMap& src, bool cols, bool inverse, int blocks,
                     hipStream_t s) {
    if (t.ntt_cached_mid) launch_ntt_pass<SL, false>(t, m, src, cols, inverse, blocks, s);
    else launch_ntt_pass<SL, true>(t, m, src, cols, inverse, blocks, s);
}

void dispatch_ntt_pass(const DevTables& t, const RowMap& m, const RowMap& src, bool cols, bool inverse, int blocks,
                       hipStream_t s) {
    const int SL = cols ? t.L1 : t.logN - t.L1;
    switch (SL) {
        case 6: launch_ntt_pass<6>(t, m, src, cols, inverse, blocks, s); break;
        case 7: launch_ntt_pass<7>(t, m, src, cols, inverse, blocks, s); break;
        case 8: launch_ntt_pass<8>(t, m, src, cols, inverse, blocks, s); break;
        case 9: launch_ntt_pass<9>(t, m, src, cols, inverse, blocks, s); break;
        default: break;   // both passes are validated to 6..9 stages (ntt_split_valid)
    }
}

// ------------------------------------------------------------------ elementwise
#define EW_PROLOGUE(map)                                                              \
    const int logN = t.logN;                                                          \
    const int N = 1 << logN;                                                          \
    const int chunks = N / (kThreads * kEwPerThread);                                 \
    int b, k, chunk;                                                                  \
    block_coords(blockIdx.x, chunks, map.batch, b, k, chunk);                         \
    const int base_i = chunk * kThreads * kEwPerThread + threadIdx.x;

__global__ void __launch_bounds__(kThreads) k_expand_signed(DevTables t, RowMap out, const int64_t* src, int n_src, int64_t sbs) {
    EW_PROLOGUE(out)
    int mod;
    uint64_t* o = map_row(out, b, k, logN, mod);
    const uint64_t q = t.mods[mod].q;
    const int64_t* s = src + (int64_t)b * sbs + (int64_t)(k % n_src) * N;
    for (int u = 0; u < kEwPerThread; ++u) {
        const int i = base_i + u * kThreads;
        o[i] = from_signed(s[i], q);
    }
}

// ModRaise: residues x mod q_0 (coefficient form) read as the centred integer
// in (-q_0/2, q_0/2] and taken modulo the row's prime.
__global__ void __launch_bounds__(kThreads) k_lift_centred(DevTables t, RowMap out, const uint64_t* src, int64_t sbs,
                                                            uint64_t q0) {
    EW_PROLOGUE(out)
    int mod;
    uint64_t* o = map_row(out, b, k, logN, mod);
    const uint64_t q = t.mods[mod].q;
    const uint64_t* s = src + (int64_t)b * sbs;
    const uint64_t half = q0 >> 1;
    for (int u = 0; u < kEwPerThread; ++u) {
        const int i = base_i + u * kThreads;
        const uint64_t x = s[i];
        o[i] = x > half ? from_signed(-(int64_t)(q0 - x), q) : from_signed((int64_t)x, q);
    }
}

__global__ void __launch_bounds__(kThreads) k_ew(DevTables t, int op, RowMap out, RowMap a, RowMap bm) {
    EW_PROLOGUE(out)
    int mod, ma, mb;
    uint64_t* o = map_row(out, b, k, logN, mod);
    const uint64_t* pa = map_row(a, b, k, logN, ma);
    const uint64_t* pb = (op == EW_ADD || op == EW_SUB) ? map_row(bm, b, k, logN, mb) : nullptr;
    const uint64_t q = t.mods[mod].q;
    for (int u = 0; u < kEwPerThread; ++u) {
        const int i = base_i + u * kThreads;
        const uint64_t x = pa[i];
        uint64_t r;
        if (op == EW_ADD) r = add_mod(x, pb[i], q);
        else if (op == EW_SUB) r = sub_mod(x, pb[i], q);
        else if (op == EW_NEG) r = neg_mod(x, q);
        else if (op == EW_F64C && q < kFp64PrimeBound) r = f64_bits(x > q / 2 ? -(double)(q - x) : (double)x);
        else if (op == EW_F64U && q < kFp64PrimeBound) {
            const double v = as_f64(x);
            r = v < 0.0 ? q - (uint64_t)(-v) : (uint64_t)v;
        } else r = x;
        o[i] = r;
    }
}

__global__ void __launch_bounds__(kThreads) k_mul_mont(DevTables t, RowMap out, RowMap a, RowMap bm, int acc) {
    EW_PROLOGUE(out)
    int mod, ma, mb;
    uint64_t* o = map_row(out, b, k, logN, mod);
    const uint64_t* pa = map_row(a, b, k, logN, ma);
    const uint64_t* pb = map_row(bm, b, k, logN, mb);
    const Modulus md = t.mods[mod];
    for (int u = 0; u < kEwPerThread; ++u) {
        const int i = base_i + u * kThreads;
        uint64_t r = mul_mont(pa[i], pb[i], md.q, md.qneg_inv);
        if (acc) r = add_mod(r, o[i], md.q);
        o[i] = r;
    }
}

__global__ void __launch_bounds__(kThreads) k_mul_const(DevTables t, RowMap out, RowMap a, const uint64_t* consts, int both) {
    EW_PROLOGUE(out)
    int mod, ma;
    uint64_t* o = map_row(out, b, k, logN, mod);
    const uint64_t* pa = map_row(a, b, k, logN, ma);
    const uint64_t q = t.mods[mod].q;
    const uint64_t c = consts[2 * k], cp = consts[2 * k + 1];
    for (int u = 0; u < kEwPerThread; ++u) {
        const int i = base_i + u * kThreads;
        o[i] = mul_shoup(pa[i], c, cp, q);
        if (both) o[i + out.poly_stride] = mul_shoup(pa[i + a.poly_stride], c, cp, q);
    }
}

__global__ void __launch_bounds__(kThreads) k_tensor(DevTables t, RowMap d, RowMap a, RowMap bm) {
    EW_PROLOGUE(d)
    int mod, ma, mb;
    uint64_t* pd = map_row(d, b, k, logN, mod);
    const uint64_t* pa = map_row(a, b, k, logN, ma);
    const uint64_t* pb = map_row(bm, b, k, logN, mb);
    const Modulus md = t.mods[mod];
    const uint64_t q = md.q, qi = md.qneg_inv;
    for (int u = 0; u < kEwPerThread; ++u) {
        const int i = base_i + u * kThreads;
        // a -> a * 2^64 (Montgomery form), so mont(aR, b) = a*b
        const uint64_t a0 = mul_shoup(pa[i], md.r_mod, md.r_mod_shoup, q);
        const uint64_t a1 = mul_shoup(pa[i + a.poly_stride], md.r_mod, md.r_mod_shoup, q);
        const uint64_t b0 = pb[i], b1 = pb[i + bm.poly_stride];
        pd[i] = mul_mont(a0, b0, q, qi);
        pd[i + d.poly_stride] = add_mod(mul_mont(a0, b1, q, qi), mul_mont(a1, b0, q, qi), q);
        pd[i + 2 * d.poly_stride] = mul_mont(a1, b1, q, qi);
    }
}

__global__ void __launch_bounds__(kThreads) k_automorphism(DevTables t, uint32_t g, RowMap out, RowMap in, int both) {
    EW_PROLOGUE(out)
    int mod, mi;
    uint64_t* o = map_row(out, b, k, logN, mod);
    const uint64_t* pi = map_row(in, b, k, logN, mi);
    for (int u = 0; u < kEwPerThread; ++u) {
        const int i = base_i + u * kThreads;
        const uint32_t src = galois_perm((uint32_t)i, g, logN);
        o[i] = pi[src];
        if (both) o[i + out.poly_stride] = pi[src + in.poly_stride];
    }
}

// Basis conversion, one coefficient per thread.  y_s = x_s * [Qhat_s^-1]_{q_s}
// (canonical, or centred in (-q_s/2, q_s/2) if kCentered: ModUp), then for
// every target t the sum of y_s * [Qhat_s]_t.
//
// y_s: for a source prime below kFp64PrimeBound one exact FP64 product
// (fmul_centred, |r| <= 0.57 q_s) brought to the centred or canonical
// representative by one rounding step; for the others a Shoup product.  Each
// y_s is kept as balanced 30-bit halves y_s = a_s + b_s 2^30 (|a_s| <= 2^29),
// as doubles.
//
// Targets t < 2^40 (the scale primes) take an exact FP64 form: C = [Qhat_s]_t
// is split into balanced 20-bit halves C = c_s + d_s 2^20 (|c_s| <= 2^19,
// 0 <= d_s <= 2^20), so every partial product is an integer of magnitude at
// most 2^49 and each of the four sums
//   A0 = sum a c,  A1 = sum a d (weight 2^20),  A2 = sum b c (2^30),
//   A3 = sum b d (2^50)
// of at most 16 sources stays within 2^53: exact in doubles, one FMA per
// product and no reduction inside the sum.  The weights are applied by exact
// products modulo t (fmul_wide, each below 3.5 t), the total (below 2^53) is
// reduced by one rounding step and one correction.  Without centring a 60-bit
// y_s has |b_s| <= 2^30, so that form is used for at most 8 sources (ModDown
// converts the special limbs).
//
// Other targets (the 60-bit primes) sum the products |y_s| * (Qhat_s 2^64 mod t)
// exactly in 128 bits and reduce once by Montgomery REDC:
// sum < NS * 2^60 * t <= t * 2^64, so REDC returns sum * 2^-64 mod t in [0, 2t);
// a term with y_s < 0 contributes |y_s| * (t - c) = y_s * c (mod t), every
// term below 2^59 * t.
//
// The constants are the same for every thread and are read with scalar
// loads: 4 words per source and one record of 2 NS + 8 words per target
// (layouts in kernels.h), which also tell the two kinds of prime apart.

// y * w mod q for an integer-valued double |y| <= 2^53 and an integer
// 0 <= w < q < 2^44 with wq within two roundings of w/q: h = fl(y w) and
// l = y w - h (exact, FMA), t = rint(fl(y wq)) is within 3.5 of y w / q (at
// most three roundings of relative size 2^-53 on a quotient below 2^53), so
// h - t q = y w - t q - l is an integer below 2^45 in magnitude and the FMA
// forms it exactly; the result y w - t q is exact, with |r| <= 3.5 q.
__device__ __forceinline__ double fmul_wide(double y, double w, double wq, double q) {
    const double h = y * w;
    const double l = fma(y, w, -h);
    const double t = rint(y * wq);
    return fma(-t, q, h) + l;
}

template <int NS, bool kCentered>
__global__ void __launch_bounds__(kThreads) k_basis_convert(DevTables t, RowMap dst, RowMap src,
                                                            const uint64_t* __restrict__ yc,
                                                            const uint64_t* __restrict__ rec) {
    const int logN = t.logN;
    const int N = 1 << logN;
    const int chunks = N / kThreads;
    const int chunk = blockIdx.x % chunks;
    const int b = blockIdx.x / chunks;
    const int i = chunk * kThreads + threadIdx.x;
    const int nt = dst.n;
    constexpr bool kFp64Sum = kCentered ? NS <= 16 : NS <= 8;
    constexpr int R = kBcRecordWords(NS);
    // all source loads first (the memory clobber keeps them above it): the
    // compiler would otherwise sink each load into its source's branch below
    // and wait for it there, one source after the other
    uint64_t xs[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        int mod;
        xs[s] = __builtin_nontemporal_load(&map_row(src, b, s, logN, mod)[i]);
    }
    asm volatile("" ::: "memory");
    double ya[NS], yb[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const uint64_t x = xs[s];
        const uint64_t* c = yc + 4 * s;
        const double qinv = as_f64(c[3]);
        if (qinv != 0.0) {   // FP64 source: w, fl(w/q), q, 1/q
            const double q = as_f64(c[2]);
            double v = fmul_centred(u52_to_f64(x), as_f64(c[0]), as_f64(c[1]), q);
            if (kCentered) v = fma(-rint(v * qinv), q, v);
            else v = v < 0.0 ? v + q : v;
            yb[s] = rint(v * 0x1p-30);
            ya[s] = fma(-yb[s], 0x1p30, v);
        } else {             // integer source: w, shoup(w), q, 0
            const uint64_t qs = c[2];
            const uint64_t v = mul_shoup(x, c[0], c[1], qs);
            const int64_t y = (kCentered && 2 * v > qs) ? (int64_t)v - (int64_t)qs : (int64_t)v;
            const int64_t lo = (int64_t)(((uint64_t)y + (1u << 29)) & ((1u << 30) - 1)) - (1 << 29);
            ya[s] = (double)(int32_t)lo;
            yb[s] = (double)(int32_t)((y - lo) >> 30);
        }
    }
    // the targets below 2^40 (record word 2 NS holds t as a double, nonzero)
    for (int tt = 0; kFp64Sum && tt < nt; ++tt) {
        const double* r = reinterpret_cast<const double*>(rec + (size_t)tt * R);
        const double* f = r + 2 * NS;   // t, 1/t, then (2^20, 2^30, 2^50 mod t) with their quotients by t
        if (f[0] == 0.0) continue;
        int mod;
        uint64_t* o = map_row(dst, b, tt, logN, mod);
        double A0 = 0.0, A1 = 0.0, A2 = 0.0, A3 = 0.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            A0 = fma(ya[s], r[2 * s], A0);
            A1 = fma(ya[s], r[2 * s + 1], A1);
            A2 = fma(yb[s], r[2 * s], A2);
            A3 = fma(yb[s], r[2 * s + 1], A3);
        }
        const double q = f[0];
        const double v = A0 + fmul_wide(A1, f[2], f[3], q) + fmul_wide(A2, f[4], f[5], q) + fmul_wide(A3, f[6], f[7], q);
        double res = fma(-rint(v * f[1]), q, v);
        res = res < 0.0 ? res + q : res;
        __builtin_nontemporal_store(f64_to_u52(res), &o[i]);
    }
    // then the 60-bit targets, from |y_s| and the signs; y_s is formed again
    // from its halves (an empty asm keeps the compiler from holding y_s
    // itself through the loop above)
    uint64_t ym[NS];
    uint32_t neg = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        double ha = ya[s], hb = yb[s];
        asm volatile("" : "+v"(ha), "+v"(hb));
        const int64_t y = (int64_t)(int32_t)ha + (int64_t)(int32_t)hb * (1ll << 30);
        neg |= (y < 0 ? 1u : 0u) << s;
        ym[s] = (uint64_t)(y < 0 ? -y : y);
    }
    for (int tt = 0; tt < nt; ++tt) {
        const uint64_t* r = rec + (size_t)tt * R;   // C_s (Montgomery form) per source, then 0 at 2 NS, t, -t^-1 mod 2^64
        if (kFp64Sum && r[2 * NS] != 0) continue;
        int mod;
        uint64_t* o = map_row(dst, b, tt, logN, mod);
        const uint64_t q = r[2 * NS + 1], qneg_inv = r[2 * NS + 2];
        // t - C_s formed from a vector copy of t: a select between two scalar
        // constants per source kept them all in vector registers at once
        uint64_t qv = q;
        asm volatile("" : "+v"(qv));
        uint64_t lo = 0, hi = 0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const uint64_t c0 = r[s];
            const uint64_t c = (((neg >> s) & 1u) && c0) ? qv - c0 : c0;
            const uint64_t pl = ym[s] * c;
            const uint64_t ph = mulhi64(ym[s], c);
            lo += pl;
            hi += ph + (lo < pl ? 1u : 0u);
        }
        const uint64_t m = lo * qneg_inv;
        const uint64_t res = hi + mulhi64(m, q) + (lo != 0 ? 1u : 0u);
        __builtin_nontemporal_store(res >= q ? res - q : res, &o[i]);
    }
}

// Inner product of the extended digits with a switching key for limb kl at
// element i: (sum_j x_j key_j0, sum_j x_j key_j1), x_j = ext_j (or, for the
// limb's own digit, the input limb itself) at the tau_g source of i.
__device__ __forceinline__ void ks_dot(const KsArgs& a, int b, int kl, int i, uint32_t src, int logN,
                                       const Modulus& md, uint64_t& acc0, uint64_t& acc1) {
    const int64_t krow = (int64_t)(kl < a.n_q ? kl : kl + a.key_shift) << logN;
    const uint64_t* pe0 = a.ext + (int64_t)b * a.ext_batch_stride + ((int64_t)kl << logN);
    // a Q limb's own digit is the input polynomial's limb itself
    const int jown = kl < a.n_q ? a.digit_of[kl] : -1;
    int omod;
    const uint64_t* pown = kl < a.n_q ? map_row(a.own, b, kl, logN, omod) : nullptr;
    acc0 = acc1 = 0;
    for (int j = 0; j < a.n_digits; ++j) {
        // the digits are streamed (nontemporal); the key limbs, shared by the
        // batch, stay cached
        const uint64_t x = j == jown ? __builtin_nontemporal_load(&pown[src])
                                     : __builtin_nontemporal_load(&pe0[(int64_t)j * a.ext_digit_stride + src]);
        const uint64_t* pk = a.key + (int64_t)j * a.key_digit_stride + krow;
        acc0 = add_mod(acc0, mul_mont(x, pk[i], md.q, md.qneg_inv), md.q);
        acc1 = add_mod(acc1, mul_mont(x, pk[i + a.key_poly_stride], md.q, md.qneg_inv), md.q);
    }
}

// The same inner product for a limb whose prime is below 2^44: the key rows
// of such a limb hold centred doubles (switching keys are stored that way),
// every product is exact (fmul_centred, |x| < q < 2^44), and the sums of at
// most 16 terms (each below 0.6 q in magnitude) stay centred doubles.
__device__ __forceinline__ void ks_dot_f64(const KsArgs& a, int b, int kl, int i, uint32_t src, int logN,
                                           const ModF& mf, double& acc0, double& acc1) {
    const int64_t krow = (int64_t)kl << logN;
    const uint64_t* pe0 = a.ext + (int64_t)b * a.ext_batch_stride + ((int64_t)kl << logN);
    const int jown = a.digit_of[kl];
    int omod;
    const uint64_t* pown = map_row(a.own, b, kl, logN, omod);
    acc0 = acc1 = 0.0;
    for (int j = 0; j < a.n_digits; ++j) {
        const double x = u52_to_f64(j == jown ? __builtin_nontemporal_load(&pown[src])
                                              : __builtin_nontemporal_load(&pe0[(int64_t)j * a.ext_digit_stride + src]));
        const uint64_t* pk = a.key + (int64_t)j * a.key_digit_stride + krow;
        const double w0 = as_f64(pk[i]), w1 = as_f64(pk[i + a.key_poly_stride]);
        acc0 += fmul_centred(x, w0, w0 * mf.qinv, mf.q);
        acc1 += fmul_centred(x, w1, w1 * mf.qinv, mf.q);
    }
}

__global__ void __launch_bounds__(kThreads) k_ks_inner(DevTables t, RowMap u, KsArgs a, uint32_t g) {
    EW_PROLOGUE(u)
    int mod;
    uint64_t* pu = map_row(u, b, k, logN, mod);
    const Modulus md = t.mods[mod];
    const int kl = k + a.row0;
    if (kl < a.n_q && md.q < kFp64PrimeBound) {   // a Q limb with FP64 key rows
        const ModF mf{(double)md.q, 1.0 / (double)md.q};
        for (int uu = 0; uu < kEwPerThread; ++uu) {
            const int i = base_i + uu * kThreads;
            const uint32_t src = (g == 1u) ? (uint32_t)i : galois_perm((uint32_t)i, g, logN);
            double acc0, acc1;
            ks_dot_f64(a, b, kl, i, src, logN, mf, acc0, acc1);
            __builtin_nontemporal_store(f64_canon(acc0, mf), &pu[i]);
            __builtin_nontemporal_store(f64_canon(acc1, mf), &pu[i + u.poly_stride]);
        }
        return;
    }
    for (int uu = 0; uu < kEwPerThread; ++uu) {
        const int i = base_i + uu * kThreads;
        const uint32_t src = (g == 1u) ? (uint32_t)i : galois_perm((uint32_t)i, g, logN);
        uint64_t acc0, acc1;
        ks_dot(a, b, kl, i, src, logN, md, acc0, acc1);
        __builtin_nontemporal_store(acc0, &pu[i]);
        __builtin_nontemporal_store(acc1, &pu[i + u.poly_stride]);
    }
}

__global__ void __launch_bounds__(kThreads) k_ks_combine(DevTables t, RowMap out, KsArgs a, uint32_t g, RowMap conv,
                                                         RowMap add, uint32_t g_add, int add_both,
                                                         const uint64_t* consts, RowMap acc) {
    EW_PROLOGUE(out)
    int mod, m2, m3, m4;
    uint64_t* o = map_row(out, b, k, logN, mod);
    const uint64_t* pc = map_row(conv, b, k, logN, m2);
    const uint64_t* pa = add.n ? map_row(add, b, k, logN, m3) : nullptr;
    const uint64_t* pacc = acc.n ? map_row(acc, b, k, logN, m4) : nullptr;
    const Modulus md = t.mods[mod];
    const uint64_t q = md.q;
    const uint64_t c = consts[2 * k], cp = consts[2 * k + 1];
    if (q < kFp64PrimeBound) {
        // exact FP64 form: (u - conv) P^-1 with centred doubles, one reduction at the end
        const ModF mf{(double)q, 1.0 / (double)q};
        const double cd = (double)c, cq = cd * mf.qinv;
        for (int uu = 0; uu < kEwPerThread; ++uu) {
            const int i = base_i + uu * kThreads;
            const uint32_t src = (g == 1u) ? (uint32_t)i : galois_perm((uint32_t)i, g, logN);
            double u0, u1;
            ks_dot_f64(a, b, k, i, src, logN, mf, u0, u1);
            const uint32_t sa = (g_add == 1u) ? (uint32_t)i : galois_perm((uint32_t)i, g_add, logN);
            double r0 = fmul_centred(u0 - u52_to_f64(__builtin_nontemporal_load(&pc[i])), cd, cq, mf.q);
            double r1 = fmul_centred(u1 - u52_to_f64(__builtin_nontemporal_load(&pc[i + conv.poly_stride])), cd, cq, mf.q);
            if (pa) {
                r0 += u52_to_f64(pa[sa]);
                if (add_both) r1 += u52_to_f64(pa[sa + add.poly_stride]);
            }
            if (pacc) {
                r0 += u52_to_f64(pacc[i]);
                r1 += u52_to_f64(pacc[i + acc.poly_stride]);
            }
            __builtin_nontemporal_store(f64_canon(r0, mf), &o[i]);
            __builtin_nontemporal_store(f64_canon(r1, mf), &o[i + out.poly_stride]);
        }
        return;
    }
    for (int uu = 0; uu < kEwPerThread; ++uu) {
        const int i = base_i + uu * kThreads;
        const uint32_t src = (g == 1u) ? (uint32_t)i : galois_perm((uint32_t)i, g, logN);
        uint64_t u0, u1;
        ks_dot(a, b, k, i, src, logN, md, u0, u1);
        const uint32_t sa = (g_add == 1u) ? (uint32_t)i : galois_perm((uint32_t)i, g_add, logN);
        uint64_t r0 = mul_shoup(sub_mod(u0, __builtin_nontemporal_load(&pc[i]), q), c, cp, q);
        uint64_t r1 = mul_shoup(sub_mod(u1, __builtin_nontemporal_load(&pc[i + conv.poly_stride]), q), c, cp, q);
        if (pa) {
            r0 = add_mod(r0, pa[sa], q);
            if (add_both) r1 = add_mod(r1, pa[sa + add.poly_stride], q);
        }
        if (pacc) {
            r0 = add_mod(r0, pacc[i], q);
            r1 = add_mod(r1, pacc[i + acc.poly_stride], q);
        }
        __builtin_nontemporal_store(r0, &o[i]);
        __builtin_nontemporal_store(r1, &o[i + out.poly_stride]);
    }
}

__global__ void __launch_bounds__(kThreads) k_rescale_spread(DevTables t, RowMap dst, RowMap top, uint32_t top_mod) {
    EW_PROLOGUE(dst)
    int mod, mt;
    uint64_t* o = map_row(dst, b, k, logN, mod);
    const uint64_t* pt = map_row(top, b, 0, logN, mt);
    const uint64_t ql = t.mods[top_mod].q;
    const uint64_t h = ql >> 1;
    const uint64_t q = t.mods[mod].q;
    const uint64_t hq = h >= q ? h % q : h;
    for (int uu = 0; uu < kEwPerThread; ++uu) {
        const int i = base_i + uu * kThreads;
        uint64_t t0 = add_mod(pt[i], h, ql);
        uint64_t t1 = add_mod(pt[i + top.poly_stride], h, ql);
        t0 = t0 >= q ? t0 % q : t0;
        t1 = t1 >= q ? t1 % q : t1;
        o[i] = sub_mod(t0, hq, q);                       // (t - h) mod q_i, coefficient form
        o[i + dst.poly_stride] = sub_mod(t1, hq, q);
    }
}

__global__ void __launch_bounds__(kThreads) k_rescale_combine(DevTables t, RowMap out, RowMap c, RowMap T, const uint64_t* consts) {
    EW_PROLOGUE(out)
    int mod, m1, m2;
    uint64_t* o = map_row(out, b, k, logN, mod);
    const uint64_t* pc = map_row(c, b, k, logN, m1);
    const uint64_t* pt = map_row(T, b, k, logN, m2);
    const uint64_t q = t.mods[mod].q;
    const uint64_t w = consts[4 * k + 1], wp = consts[4 * k + 2];
    for (int uu = 0; uu < kEwPerThread; ++uu) {
        const int i = base_i + uu * kThreads;
        o[i] = mul_shoup(sub_mod(pc[i], pt[i], q), w, wp, q);
        o[i + out.poly_stride] = mul_shoup(sub_mod(pc[i + c.poly_stride], pt[i + T.poly_stride], q), w, wp, q);
    }
}

// bytes of `rows` polynomial rows (algorithmic traffic accounting for the profiler)
#define NB(rows) ((double)(rows) * (double)(1 << t.logN) * 8.0)

// Multi-task masked MAC for block permutations: task t accumulates into acc_t
// (both polynomials, limbs 0..n_limbs-1) the groups [grp_begin[t], grp_begin[t+1]) of
//     src_g (.) M_g,   M_g[x] = sum_{m in group} cw[m][k] * I0_k[perm_{g_m}(x)]
// (cw = W_m * 2^64 mod q_k with its Shoup factor, so the product with src is a
// Montgomery multiply; g_m = 0 adds cw[m][k] itself, a constant plaintext);
// group g reads src_ptr[g] (c1 at +poly_stride) and its terms
// [term_begin[g], term_begin[g+1]).  If first[t] != 0 the accumulator starts at 0.


// The MAC's per-task metadata (group and term tables, weights, source
// pointers) is written by the host before the launch and only read here:
// read through the constant address space, uniform loads of it become scalar
// loads, which wait on their own counter instead of behind the vector loads
// of the mask rows and sources.
template <typename T> using ConstPtr = const __attribute__((address_space(4))) T*;
template <typename T> __device__ __forceinline__ ConstPtr<T> as_const(const T* p) { return (ConstPtr<T>)p; }

// FP64 form of the masked MAC for a limb whose prime is below 2^44 (the mask
// row and the weight rows of such a limb hold centred doubles: the mask value,
// and w with fl(w/q)).  Every product is exact (FMA two-product, reduced by
// rint(h/q)), reduced terms stay below q in magnitude, and the double sums are
// re-centred every kF64Batch additions, so they never exceed 2^53.  The
// canonical residues that come out equal those of the integer path.
constexpr int kF64Batch = 256;

__device__ __forceinline__ double f64_centre(double v, double q, double qinv) { return fma(-rint(v * qinv), q, v); }

__device__ __forceinline__ double f64_mulmod(double a, double b, double q, double qinv) {
    const double h = a * b;
    const double l = fma(a, b, -h);
    return fma(-rint(h * qinv), q, h) + l;
}

__device__ __forceinline__ void mask_mac_f64(const MaskTasks& T, int task, int k, int base_i, int g0, int g1,
                                             const uint64_t* row, uint64_t* pa, uint64_t q64, int logN) {
    const double q = (double)q64, qinv = 1.0 / q;
    const ModF mf{q, qinv};
    double a0[kMacPerThread], a1[kMacPerThread];
    if (T.first[task]) {
#pragma unroll
        for (int u = 0; u < kMacPerThread; ++u) a0[u] = a1[u] = 0.0;
    } else {
#pragma unroll
        for (int u = 0; u < kMacPerThread; ++u) {
            a0[u] = u52_to_f64(pa[base_i + u]);
            a1[u] = u52_to_f64(pa[base_i + u + T.poly_stride]);
        }
    }
    int n_acc = 0;
    const ConstPtr<int32_t> term_begin = as_const(T.term_begin), wi = as_const(T.wi);
    const ConstPtr<uint32_t> gs = as_const(T.gs);
    const ConstPtr<uint64_t> cw = as_const(T.cw);
    const ConstPtr<const uint64_t*> srcs = as_const(T.src);
    for (int g = g0; g < g1; ++g) {
        // the group's source rows first: their loads overlap the mask gathers
        const uint64_t* ps = srcs[g] + ((size_t)k << logN);
        double s0[kMacPerThread], s1[kMacPerThread];
#pragma unroll
        for (int u = 0; u < kMacPerThread; ++u) {
            s0[u] = u52_to_f64(ps[base_i + u]);
            s1[u] = u52_to_f64(ps[base_i + u + T.poly_stride]);
        }
        asm volatile("" ::: "memory");   // issued here, not sunk below the term loop
        double M[kMacPerThread];
#pragma unroll
        for (int u = 0; u < kMacPerThread; ++u) M[u] = 0.0;
        const int m0 = term_begin[g], m1 = term_begin[g + 1];
        for (int m = m0; m < m1; ++m) {
            const ConstPtr<uint64_t> c = cw + 2 * ((size_t)wi[m] * T.cw_stride + k);
            const double w = as_f64(c[0]), wq = as_f64(c[1]);
            const uint32_t gm = gs[m];
            // Galois element 0 marks a constant term (the plaintext W, no mask)
            if (gm) {
#pragma unroll
                for (int u = 0; u < kMacPerThread; ++u)
                    M[u] += fmul_centred(as_f64(row[galois_perm((uint32_t)(base_i + u), gm, logN)]), w, wq, q);
            } else {
#pragma unroll
                for (int u = 0; u < kMacPerThread; ++u) M[u] += w;
            }
            if ((m - m0) % kF64Batch == kF64Batch - 1) {
#pragma unroll
                for (int u = 0; u < kMacPerThread; ++u) M[u] = f64_centre(M[u], q, qinv);
            }
        }
#pragma unroll
        for (int u = 0; u < kMacPerThread; ++u) {
            const double Mc = f64_centre(M[u], q, qinv);
            a0[u] += f64_mulmod(s0[u], Mc, q, qinv);
            a1[u] += f64_mulmod(s1[u], Mc, q, qinv);
        }
        if (++n_acc == kF64Batch) {
            n_acc = 0;
#pragma unroll
            for (int u = 0; u < kMacPerThread; ++u) {
                a0[u] = f64_centre(a0[u], q, qinv);
                a1[u] = f64_centre(a1[u], q, qinv);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < kMacPerThread; ++u) {
        pa[base_i + u] = f64_canon(a0[u], mf);
        pa[base_i + u + T.poly_stride] = f64_canon(a1[u], mf);
    }
}

// Grid order (XCD-aware): work-groups are dispatched to the 8 XCDs round
// robin, so block b runs on XCD b % 8.  A tile (limb k, chunk of elements)
// is given to one XCD and all tasks of that tile run there back to back:
//   xcd = b % 8,  task = (b / 8) % n_tasks,  tile = ((b / 8) / n_tasks) * 8 + xcd,
// so the tile of every source (babies read by many tasks) stays in that XCD's
// L2 while its tasks run, instead of being fetched once per task.
__global__ void __launch_bounds__(kThreads) k_mask_mac_tasks(DevTables t, MaskTasks T, const uint64_t* i0) {
    const int logN = t.logN;
    const int N = 1 << logN;
    const int chunks = N / (kThreads * kMacPerThread);
    const int xcd = blockIdx.x & (kXcds - 1);
    const int j = blockIdx.x / kXcds;
    const int task = j % T.n_tasks;
    const int tile = (j / T.n_tasks) * kXcds + xcd;
    if (tile >= T.n_limbs * chunks) return;
    const int k = tile / chunks;             // limb
    const int chunk = tile % chunks;
    // each thread owns kMacPerThread adjacent elements (one 16-byte load per
    // source row and accumulator row; 17 % faster than a stride of kThreads),
    // so a group's and a term's metadata is loaded once for all of them
    const int base_i = (chunk * kThreads + threadIdx.x) * kMacPerThread;
    const Modulus md = t.mods[k];
    const uint64_t* row = i0 + ((size_t)k << logN);
    uint64_t* pa = T.acc[task] + ((size_t)k << logN);
    const int g0 = T.grp_begin[task], g1 = T.grp_begin[task + 1];
    if (md.q < kFp64PrimeBound) {
        mask_mac_f64(T, task, k, base_i, g0, g1, row, pa, md.q, logN);
        return;
    }
    uint64_t a0[kMacPerThread], a1[kMacPerThread];
    if (T.first[task]) {
#pragma unroll
        for (int u = 0; u < kMacPerThread; ++u) a0[u] = a1[u] = 0;
    } else {
#pragma unroll
        for (int u = 0; u < kMacPerThread; ++u) {
            a0[u] = pa[base_i + u];
            a1[u] = pa[base_i + u + T.poly_stride];
        }
    }
    const ConstPtr<int32_t> term_begin = as_const(T.term_begin), wi = as_const(T.wi);
    const ConstPtr<uint32_t> gs = as_const(T.gs);
    const ConstPtr<uint64_t> cw = as_const(T.cw);
    const ConstPtr<const uint64_t*> srcs = as_const(T.src);
    for (int g = g0; g < g1; ++g) {
        const uint64_t* ps = srcs[g] + ((size_t)k << logN);
        uint64_t s0[kMacPerThread], s1[kMacPerThread];
#pragma unroll
        for (int u = 0; u < kMacPerThread; ++u) {
            s0[u] = ps[base_i + u];
            s1[u] = ps[base_i + u + T.poly_stride];
        }
        asm volatile("" ::: "memory");
        uint64_t M[kMacPerThread];
#pragma unroll
        for (int u = 0; u < kMacPerThread; ++u) M[u] = 0;
        const int m1 = term_begin[g + 1];
        for (int m = term_begin[g]; m < m1; ++m) {
            const ConstPtr<uint64_t> c = cw + 2 * ((size_t)wi[m] * T.cw_stride + k);
            const uint64_t w = c[0], ws = c[1];
            const uint32_t gm = gs[m];
            // Galois element 0 marks a constant term (the plaintext W, no mask)
            if (gm) {
#pragma unroll
                for (int u = 0; u < kMacPerThread; ++u)
                    M[u] = add_mod(M[u], mul_shoup(row[galois_perm((uint32_t)(base_i + u), gm, logN)], w, ws,
                                                   md.q), md.q);
            } else {
#pragma unroll
                for (int u = 0; u < kMacPerThread; ++u) M[u] = add_mod(M[u], w, md.q);
            }
        }
#pragma unroll
        for (int u = 0; u < kMacPerThread; ++u) {
            a0[u] = add_mod(a0[u], mul_mont(s0[u], M[u], md.q, md.qneg_inv), md.q);
            a1[u] = add_mod(a1[u], mul_mont(s1[u], M[u], md.q, md.qneg_inv), md.q);
        }
    }
#pragma unroll
    for (int u = 0; u < kMacPerThread; ++u) {
        pa[base_i + u] = a0[u];
        pa[base_i + u + T.poly_stride] = a1[u];
    }
}

inline int ew_blocks(const DevTables& t, const RowMap& m) {
    return m.rows() * ((1 << t.logN) / (kThreads * kEwPerThread));
}

}  // namespace

// ------------------------------------------------------------------ launchers
// t.ntt_chunk_rows: rows per pair of passes (0: the whole batch at once).
// With a chunk, both passes of a sub-batch run back to back so the second
// pass can find the first pass's output in the last-level cache.  Chosen per
// context by the autotuner.

void launch_ntt(const DevTables& t, const RowMap& m, bool inverse, hipStream_t s) {
    launch_ntt_from(t, m, RowMap(), inverse, s);
}

void launch_ntt_from(const DevTables& t, const RowMap& m, const RowMap& src, bool inverse, hipStream_t s) {
    if (m.rows() == 0) return;
    if (src.n && (src.n != m.n || src.batch != m.batch)) throw std::length_error("transform source map differs in shape");
    const int per_b = m.n;
    int bchunk = m.batch;
    const int cr = t.ntt_chunk_rows;
    if (cr > 0) bchunk = per_b >= cr ? 1 : cr / per_b;
    if (bchunk > m.batch) bchunk = m.batch;
    const RowMap none{};
    for (int b0 = 0; b0 < m.batch; b0 += bchunk) {
        RowMap sub = m, ssub = src;
        sub.batch = ssub.batch = (m.batch - b0) < bchunk ? (m.batch - b0) : bchunk;
        if (m.ptrs) sub.ptrs = m.ptrs + b0;
        else sub.base = m.base + (int64_t)b0 * m.batch_stride;
        if (src.ptrs) ssub.ptrs = src.ptrs + b0;
        else if (src.n) ssub.base = src.base + (int64_t)b0 * src.batch_stride;
        const int blocks = sub.rows() * (int)(((size_t)1 << t.logN) / kNttBlockElems);
        // algorithmic bytes: a transform reads and writes each row once, half
        // of that is charged to each of its two passes
        const double bytes = NB(sub.rows());
        if (!inverse) {
            { ProfScope ps_("k_ntt_pass<cols,fwd>", s, bytes); dispatch_ntt_pass(t, sub, ssub, true, false, blocks, s); }
            { ProfScope ps_("k_ntt_pass<rows,fwd>", s, bytes); dispatch_ntt_pass(t, sub, none, false, false, blocks, s); }
        } else {
            { ProfScope ps_("k_ntt_pass<rows,inv>", s, bytes); dispatch_ntt_pass(t, sub, ssub, false, true, blocks, s); }
            { ProfScope ps_("k_ntt_pass<cols,inv>", s, bytes); dispatch_ntt_pass(t, sub, none, true, true, blocks, s); }
        }
    }
}

void launch_expand_signed(const DevTables& t, const RowMap& out, const int64_t* src, int n_src, int64_t sbs,
                          hipStream_t s) {
    if (!out.rows()) return;
    { ProfScope ps_("k_expand_signed", s, NB(out.rows()) * 2); hipLaunchKernelGGL(k_expand_signed, dim3(ew_blocks(t, out)), dim3(kThreads), 0, s, t, out, src, n_src, sbs); }
}

void launch_lift_centred(const DevTables& t, const RowMap& out, const uint64_t* src, int64_t sbs, uint64_t q0,
                         hipStream_t s) {
    if (!out.rows()) return;
    { ProfScope ps_("k_lift_centred", s, NB(out.rows()) * 2); hipLaunchKernelGGL(k_lift_centred, dim3(ew_blocks(t, out)), dim3(kThreads), 0, s, t, out, src, sbs, q0); }
}

void launch_ew(const DevTables& t, EwOp op, const RowMap& out, const RowMap& a, const RowMap& b, hipStream_t s) {
    if (!out.rows()) return;
    { ProfScope ps_("k_ew", s, NB(out.rows()) * 3); hipLaunchKernelGGL(k_ew, dim3(ew_blocks(t, out)), dim3(kThreads), 0, s, t, (int)op, out, a, b); }
}

void launch_mul_mont(const DevTables& t, const RowMap& out, const RowMap& a, const RowMap& b, bool acc, hipStream_t s) {
    if (!out.rows()) return;
    { ProfScope ps_("k_mul_mont", s, NB(out.rows()) * 3); hipLaunchKernelGGL(k_mul_mont, dim3(ew_blocks(t, out)), dim3(kThreads), 0, s, t, out, a, b, acc ? 1 : 0); }
}

void launch_mul_const(const DevTables& t, const RowMap& out, const RowMap& a, const uint64_t* consts, bool both, hipStream_t s) {
    if (!out.rows()) return;
    { ProfScope ps_("k_mul_const", s, NB(out.rows()) * (both ? 4 : 2)); hipLaunchKernelGGL(k_mul_const, dim3(ew_blocks(t, out)), dim3(kThreads), 0, s, t, out, a, consts, both ? 1 : 0); }
}

void launch_tensor(const DevTables& t, const RowMap& d, const RowMap& a, const RowMap& b, hipStream_t s) {
    if (!d.rows()) return;
    { ProfScope ps_("k_tensor", s, NB(d.rows()) * 7); hipLaunchKernelGGL(k_tensor, dim3(ew_blocks(t, d)), dim3(kThreads), 0, s, t, d, a, b); }
}

void launch_automorphism(const DevTables& t, uint32_t g, const RowMap& out, const RowMap& in, bool both, hipStream_t s) {
    if (!out.rows()) return;
    { ProfScope ps_("k_automorphism", s, NB(out.rows()) * (both ? 4 : 2)); hipLaunchKernelGGL(k_automorphism, dim3(ew_blocks(t, out)), dim3(kThreads), 0, s, t, g, out, in, both ? 1 : 0); }
}

template <int NS>
static void launch_bc(const DevTables& t, const RowMap& dst, const RowMap& src, const uint64_t* yc,
                      const uint64_t* cc, bool centered, int blocks, hipStream_t s) {
    if (centered) hipLaunchKernelGGL((k_basis_convert<NS, true>), dim3(blocks), dim3(kThreads), 0, s, t, dst, src, yc, cc);
    else hipLaunchKernelGGL((k_basis_convert<NS, false>), dim3(blocks), dim3(kThreads), 0, s, t, dst, src, yc, cc);
}

void launch_basis_convert(const DevTables& t, const RowMap& dst, const RowMap& src, const uint64_t* yc,
                          const uint64_t* cc, bool centered, hipStream_t s) {
    if (!dst.n || !src.n) return;
    const int blocks = dst.batch * ((1 << t.logN) / kThreads);
    ProfScope ps_("k_basis_convert", s, NB(dst.batch) * (src.n + dst.n));
    const bool ce = centered;
    switch (src.n) {
        case 1: launch_bc<1>(t, dst, src, yc, cc, ce, blocks, s); break;
        case 2: launch_bc<2>(t, dst, src, yc, cc, ce, blocks, s); break;
        case 3: launch_bc<3>(t, dst, src, yc, cc, ce, blocks, s); break;
        case 4: launch_bc<4>(t, dst, src, yc, cc, ce, blocks, s); break;
        case 5: launch_bc<5>(t, dst, src, yc, cc, ce, blocks, s); break;
        case 6: launch_bc<6>(t, dst, src, yc, cc, ce, blocks, s); break;
        case 7: launch_bc<7>(t, dst, src, yc, cc, ce, blocks, s); break;
        case 8: launch_bc<8>(t, dst, src, yc, cc, ce, blocks, s); break;
        case 9: launch_bc<9>(t, dst, src, yc, cc, ce, blocks, s); break;
        case 10: launch_bc<10>(t, dst, src, yc, cc, ce, blocks, s); break;
        case 11: launch_bc<11>(t, dst, src, yc, cc, ce, blocks, s); break;
        case 12: launch_bc<12>(t, dst, src, yc, cc, ce, blocks, s); break;
        case 13: launch_bc<13>(t, dst, src, yc, cc, ce, blocks, s); break;
        case 14: launch_bc<14>(t, dst, src, yc, cc, ce, blocks, s); break;
        case 15: launch_bc<15>(t, dst, src, yc, cc, ce, blocks, s); break;
        case 16: launch_bc<16>(t, dst, src, yc, cc, ce, blocks, s); break;
        default: break;   // digit sizes are validated at context creation
    }
}

void launch_ks_inner(const DevTables& t, const RowMap& u, const KsArgs& a, uint32_t g, hipStream_t s) {
    if (!u.rows()) return;
    { ProfScope ps_("k_ks_inner", s, NB(u.rows()) * (a.n_digits + 2) + NB(u.n) * 2 * a.n_digits); hipLaunchKernelGGL(k_ks_inner, dim3(ew_blocks(t, u)), dim3(kThreads), 0, s, t, u, a, g); }
}

void launch_ks_combine(const DevTables& t, const RowMap& out, const KsArgs& a, uint32_t g, const RowMap& conv,
                       const RowMap& addend, uint32_t g_add, bool addend_both, const uint64_t* consts,
                       const RowMap& acc, hipStream_t s) {
    if (!out.rows()) return;
    if (a.row0 != 0) throw std::length_error("fused key-switch tail covers the Q limbs from limb 0");
    if (acc.n && (acc.n != out.n || acc.batch != out.batch)) throw std::length_error("accumulator map differs in shape");
    const double bytes = NB(out.rows()) * (a.n_digits + 4 + (addend.n ? (addend_both ? 2 : 1) : 0) + (acc.n ? 2 : 0)) +
                         NB(out.n) * 2 * a.n_digits;
    { ProfScope ps_("k_ks_combine", s, bytes); hipLaunchKernelGGL(k_ks_combine, dim3(ew_blocks(t, out)), dim3(kThreads), 0, s, t, out, a, g, conv,
                       addend, g_add, addend_both ? 1 : 0, consts, acc); }
}

void launch_mask_mac_tasks(const DevTables& t, const MaskTasks& T, const uint64_t* i0, double bytes, hipStream_t s) {
    if (T.n_tasks <= 0) return;
    ProfScope ps_("k_mask_mac_tasks", s, bytes);
    const int tiles = T.n_limbs * ((1 << t.logN) / (kThreads * kMacPerThread));
    const int blocks = kXcds * T.n_tasks * ((tiles + kXcds - 1) / kXcds);
    hipLaunchKernelGGL(k_mask_mac_tasks, dim3(blocks), dim3(kThreads), 0, s, t, T, i0);
}

void launch_rescale_spread(const DevTables& t, const RowMap& dst, const RowMap& top, uint32_t top_mod, hipStream_t s) {
    if (!dst.rows()) return;
    { ProfScope ps_("k_rescale_spread", s, NB(dst.rows()) * 3); hipLaunchKernelGGL(k_rescale_spread, dim3(ew_blocks(t, dst)), dim3(kThreads), 0, s, t, dst, top, top_mod); }
}

void launch_rescale_combine(const DevTables& t, const RowMap& out, const RowMap& c, const RowMap& T,
                            const uint64_t* consts, hipStream_t s) {
    if (!out.rows()) return;
    { ProfScope ps_("k_rescale_combine", s, NB(out.rows()) * 6); hipLaunchKernelGGL(k_rescale_combine, dim3(ew_blocks(t, out)), dim3(kThreads), 0, s, t, out, c, T, consts); }
}

}  // namespace csrmf
