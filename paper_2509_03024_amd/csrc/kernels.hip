// gfx950 kernels for RNS-CKKS: negacyclic NTT/INTT, elementwise modular
// arithmetic, tensor product, automorphism, fast basis conversion, key
// switching inner product, ModDown and rescale.
//
// Layout: every polynomial row is N contiguous uint64 residues (limb-major);
// a launch covers a RowMap of rows.  Blocks are ordered limb-major over the
// batch (consecutive blocks share a modulus and its tables in L2).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace csrmf {

namespace {

constexpr int kThreads = 256;
constexpr int kNttTile = 4096;    // residues staged in LDS per block (32 KiB)
constexpr int kColTile = 16;      // columns per block in the column pass (128-byte runs)
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
// bit-reversed output).  Stage s (0-based) pairs j and j + N/2^(s+1) inside
// block i = j / (N/2^s) with twiddle psi^brev(2^s + i).  Pass A (columns)
// runs stages 0..L1-1 on the 2^L1 residues sharing j mod 2^L2; pass B (rows)
// runs stages L1..logN-1 on contiguous runs of 2^L2 residues.

__global__ void __launch_bounds__(kThreads) k_ntt_cols(DevTables t, RowMap m, int inverse) {
    __shared__ uint64_t lds[kNttTile];
    const int logN = t.logN, L1 = t.L1, L2 = logN - L1;
    const int R = 1 << L1, C = kColTile;
    const int chunks = (1 << L2) / C;
    int b, k, chunk, mod;
    block_coords(blockIdx.x, chunks, m.batch, b, k, chunk);
    uint64_t* data = map_row(m, b, k, logN, mod);
    const Modulus md = t.mods[mod];
    const uint64_t q = md.q;
    const size_t N = (size_t)1 << logN;
    const uint64_t* W = t.tw + (size_t)mod * 4 * N + (inverse ? 2 * N : 0);
    const uint64_t* Wp = W + N;
    const int c0 = chunk * C;
    for (int e = threadIdx.x; e < C * R; e += kThreads) {
        const int r = e / C, c = e % C;
        lds[e] = data[((size_t)r << L2) + c0 + c];
    }
    __syncthreads();
    if (!inverse) {
        for (int s = 0; s < L1; ++s) {
            const int tl = R >> (s + 1);
            const int m0 = 1 << s;
            for (int bf = threadIdx.x; bf < C * R / 2; bf += kThreads) {
                const int c = bf % C, bb = bf / C;
                const int i = bb / tl, jj = bb % tl;
                const int r = 2 * i * tl + jj;
                const uint64_t x = lds[r * C + c];
                const uint64_t v = mul_shoup(lds[(r + tl) * C + c], W[m0 + i], Wp[m0 + i], q);
                lds[r * C + c] = add_mod(x, v, q);
                lds[(r + tl) * C + c] = sub_mod(x, v, q);
            }
            __syncthreads();
        }
        for (int e = threadIdx.x; e < C * R; e += kThreads) {
            const int r = e / C, c = e % C;
            data[((size_t)r << L2) + c0 + c] = lds[e];
        }
    } else {
        for (int s = L1 - 1; s >= 0; --s) {
            const int tl = R >> (s + 1);
            const int m0 = 1 << s;
            for (int bf = threadIdx.x; bf < C * R / 2; bf += kThreads) {
                const int c = bf % C, bb = bf / C;
                const int i = bb / tl, jj = bb % tl;
                const int r = 2 * i * tl + jj;
                const uint64_t x = lds[r * C + c];
                const uint64_t y = lds[(r + tl) * C + c];
                lds[r * C + c] = add_mod(x, y, q);
                lds[(r + tl) * C + c] = mul_shoup(sub_mod(x, y, q), W[m0 + i], Wp[m0 + i], q);
            }
            __syncthreads();
        }
        for (int e = threadIdx.x; e < C * R; e += kThreads) {
            const int r = e / C, c = e % C;
            data[((size_t)r << L2) + c0 + c] = mul_shoup(lds[e], md.n_inv, md.n_inv_shoup, q);
        }
    }
}

__global__ void __launch_bounds__(kThreads) k_ntt_rows(DevTables t, RowMap m, int inverse) {
    __shared__ uint64_t lds[kNttTile];
    const int logN = t.logN, L1 = t.L1, L2 = logN - L1;
    const size_t N = (size_t)1 << logN;
    const int BL = 1 << L2;
    const int TILE = (int)(N < (size_t)kNttTile ? N : (size_t)kNttTile);
    const int chunks = (int)(N / TILE);
    const int bpt = TILE / BL;           // runs per tile
    int b, k, chunk, mod;
    block_coords(blockIdx.x, chunks, m.batch, b, k, chunk);
    uint64_t* data = map_row(m, b, k, logN, mod) + (size_t)chunk * TILE;
    const uint64_t q = t.mods[mod].q;
    const uint64_t* W = t.tw + (size_t)mod * 4 * N + (inverse ? 2 * N : 0);
    const uint64_t* Wp = W + N;
    for (int e = threadIdx.x; e < TILE; e += kThreads) lds[e] = data[e];
    __syncthreads();
    const int half_mask = (BL >> 1) - 1;
    for (int st = 0; st < L2; ++st) {
        const int s2 = inverse ? (L2 - 1 - st) : st;
        const int s = L1 + s2;
        const int m0 = 1 << s;
        const int tt = BL >> (s2 + 1);
        for (int bf = threadIdx.x; bf < TILE / 2; bf += kThreads) {
            const int bl = bf >> (L2 - 1);
            const int kk = bf & half_mask;
            const int ip = kk / tt, jj = kk % tt;
            const int jl = 2 * ip * tt + jj;
            const int gb = chunk * bpt + bl;
            const int i = gb * (BL / (2 * tt)) + ip;
            const int a0 = bl * BL + jl;
            const uint64_t x = lds[a0], y = lds[a0 + tt];
            if (!inverse) {
                const uint64_t v = mul_shoup(y, W[m0 + i], Wp[m0 + i], q);
                lds[a0] = add_mod(x, v, q);
                lds[a0 + tt] = sub_mod(x, v, q);
            } else {
                lds[a0] = add_mod(x, y, q);
                lds[a0 + tt] = mul_shoup(sub_mod(x, y, q), W[m0 + i], Wp[m0 + i], q);
            }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < TILE; e += kThreads) data[e] = lds[e];
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
        else r = x;
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

// Basis conversion: one thread per coefficient, loops over source and target limbs.
__global__ void __launch_bounds__(kThreads) k_basis_convert(DevTables t, RowMap dst, RowMap src, const uint64_t* yc, const uint64_t* cc) {
    const int logN = t.logN;
    const int N = 1 << logN;
    const int chunks = N / kThreads;
    const int chunk = blockIdx.x % chunks;
    const int b = blockIdx.x / chunks;
    const int i = chunk * kThreads + threadIdx.x;
    const int ns = src.n, nt = dst.n;
    uint64_t y[16];
    for (int s = 0; s < ns; ++s) {
        int mod;
        const uint64_t* p = map_row(src, b, s, logN, mod);
        y[s] = mul_shoup(p[i], yc[2 * s], yc[2 * s + 1], t.mods[mod].q);
    }
    for (int tt = 0; tt < nt; ++tt) {
        int mod;
        uint64_t* o = map_row(dst, b, tt, logN, mod);
        const uint64_t q = t.mods[mod].q;
        uint64_t acc = 0;
        for (int s = 0; s < ns; ++s) {
            const uint64_t* c = cc + 2 * (s * nt + tt);
            acc = add_mod(acc, mul_shoup(y[s], c[0], c[1], q), q);
        }
        o[i] = acc;
    }
}

__global__ void __launch_bounds__(kThreads) k_ks_inner(DevTables t, RowMap u, KsArgs a, uint32_t g) {
    EW_PROLOGUE(u)
    int mod;
    uint64_t* pu = map_row(u, b, k, logN, mod);
    const Modulus md = t.mods[mod];
    const int64_t krow = (int64_t)(k < a.n_q ? k : k + a.key_shift) << logN;
    const uint64_t* pe0 = a.ext + (int64_t)b * a.ext_batch_stride + ((int64_t)k << logN);
    for (int uu = 0; uu < kEwPerThread; ++uu) {
        const int i = base_i + uu * kThreads;
        const uint32_t src = (g == 1u) ? (uint32_t)i : galois_perm((uint32_t)i, g, logN);
        uint64_t acc0 = 0, acc1 = 0;
        for (int j = 0; j < a.n_digits; ++j) {
            const uint64_t x = pe0[(int64_t)j * a.ext_digit_stride + src];
            const uint64_t* pk = a.key + (int64_t)j * a.key_digit_stride + krow;
            acc0 = add_mod(acc0, mul_mont(x, pk[i], md.q, md.qneg_inv), md.q);
            acc1 = add_mod(acc1, mul_mont(x, pk[i + a.key_poly_stride], md.q, md.qneg_inv), md.q);
        }
        pu[i] = acc0;
        pu[i + u.poly_stride] = acc1;
    }
}

__global__ void __launch_bounds__(kThreads) k_moddown_combine(DevTables t, RowMap out, RowMap u, RowMap conv, RowMap add, uint32_t g_add, int add_both, const uint64_t* consts) {
    EW_PROLOGUE(out)
    int mod, m1, m2, m3;
    uint64_t* o = map_row(out, b, k, logN, mod);
    const uint64_t* pu = map_row(u, b, k, logN, m1);
    const uint64_t* pc = map_row(conv, b, k, logN, m2);
    const uint64_t* pa = add.n ? map_row(add, b, k, logN, m3) : nullptr;
    const uint64_t q = t.mods[mod].q;
    const uint64_t c = consts[2 * k], cp = consts[2 * k + 1];
    for (int uu = 0; uu < kEwPerThread; ++uu) {
        const int i = base_i + uu * kThreads;
        const uint32_t src = (g_add == 1u) ? (uint32_t)i : galois_perm((uint32_t)i, g_add, logN);
        uint64_t r0 = mul_shoup(sub_mod(pu[i], pc[i], q), c, cp, q);
        uint64_t r1 = mul_shoup(sub_mod(pu[i + u.poly_stride], pc[i + conv.poly_stride], q), c, cp, q);
        if (pa) {
            r0 = add_mod(r0, pa[src], q);
            if (add_both) r1 = add_mod(r1, pa[src + add.poly_stride], q);
        }
        o[i] = r0;
        o[i + out.poly_stride] = r1;
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

inline int ew_blocks(const DevTables& t, const RowMap& m) {
    return m.rows() * ((1 << t.logN) / (kThreads * kEwPerThread));
}

}  // namespace

// ------------------------------------------------------------------ launchers
void launch_ntt(const DevTables& t, const RowMap& m, bool inverse, hipStream_t s) {
    if (m.rows() == 0) return;
    const int L2 = t.logN - t.L1;
    const int col_blocks = m.rows() * ((1 << L2) / kColTile);
    const int tile = (1 << t.logN) < kNttTile ? (1 << t.logN) : kNttTile;
    const int row_blocks = m.rows() * ((1 << t.logN) / tile);
    if (!inverse) {
        hipLaunchKernelGGL(k_ntt_cols, dim3(col_blocks), dim3(kThreads), 0, s, t, m, 0);
        hipLaunchKernelGGL(k_ntt_rows, dim3(row_blocks), dim3(kThreads), 0, s, t, m, 0);
    } else {
        hipLaunchKernelGGL(k_ntt_rows, dim3(row_blocks), dim3(kThreads), 0, s, t, m, 1);
        hipLaunchKernelGGL(k_ntt_cols, dim3(col_blocks), dim3(kThreads), 0, s, t, m, 1);
    }
}

void launch_expand_signed(const DevTables& t, const RowMap& out, const int64_t* src, int n_src, int64_t sbs,
                          hipStream_t s) {
    if (!out.rows()) return;
    hipLaunchKernelGGL(k_expand_signed, dim3(ew_blocks(t, out)), dim3(kThreads), 0, s, t, out, src, n_src, sbs);
}

void launch_ew(const DevTables& t, EwOp op, const RowMap& out, const RowMap& a, const RowMap& b, hipStream_t s) {
    if (!out.rows()) return;
    hipLaunchKernelGGL(k_ew, dim3(ew_blocks(t, out)), dim3(kThreads), 0, s, t, (int)op, out, a, b);
}

void launch_mul_mont(const DevTables& t, const RowMap& out, const RowMap& a, const RowMap& b, bool acc, hipStream_t s) {
    if (!out.rows()) return;
    hipLaunchKernelGGL(k_mul_mont, dim3(ew_blocks(t, out)), dim3(kThreads), 0, s, t, out, a, b, acc ? 1 : 0);
}

void launch_mul_const(const DevTables& t, const RowMap& out, const RowMap& a, const uint64_t* consts, bool both, hipStream_t s) {
    if (!out.rows()) return;
    hipLaunchKernelGGL(k_mul_const, dim3(ew_blocks(t, out)), dim3(kThreads), 0, s, t, out, a, consts, both ? 1 : 0);
}

void launch_tensor(const DevTables& t, const RowMap& d, const RowMap& a, const RowMap& b, hipStream_t s) {
    if (!d.rows()) return;
    hipLaunchKernelGGL(k_tensor, dim3(ew_blocks(t, d)), dim3(kThreads), 0, s, t, d, a, b);
}

void launch_automorphism(const DevTables& t, uint32_t g, const RowMap& out, const RowMap& in, bool both, hipStream_t s) {
    if (!out.rows()) return;
    hipLaunchKernelGGL(k_automorphism, dim3(ew_blocks(t, out)), dim3(kThreads), 0, s, t, g, out, in, both ? 1 : 0);
}

void launch_basis_convert(const DevTables& t, const RowMap& dst, const RowMap& src, const uint64_t* yc,
                          const uint64_t* cc, hipStream_t s) {
    if (!dst.n || !src.n) return;
    const int blocks = dst.batch * ((1 << t.logN) / kThreads);
    hipLaunchKernelGGL(k_basis_convert, dim3(blocks), dim3(kThreads), 0, s, t, dst, src, yc, cc);
}

void launch_ks_inner(const DevTables& t, const RowMap& u, const KsArgs& a, uint32_t g, hipStream_t s) {
    if (!u.rows()) return;
    hipLaunchKernelGGL(k_ks_inner, dim3(ew_blocks(t, u)), dim3(kThreads), 0, s, t, u, a, g);
}

void launch_moddown_combine(const DevTables& t, const RowMap& out, const RowMap& u, const RowMap& conv,
                            const RowMap& addend, uint32_t g_add, bool addend_both, const uint64_t* consts,
                            hipStream_t s) {
    if (!out.rows()) return;
    hipLaunchKernelGGL(k_moddown_combine, dim3(ew_blocks(t, out)), dim3(kThreads), 0, s, t, out, u, conv,
                       addend, g_add, addend_both ? 1 : 0, consts);
}

void launch_rescale_spread(const DevTables& t, const RowMap& dst, const RowMap& top, uint32_t top_mod, hipStream_t s) {
    if (!dst.rows()) return;
    hipLaunchKernelGGL(k_rescale_spread, dim3(ew_blocks(t, dst)), dim3(kThreads), 0, s, t, dst, top, top_mod);
}

void launch_rescale_combine(const DevTables& t, const RowMap& out, const RowMap& c, const RowMap& T,
                            const uint64_t* consts, hipStream_t s) {
    if (!out.rows()) return;
    hipLaunchKernelGGL(k_rescale_combine, dim3(ew_blocks(t, out)), dim3(kThreads), 0, s, t, out, c, T, consts);
}

}  // namespace csrmf
