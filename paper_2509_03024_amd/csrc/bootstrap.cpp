// CKKS bootstrapping of sparsely packed ciphertexts on the device.
//
// The paper's Sec. IV-C claims that its factorisation runs without
// communication, yet names no way to renew the levels each epoch uses.  This
// program renews them inside the ciphertext, by the published method for
// approximate homomorphic encryption (Cheon, Han, Kim, Kim, Song,
// EUROCRYPT 2018) in its sparse-packing form, the exponential evaluated by a
// Taylor series and repeated squaring:
//
//   ModRaise     level 0 -> level L: the ciphertext decrypts to t = m + q_0 I;
//   SubSum       sum of rotations by n 2^j: N/2n times the coefficients
//                t'_i = t_{i N/2n} of the trace onto Z[X^(N/2n)];
//   CoeffToSlot  the 2n real t'_i into 2n-periodic slots, read as
//                theta = 2 pi t' / (q_0 2^r): A + conj(A) for the diagonal sum A
//                over n rotations (baby-step giant-step), then two rescales;
//   EvalMod      exp(i theta) = sum_{k<=d} (i theta)^k / k!, squared r times,
//                minus its conjugate: D = 2 i sin(2 pi m / q_0), free of q_0 I;
//   (arcsine)    optionally D - D^3/24 = 2 i (s + s^3/6), the first two terms of
//                arcsin, so that the message may use more of q_0;
//   SlotToCoeff  back to the n slots with q_0 / (4 pi i) folded in (2n diagonals
//                by baby-step giant-step, one rescale).
//
// Every operation runs in the library's kernels on the whole batch.  The
// sequence of operations, the plaintext encodings and the scale bookkeeping
// are fixed as follows, so that the result is one ciphertext bit for bit:
//   e(k) = exp(i pi k / P2) as cos, sin of (pi * k) / P2, k reduced mod 2 P2;
//   a P-periodic slot vector z encodes to m_{t N/2P} =
//     round_half_even(((sum_{u<P} (Re z_u cos - Im z_u sin)) * Delta) / P),
//     (cos, sin) of e(-(5^u mod 4P) t) with P2 = 2P, summed in order u;
//   a constant c encodes to m_0 = rhe(Delta Re c), m_{N/2} = rhe(Delta Im c);
//   each plaintext scale is set so that the rescale after it lands on
//   2^log2_scale (see the steps below).
#include "bootstrap.h"

#include <algorithm>
#include <cmath>
#include <utility>

#pragma clang fp contract(off)

namespace csrmf {

namespace {

// Ciphertexts of one batch, owned here (their blocks go back to the pool).
class Batch {
public:
    Batch(Context* c, int n) : c_(c), v_(n) {}
    Batch(Batch&& o) noexcept : c_(o.c_), v_(std::move(o.v_)) { o.v_.clear(); }
    Batch& operator=(Batch&& o) noexcept {
        if (this != &o) {
            release();
            c_ = o.c_;
            v_ = std::move(o.v_);
            o.v_.clear();
        }
        return *this;
    }
    Batch(const Batch&) = delete;
    Batch& operator=(const Batch&) = delete;
    ~Batch() { release(); }
    std::vector<Ct*> ptrs() {
        std::vector<Ct*> p;
        for (Ct& x : v_) p.push_back(&x);
        return p;
    }
    Ct& operator[](size_t i) { return v_[i]; }
    int size() const { return (int)v_.size(); }
    int level() const { return v_[0].level; }
    double scale() const { return v_[0].scale; }
    std::vector<Ct> take() {
        std::vector<Ct> out = std::move(v_);
        v_.clear();
        return out;
    }

private:
    void release() {
        for (Ct& x : v_)
            if (x.d) c_->pool.put(x.d);
        v_.clear();
    }
    Context* c_;
    std::vector<Ct> v_;
};

struct Cplx {
    double re, im;
};

void root(int64_t k, int64_t P2, double& c, double& s) {
    const int64_t m = 2 * P2;
    k %= m;
    if (k < 0) k += m;
    const double ang = (M_PI * (double)k) / (double)P2;
    c = std::cos(ang);
    s = std::sin(ang);
}

int64_t pow5_mod(int64_t e, int64_t m) {
    int64_t x = 1 % m;
    for (int64_t i = 0; i < e; ++i) x = x * 5 % m;
    return x;
}

std::vector<int64_t> encode_periodic(uint64_t N, const std::vector<Cplx>& z, double scale) {
    const int64_t P = (int64_t)z.size();
    std::vector<int64_t> m(N, 0);
    const int64_t step = (int64_t)N / (2 * P), M2 = 4 * P;
    for (int64_t t = 0; t < 2 * P; ++t) {
        double acc = 0.0;
        int64_t g = 1;
        for (int64_t u = 0; u < P; ++u) {
            double c, s;
            root(-(g * t), 2 * P, c, s);
            const double t1 = z[u].re * c;
            const double t2 = z[u].im * s;
            const double t3 = t1 - t2;
            acc = acc + t3;
            g = g * 5 % M2;
        }
        m[t * step] = (int64_t)std::nearbyint((acc * scale) / (double)P);
    }
    return m;
}

std::vector<int64_t> encode_const(uint64_t N, Cplx c, double scale) {
    std::vector<int64_t> m(N, 0);
    m[0] = (int64_t)std::nearbyint(scale * c.re);
    m[N / 2] = (int64_t)std::nearbyint(scale * c.im);
    return m;
}

// CoeffToSlot's diagonals d < n (on x), 2n-periodic: with a_{j,c} = e(-2 5^c j)/n
// (P2 = 4n), the entries of the inverse of the embedding restricted to
// Z[X^(N/2n)], D_d[j] = a_{j mod n, (j+d) mod n} / 2 times 1 (j < n) or -i
// (j >= n), so that A + conj(A), A = sum_d D_d rot(x, d), puts
// Re(sum_c a_{j,c} x_c) in slot j < n and Im(sum_c a_{j,c} x_c) in slot n + j.
std::vector<std::vector<Cplx>> cts_diagonals(int n) {
    const double inv = 1.0 / (2.0 * n);
    std::vector<std::vector<Cplx>> D(n, std::vector<Cplx>(2 * n));
    for (int d = 0; d < n; ++d)
        for (int j = 0; j < 2 * n; ++j) {
            const int c = (j + d) % n;
            double co, si;
            root(-2 * pow5_mod(c, 8 * n) * (j % n), 4 * n, co, si);
            co = co * inv;
            si = si * inv;
            D[d][j] = j < n ? Cplx{co, si} : Cplx{si, -co};
        }
    return D;
}

// SlotToCoeff's diagonals d < 2n of B'_{j,c} = e(2 5^(j mod n) (c mod n)) times
// -i (c < n) or 1 (c >= n), 2n-periodic.
std::vector<std::vector<Cplx>> stc_diagonals(int n) {
    std::vector<std::vector<Cplx>> out(2 * n, std::vector<Cplx>(2 * n));
    for (int d = 0; d < 2 * n; ++d)
        for (int j = 0; j < 2 * n; ++j) {
            const int c = (j + d) % (2 * n);
            double co, si;
            root(2 * pow5_mod(j % n, 8 * n) * (c % n), 4 * n, co, si);
            out[d][j] = c < n ? Cplx{si, -co} : Cplx{co, si};
        }
    return out;
}

int log2_exact(uint64_t x) {
    int l = 0;
    while ((1ull << l) < x) ++l;
    return l;
}

// ---------------------------------------------------------------- batch ops
Batch rotate(Context* c, Batch& in, uint32_t g) {
    Batch out(c, in.size());
    std::vector<Ct*> pi = in.ptrs(), po = out.ptrs();
    c->rotate(pi, g, po);
    return out;
}

Batch add(Context* c, Batch& a, Batch& b, bool sub = false) {
    Batch out(c, a.size());
    std::vector<Ct*> pa = a.ptrs(), pb = b.ptrs(), po = out.ptrs();
    c->add_batch(pa, pb, po, sub);
    return out;
}

Batch mul_plain(Context* c, Batch& a, const std::vector<int64_t>& m, double pt_scale) {
    Batch out(c, a.size());
    std::vector<Ct*> pa = a.ptrs(), po = out.ptrs();
    c->mul_plain_batch(pa, m.data(), pt_scale, po);
    return out;
}

void rescale(Context* c, Batch& a) {
    std::vector<Ct*> p = a.ptrs();
    c->rescale(p);
}

Batch hmult(Context* c, Batch& a, Batch& b) {
    Batch out(c, a.size());
    std::vector<Ct*> pa = a.ptrs(), pb = b.ptrs(), po = out.ptrs();
    c->mul_relin(pa, pb, po);
    c->rescale(po);
    return out;
}

// acc (+)= sum_{d < count} diag_d (.) rot(in, d) by baby-step giant-step: with
// d = g B + b, diag_d (.) rot(x, d) = rot(rot(diag_d, -g B) (.) rot(x, b), g B), so
// the B baby rotations share one ModUp (hoisted) and each giant step g > 0
// rotates the sum of its B products once.  Each product is accumulated by the
// multiply kernel itself (modular sums are exact, so the bits are those of
// separate products and additions).
void bsgs_mac(Context* c, Batch& in, const std::vector<std::vector<Cplx>>& diags, double enc_scale, double pt_scale,
              Batch& acc, bool& have) {
    const uint64_t N = c->N;
    const int count = (int)diags.size(), P = (int)diags[0].size();
    const int B = 1 << ((log2_exact((uint64_t)count) + 1) / 2), G = (count + B - 1) / B;
    Context::Hoist h;
    std::vector<Batch> R;
    if (B > 1) {
        std::vector<Ct*> pi = in.ptrs();
        c->hoist_begin(h, pi);
        for (int b = 1; b < B; ++b) {
            R.emplace_back(c, in.size());
            std::vector<Ct*> po = R.back().ptrs();
            c->hoist_rotate(h, c->galois_for_step(b), po);
        }
    }
    std::vector<Cplx> shifted(P);
    for (int g = 0; g < G; ++g) {
        Batch part(c, 0);
        bool hp = false;
        for (int b = 0; b < B && g * B + b < count; ++b) {
            const auto& dg = diags[g * B + b];
            for (int j = 0; j < P; ++j) shifted[j] = dg[((j - g * B) % P + P) % P];
            const std::vector<int64_t> pt = encode_periodic(N, shifted, enc_scale);
            Batch& src = b == 0 ? in : R[b - 1];
            if (!hp) {
                part = mul_plain(c, src, pt, pt_scale);
                hp = true;
            } else {
                std::vector<Ct*> ps = src.ptrs(), pa = part.ptrs();
                c->mul_plain_batch(ps, pt.data(), pt_scale, pa, true);
            }
        }
        if (g > 0) part = rotate(c, part, c->galois_for_step((int64_t)g * B));
        if (!have) {
            acc = std::move(part);
            have = true;
        } else {
            acc = add(c, acc, part);
        }
    }
}

}  // namespace

int boot_levels(const BootCfg& cfg) {
    return 2 + log2_exact((uint64_t)cfg.d) + 1 + cfg.r + (cfg.arcsine ? 2 : 0) + 1;
}

std::vector<int32_t> boot_rotation_steps(uint64_t N, int n) {
    std::vector<int32_t> s;
    const int64_t half = (int64_t)N / 2;
    for (int64_t k = 1; k < 2 * (int64_t)n; ++k)
        if (k % half) s.push_back((int32_t)k);
    for (int j = 0; ((int64_t)n << j) < half; ++j) {
        const int64_t k = (int64_t)n << j;
        if (k >= 2 * (int64_t)n) s.push_back((int32_t)k);
    }
    std::sort(s.begin(), s.end());
    s.erase(std::unique(s.begin(), s.end()), s.end());
    return s;
}

void boot_check(const Context* c, const BootCfg& cfg) {
    const int64_t n = cfg.n;
    if (n < 1 || (n & (n - 1)) || (uint64_t)n > c->N / 4)
        throw Error(CSRMF_E_INVAL, "bootstrap: n_slots must be a power of two in [1, N/4]");
    if (cfg.d < 1 || cfg.d > 18) throw Error(CSRMF_E_INVAL, "bootstrap: degree must be in [1, 18]");
    if (cfg.r < 0 || cfg.r > 40) throw Error(CSRMF_E_INVAL, "bootstrap: squarings must be in [0, 40]");
    if (cfg.pre_bits < 0 || cfg.pre_bits > 30) throw Error(CSRMF_E_INVAL, "bootstrap: pre_bits must be in [0, 30]");
    if (boot_levels(cfg) > c->L)
        throw Error(CSRMF_E_LEVEL, "bootstrap: the chain has " + std::to_string(c->L) + " levels, the bootstrap uses " +
                                       std::to_string(boot_levels(cfg)));
}

void bootstrap(Context* c, const BootCfg& cfg, const std::vector<Ct*>& in, std::vector<Ct>& result) {
    boot_check(c, cfg);
    const int B = (int)in.size();
    if (B == 0) return;
    if (!c->have_keys) throw Error(CSRMF_E_STATE, "keygen first");
    for (Ct* x : in)
        if (x->scale != in[0]->scale) throw Error(CSRMF_E_SCALE, "bootstrap: the batch must share one scale");
    const uint64_t N = c->N;
    const int n = cfg.n;
    const double target = std::ldexp(1.0, c->prm.log2_scale);
    const uint64_t q0 = c->moduli[0];
    const uint32_t g_conj = (uint32_t)(2 * N - 1);
    // keys first, so that a missing one fails before any work is enqueued
    c->key_for(g_conj);
    for (int32_t s : boot_rotation_steps(N, n)) c->key_for(c->galois_for_step(s));

    // level 0, times 2^pre_bits
    Batch x(c, B);
    for (int i = 0; i < B; ++i) {
        Ct v = *in[i];
        v.level = 0;
        c->mul_int(v, (int64_t)1 << cfg.pre_bits, x[i]);
    }
    const double dm = x.scale();
    const double gamma = (double)q0 / (4.0 * M_PI * dm);

    // ModRaise, declared scale (N q_0 2^r) / (4 pi n): the slots of U0^{-1}
    // applied to the trace then read theta
    const double s_raise = (((double)N * (double)q0) * std::ldexp(1.0, cfg.r)) / (4.0 * M_PI * (double)n);
    Batch y(c, B);
    {
        std::vector<Ct*> px = x.ptrs(), py = y.ptrs();
        c->mod_raise(px, s_raise, py);
    }
    x = Batch(c, 0);

    // SubSum
    for (int j = 0; ((uint64_t)n << j) < N / 2; ++j) {
        Batch rt = rotate(c, y, c->galois_for_step((int64_t)n << j));
        y = add(c, y, rt);
    }

    // CoeffToSlot: plaintext scale (target q_l) q_{l-1} / scale, two rescales
    Batch theta(c, 0);
    {
        const int lv = y.level();
        const double delta = ((target * (double)c->moduli[lv]) * (double)c->moduli[lv - 1]) / y.scale();
        // the map on conj(x) has the conjugate diagonals and conjugation
        // commutes with rotation: the map is A + conj(A), A = sum_d D_d rot(x, d)
        bool have = false;
        bsgs_mac(c, y, cts_diagonals(n), delta, delta, theta, have);
        // the conjugation at A's scale, where its key-switching noise is negligible
        Batch tj = rotate(c, theta, g_conj);
        theta = add(c, theta, tj);
        rescale(c, theta);
        rescale(c, theta);
    }
    y = Batch(c, 0);

    // EvalMod: the series, each term rescaled onto the target scale
    Batch e(c, 0);
    {
        std::vector<Batch> p;
        p.emplace_back(c, 0);                   // p[0] unused
        p.push_back(std::move(theta));
        for (int k = 2; k <= cfg.d; ++k) {
            int a = 1;
            while (2 * a <= k) a *= 2;
            const int b = (a == k) ? k / 2 : k - a;
            if (a == k) a = k / 2;
            p.push_back(hmult(c, p[a], p[b]));
        }
        bool have = false;
        double fact = 1.0;
        for (int k = 1; k <= cfg.d; ++k) {
            fact = fact * (double)k;
            Batch& pk = p[k];
            const double delta = (target * (double)c->moduli[pk.level()]) / pk.scale();
            const double inv = 1.0 / fact;
            static const int re_sign[4] = {1, 0, -1, 0}, im_sign[4] = {0, 1, 0, -1};
            const Cplx cf{re_sign[k % 4] * inv, im_sign[k % 4] * inv};
            Batch t = mul_plain(c, pk, encode_const(N, cf, delta), delta);
            rescale(c, t);
            if (!have) {
                e = std::move(t);
                have = true;
            } else {
                e = add(c, e, t);
            }
        }
        Batch e1(c, B);
        const std::vector<int64_t> one = encode_const(N, Cplx{1.0, 0.0}, e.scale());
        for (int i = 0; i < B; ++i) c->add_plain(e[i], one.data(), e1[i]);
        e = std::move(e1);
    }
    for (int s = 0; s < cfg.r; ++s) e = hmult(c, e, e);
    {
        Batch ej = rotate(c, e, g_conj);
        e = add(c, e, ej, true);
    }
    if (cfg.arcsine) {
        // D^2; D times -1/24 at plaintext scale q_l q_{l-1} / scale(D^2), so that
        // the product of the two lands on D's scale; D + that keeps D's scale
        Batch d2 = hmult(c, e, e);
        const double delta = ((double)c->moduli[e.level()] * (double)c->moduli[e.level() - 1]) / d2.scale();
        Batch t = mul_plain(c, e, encode_const(N, Cplx{-1.0 / 24.0, 0.0}, delta), delta);
        rescale(c, t);
        Batch d3 = hmult(c, d2, t);
        e = add(c, e, d3);
    }

    // SlotToCoeff: integers carry gamma, the declared plaintext scale does not
    Batch out(c, 0);
    {
        const double delta = (target * (double)c->moduli[e.level()]) / e.scale();
        const double dg = delta * gamma;
        bool have = false;
        bsgs_mac(c, e, stc_diagonals(n), dg, delta, out, have);
        rescale(c, out);
    }
    result = out.take();
}

}  // namespace csrmf
