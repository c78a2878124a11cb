"""CKKS bootstrapping of a sparsely packed ciphertext (oracle; test infrastructure only).

The paper keeps every ciphertext alive through the epochs of its matrix
factorisation and claims that the computation needs no communication while it
runs (Sec. IV-C); it names no mechanism for renewing the levels an epoch uses.
The library renews them by the masked refresh of the three-party protocol, or
by this bootstrapping, which restores the levels inside the ciphertext.  The
method is the published one for approximate homomorphic encryption
(Cheon, Han, Kim, Kim and Song, "Bootstrapping for approximate homomorphic
encryption", EUROCRYPT 2018), in its sparse-packing form, with the exponential
evaluated by a Taylor series and repeated squaring:

  ModRaise    the level-0 ciphertext's residues mod q_0, read as centred integers,
              are taken modulo every q_i: it then decrypts to t = m + q_0 I over
              the whole chain (I a small integer polynomial);
  SubSum      sum of the rotations by n 2^j: the trace onto Z[Y], Y = X^(N/2n),
              keeps the 2n coefficients t'_i = t_{i N/2n}, times N/2n;
  CoeffToSlot the linear map from the n slots to the 2n real coefficients,
              laid out 2n-periodically as [t'_0..t'_{n-1} | t'_n..t'_{2n-1}], read
              as theta = 2 pi t' / (q_0 2^r): A + conj(A) for one diagonal sum A
              over n rotations (baby-step giant-step), then two rescales;
  EvalMod     exp(i theta) by its Taylor series of degree d, squared r times:
              exp(2 pi i t'/q_0), whose imaginary part sin(2 pi m/q_0) no longer
              sees q_0 I;
  (arcsine)   optionally D - D^3/24 in place of D = 2 i sin: (s + s^3/6) 2 i, the
              first two terms of arcsin, so that a larger message (more of q_0)
              keeps the linearisation error small;
  SlotToCoeff the linear map from those 2n values back to the n slots, with the
              factor q_0 / (2 pi) folded in.

Every non-associative choice is fixed here, and the library follows the same
sequence of operations, so the two give the same ciphertext bit for bit:

* roots:  e(k) = exp(i pi k / 4n) for an integer k reduced mod 8n, evaluated as
  cos and sin of (pi * k) / (4n) in IEEE double;
* encoding of a P-periodic slot vector (P | N/2): only the coefficients
  nu = t N/(2P), t < 2P, are non-zero (the closed form of the canonical
  embedding's inverse for periodic vectors),
      m_{t N/2P} = round_half_even(((sum_u z_u e'(-5^u t)) * Delta) / P),
  with e'(k) = exp(i pi k / 2P), the sum taken in order u = 0..P-1 as
  acc = acc + (Re z_u cos - Im z_u sin), each operation rounded once;
* encoding of a constant c: m_0 = round_half_even(Delta Re c),
  m_{N/2} = round_half_even(Delta Im c), all other coefficients 0;
* scales: IEEE double bookkeeping of ``ckks`` (products and quotients by q_l),
  and every plaintext scale is chosen so that the next rescale lands on a fixed
  target (below).

Precondition: |I| < K, where 2^r >= 2 pi (K + 1/2) / R keeps the series' argument
below R (about 0.8 for the parameters the tests use).  With the dense ternary
secret of ``ckks`` the coefficients of I are about sqrt(N/18) in size.
"""
import math
from dataclasses import dataclass

import numpy as np

from . import ring
from .ckks import Ciphertext, galois_for_step


@dataclass(frozen=True)
class BootConfig:
    n: int           # slots of the sparse packing (power of two, 1 <= n <= N/4)
    r: int           # squarings of the exponential
    d: int           # degree of the Taylor series of exp
    pre_bits: int    # the level-0 input is multiplied by 2^pre_bits before ModRaise
    arcsine: bool = False   # add the cubic term of arcsin after EvalMod (2 more levels)


def levels_used(cfg):
    """Levels one bootstrap consumes: 2 (CoeffToSlot) + ceil(log2 d) + 1 (series)
    + r (squarings) + 2 with the arcsine term + 1 (SlotToCoeff)."""
    return 2 + (cfg.d - 1).bit_length() + 1 + cfg.r + (2 if cfg.arcsine else 0) + 1


def rotation_steps(N, n):
    """Rotation keys a bootstrap needs: n 2^j (SubSum) and 1..2n-1 (the two linear
    maps); conjugation as well."""
    steps = set(range(1, 2 * n)) | {n << j for j in range(_log2(N // (2 * n)))}
    return sorted(s for s in steps if s % (N // 2))


def _log2(x):
    assert x > 0 and x & (x - 1) == 0
    return x.bit_length() - 1


# ------------------------------------------------------------------ encoding
def root(k, P2):
    """exp(i pi k / P2) for an integer k (reduced mod 2 P2) as (cos, sin)."""
    k %= 2 * P2
    ang = (math.pi * float(k)) / float(P2)
    return math.cos(ang), math.sin(ang)


def encode_periodic(N, z, scale):
    """Integer plaintext of the P-periodic complex slot vector z (length P)."""
    P = len(z)
    assert P & (P - 1) == 0 and 1 <= P <= N // 2
    m = np.zeros(N, dtype=np.int64)
    step = N // (2 * P)
    M2 = 4 * P                      # 5^u is reduced mod 4P (exp(i pi k / 2P) has period 4P)
    for t in range(2 * P):
        acc = 0.0
        g = 1
        for u in range(P):
            c, s = root(-(g * t), 2 * P)
            zr, zi = z[u]
            acc = acc + (zr * c - zi * s)
            g = g * 5 % M2
        m[t * step] = int(round((acc * scale) / float(P)))
    return m


def encode_const(N, c, scale):
    """Integer plaintext of the constant complex c = (re, im) in every slot."""
    m = np.zeros(N, dtype=np.int64)
    m[0] = int(round(scale * c[0]))
    m[N // 2] = int(round(scale * c[1]))
    return m


# -------------------------------------------------------------- the matrices
def cts_diagonals(n):
    """Diagonals of CoeffToSlot's two maps (on x and on conj(x)), 2n-periodic.

    With a_{j,c} = e(-2 5^c j)/n the entries of U0^{-1} (U0_{j,i} = e(2 5^j i),
    j, i < n, the embedding restricted to Z[Y]), output slot j < n is
    Re(sum_c a_{j,c} x_c) and slot n + j is Im(sum_c a_{j,c} x_c).  Diagonal
    d < n of the map on x is D1_d[j] = a_{j mod n, (j+d) mod n} / 2 times 1
    (j < n) or -i (j >= n); on conj(x), D2_d[j] = conj(a) / 2 times 1 or i."""
    P2 = 4 * n                      # e(k) = exp(i pi k / 4n)
    inv = 1.0 / (2 * n)
    D1, D2 = [], []
    for d in range(n):
        v1, v2 = [], []
        for j in range(2 * n):
            c = (j + d) % n
            co, si = root(-2 * pow(5, c, 8 * n) * (j % n), P2)
            co, si = co * inv, si * inv
            if j < n:
                v1.append((co, si))
                v2.append((co, -si))
            else:
                v1.append((si, -co))
                v2.append((si, co))
        D1.append(v1)
        D2.append(v2)
    return D1, D2


def stc_diagonals(n):
    """Diagonals d < 2n of SlotToCoeff's map B'_{j,c} = e(2 5^(j mod n) (c mod n))
    times -i (c < n) or 1 (c >= n), 2n-periodic."""
    P2 = 4 * n
    out = []
    for d in range(2 * n):
        v = []
        for j in range(2 * n):
            c = (j + d) % (2 * n)
            co, si = root(2 * pow(5, j % n, 8 * n) * (c % n), P2)
            v.append((si, -co) if c < n else (co, si))
        out.append(v)
    return out


# ---------------------------------------------------------------- the steps
def mod_raise(ctx, ct, scale):
    """Level-0 ciphertext -> level L: centred residues mod q_0 taken mod every q_i."""
    assert ct.level == 0
    q0 = ctx.prm.q[0]
    qm = ctx.qmods(ctx.prm.L)

    def lift(row):
        r = row.astype(np.int64)                      # q_0 < 2^63
        return ring.from_signed(np.where(r > q0 // 2, r - np.int64(q0), r), qm)

    return Ciphertext(lift(ct.c0[0]), lift(ct.c1[0]), float(scale))


def sub_sum(ctx, ct, n):
    """ct <- ct + rot(ct, n 2^j) for j = 0 .. log2(N/2n) - 1."""
    for j in range(_log2(ctx.N // (2 * n))):
        ct = ctx.add(ct, ctx.rotate(ct, n << j))
    return ct


def _rescale_to(ctx, ct, times):
    for _ in range(times):
        ct = ctx.rescale(ct)
    return ct


def bsgs_split(count):
    """Baby steps B = 2^ceil(log2(count) / 2) and giant steps G = ceil(count / B)."""
    B = 1 << (((count - 1).bit_length() + 1) // 2)
    return B, -(-count // B)


def linear_map(ctx, ct, diags, enc_scale, pt_scale):
    """sum_{d < count} diag_d (.) rot(ct, d), no rescale, by baby-step giant-step:
    with d = g B + b, diag_d (.) rot(x, d) = rot(rot(diag_d, -g B) (.) rot(x, b), g B),
    so the B baby rotations share one ModUp (hoisted) and each giant step g > 0
    rotates the sum of its B products once.  The diagonals are P-periodic complex
    vectors; rot(v, -k)_j = v_{(j - k) mod P}."""
    count, P = len(diags), len(diags[0])
    B, G = bsgs_split(count)
    R = ctx.hoisted_rotations(ct, list(range(B)))
    acc = None
    for g in range(G):
        part = None
        for b in range(B):
            d = g * B + b
            if d >= count:
                break
            shifted = [diags[d][(j - g * B) % P] for j in range(P)]
            t = ctx.mul_plain(R[b], encode_periodic(ctx.N, shifted, enc_scale), pt_scale)
            part = t if part is None else ctx.add(part, t)
        if g > 0:
            part = ctx.rotate(part, g * B)
        acc = part if acc is None else ctx.add(acc, part)
    return acc


def coeff_to_slot(ctx, ct, n, target):
    """[theta_lo | theta_hi] in 2n-periodic real slots, scale about `target`,
    two levels lower.  The map on conj(x) has the conjugate diagonals
    (D2_d = conj(D1_d)) and conjugation commutes with rotation, so the whole
    map is A + conj(A) with A = sum_d D1_d rot(x, d): one fan-out of rotations
    and one conjugation, the latter before the two rescales (at A's scale its
    key-switching noise is negligible; after them the squarings of EvalMod
    would amplify it).  The plaintext scale puts the scale after the rescales
    at target: Delta = (target q_l) q_{l-1} / scale."""
    lv = ct.level
    q = ctx.prm.q
    delta = ((target * float(q[lv])) * float(q[lv - 1])) / ct.scale
    D1, _ = cts_diagonals(n)
    acc = linear_map(ctx, ct, D1, delta, delta)
    return _rescale_to(ctx, ctx.add(acc, ctx.conjugate(acc)), 2)


def _power_split(k):
    """x^k = x^a * x^b with a the largest power of two below k (a = b = k/2 for a
    power of two): depth ceil(log2 k)."""
    a = 1 << (k.bit_length() - 1)
    if a == k:
        return k // 2, k // 2
    return a, k - a


def exp_series(ctx, x, d, target):
    """sum_{k<=d} (i x)^k / k! with every term rescaled onto scale `target`."""
    p = {1: x}
    for k in range(2, d + 1):
        a, b = _power_split(k)
        p[k] = ctx.hmult(p[a], p[b])
    q = ctx.prm.q
    acc = None
    for k in range(1, d + 1):
        pk = p[k]
        delta = (target * float(q[pk.level])) / pk.scale
        inv = 1.0 / float(math.factorial(k))
        c = [(inv, 0.0), (0.0, inv), (-inv, 0.0), (0.0, -inv)][k % 4]
        t = ctx.rescale(ctx.mul_plain(pk, encode_const(ctx.N, c, delta), delta))
        if acc is None:
            acc = t
        else:
            lv = min(acc.level, t.level)
            acc = ctx.add(ctx.mod_drop(acc, lv), ctx.mod_drop(t, lv))
    return ctx.add_plain(acc, encode_const(ctx.N, (1.0, 0.0), acc.scale))


def eval_mod(ctx, x, d, r, target):
    """E = exp(i x) (series), E <- E^2 r times, then E - conj(E) = 2 i sin(2^r x)."""
    e = exp_series(ctx, x, d, target)
    for _ in range(r):
        e = ctx.hmult(e, e)
    return ctx.sub(e, ctx.conjugate(e))


def arcsine_term(ctx, D):
    """D - D^3 / 24 for D = 2 i s: 2 i (s + s^3 / 6).  D^2 = D D; the constant
    -1/24 multiplies D with the plaintext scale q_l q_{l-1} / scale(D^2), so that
    D^2 times it lands on D's scale; the sum keeps D's scale."""
    q = ctx.prm.q
    d2 = ctx.hmult(D, D)
    delta = (float(q[D.level]) * float(q[D.level - 1])) / d2.scale
    t = ctx.rescale(ctx.mul_plain(D, encode_const(ctx.N, (-1.0 / 24.0, 0.0), delta), delta))
    d3 = ctx.hmult(d2, t)
    return ctx.add(ctx.mod_drop(D, d3.level), d3)


def slot_to_coeff(ctx, ct, n, gamma, target):
    """Sum over d < 2n of rot(ct, d) times diagonal d of gamma B', one rescale onto
    `target`: the integers carry gamma, the declared plaintext scale does not."""
    q = ctx.prm.q
    delta = (target * float(q[ct.level])) / ct.scale
    dg = delta * gamma
    return ctx.rescale(linear_map(ctx, ct, stc_diagonals(n), dg, delta))


def raise_scale(N, q0, n, r):
    """Declared scale after ModRaise: the trace multiplies by N/2n, so the slots of
    U0^{-1} read theta = 2 pi t'/(q_0 2^r) at scale (N q_0 2^r) / (4 pi n)."""
    return ((float(N) * float(q0)) * float(2 ** r)) / (4.0 * math.pi * float(n))


def bootstrap(ctx, ct, cfg, target=None):
    """Bootstrap ct (any level, its slots n-periodic) onto level L - levels_used."""
    N = ctx.N
    assert cfg.n & (cfg.n - 1) == 0 and 1 <= cfg.n <= N // 4     # 2n-periodic vectors fit N/2 slots
    if levels_used(cfg) > ctx.prm.L:
        raise ValueError("not enough levels for this bootstrap")
    target = ctx.prm.scale if target is None else target
    q0 = ctx.prm.q[0]
    c = ctx.mod_drop(ct, 0)
    c = ctx.mul_int(c, 1 << cfg.pre_bits)
    dm = c.scale
    gamma = float(q0) / (4.0 * math.pi * dm)
    c = mod_raise(ctx, c, raise_scale(N, q0, cfg.n, cfg.r))
    c = sub_sum(ctx, c, cfg.n)
    c = coeff_to_slot(ctx, c, cfg.n, target)
    c = eval_mod(ctx, c, cfg.d, cfg.r, target)
    if cfg.arcsine:
        c = arcsine_term(ctx, c)
    return slot_to_coeff(ctx, c, cfg.n, gamma, target)


def keygen_for(ctx, cfg):
    """Relinearisation, conjugation and the rotation keys of ``rotation_steps``."""
    ctx.keygen(rot_steps=rotation_steps(ctx.N, cfg.n), conj=True)


def rotation_galois(N, n):
    return [galois_for_step(s, N) for s in rotation_steps(N, n)]
