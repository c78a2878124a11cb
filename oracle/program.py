"""Encrypted CSR matrix-factorisation epoch (oracle; test infrastructure only).

What it computes: the synchronous gradient epoch of ``oracle.mf`` (Eq. 2-5,
Alg. 1 with the per-entity accumulator of Alg. 2) on CKKS ciphertexts whose
slots hold the CSR ratings (Sec. III-C: non-zero ratings packed in CSR order,
profile vectors of k factors packed together).

Layout (k' = 2^ceil(log2 k), block width B = 2k', D = N/(2B) blocks per
ciphertext):
* rating ciphertexts: rows packed greedily in CSR order; a row that does not
  fit in the current ciphertext starts a new one; a row longer than D is cut
  into chunks of D.  Block t of rating ciphertext c holding rating (i, j)
  carries r_ij (R), u_i (Ug) and v_j (Vg) in slots tB .. tB+k-1; other slots 0.
* factor tables: table ciphertext a holds user (item) a*D + b at block b.

One epoch, Ug and Vg at level l:
 1. P = HMult(Ug, Vg)
 2. windowed block sum: T_0 = P, T_{s+1} = T_s + Rot(T_s, 2^s) for s < log2 B,
    Sdot = Rot(T_{log2 B}, -k'); slot tB+f (f < k) now holds <u_i, v_j>
 3. R_e = Rescale(R * W_R), W_R = rint((S_P * q_L) / S_R), dropped to Sdot's
    level; E = R_e - Sdot
 4. G_U = HMult(E, Vg), G_V = HMult(E, Ug)
 5. scatter: table <- BlockPermute(G -> table layout, learning-rate weights)
    plus the self term (1 - a_t*lambda*d) * table, one rescale
 6. gather (not after the last epoch): Ug, Vg <- BlockPermute(tables ->
    rating layout, weight 1), one rescale.

BlockPermute: a move (source ciphertext c, source block a -> destination
block b, weight w) has delta = (a - b) mod D = gamma*G + beta, with the
baby-step size G of the call fixed by the schedule (see "the permutation
schedule" below).  For destination d:
    acc_d = sum_gamma Rot_{gamma G B}( sum_{c, beta} Rot_{beta B}(src_c) (.) M_{d,c,gamma,beta} )
            + T_d (.) (W_c + sum_{b in C_d} W_b I_b)                  (scatter only)
with the baby rotations built once per source, the giant rotation applied
once per (d, gamma) after the inner sum, zero steps skipped, and the plaintext mask
    M_{d,c,gamma,beta} = sum_{moves in the group} W * I_{(b + gamma G) mod D},
    I_p = tau_{g_p}(I_0), g_p = 5^((-p B) mod N/2) mod 2N,
I_0 the encoding of the indicator of slots 0..k-1 at the call's mask scale S_I
and the integer weight W = rint((w * S_t * q_ell) / (S_src * S_I)) for the
target scale S_t (q_ell the top prime of the accumulator).  One rescale per
destination.  Gathers target S_t = Delta = 2^40 (the factors that enter the
products); scatters target S_t = 2^50, the scale the factor tables are held
at, which leaves room for the small weights alpha/d (~1e-5): W ~ w * 2^26
with S_I = 2^24 (at a 2^40 target and S_I = 2^20 it would be w * 2^20 ~ 10,
a rounding of up to 5 percent, the same way every epoch).

Mask precision.  Encoding I_0 rounds its N coefficients, so every slot of I_p
is off by about sqrt(N/24)/S_I (5e-5 at N = 2^15, S_I = 2^20) and a sum of D
masks with weight ~1 is off by sqrt(D) times that.  Three choices keep the
result within the 1e-4 value contract at N = 2^15 and 2^16:
* gather (every weight 1, one source scale): I_0 at S_I = 2^30; the
  accumulator's scale is declared as S_src * S_I * W_1 with
  W_1 = rint((S_t * q_ell) / (S_src * S_I)), the exact scale of every term,
  so no weight is rounded and the result's scale is within 2^-10 of S_t;
* scatter: I_0 at S_I = 2^24, target 2^50.  The self term's weights w_b (one per table
  entry) are split into a constant c, the lower median of the w_b of the
  present entries, applied as the constant polynomial
  W_c = rint((c * S_t * q_ell) / S_T) (S_T the table's scale), plus masked corrections w_b - c for the
  entries whose weight differs (C_d).  Mask rounding then scales with the
  correction, not with the weight ~1.  Slots of absent entries and the
  padding slots of a table are multiplied by c (they hold no data).

The same program runs on two back ends: ``CkksBackend`` (the oracle CKKS
context) and ``ClearBackend`` (plain slot vectors with exact 0/1 masks and
exact weights), which pins the rotation and mask index algebra.
"""
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

from . import chacha, ckks, ring

S_I = 2.0 ** 24      # mask scale of a scatter
S_IG = 2.0 ** 30     # mask scale of a gather
S_T = 2.0 ** 40      # target scale of a gather (the gathered factors)
S_TAB = 2.0 ** 50    # target scale of a scatter (the factor tables)
REFRESH_LEVEL = 4    # tables below this level are refreshed before the next gather
REFRESH_SERIAL = 0x20000000   # encryption serials of refreshed tables: + round * 1024 + table
MASK_BITS = 50       # refresh masks: integer coefficients in [-2^50, 2^50)


def block_masks(ctx, k):
    """{mask scale: I_0 encoded at that scale} for the scatter and gather scales."""
    ind = np.zeros(ctx.N // 2)
    ind[:k] = 1.0
    return {S_I: ctx.encode(ind, S_I), S_IG: ctx.encode(ind, S_IG)}


def next_pow2(k):
    p = 1
    while p < k:
        p *= 2
    return p


@dataclass
class Layout:
    N: int
    k: int
    kp: int
    B: int
    D: int
    G: int
    n_users: int
    n_items: int
    n_ct: int = 0
    # per rating (CSR order): rating ciphertext and block
    ct_of: np.ndarray = None
    blk_of: np.ndarray = None
    rows: np.ndarray = None      # user of each rating
    cols: np.ndarray = None      # item of each rating

    @property
    def n_utab(self):
        return -(-self.n_users // self.D)

    @property
    def n_vtab(self):
        return -(-self.n_items // self.D)


def make_layout(N, k, n_users, n_items, row_ptr, col_idx):
    kp = next_pow2(k)
    B = 2 * kp
    D = N // (2 * B)
    logD = D.bit_length() - 1
    G = 1 << ((logD + 1) // 2)
    row_ptr = np.asarray(row_ptr, np.int64)
    nnz = int(row_ptr[-1])
    ct_of = np.zeros(nnz, np.int64)
    blk_of = np.zeros(nnz, np.int64)
    c, used = 0, 0
    started = False
    for i in range(n_users):
        s, e = int(row_ptr[i]), int(row_ptr[i + 1])
        pos = s
        while pos < e:
            chunk = min(D, e - pos)
            if not started:
                started = True
            elif used + chunk > D:
                c += 1
                used = 0
            ct_of[pos:pos + chunk] = c
            blk_of[pos:pos + chunk] = used + np.arange(chunk)
            used += chunk
            pos += chunk
    lay = Layout(N, k, kp, B, D, G, n_users, n_items)
    lay.n_ct = c + 1 if started else 0
    lay.ct_of, lay.blk_of = ct_of, blk_of
    lay.rows = np.repeat(np.arange(n_users), np.diff(row_ptr))
    lay.cols = np.asarray(col_idx, np.int64)
    return lay


def slot_vectors(lay, values_per_rating=None, users=None, items=None, which="R"):
    """Cleartext slot contents of the rating-layout ciphertexts ([n_ct][N/2])."""
    out = np.zeros((lay.n_ct, lay.N // 2))
    for r in range(len(lay.rows)):
        c, t = lay.ct_of[r], lay.blk_of[r]
        sl = slice(t * lay.B, t * lay.B + lay.k)
        if which == "R":
            out[c, sl] = values_per_rating[r]
        elif which == "U":
            out[c, sl] = users[lay.rows[r]]
        else:
            out[c, sl] = items[lay.cols[r]]
    return out


def table_vectors(lay, F, n_tab):
    out = np.zeros((n_tab, lay.N // 2))
    for e in range(F.shape[0]):
        a, b = divmod(e, lay.D)
        out[a, b * lay.B: b * lay.B + lay.k] = F[e]
    return out


def rotation_steps(lay):
    """Every rotation the program uses (left steps): the windowed sum
    (1, 2, .., B/2 and -k') and the block steps 2^j B, j < log2 D, of the
    baby and giant trees."""
    st = set()
    s = 1
    while s < lay.B:
        st.add(s)
        s *= 2
    st.add(-lay.kp)
    s = 1
    while s < lay.D:
        st.add(s * lay.B)
        s *= 2
    return sorted(st)


# ---------------------------------------------------------------- back ends
class CkksBackend:
    """Evaluates the program on oracle ciphertexts."""

    def __init__(self, ctx: ckks.Context, masks):
        """masks: {mask scale: integer coefficients of I_0 encoded at that scale}."""
        self.ctx = ctx
        self.masks = {float(s): np.asarray(m, np.int64) for s, m in masks.items()}
        self.N = ctx.N

    def level(self, x):
        return x.level

    def scale(self, x):
        return x.scale

    def top_prime(self, level):
        return self.ctx.prm.q[level]

    def hmult(self, a, b):
        return self.ctx.hmult(a, b)

    def add(self, a, b):
        return self.ctx.add(a, b)

    def sub(self, a, b):
        return self.ctx.sub(a, b)

    def rotate(self, a, r):
        return self.ctx.rotate(a, r)

    def mul_int(self, a, w):
        return self.ctx.mul_int(a, w)

    def rescale(self, a):
        return self.ctx.rescale(a)

    def drop(self, a, level):
        return self.ctx.mod_drop(a, level)

    def mask_mul(self, a, terms, scale, mask_scale, const=0):
        """a (.) (const + sum_m W_m * I_{p_m}), I_0 encoded at mask_scale; the
        result carries the given scale."""
        N = self.N
        m = np.zeros(N, dtype=object)
        m[0] = int(const)
        for p, W in terms:
            m = m + int(W) * self._mask(p, mask_scale)
        qm = self.ctx.qmods(a.level)
        mm = np.stack([np.array([int(v) % q for v in m], dtype=np.uint64) for q in qm])
        idx = list(range(a.level + 1))
        return ckks.Ciphertext(self.ctx.mul(a.c0, mm, idx), self.ctx.mul(a.c1, mm, idx), scale)

    def set_block(self, B):
        self.B = B
        self._cache = {}

    def refresh(self, ct, obj):
        c = self.ctx
        mask = refresh_mask(c.seed, self.N, obj)
        masked = c.add_plain(ct, mask)                 # evaluating party
        m = c.decrypt_int(masked)                      # key holder: integers mod q_0
        saved = c.serial
        c.serial = REFRESH_SERIAL + obj
        fresh = c.encrypt_int(m, c.prm.L, ct.scale)
        c.serial = saved
        return c.add_plain(fresh, -mask)               # evaluating party

    def _mask(self, p, mask_scale):
        key = (float(mask_scale), p)
        if key not in self._cache:
            N = self.N
            g = pow(5, (-p * self.B) % (N // 2), 2 * N)
            dst, neg = ring.automorphism_map(g, N)
            v = np.zeros(N, dtype=object)
            src = self.masks[float(mask_scale)].astype(object)
            v[dst] = np.where(neg, -src, src)
            self._cache[key] = v
        return self._cache[key]


class ClearBackend:
    """Plain slot vectors: exact 0/1 block masks and exact weights."""

    @dataclass
    class V:
        z: np.ndarray
        level: int
        scale: float

    def __init__(self, N, q_chain, B, k, L=None):
        self.N = N
        self.q = q_chain
        self.B = B
        self.k = k
        self.L = L        # top level (refresh target); default: the last prime of q_chain

    def wrap(self, z, level, scale):
        return ClearBackend.V(np.asarray(z, np.float64), level, scale)

    def level(self, x):
        return x.level

    def scale(self, x):
        return x.scale

    def top_prime(self, level):
        return self.q[level]

    def hmult(self, a, b):
        lv = min(a.level, b.level)
        return self.V(a.z * b.z, lv - 1, a.scale * b.scale / float(self.q[lv]))

    def add(self, a, b):
        return self.V(a.z + b.z, min(a.level, b.level), a.scale)

    def sub(self, a, b):
        return self.V(a.z - b.z, min(a.level, b.level), a.scale)

    def rotate(self, a, r):
        return self.V(np.roll(a.z, -r), a.level, a.scale)

    def mul_int(self, a, w):
        return self.V(a.z, a.level, a.scale * float(w))   # value unchanged; scale absorbs w

    def rescale(self, a):
        return self.V(a.z, a.level - 1, a.scale / float(self.q[a.level]))

    def drop(self, a, level):
        return self.V(a.z, level, a.scale)

    def mask_mul(self, a, terms, scale, mask_scale, const=0.0):
        m = np.full(self.N // 2, float(const))
        for p, w in terms:            # here the weights are the exact reals, not the integers W
            m[p * self.B: p * self.B + self.k] += w
        return self.V(a.z * m, a.level, scale)

    def set_block(self, B):
        pass

    def refresh(self, ct, obj):
        return self.V(ct.z, len(self.q) - 1 if self.L is None else self.L, ct.scale)


# ---------------------------------------------------------------- the program
@dataclass
class Move:
    src: int      # source ciphertext
    a: int        # source block
    b: int        # destination block
    w: float      # real weight


# ---------------------------------------------------------------- the permutation schedule
# Every arrangement of BlockPermute's rotations gives the same slot values, but
# not the same bits: each key switch rounds in its own way.  The paper leaves
# this data movement to the implementation, so the schedule is part of the
# definition here (a reading), and an implementation that is to match bit for
# bit follows it:
#   * baby-step size G: choose_G, the power of two with the fewest rotations
#     among those that keep at most MAX_ACCUMULATORS inner sums
#     (destinations x D/G) alive, ties to the smaller G;
#   * babies Rot_{beta B}(src) for beta up to the largest one the source needs,
#     in blocks of BABY_BLOCK steps: block base Rot_{k B}(src) (k a multiple of
#     BABY_BLOCK, the next base Rot_{BABY_BLOCK B} of the previous one), inside
#     a block baby k+s+j = Rot_{s B}(baby k+j) for s = 1, 2, 4, ..;
#   * per destination, inner sums over (source, beta) in that order, then the
#     giant steps as a pairwise tree (level j: node t = node 2t +
#     Rot_{2^j G B}(node 2t+1)), the self term, one rescale.
# What does not change a ciphertext is left free: batching of rotations, the
# order of exact modular sums, and how many sources are processed at once.
BABY_BLOCK = 64           # babies are built in blocks of this many consecutive steps
MAX_ACCUMULATORS = 1024   # bound on destinations * D/G inner sums alive at once


def _next_pow2(x):
    p = 1
    while p < x:
        p *= 2
    return p


def baby_rotations(n):
    """Rotations that build babies 1..n-1 of one source: every baby is made by
    one rotation (inside a block of BABY_BLOCK from a smaller one by a doubling
    step, or as the next block's base)."""
    return max(0, n - 1)


def giant_rotations(present, width):
    """Rotations of the pairwise giant-step tree over positions 0..width-1 of
    which `present` hold a nonempty inner sum."""
    nodes = set(present)
    count = 0
    while width > 1:
        nxt = set()
        for t in range(width // 2):
            if 2 * t + 1 in nodes:
                count += 1
            if 2 * t in nodes or 2 * t + 1 in nodes:
                nxt.add(t)
        nodes, width = nxt, width // 2
    return count


def choose_G(dests_moves, D):
    """Baby-step size of one permutation: the power of two G <= D with the
    fewest rotations (babies: blocks of doubling trees up to the largest baby
    step a source needs; giants: pairwise trees over D/G positions per
    destination), among those with len(dests) * D/G <= MAX_ACCUMULATORS;
    ties go to the smaller G; G = D if no G meets the bound."""
    best = None
    G = 1
    while G <= D:
        if len(dests_moves) * (D // G) <= MAX_ACCUMULATORS:
            top = {}
            gam = {}
            for d, moves in enumerate(dests_moves):
                for mv in moves:
                    gamma, beta = divmod((mv.a - mv.b) % D, G)
                    top[mv.src] = max(top.get(mv.src, 0), beta)
                    gam.setdefault(d, set()).add(gamma)
            cost = sum(baby_rotations(m + 1) for m in top.values())
            cost += sum(giant_rotations(s, D // G) for s in gam.values())
            if best is None or cost < best[0]:
                best = (cost, G)
        G *= 2
    return best[1] if best is not None else D


def block_permute(be, lay, srcs, dests_moves, self_terms, level, mask_scale, target, unit=False,
                  exact_weights=False, G=None):
    """dests_moves[d] = list of Move; self_terms[d] = (table ciphertext, c,
    [(block, w_b - c)]) or None.  All sources share level and scale.  unit:
    every move has weight 1 and the accumulator takes the exact scale of the
    terms.  G: baby-step size (None: choose_G).  Returns the rescaled
    accumulators."""
    D, B = lay.D, lay.B
    if G is None:
        G = choose_G(dests_moves, D)
    src_scale = be.scale(srcs[0]) if srcs else None
    q_acc = float(be.top_prime(level))
    if unit:
        assert all(mv.w == 1.0 for moves in dests_moves for mv in moves)
        W1 = weight(1.0, src_scale, q_acc, mask_scale, False, target)
        acc_scale = src_scale * mask_scale * float(W1)
    else:
        acc_scale = target * q_acc
    # babies Rot_{beta B}(src) for beta up to the largest one a source needs
    top = {}
    for moves in dests_moves:
        for mv in moves:
            top[mv.src] = max(top.get(mv.src, 0), ((mv.a - mv.b) % D) % G)
    baby = {}
    for c, m in top.items():
        n = m + 1
        b = {}
        base = be.drop(srcs[c], level)
        for k in range(0, n, BABY_BLOCK):
            b[k] = base
            width = min(BABY_BLOCK, n - k)
            s = 1
            while s < width:
                for j in range(s):
                    if s + j < width:
                        b[k + s + j] = be.rotate(b[k + j], s * B)
                s *= 2
            if k + BABY_BLOCK < n:
                base = be.rotate(base, BABY_BLOCK * B)
        baby[c] = b
    out = []
    for d, moves in enumerate(dests_moves):
        groups = {}
        for mv in moves:
            delta = (mv.a - mv.b) % D
            gamma, beta = divmod(delta, G)
            groups.setdefault(gamma, {}).setdefault((mv.src, beta), []).append(mv)
        nodes = {}
        for gamma in sorted(groups):
            inner = None
            for (c, beta) in sorted(groups[gamma]):
                terms = []
                for mv in groups[gamma][(c, beta)]:
                    p = (mv.b + gamma * G) % D
                    terms.append((p, weight(mv.w, src_scale, q_acc, mask_scale, exact_weights, target)))
                t = be.mask_mul(baby[c][beta], terms, acc_scale, mask_scale)
                inner = t if inner is None else be.add(inner, t)
            nodes[gamma] = inner
        # giant steps: sum_gamma Rot_{gamma G B}(inner_gamma) as a pairwise tree
        width, step = D // G, G * B
        while width > 1:
            nxt = {}
            for tt in range(width // 2):
                left, right = nodes.get(2 * tt), nodes.get(2 * tt + 1)
                if right is not None:
                    right = be.rotate(right, step)
                if left is not None and right is not None:
                    nxt[tt] = be.add(left, right)
                elif left is not None or right is not None:
                    nxt[tt] = left if left is not None else right
            nodes, width, step = nxt, width // 2, step * 2
        acc = nodes.get(0)
        st = self_terms[d] if self_terms else None
        if st is not None:
            ct, cst, blocks = st
            ctd = be.drop(ct, level)
            s_self = be.scale(ctd)
            Wc = weight(cst, s_self, q_acc, 1.0, exact_weights, target)
            terms = [(b, weight(w, s_self, q_acc, mask_scale, exact_weights, target)) for b, w in blocks]
            t = be.mask_mul(ctd, terms, acc_scale, mask_scale, const=Wc)
            acc = t if acc is None else be.add(acc, t)
        out.append(be.rescale(acc))
    return out


def weight(w, s_src, q_acc, mask_scale, exact, target):
    """The integer W that carries weight w from scale s_src to target * q_acc."""
    if exact:
        return w
    return int(np.rint((w * target * q_acc) / (s_src * mask_scale)))


@dataclass
class EpochResult:
    utab: list
    vtab: list
    ug: list = None
    vg: list = None
    sdot: list = None
    refresh_round: int = 0


def run_epochs(be, lay, R, Ug, Vg, Utab, Vtab, n_epochs, alpha, lam, damp=0.0, rule="R1",
               exact_weights=False, refresh=False, refresh_round=0, epoch0=0):
    """Run n_epochs from gathered factors Ug, Vg (None: gather first); every
    later epoch first gathers from the tables, refreshing them when their
    level is below REFRESH_LEVEL (only if refresh is allowed).  epoch0: epochs
    run before (the dampening index).  Returns the final tables and the last
    forward dot products."""
    be.set_block(lay.B)
    d_user = np.bincount(lay.rows, minlength=lay.n_users)
    c_item = np.bincount(lay.cols, minlength=lay.n_items)
    sdot = None
    for t in range(n_epochs):
        a_t = alpha / (1.0 + damp * (epoch0 + t))
        if t > 0 or Ug is None:
            # 6: gather for this epoch, after a refresh if the tables are too low
            if be.level(Utab[0]) < REFRESH_LEVEL:
                if not refresh:
                    raise ValueError("level budget exhausted and refresh not allowed")
                Utab, Vtab = refresh_tables(be, Utab, Vtab, refresh_round)
                refresh_round += 1
            Ug = _gather(be, lay, Utab, lay.rows, exact_weights)
            Vg = _gather(be, lay, Vtab, lay.cols, exact_weights)
        # 1-3: block dot products and errors
        E, sdot = [], []
        for c in range(lay.n_ct):
            P = be.hmult(Ug[c], Vg[c])
            T = P
            s = 1
            while s < lay.B:
                T = be.add(T, be.rotate(T, s))
                s *= 2
            S = be.rotate(T, -lay.kp)
            sdot.append(S)
            SP = be.scale(P)
            WR = int(np.rint((SP * float(be.top_prime(be.level(R[c])))) / be.scale(R[c])))
            Re = be.rescale(be.mul_int(R[c], WR))
            Re = be.drop(Re, be.level(S))
            E.append(be.sub(Re, S))
        # 4: gradient terms
        GU = [be.hmult(E[c], be.drop(Vg[c], be.level(E[c]))) for c in range(lay.n_ct)]
        GV = [be.hmult(E[c], be.drop(Ug[c], be.level(E[c]))) for c in range(lay.n_ct)]
        glevel = be.level(GU[0])
        # 5: scatter into the tables
        Utab = _scatter(be, lay, GU, Utab, lay.rows, d_user, lay.n_users, a_t, lam, rule, glevel, exact_weights)
        Vtab = _scatter(be, lay, GV, Vtab, lay.cols, c_item, lay.n_items, a_t, lam, rule, glevel, exact_weights)
    return EpochResult(Utab, Vtab, Ug, Vg, sdot, refresh_round)


def refresh_tables(be, Utab, Vtab, rnd):
    """Refresh of level-exhausted tables through the masking step of the
    protocol (Sec. III-B): the evaluating party adds a mask polynomial, the key
    holder decrypts to integers (mod q_0) and encrypts the same integers anew
    at the top level and the same scale, the evaluating party removes the
    mask.  Table j of round rnd (U tables first) uses mask stream id
    rnd * 1024 + j and encryption serial REFRESH_SERIAL + rnd * 1024 + j."""
    tabs = list(Utab) + list(Vtab)
    out = [be.refresh(ct, rnd * 1024 + j) for j, ct in enumerate(tabs)]
    return out[:len(Utab)], out[len(Utab):]


def refresh_mask(seed, N, obj):
    """Mask polynomial (ChaCha20 purpose 9, object obj, limb 0): coefficient
    n = (w_n mod 2^51) - 2^50."""
    w = chacha.words_u64(seed, chacha.P_REFRESH_MASK, obj, 0, N)
    return (w % np.uint64(1 << (MASK_BITS + 1))).astype(np.int64) - (1 << MASK_BITS)


def _scatter(be, lay, Gs, tabs, owner, deg, n_ent, a_t, lam, rule, level, exact):
    D = lay.D
    moves = [[] for _ in tabs]
    for r in range(len(owner)):
        e = int(owner[r])
        d, b = divmod(e, D)
        w = a_t if rule == "R1" else a_t / deg[e]
        moves[d].append(Move(int(lay.ct_of[r]), int(lay.blk_of[r]), b, w))
    return block_permute(be, lay, Gs, moves, self_terms(lay, tabs, deg, n_ent, a_t, lam, rule), level,
                         S_I, S_TAB, False, exact)


def self_terms(lay, tabs, deg, n_ent, a_t, lam, rule):
    """Per table ciphertext: (ciphertext, c, [(block, w_b - c)]) with w_b the
    entry's weight (R1: 1 - a_t*lambda*d; R2: 1 - a_t*lambda, 1 for an empty
    entry), c the lower median of the w_b, corrections where w_b != c."""
    D = lay.D
    out = []
    for d in range(len(tabs)):
        ws = []
        for b in range(D):
            e = d * D + b
            if e >= n_ent:
                break
            if rule == "R1":
                w = 1.0 - a_t * lam * deg[e]
            else:
                w = (1.0 - a_t * lam) if deg[e] > 0 else 1.0
            ws.append((b, w))
        srt = sorted(w for _, w in ws)
        c = srt[(len(srt) - 1) // 2]
        out.append((tabs[d], c, [(b, w - c) for b, w in ws if w != c]))
    return out


def _gather(be, lay, tabs, owner, exact):
    D = lay.D
    moves = [[] for _ in range(lay.n_ct)]
    for r in range(len(owner)):
        e = int(owner[r])
        a_ct, a = divmod(e, D)
        moves[int(lay.ct_of[r])].append(Move(a_ct, a, int(lay.blk_of[r]), 1.0))
    level = be.level(tabs[0])
    return block_permute(be, lay, tabs, moves, None, level, S_IG, S_T, True, exact)


def decode_tables(vals, lay, n_ent):
    """Slot vectors of table ciphertexts -> factor matrix [n_ent][k]."""
    F = np.zeros((n_ent, lay.k))
    for e in range(n_ent):
        a, b = divmod(e, lay.D)
        F[e] = vals[a][b * lay.B: b * lay.B + lay.k]
    return F


def decode_predictions(vals, lay):
    """Slot vectors of the forward dot products -> r_hat per rating (CSR order)."""
    return np.array([vals[int(c)][int(t) * lay.B] for c, t in zip(lay.ct_of, lay.blk_of)])


# ---------------------------------------------------------------- Alg. 2 on ciphertexts
# The user-item batch pairs of Sec. III-D with a batch = one factor-table
# ciphertext (the D profiles it holds): user i is local index i mod D of batch
# i div D, items likewise.  The ratings of each pair, in CSR order, are packed
# into rating ciphertexts of their own (D blocks each); pairs come in the order
# of their first rating.  An epoch runs the pairs one after the other, each
# from the tables as they are when it starts (Alg. 2):
#   Ug, Vg <- gather of the pair's user table and item table into the pair's
#             rating layout (BlockPermute, weight 1);
#   Sdot, E, G_U = HMult(E, Vg), G_V = HMult(E, Ug) as in the epoch above;
#   user table <- BlockPermute(G_U -> table, weight a') + self term
#                 (1 - a' lambda c_i) u_i, c_i = ratings of user i in the pair
#                 (1 for users of the table without one);  items likewise;
# with a' = alpha / (1 + damp t) and the per-rating lambda of Alg. 2.  Before a
# pair whose tables are below REFRESH_LEVEL, all tables are refreshed.
@dataclass
class Pair:
    ub: int               # user table (batch) index
    vb: int               # item table index
    cts: list             # its rating ciphertexts
    ratings: np.ndarray   # its ratings (CSR indices)


def make_pair_layout(N, k, n_users, n_items, row_ptr, col_idx):
    from .mf import batch_pairs
    lay = make_layout(N, k, n_users, n_items, row_ptr, col_idx)   # shape of the blocks and tables
    D = lay.D
    ct_of = np.zeros(len(lay.rows), np.int64)
    blk_of = np.zeros(len(lay.rows), np.int64)
    pairs, c = [], 0
    for (ub, vb), idx in batch_pairs(row_ptr, col_idx, D, D):
        idx = np.asarray(idx, np.int64)
        n = -(-len(idx) // D)
        ct_of[idx] = c + np.arange(len(idx)) // D
        blk_of[idx] = np.arange(len(idx)) % D
        pairs.append(Pair(ub, vb, list(range(c, c + n)), idx))
        c += n
    lay.ct_of, lay.blk_of, lay.n_ct = ct_of, blk_of, c
    lay.pairs = pairs
    return lay


def _pair_moves(lay, pair, owner, to_table):
    """Moves of one pair: gather (table block -> the pair's rating blocks) or
    scatter (rating blocks -> table block, weight set by the caller)."""
    D, c0 = lay.D, pair.cts[0]
    if to_table:
        return [Move(int(lay.ct_of[r]) - c0, int(lay.blk_of[r]), int(owner[r]) % D, 1.0) for r in pair.ratings]
    moves = [[] for _ in pair.cts]
    for r in pair.ratings:
        moves[int(lay.ct_of[r]) - c0].append(Move(0, int(owner[r]) % D, int(lay.blk_of[r]), 1.0))
    return moves


def run_pair_epochs(be, lay, R, Utab, Vtab, n_epochs, alpha, lam, damp=0.1, exact_weights=False, refresh=True,
                    refresh_round=0, epoch0=0):
    """Alg. 2 epochs on a pair layout; returns the tables and the dot products
    of every rating ciphertext from the last epoch (at the start of its pair)."""
    be.set_block(lay.B)
    Utab, Vtab = list(Utab), list(Vtab)
    sdot = [None] * lay.n_ct
    for t in range(n_epochs):
        a_t = alpha / (1.0 + damp * (epoch0 + t))
        for pr in lay.pairs:
            if min(be.level(Utab[pr.ub]), be.level(Vtab[pr.vb])) < REFRESH_LEVEL:
                if not refresh:
                    raise ValueError("level budget exhausted and refresh not allowed")
                Utab, Vtab = refresh_tables(be, Utab, Vtab, refresh_round)
                refresh_round += 1
            ut, vt = Utab[pr.ub], Vtab[pr.vb]
            Ug = block_permute(be, lay, [ut], _pair_moves(lay, pr, lay.rows, False), None, be.level(ut),
                               S_IG, S_T, True, exact_weights)
            Vg = block_permute(be, lay, [vt], _pair_moves(lay, pr, lay.cols, False), None, be.level(vt),
                               S_IG, S_T, True, exact_weights)
            E = []
            for i, c in enumerate(pr.cts):
                P = be.hmult(Ug[i], Vg[i])
                T = P
                s = 1
                while s < lay.B:
                    T = be.add(T, be.rotate(T, s))
                    s *= 2
                S = be.rotate(T, -lay.kp)
                sdot[c] = S
                WR = int(np.rint((be.scale(P) * float(be.top_prime(be.level(R[c])))) / be.scale(R[c])))
                Re = be.drop(be.rescale(be.mul_int(R[c], WR)), be.level(S))
                E.append(be.sub(Re, S))
            GU = [be.hmult(E[i], be.drop(Vg[i], be.level(E[i]))) for i in range(len(pr.cts))]
            GV = [be.hmult(E[i], be.drop(Ug[i], be.level(E[i]))) for i in range(len(pr.cts))]
            glevel = be.level(GU[0])
            for tabs, G, owner, b in ((Utab, GU, lay.rows, pr.ub), (Vtab, GV, lay.cols, pr.vb)):
                n_ent = lay.n_users if owner is lay.rows else lay.n_items
                cnt = np.zeros(n_ent)
                np.add.at(cnt, np.asarray(owner)[pr.ratings], 1.0)
                moves = _pair_moves(lay, pr, owner, True)
                for mv in moves:
                    mv.w = a_t
                st = _pair_self_term(lay, tabs[b], b, cnt, n_ent, a_t, lam)
                tabs[b] = block_permute(be, lay, G, [moves], [st], glevel, S_I, S_TAB, False, exact_weights)[0]
    return EpochResult(Utab, Vtab, None, None, sdot, refresh_round)


def _pair_self_term(lay, tab, d, cnt, n_ent, a_t, lam):
    """Self term of table d for one pair: w_b = 1 - a' lambda c_e (c_e the
    entity's ratings in the pair), as a constant (lower median) plus corrections."""
    ws = []
    for b in range(lay.D):
        e = d * lay.D + b
        if e >= n_ent:
            break
        ws.append((b, 1.0 - a_t * lam * cnt[e]))
    srt = sorted(w for _, w in ws)
    c = srt[(len(srt) - 1) // 2]
    return (tab, c, [(b, w - c) for b, w in ws if w != c])
