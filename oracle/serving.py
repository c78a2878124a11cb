"""Per-user encrypted requests against resident factor tables (oracle; test
infrastructure only).

The paper's recommendation phase (Sec. III-B) has the server answer from the
encrypted factors, and its update rule (Eq. 2-3, Alg. 1) applied to one user
row is an UPDATE of that user's profile with the items fixed.  A request
carries user i and its CSR row (items j_1 < .. < j_d; ratings for an UPDATE);
the row is cut into chunks of at most D items (chunk c holds items
c*D .. c*D+D-1 of the row, item t of the chunk in block t).

Per chunk (tables Utab, Vtab resident at the top level; baby-step size
G = 2^ceil(log2(D)/2)):
 * gather Ug (u_i in every used block) and Vg (v_j in block t) by block
   permutation with weight 1: a move (table a, table block e mod D -> block t)
   has delta = (e mod D - t) mod D = gamma*G + beta; per (gamma, table, beta)
   the group's terms (p = (t + gamma G) mod D, W_1) form the mask
   sum_m W_1 I_p applied to the baby Rot_{beta B}(table) (hoisted from the
   table, beta = 0: the table itself); the gamma = 0 groups sum into the
   accumulator, each gamma > 0 into its own inner sum, which is rotated by
   gamma*G*B and added (gamma ascending; an accumulator without gamma = 0
   terms starts with the first rotated inner sum); one rescale.  The
   accumulator's scale is the exact scale of its terms S_src * S_I * W_1
   with W_1 = rint((S_T * q_L) / (S_src * S_I)), S_I = 2^30, S_T = 2^40;
 * Sdot = windowed block sum of HMult(Ug, Vg): slot tB holds <u_i, v_j>.
PREDICT returns Sdot per chunk.  UPDATE (rule R2 of the epoch, one user):
 * R_c = Enc(encoded rating chunk) at the top level, scale 2^40, encryption
   serial 0x40000000 + 8 * client_serial + c;
 * E = drop(Rescale(R * W_R)) - Sdot, W_R = rint((S_P * q_L) / S_R);
 * G = HMult(E, drop(Vg)); T = G summed over all D blocks (T <- T + Rot(T, s)
   for s = B, 2B, .., B*D/2); chunk sums added in chunk order;
 * u' = Rescale((1 - lr*lambda) * Ug + (lr/d) * T) with integer weights
   W_s = rint(((1 - lr*lambda) * 2^40 * q) / S_Ug), W_g = rint(((lr/d) * 2^40 * q) / S_T)
   at the declared scale 2^40 * q (q the top prime of T's level), so u' has
   scale 2^40; it is returned in broadcast layout (block 0 holds u_i').
"""
import numpy as np

from . import ckks
from .program import S_IG, S_T, Move, weight, next_pow2

SERVE_SERIAL = 0x40000000


def chunk_serial(client_serial, chunk):
    return SERVE_SERIAL + client_serial * 8 + chunk


class ServingState:
    """Resident tables and their cached baby-step rotations."""

    def __init__(self, ctx: ckks.Context, k, utab, vtab, mask_gather, lr, lam):
        self.ctx = ctx
        self.k = k
        self.kp = next_pow2(k)
        self.B = 2 * self.kp
        self.D = ctx.N // (2 * self.B)
        logD = self.D.bit_length() - 1
        self.G = 1 << ((logD + 1) // 2)
        self.utab, self.vtab = list(utab), list(vtab)
        self.mask = np.asarray(mask_gather, np.int64)
        self.lr, self.lam = lr, lam
        self.babies = {}
        for name, tabs in (("u", self.utab), ("v", self.vtab)):
            for a, t in enumerate(tabs):
                hs = ctx.hoisted_rotations(t, [b * self.B for b in range(1, self.G)])
                for b in range(1, self.G):
                    self.babies[(name, a, b)] = hs[b * self.B]

    def _mask_poly(self, p):
        """I_p = tau_{g_p}(I_0), g_p = 5^((-p B) mod N/2) mod 2N."""
        from . import ring
        N = self.ctx.N
        g = pow(5, (-p * self.B) % (N // 2), 2 * N)
        dst, neg = ring.automorphism_map(g, N)
        v = np.zeros(N, dtype=object)
        src = self.mask.astype(object)
        v[dst] = np.where(neg, -src, src)
        return v

    def _mask_mul(self, ct, terms, scale):
        ctx = self.ctx
        m = np.zeros(ctx.N, dtype=object)
        for p, W in terms:
            m = m + int(W) * self._mask_poly(p)
        qm = ctx.qmods(ct.level)
        mm = np.stack([np.array([int(v) % q for v in m], dtype=np.uint64) for q in qm])
        idx = list(range(ct.level + 1))
        return ckks.Ciphertext(ctx.mul(ct.c0, mm, idx), ctx.mul(ct.c1, mm, idx), scale)

    def gather(self, name, moves):
        """One destination: moves = [Move(table, block, dst block, 1.0)]."""
        ctx, D, G, B = self.ctx, self.D, self.G, self.B
        tabs = self.utab if name == "u" else self.vtab
        level = tabs[0].level
        s_src = tabs[0].scale
        q_acc = float(ctx.prm.q[level])
        W1 = weight(1.0, s_src, q_acc, S_IG, False, S_T)
        acc_scale = s_src * S_IG * float(W1)
        groups = {}
        for mv in moves:
            gamma, beta = divmod((mv.a - mv.b) % D, G)
            groups.setdefault(gamma, {}).setdefault((mv.src, beta), []).append(((mv.b + gamma * G) % D, W1))
        sums = {}
        for gamma in sorted(groups):
            for (a, beta), terms in sorted(groups[gamma].items()):
                baby = tabs[a] if beta == 0 else self.babies[(name, a, beta)]
                t = self._mask_mul(baby, terms, acc_scale)
                sums[gamma] = t if gamma not in sums else ctx.add(sums[gamma], t)
        acc = sums.get(0)
        for gamma in sorted(g for g in sums if g > 0):
            r = ctx.rotate(sums[gamma], gamma * G * B)
            acc = r if acc is None else ctx.add(acc, r)
        return ctx.rescale(acc)

    def _chunks(self, user, items):
        D = self.D
        a_u, e_u = divmod(user, D)
        out = []
        for s in range(0, len(items), D):
            part = items[s:s + D]
            mu = [Move(a_u, e_u, t, 1.0) for t in range(len(part))]
            mv = [Move(int(j) // D, int(j) % D, t, 1.0) for t, j in enumerate(part)]
            out.append((mu, mv))
        return out

    def _dots(self, ug, vg):
        ctx = self.ctx
        P = ctx.hmult(ug, vg)
        T = P
        s = 1
        while s < self.B:
            T = ctx.add(T, ctx.rotate(T, s))
            s *= 2
        return P.scale, ctx.rotate(T, -self.kp)

    def predict(self, user, items):
        """Sdot per chunk (slot t*B holds <u_user, v_(item t of the chunk)>)."""
        out = []
        for mu, mv in self._chunks(user, items):
            out.append(self._dots(self.gather("u", mu), self.gather("v", mv))[1])
        return out

    def update(self, user, items, plain_chunks, client_serial):
        """u' (rule R2 step for one user) from the client's encoded rating chunks."""
        ctx, L, B, D = self.ctx, self.ctx.prm.L, self.B, self.D
        tots, ug0 = [], None
        for c, (mu, mv) in enumerate(self._chunks(user, items)):
            ug, vg = self.gather("u", mu), self.gather("v", mv)
            if ug0 is None:
                ug0 = ug
            sp, S = self._dots(ug, vg)
            saved = ctx.serial
            ctx.serial = chunk_serial(client_serial, c)
            R = ctx.encrypt_int(plain_chunks[c], L, S_T)
            ctx.serial = saved
            WR = int(np.rint((sp * float(ctx.prm.q[L])) / R.scale))
            Re = ctx.mod_drop(ctx.rescale(ctx.mul_int(R, WR)), S.level)
            E = ctx.sub(Re, S)
            T = ctx.hmult(E, ctx.mod_drop(vg, E.level))
            s = B
            while s < B * D:
                T = ctx.add(T, ctx.rotate(T, s))
                s *= 2
            tots.append(T)
        tot = tots[0]
        for T in tots[1:]:
            tot = ctx.add(tot, T)
        lvl = tot.level
        q = float(ctx.prm.q[lvl])
        target = S_T * q
        d = float(len(items))
        self_ = ctx.mod_drop(ug0, lvl)
        Ws = int(np.rint(((1.0 - self.lr * self.lam) * S_T * q) / self_.scale))
        Wg = int(np.rint(((self.lr / d) * S_T * q) / tot.scale))
        a = ctx.mul_int(self_, Ws)
        b = ctx.mul_int(tot, Wg)
        a = ckks.Ciphertext(a.c0, a.c1, target)
        b = ckks.Ciphertext(b.c0, b.c1, target)
        return ctx.rescale(ctx.add(a, b))
