"""RNS-CKKS, written out plainly (oracle; test infrastructure only).

The paper encrypts ratings and latent factors with CKKS (Sec. II-A.2, Sec. IV-A)
and uses exactly four homomorphic properties, Eq. 6-9: ciphertext + ciphertext,
ciphertext x ciphertext, ciphertext + plaintext and ciphertext x plaintext.  Its
Alg. 1 also needs slot rotations (to reduce a packed product to a dot product)
and its leveled use needs rescaling.  The definitions below are textbook CKKS
(Cheon-Kim-Kim-Song 2017) in its full-RNS form with hybrid key switching; every
non-associative choice is fixed so that an independent implementation can
reproduce the ciphertexts bit for bit:

keys     s ternary; pk = (b, a), b = -a*s + e over Q_L; switching key s' -> s per
         digit j: b_j = -a_j*s + e_j + [P]_{q_i} * s' * 1[i in D_j] on Q limbs,
         b_j = -a_j*s + e_j on P limbs.  Relinearisation key: s' = s^2.
         Rotation key for Galois element g: s' = tau_g(s).
encrypt  c0 = v*b + m + e0, c1 = v*a + e1 over q_0..q_l.
decrypt  c0 + c1*s kept mod q_0 only, centred.
KS(d)    ModUp every digit of d to Q_l u P, inner product with the key digits,
         ModDown both halves.
HMult    tensor -> relinearise -> rescale, in that order.
rotate   non-hoisted: (tau_g(c0) + u0, u1) with (u0, u1) = KS_{tau_g(s)->s}(tau_g(c1));
         hoisted: ModUp the unrotated c1 once, apply tau_g to every extended digit.
scales   IEEE double bookkeeping: products S_a*S_b, rescale S/q_l.

Randomness comes from ChaCha20 streams keyed by the master seed (see ``chacha``):
purpose 1 secret, 2/3 pk a/e, 4/5 switching-key a/e with object id
key_index*dnum + digit (key_index 0 = relinearisation, g = rotation by Galois
element g), 6/7/8 encryption v/e0/e1 with object id = ciphertext serial number
(assigned 0, 1, 2, ... in creation order).
"""
from dataclasses import dataclass

import numpy as np

from . import chacha, sampling, ring, rns
from .modarith import mulmod, addmod

SCALE_TOL = 2.0 ** -30


class CkksError(Exception):
    pass


class ScaleMismatch(CkksError):
    pass


@dataclass
class Ciphertext:
    c0: np.ndarray      # [level+1, N] uint64, coefficient form
    c1: np.ndarray
    scale: float

    @property
    def level(self):
        return self.c0.shape[0] - 1


def galois_for_step(r, N):
    """Galois element of a left rotation by r slots: 5^(r mod N/2) mod 2N."""
    return pow(5, r % (N // 2), 2 * N)


class Context:
    def __init__(self, prm, seed: bytes):
        assert len(seed) == 32
        self.prm = prm
        self.seed = seed
        self.serial = 0
        self.N = prm.N
        self.moduli = prm.moduli
        self.psis = prm.psi
        self.s_signed = None
        self.rot_keys = {}

    # ------------------------------------------------------------------ helpers
    def qmods(self, level):
        return self.prm.q[: level + 1]

    def _limb_index_set(self, level):
        """Global limb indices of Q_level u P."""
        L = self.prm.L
        return list(range(level + 1)) + list(range(L + 1, L + 1 + self.prm.alpha))

    def _mods(self, idx):
        return [self.moduli[i] for i in idx]

    def _psis(self, idx):
        return [self.psis[i] for i in idx]

    def mul(self, a, b, idx):
        return ring.polymul(a, b, self._mods(idx), self._psis(idx))

    # ------------------------------------------------------------------- keygen
    def keygen(self, rot_steps=(), conj=False):
        prm, N = self.prm, self.N
        s = sampling.ternary(self.seed, chacha.P_SECRET, 0, N)
        self.s_signed = s
        self.s = ring.from_signed(s, self.moduli)           # all limbs Q u P
        qidx = list(range(prm.L + 1))
        a = np.stack([sampling.uniform_mod(self.seed, chacha.P_PK_A, 0, i, N, prm.q[i])
                      for i in qidx])
        e = sampling.cbd21(self.seed, chacha.P_PK_E, 0, N)
        qm = prm.q
        b = ring.polyadd(ring.polyneg(self.mul(a, self.s[qidx], qidx), qm),
                         ring.from_signed(e, qm), qm)
        self.pk = (b, a)
        s2 = self.mul(self.s[qidx], self.s[qidx], qidx)
        self.relin_key = self.switching_key(s2, 0)
        for r in rot_steps:
            self.add_rotation_key(galois_for_step(r, N))
        if conj:
            self.add_rotation_key(2 * N - 1)

    def add_rotation_key(self, g):
        if g in self.rot_keys:
            return
        qidx = list(range(self.prm.L + 1))
        sg = ring.apply_automorphism(self.s[qidx], g, self.prm.q)
        self.rot_keys[g] = self.switching_key(sg, g)

    def switching_key(self, sprime, key_index):
        """Key digits [(b_j, a_j)] over all limbs for s' (given on Q limbs)."""
        prm, N = self.prm, self.N
        P = rns.prod(prm.p)
        allidx = list(range(len(self.moduli)))
        key = []
        for j, D in prm.digits(prm.L):
            obj = key_index * prm.dnum + j
            a = np.stack([sampling.uniform_mod(self.seed, chacha.P_KSK_A, obj, t, N, self.moduli[t])
                          for t in allidx])
            e = sampling.cbd21(self.seed, chacha.P_KSK_E, obj, N)
            b = ring.polyadd(ring.polyneg(self.mul(a, self.s, allidx), self.moduli),
                             ring.from_signed(e, self.moduli), self.moduli)
            for i in D:
                q = prm.q[i]
                b[i] = addmod(b[i], mulmod(sprime[i], np.uint64(P % q), q), q)
            key.append((j, b, a))
        return key

    # ----------------------------------------------------------- encode/decode
    def encode(self, z, scale):
        """m_n = round_half_even(scale * (2/N) * Re sum_j z_j zeta_j^-n),
        zeta_j = exp(i pi 5^j / N); evaluated with a length-2N FFT."""
        N = self.N
        z = np.asarray(z, dtype=np.float64)
        A = np.zeros(2 * N, dtype=np.complex128)
        pos = self.slot_positions()
        A[pos[: len(z)]] = z
        F = np.fft.fft(A)
        return np.rint(scale * (2.0 / N) * F[:N].real).astype(np.int64)

    def slot_positions(self):
        N = self.N
        out = np.empty(N // 2, dtype=np.int64)
        x = 1
        for j in range(N // 2):
            out[j] = x
            x = x * 5 % (2 * N)
        return out

    def decode(self, m, scale):
        N = self.N
        B = np.zeros(2 * N, dtype=np.complex128)
        B[:N] = np.asarray(m, dtype=np.float64)
        G = np.fft.ifft(B) * (2 * N)
        return G[self.slot_positions()].real / scale

    # --------------------------------------------------------- encrypt/decrypt
    def encrypt_int(self, m, level, scale):
        """Encrypt an integer plaintext polynomial m (length N, signed)."""
        N = self.N
        serial = self.serial
        self.serial += 1
        v = sampling.ternary(self.seed, chacha.P_ENC_V, serial, N)
        e0 = sampling.cbd21(self.seed, chacha.P_ENC_E0, serial, N)
        e1 = sampling.cbd21(self.seed, chacha.P_ENC_E1, serial, N)
        idx = list(range(level + 1))
        qm = self.qmods(level)
        vv = ring.from_signed(v, qm)
        b, a = self.pk
        c0 = ring.polyadd(ring.polyadd(self.mul(vv, b[idx], idx), ring.from_signed(m, qm), qm),
                          ring.from_signed(e0, qm), qm)
        c1 = ring.polyadd(self.mul(vv, a[idx], idx), ring.from_signed(e1, qm), qm)
        return Ciphertext(c0, c1, float(scale))

    def decrypt_int(self, ct):
        q0 = self.prm.q[0]
        m = addmod(ct.c0[0], ring.polymul(ct.c1[:1], self.s[:1], [q0], [self.psis[0]])[0], q0)
        m = m.astype(object)
        return np.array([int(v) - q0 if int(v) > q0 // 2 else int(v) for v in m], dtype=np.int64)

    def encrypt(self, z, level=None, scale=None):
        level = self.prm.L if level is None else level
        scale = self.prm.scale if scale is None else scale
        return self.encrypt_int(self.encode(z, scale), level, scale)

    def decrypt(self, ct):
        return self.decode(self.decrypt_int(ct), ct.scale)

    # ---------------------------------------------------------------- ops
    def mod_drop(self, ct, level):
        if level > ct.level:
            raise CkksError("cannot raise a level")
        return Ciphertext(ct.c0[: level + 1].copy(), ct.c1[: level + 1].copy(), ct.scale)

    def _align(self, a, b):
        lv = min(a.level, b.level)
        if abs(a.scale / b.scale - 1.0) > SCALE_TOL:
            raise ScaleMismatch(f"scales {a.scale} and {b.scale} differ")
        return self.mod_drop(a, lv), self.mod_drop(b, lv)

    def add(self, a, b):
        a, b = self._align(a, b)
        qm = self.qmods(a.level)
        return Ciphertext(ring.polyadd(a.c0, b.c0, qm), ring.polyadd(a.c1, b.c1, qm), a.scale)

    def sub(self, a, b):
        a, b = self._align(a, b)
        qm = self.qmods(a.level)
        return Ciphertext(ring.polysub(a.c0, b.c0, qm), ring.polysub(a.c1, b.c1, qm), a.scale)

    def mul_int(self, ct, w):
        """Multiply by the integer constant w; the scale becomes scale * w."""
        qm = self.qmods(ct.level)
        return Ciphertext(ring.scalar_mul(ct.c0, w, qm), ring.scalar_mul(ct.c1, w, qm),
                          ct.scale * float(w))

    def mul_plain(self, ct, m, pt_scale):
        """ct (x) plaintext polynomial m (signed integer coefficients); Eq. 9."""
        qm = self.qmods(ct.level)
        idx = list(range(ct.level + 1))
        mm = ring.from_signed(m, qm)
        return Ciphertext(self.mul(ct.c0, mm, idx), self.mul(ct.c1, mm, idx), ct.scale * pt_scale)

    def add_plain(self, ct, m):
        qm = self.qmods(ct.level)
        return Ciphertext(ring.polyadd(ct.c0, ring.from_signed(m, qm), qm), ct.c1.copy(), ct.scale)

    def tensor(self, a, b):
        lv = min(a.level, b.level)
        a = self.mod_drop(a, lv)
        b = self.mod_drop(b, lv)
        idx = list(range(lv + 1))
        qm = self.qmods(lv)
        d0 = self.mul(a.c0, b.c0, idx)
        d1 = ring.polyadd(self.mul(a.c0, b.c1, idx), self.mul(a.c1, b.c0, idx), qm)
        d2 = self.mul(a.c1, b.c1, idx)
        return d0, d1, d2, a.scale * b.scale

    def key_switch(self, d, key, level):
        """KS(d) for d over q_0..q_level (coefficient form) -> (u0, u1) over Q_level."""
        return self._ks_inner(self._mod_up_digits(d, level), key, level)

    def _mod_up_digits(self, d, level):
        qm = self.qmods(level)
        return [(j, rns.mod_up(d, qm, D, self.prm.p)) for j, D in self.prm.digits(level)]

    def _ks_inner(self, exts, key, level):
        idx = self._limb_index_set(level)
        mods = self._mods(idx)
        kd = {j: (b, a) for j, b, a in key}
        acc0 = np.zeros((len(idx), self.N), dtype=np.uint64)
        acc1 = np.zeros((len(idx), self.N), dtype=np.uint64)
        for j, ext in exts:
            b, a = kd[j]
            acc0 = ring.polyadd(acc0, self.mul(ext, b[idx], idx), mods)
            acc1 = ring.polyadd(acc1, self.mul(ext, a[idx], idx), mods)
        qm = self.qmods(level)
        return (rns.mod_down(acc0, qm, self.prm.p), rns.mod_down(acc1, qm, self.prm.p))

    def relinearize(self, d0, d1, d2, scale):
        lv = d0.shape[0] - 1
        qm = self.qmods(lv)
        u0, u1 = self.key_switch(d2, self.relin_key, lv)
        return Ciphertext(ring.polyadd(d0, u0, qm), ring.polyadd(d1, u1, qm), scale)

    def rescale(self, ct):
        if ct.level < 1:
            raise CkksError("no level left to rescale")
        qm = self.qmods(ct.level)
        ql = float(qm[-1])
        return Ciphertext(rns.rescale(ct.c0, qm), rns.rescale(ct.c1, qm), ct.scale / ql)

    def hmult(self, a, b):
        """Eq. 7: tensor, relinearise, rescale (in that order)."""
        return self.rescale(self.relinearize(*self.tensor(a, b)))

    def apply_galois(self, ct, g):
        """Rotation by Galois element g, non-hoisted."""
        if g not in self.rot_keys:
            raise CkksError(f"no rotation key for g={g}")
        qm = self.qmods(ct.level)
        c0 = ring.apply_automorphism(ct.c0, g, qm)
        c1 = ring.apply_automorphism(ct.c1, g, qm)
        u0, u1 = self.key_switch(c1, self.rot_keys[g], ct.level)
        return Ciphertext(ring.polyadd(c0, u0, qm), u1, ct.scale)

    def rotate(self, ct, r):
        """Left rotation by r slots (slot j takes old slot j + r)."""
        if r % (self.N // 2) == 0:
            return Ciphertext(ct.c0.copy(), ct.c1.copy(), ct.scale)
        return self.apply_galois(ct, galois_for_step(r, self.N))

    def conjugate(self, ct):
        return self.apply_galois(ct, 2 * self.N - 1)

    def hoisted_rotations(self, ct, steps):
        """Rotations of one ciphertext sharing a single ModUp of c1 (hoisting).
        tau_g is applied to every extended digit; the result is a valid
        encryption of the rotated message but not bit-equal to `rotate`."""
        lv = ct.level
        qm = self.qmods(lv)
        idx = self._limb_index_set(lv)
        mods = self._mods(idx)
        exts = self._mod_up_digits(ct.c1, lv)
        out = {}
        for r in steps:
            if r % (self.N // 2) == 0:
                out[r] = Ciphertext(ct.c0.copy(), ct.c1.copy(), ct.scale)
                continue
            g = galois_for_step(r, self.N)
            if g not in self.rot_keys:
                raise CkksError(f"no rotation key for g={g}")
            exts_g = [(j, ring.apply_automorphism(e, g, mods)) for j, e in exts]
            u0, u1 = self._ks_inner(exts_g, self.rot_keys[g], lv)
            c0 = ring.apply_automorphism(ct.c0, g, qm)
            out[r] = Ciphertext(ring.polyadd(c0, u0, qm), u1, ct.scale)
        return out
