"""Negacyclic polynomial arithmetic in Z_q[X]/(X^N + 1) (oracle; test infrastructure only).

A polynomial in RNS form is a uint64 array of shape [n_limbs, N] in coefficient
form, row i holding the residues mod moduli[i].

Products use the textbook route: the negacyclic product equals a cyclic
convolution after the "twist" a_n -> a_n psi^n with psi a primitive 2N-th root
(psi^N = -1), and the cyclic convolution is done by a radix-2 decimation-in-time
DFT over Z_q with omega = psi^2.  Nothing here is fused or reordered beyond
that; the GPU path uses its own, unrelated transform.  The tests pin this
against an exact schoolbook product computed with Python big integers.
"""
import numpy as np

from .modarith import addmod, submod, mulmod, negmod, reduce_signed

_tables = {}


def _bitrev(N):
    logn = N.bit_length() - 1
    r = np.zeros(N, dtype=np.int64)
    for i in range(N):
        x = i
        y = 0
        for _ in range(logn):
            y = (y << 1) | (x & 1)
            x >>= 1
        r[i] = y
    return r


def _pow_table(base, n, q):
    out = np.empty(n, dtype=np.uint64)
    x = 1
    for i in range(n):
        out[i] = x
        x = x * base % q
    return out


def _get_tables(N, q, psi):
    key = (N, q, psi)
    t = _tables.get(key)
    if t is None:
        omega = psi * psi % q
        t = {
            "twist": _pow_table(psi, N, q),
            "untwist": _pow_table(pow(psi, -1, q), N, q),
            "omega": omega,
            "omega_inv": pow(omega, -1, q),
            "n_inv": pow(N, -1, q),
            "bitrev": _bitrev_cached(N),
        }
        _tables[key] = t
    return t


_br = {}


def _bitrev_cached(N):
    if N not in _br:
        _br[N] = _bitrev(N)
    return _br[N]


_stw = {}


def _stage_twiddles(omega, N, m, q):
    key = (omega, N, m, q)
    if key not in _stw:
        _stw[key] = _pow_table(pow(omega, N // (2 * m), q), m, q)
    return _stw[key]


def _cyclic_dft(a, omega, q):
    """Radix-2 DIT DFT over Z_q: A_t = sum_n a_n omega^(t n); natural order in and out."""
    N = a.shape[-1]
    x = a[..., _bitrev_cached(N)].copy()
    m = 1
    while m < N:
        w = _stage_twiddles(omega, N, m, q)
        x = x.reshape(x.shape[:-1] + (N // (2 * m), 2 * m))
        lo = x[..., :m]
        hi = mulmod(x[..., m:], w, q)
        x = np.concatenate([addmod(lo, hi, q), submod(lo, hi, q)], axis=-1)
        x = x.reshape(x.shape[:-2] + (N,))
        m *= 2
    return x


def ntt(a, q, psi):
    """Negacyclic transform of one limb: A_t = sum_n a_n psi^((2t+1) n) mod q."""
    N = a.shape[-1]
    t = _get_tables(N, q, psi)
    return _cyclic_dft(mulmod(a, t["twist"], q), t["omega"], q)


def intt(A, q, psi):
    N = A.shape[-1]
    t = _get_tables(N, q, psi)
    a = _cyclic_dft(A, t["omega_inv"], q)
    a = mulmod(a, np.uint64(t["n_inv"]), q)
    return mulmod(a, t["untwist"], q)


def polymul(a, b, moduli, psis):
    """Negacyclic product of two RNS polynomials [n_limbs, N] (coefficient form)."""
    out = np.empty_like(a)
    for i, (q, psi) in enumerate(zip(moduli, psis)):
        A = ntt(a[i], q, psi)
        B = ntt(b[i], q, psi)
        out[i] = intt(mulmod(A, B, q), q, psi)
    return out


def polyadd(a, b, moduli):
    return np.stack([addmod(a[i], b[i], q) for i, q in enumerate(moduli)])


def polysub(a, b, moduli):
    return np.stack([submod(a[i], b[i], q) for i, q in enumerate(moduli)])


def polyneg(a, moduli):
    return np.stack([negmod(a[i], q) for i, q in enumerate(moduli)])


def scalar_mul(a, c, moduli):
    """Multiply by an integer constant c (any sign)."""
    return np.stack([mulmod(a[i], np.uint64(int(c) % q), q) for i, q in enumerate(moduli)])


def from_signed(x, moduli):
    """Signed integer coefficient vector -> RNS polynomial."""
    return np.stack([reduce_signed(x, q) for q in moduli])


def automorphism_map(g, N):
    """tau_g : X -> X^g on coefficient form.  Coefficient n moves to n*g mod 2N,
    negated when that index is >= N (X^N = -1).  Returns (destination, negate)."""
    n = np.arange(N, dtype=np.int64)
    t = (n * g) % (2 * N)
    neg = t >= N
    dst = np.where(neg, t - N, t)
    return dst, neg


def apply_automorphism(a, g, moduli):
    N = a.shape[-1]
    dst, neg = automorphism_map(g, N)
    out = np.empty_like(a)
    for i, q in enumerate(moduli):
        v = a[i]
        v = np.where(neg, negmod(v, q), v)
        out[i, dst] = v
    return out
