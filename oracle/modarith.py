"""Exact modular arithmetic on numpy uint64 arrays (oracle; test infrastructure only).

All residues are integers in [0, q) with q < 2^62.  The product a*b needs up to
124 bits, which numpy has no integer type for.  ``mulmod`` therefore estimates
the quotient floor(a*b/q) in x87 extended precision (64-bit mantissa) and then
forms the remainder exactly in wrapping uint64 arithmetic:

    quotient estimate  t ~ a*b/q      relative error < 2^-62, so |t - a*b/q| < 1
    remainder          r = a*b - t*q  computed mod 2^64, true value in (-q, 2q)

and one conditional add/subtract of q finishes the reduction.  Because the true
remainder lies in (-2^63, 2^63), reading the wrapped uint64 as int64 is exact.
The routine is checked against Python's unbounded integers in the tests.
"""
import numpy as np

U64 = np.uint64

if np.finfo(np.longdouble).nmant < 63:  # pragma: no cover - platform guard
    raise RuntimeError("oracle.modarith needs an 80-bit long double (x86-64)")


def as_u64(x):
    return np.asarray(x, dtype=np.uint64)


def addmod(a, b, q):
    """(a + b) mod q for a, b in [0, q), q < 2^63."""
    a = as_u64(a)
    b = as_u64(b)
    q = as_u64(q)
    s = a + b
    return np.where(s >= q, s - q, s)


def submod(a, b, q):
    """(a - b) mod q for a, b in [0, q)."""
    a = as_u64(a)
    b = as_u64(b)
    q = as_u64(q)
    return np.where(a >= b, a - b, a + (q - b))


def negmod(a, q):
    a = as_u64(a)
    q = as_u64(q)
    return np.where(a == 0, a, q - a)


def mulmod(a, b, q):
    """(a * b) mod q, elementwise with broadcasting; requires a, b < 2^62 and
    a*b/q < 2^62 (true whenever a, b < q < 2^62)."""
    a = as_u64(a)
    b = as_u64(b)
    qq = as_u64(q)
    est = np.floor(a.astype(np.longdouble) * b.astype(np.longdouble) / qq.astype(np.longdouble))
    t = est.astype(np.uint64)
    with np.errstate(over="ignore"):
        r = (a * b - t * qq).view(np.int64)
    qi = qq.astype(np.int64)
    r = np.where(r < 0, r + qi, r)
    r = np.where(r >= qi, r - qi, r)
    return r.astype(np.uint64)


def reduce_signed(x, q):
    """Map signed integers (int64 array, or Python ints via object arrays) to [0, q)."""
    x = np.asarray(x)
    if x.dtype == object:
        return np.array([int(v) % int(q) for v in x.ravel()], dtype=np.uint64).reshape(x.shape)
    x = x.astype(np.int64)
    qi = np.int64(q)
    r = np.remainder(x, qi)
    return r.astype(np.uint64)


def powmod(base, e, q):
    return pow(int(base), int(e), int(q))


def invmod(a, q):
    return pow(int(a), -1, int(q))
