"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws inputs (rating matrices in CSR form, initial factors,
random residues, request streams).  It holds none of the method's arithmetic.
MovieLens is not available here; the larger matrices are synthetic stand-ins
with the shapes and value distributions of the paper's workload (Sec. IV-A).
"""
import hashlib
from dataclasses import dataclass

import numpy as np

CRYPTO_SEED = hashlib.sha256(b"csrmf-2509.03024").digest()


@dataclass
class Csr:
    n_rows: int
    n_cols: int
    row_ptr: np.ndarray   # int64 [n_rows + 1]
    col_idx: np.ndarray   # int32 [nnz], sorted within each row
    values: np.ndarray    # float64 [nnz]

    @property
    def nnz(self):
        return int(self.row_ptr[-1])


def _csr_from_cells(n, m, rows, cols, vals):
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    return Csr(n, m, np.cumsum(row_ptr), cols.astype(np.int32), vals.astype(np.float64))


def tiny_ratings(seed=0, n=32, m=64, density=0.10):
    """32 x 64, exactly round(0.1*n*m) distinct cells uniform without replacement,
    ratings uniform integers 1..5."""
    rng = np.random.default_rng(seed)
    nnz = int(round(density * n * m))
    cells = rng.choice(n * m, size=nnz, replace=False)
    vals = rng.integers(1, 6, size=nnz).astype(np.float64)
    return _csr_from_cells(n, m, cells // m, cells % m, vals)


def edge_ratings():
    """8 users x 1100 items with the degenerate shapes of a CSR matrix: empty
    rows (users 0, 3, 6), single-rating rows (1, 7), a row of 1030 ratings
    (longer than the 1024 blocks of one ciphertext at N = 2^12, k = 1, so it is
    cut in chunks of 1024 and 6), short rows (4, 5), empty columns
    (1030..1097), and the first and last item; ratings uniform integers 1..5
    (numpy PCG64 seed 3)."""
    rng = np.random.default_rng(3)
    rows_items = {1: [5], 2: list(range(1030)), 4: [7, 1098, 1099], 5: [17, 1029], 7: [1099]}
    rows = np.concatenate([np.full(len(v), u) for u, v in rows_items.items()])
    cols = np.concatenate([np.asarray(v) for v in rows_items.values()])
    vals = rng.integers(1, 6, size=len(rows)).astype(np.float64)
    return _csr_from_cells(8, 1100, rows, cols, vals)


def init_factors(n, m, k, seed=1, sigma=0.1):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, sigma, (n, k)), rng.normal(0.0, sigma, (m, k))


def _zipf_items(rng, m, a):
    w = np.arange(1, m + 1, dtype=np.float64) ** (-a)
    perm = rng.permutation(m)
    weights = np.empty(m)
    weights[perm] = w
    return weights


def _rows_weighted_without_replacement(rng, weights, lengths):
    """Each row draws `length` distinct items with probability proportional to the
    weights (Efraimidis-Spirakis keys u^(1/w), top-d)."""
    m = len(weights)
    cols = []
    for d in lengths:
        u = rng.random(m)
        keys = np.log(u) / weights
        cols.append(np.sort(np.argpartition(-keys, d - 1)[:d]))
    return cols


def _ratings(rng, size):
    return np.rint(np.clip(rng.normal(3.5, 1.1, size), 1.0, 5.0))


def lognormal_rows(rng, n, mu, sigma, lo, hi):
    return np.clip(np.rint(rng.lognormal(mu, sigma, n)), lo, hi).astype(np.int64)


def movielens100k_shaped(seed=0):
    """943 x 1682 at 6.3% density (99,926 ratings); row lengths
    clip(round(lognormal(mu, 1)), 20, 1682) with mu fitted by bisection so the
    lengths sum to the target; Zipf(1.0) item popularity."""
    n, m = 943, 1682
    target = int(round(0.063 * n * m))
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(n)
    lo, hi = 0.0, 8.0
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        s = np.clip(np.rint(np.exp(mid + z)), 20, m).sum()
        if s < target:
            lo = mid
        else:
            hi = mid
    lengths = np.clip(np.rint(np.exp(hi + z)), 20, m).astype(np.int64)
    # fix the sum exactly by nudging the longest rows
    diff = int(lengths.sum() - target)
    order = np.argsort(-lengths)
    i = 0
    while diff != 0:
        j = order[i % n]
        step = 1 if diff > 0 else -1
        if 20 <= lengths[j] - step <= m:
            lengths[j] -= step
            diff -= step
        i += 1
    weights = _zipf_items(rng, m, 1.0)
    cols = _rows_weighted_without_replacement(rng, weights, lengths)
    rows = np.repeat(np.arange(n), lengths)
    cc = np.concatenate(cols)
    return _csr_from_cells(n, m, rows, cc, _ratings(rng, len(cc)))


def movielens1m_shaped(seed=0):
    """6040 x 3706; row lengths clip(round(lognormal(4.5, 1)), 20, 2000); Zipf(1.1)."""
    n, m = 6040, 3706
    rng = np.random.default_rng(seed)
    lengths = lognormal_rows(rng, n, 4.5, 1.0, 20, 2000)
    weights = _zipf_items(rng, m, 1.1)
    cols = _rows_weighted_without_replacement(rng, weights, lengths)
    rows = np.repeat(np.arange(n), lengths)
    cc = np.concatenate(cols)
    return _csr_from_cells(n, m, rows, cc, _ratings(rng, len(cc)))


def random_residues(moduli, N, count, seed=11):
    """`count` polynomials of uniform residues, shape [count, len(moduli), N]."""
    rng = np.random.default_rng(seed)
    out = np.empty((count, len(moduli), N), dtype=np.uint64)
    for i, q in enumerate(moduli):
        out[:, i, :] = rng.integers(0, int(q), size=(count, N), dtype=np.uint64)
    return out
