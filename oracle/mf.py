"""FP64 CSR matrix factorisation (oracle; test infrastructure only).

Notation of Sec. II-A.1: n users (rows), m items (columns), k latent factors,
U (n x k), V (m x k), NZR the set of observed ratings, M = |NZR|.

``loss_eq1`` and ``grad_eq4_eq5`` are Eq. 1 and Eq. 4-5 written out.

``epoch`` is one synchronous gradient step, the reading of Alg. 1 used by the
encrypted path: every rating's error uses the factors at the start of the
epoch (the schedule of Eq. 2-3), and all per-rating gradient terms of one user
or item are summed before being applied once (the accumulator of Alg. 2).  As
in Alg. 1 and Alg. 2 there is no 1/M and one lambda serves users and items.
Two update rules:

R1  (Alg. 1 summed over the epoch; lambda applied once per rating)
    u_i <- (1 - a_t*lambda*d_i) u_i + a_t * sum_{j in row i} e_ij v_j
    v_j <- (1 - a_t*lambda*c_j) v_j + a_t * sum_{i in col j} e_ij u_i
R2  (degree-normalised; empty rows/columns unchanged)
    u_i <- (1 - a_t*lambda) u_i + (a_t/d_i) * sum_j e_ij v_j      (same for v_j)

with e_ij = r_ij - <u_i, v_j>, d_i the row length, c_j the column count and the
dampened rate a_t = alpha / (1 + damp*t) of Alg. 2 (t = epoch index from 0,
damp = 0 reproduces the undampened Alg. 1).
"""
import numpy as np


def csr_rows(row_ptr):
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    return np.repeat(np.arange(len(row_ptr) - 1), np.diff(row_ptr))


def predict(U, V, row_ptr, col_idx):
    """r_hat_ij = <u_i, v_j> for every stored rating, in CSR order."""
    rows = csr_rows(row_ptr)
    return np.einsum("ij,ij->i", U[rows], V[np.asarray(col_idx)])


def rmse(rhat, r):
    """Eq. 10."""
    rhat = np.asarray(rhat, np.float64)
    r = np.asarray(r, np.float64)
    return float(np.sqrt(np.mean((rhat - r) ** 2)))


def loss_eq1(U, V, row_ptr, col_idx, vals, lam, mu):
    """Eq. 1: (1/M) sum (r - <u,v>)^2 + lam sum ||u_i||^2 + mu sum ||v_j||^2."""
    e = np.asarray(vals) - predict(U, V, row_ptr, col_idx)
    return float(np.mean(e ** 2) + lam * np.sum(U ** 2) + mu * np.sum(V ** 2))


def grad_eq4_eq5(U, V, row_ptr, col_idx, vals, lam, mu):
    """Eq. 4-5 as printed: (1/M) sum_j v_j (<u_i,v_j> - r_ij) + lam u_i, and the item analogue."""
    rows = csr_rows(row_ptr)
    cols = np.asarray(col_idx)
    M = len(vals)
    e = predict(U, V, row_ptr, col_idx) - np.asarray(vals)
    gU = np.zeros_like(U)
    gV = np.zeros_like(V)
    np.add.at(gU, rows, e[:, None] * V[cols])
    np.add.at(gV, cols, e[:, None] * U[rows])
    return gU / M + lam * U, gV / M + mu * V


def epoch(U, V, row_ptr, col_idx, vals, alpha, lam, t=0, damp=0.0, rule="R1"):
    """One synchronous epoch; returns (U', V', forward predictions at the epoch start)."""
    rows = csr_rows(row_ptr)
    cols = np.asarray(col_idx)
    n, m = U.shape[0], V.shape[0]
    a_t = alpha / (1.0 + damp * t)
    rhat = predict(U, V, row_ptr, col_idx)
    e = np.asarray(vals, np.float64) - rhat
    sU = np.zeros_like(U)
    sV = np.zeros_like(V)
    np.add.at(sU, rows, e[:, None] * V[cols])
    np.add.at(sV, cols, e[:, None] * U[rows])
    d = np.bincount(rows, minlength=n).astype(np.float64)
    c = np.bincount(cols, minlength=m).astype(np.float64)
    if rule == "R1":
        U2 = (1.0 - a_t * lam * d)[:, None] * U + a_t * sU
        V2 = (1.0 - a_t * lam * c)[:, None] * V + a_t * sV
    elif rule == "R2":
        dU = np.where(d > 0, 1.0 / np.maximum(d, 1), 0.0)
        dV = np.where(c > 0, 1.0 / np.maximum(c, 1), 0.0)
        U2 = np.where((d > 0)[:, None], (1.0 - a_t * lam) * U + (a_t * dU)[:, None] * sU, U)
        V2 = np.where((c > 0)[:, None], (1.0 - a_t * lam) * V + (a_t * dV)[:, None] * sV, V)
    else:
        raise ValueError(rule)
    return U2, V2, rhat


def train(U, V, row_ptr, col_idx, vals, alpha, lam, epochs, damp=0.0, rule="R1"):
    """Run `epochs` synchronous epochs; returns (U, V, forward predictions of the last epoch)."""
    rhat = None
    for t in range(epochs):
        U, V, rhat = epoch(U, V, row_ptr, col_idx, vals, alpha, lam, t, damp, rule)
    return U, V, rhat


def sequential_alg1(U, V, row_ptr, col_idx, vals, alpha, lam, epochs):
    """Alg. 1 taken literally: the factors change after every single rating.
    Kept for comparison with the synchronous schedule; not what the encrypted
    path evaluates (a leveled scheme cannot chain that many dependent products)."""
    U = U.copy()
    V = V.copy()
    rows = csr_rows(row_ptr)
    for _ in range(epochs):
        for idx, (i, j) in enumerate(zip(rows, col_idx)):
            err = vals[idx] - U[i] @ V[j]
            gu = err * V[j] - lam * U[i]
            gv = err * U[i] - lam * V[j]
            U[i] = U[i] + alpha * gu
            V[j] = V[j] + alpha * gv
    return U, V


# ---------------------------------------------------------------- Alg. 2: user-item batch pairs
def batch_pairs(row_ptr, col_idx, u_batch, v_batch):
    """Group the ratings by user-item batch pair (Sec. III-D): user i is in
    user batch i // u_batch at local index i % u_batch, item j likewise with
    v_batch.  Returns [((ub, vb), [rating indices in CSR order])] with the
    pairs in order of their first rating in CSR order (the order in which the
    grouping of Alg. 2 meets them)."""
    rows = csr_rows(row_ptr)
    groups = {}
    for r, (i, j) in enumerate(zip(rows, np.asarray(col_idx))):
        groups.setdefault((int(i) // u_batch, int(j) // v_batch), []).append(r)
    return list(groups.items())


def batch_pair_epoch(U, V, row_ptr, col_idx, vals, alpha, lam, u_batch, v_batch, t=0, damp=0.1):
    """One epoch of Alg. 2: for each batch pair in turn, every rating of the
    pair uses the factors as they are when the pair starts; the per-rating
    terms grad_u = a'(e v - lambda u), grad_v = a'(e u - lambda v) are summed
    per local index (the accumulators) and added to the batch once the pair's
    ratings are done, before the next pair; a' = alpha / (1 + damp * t).
    Returns (U', V', predictions of each rating at the start of its pair)."""
    U = np.array(U, np.float64, copy=True)
    V = np.array(V, np.float64, copy=True)
    rows = csr_rows(row_ptr)
    cols = np.asarray(col_idx)
    vals = np.asarray(vals, np.float64)
    a_t = alpha / (1.0 + damp * t)
    rhat = np.zeros(len(vals))
    for _, idx in batch_pairs(row_ptr, col_idx, u_batch, v_batch):
        idx = np.asarray(idx)
        i, j = rows[idx], cols[idx]
        p = np.einsum("ij,ij->i", U[i], V[j])
        rhat[idx] = p
        e = vals[idx] - p
        dU = np.zeros_like(U)
        dV = np.zeros_like(V)
        np.add.at(dU, i, a_t * (e[:, None] * V[j] - lam * U[i]))
        np.add.at(dV, j, a_t * (e[:, None] * U[i] - lam * V[j]))
        U += dU
        V += dV
    return U, V, rhat


def train_batch_pairs(U, V, row_ptr, col_idx, vals, alpha, lam, epochs, u_batch, v_batch, damp=0.1):
    """`epochs` epochs of Alg. 2; returns (U, V, predictions of the last epoch)."""
    rhat = None
    for t in range(epochs):
        U, V, rhat = batch_pair_epoch(U, V, row_ptr, col_idx, vals, alpha, lam, u_batch, v_batch, t, damp)
    return U, V, rhat
