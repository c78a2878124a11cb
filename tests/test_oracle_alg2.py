"""Pins of Alg. 2 (CSR with optimized batching, Sec. III-D) in the oracle:

* the batch-pair grouping on the paper's worked example (batch size 5: pairs
  (UB_0, VB_0) with 4 ratings and (UB_0, VB_1) with 3, user local index 0 three
  times in the first);
* the per-pair accumulator on hand-computed one-factor cases: ratings of one
  pair use the factors of the pair's start, pairs run one after the other,
  lambda is applied once per rating, the dampened rate a' = a / (1 + 0.1 t);
* the encrypted program's index algebra (per-pair rating ciphertexts, gathers
  from one user and one item table, scatters with the per-pair self term, the
  table refreshes between pairs) on plain slot vectors equals the FP64 Alg. 2
  epochs with a batch of D profiles.
"""
import numpy as np
import pytest

from oracle import mf, program
import workloads


def test_worked_example_groups():
    S = [(0, 0), (0, 2), (0, 4), (1, 2), (1, 6), (2, 5), (2, 8)]
    row_ptr = np.array([0, 3, 5, 7])
    col_idx = np.array([j for _, j in S])
    pairs = mf.batch_pairs(row_ptr, col_idx, 5, 5)
    assert [p for p, _ in pairs] == [(0, 0), (0, 1)]
    assert [len(r) for _, r in pairs] == [4, 3]
    rows = mf.csr_rows(row_ptr)
    first = rows[pairs[0][1]] % 5
    assert list(first).count(0) == 3                     # u_0 three times in (UB_0, VB_0)
    assert [S[r] for r in pairs[1][1]] == [(1, 6), (2, 5), (2, 8)]


def _one_factor(u, v):
    return np.array([[x] for x in u], float), np.array([[x] for x in v], float)


def test_pairs_run_in_turn_from_updated_factors():
    # one user, two items, ratings 3 and 2; batches of one entity: pairs (0,0) then (0,1)
    U, V = _one_factor([1.0], [2.0, 1.0])
    U2, V2, rhat = mf.batch_pair_epoch(U, V, [0, 2], [0, 1], [3.0, 2.0], 0.1, 0.0, 1, 1, t=0, damp=0.0)
    # pair (0,0): e = 3 - 1*2 = 1; u = 1 + 0.1*1*2 = 1.2; v0 = 2 + 0.1*1*1 = 2.1
    # pair (0,1) from u = 1.2: e = 2 - 1.2 = 0.8; u = 1.2 + 0.08 = 1.28; v1 = 1 + 0.1*0.8*1.2 = 1.096
    assert np.allclose(U2, [[1.28]]) and np.allclose(V2, [[2.1], [1.096]])
    assert np.allclose(rhat, [2.0, 1.2])


def test_one_pair_is_synchronous_and_accumulates():
    # the same ratings in one pair (batches of two): both errors from the start factors
    U, V = _one_factor([1.0], [2.0, 1.0])
    U2, V2, _ = mf.batch_pair_epoch(U, V, [0, 2], [0, 1], [3.0, 2.0], 0.1, 0.0, 2, 2, t=0, damp=0.0)
    # e = (1, 1); u = 1 + 0.1*(1*2 + 1*1) = 1.3; v0 = 2.1; v1 = 1.1
    assert np.allclose(U2, [[1.3]]) and np.allclose(V2, [[2.1], [1.1]])


def test_lambda_per_rating_and_dampening():
    U, V = _one_factor([1.0], [2.0])
    # grad_u = a'(e v - lambda u) = 0.1 (1*2 - 0.5*1) = 0.15; grad_v = 0.1 (1*1 - 0.5*2) = 0
    U2, V2, _ = mf.batch_pair_epoch(U, V, [0, 1], [0], [3.0], 0.1, 0.5, 1, 1, t=0, damp=0.1)
    assert np.allclose(U2, [[1.15]]) and np.allclose(V2, [[2.0]])
    # epoch t = 5: a' = 0.1 / 1.5
    U3, _, _ = mf.batch_pair_epoch(U, V, [0, 1], [0], [3.0], 0.1, 0.5, 1, 1, t=5, damp=0.1)
    assert np.allclose(U3, [[1.0 + 1.5 * 0.1 / 1.5]])


@pytest.mark.parametrize("N,k,epochs", [(128, 3, 2), (256, 4, 3)])
def test_clear_pair_program_equals_fp64_alg2(N, k, epochs):
    csr = workloads.tiny_ratings()
    U0, V0 = workloads.init_factors(32, 64, k, seed=6)
    lay = program.make_pair_layout(N, k, 32, 64, csr.row_ptr, csr.col_idx)
    assert len(lay.pairs) > 4 and lay.n_utab > 1 and lay.n_vtab > 1
    be = program.ClearBackend(N, [1] + [2 ** 40 + 7] * 9, lay.B, k, L=9)
    S = 2.0 ** 40
    R = [be.wrap(z, 9, S) for z in program.slot_vectors(lay, csr.values, which="R")]
    Ut = [be.wrap(z, 9, S) for z in program.table_vectors(lay, U0, lay.n_utab)]
    Vt = [be.wrap(z, 9, S) for z in program.table_vectors(lay, V0, lay.n_vtab)]
    res = program.run_pair_epochs(be, lay, R, Ut, Vt, epochs, 0.05, 0.02, damp=0.1, exact_weights=True)
    assert res.refresh_round > 0                          # tables were refreshed between pairs
    U = program.decode_tables([v.z for v in res.utab], lay, 32)
    V = program.decode_tables([v.z for v in res.vtab], lay, 64)
    rhat = program.decode_predictions([v.z for v in res.sdot], lay)
    Uf, Vf, rf = mf.train_batch_pairs(U0, V0, csr.row_ptr, csr.col_idx, csr.values, 0.05, 0.02, epochs,
                                      lay.D, lay.D, damp=0.1)
    assert np.max(np.abs(U - Uf)) < 1e-12 and np.max(np.abs(V - Vf)) < 1e-12
    assert np.max(np.abs(rhat - rf)) < 1e-12
