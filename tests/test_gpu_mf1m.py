"""Encrypted MF at the MovieLens-1M-shaped workload (6040 x 3706, ~0.89 M
ratings, k = 16, N = 2^16, 25 limbs, dnum 7, rule R2): five epochs without
refresh (3 + 4*4 = 19 of 24 levels); decrypted factors and forward
predictions within 1e-4 of the FP64 synchronous epochs (oracle.mf)."""
import numpy as np
import pytest

from oracle import mf
import workloads

pytestmark = pytest.mark.gpu

K, LR, LAM, EPOCHS = 16, 0.01, 0.02, 5


def test_mf1m_five_epochs_within_1e4_of_fp64():
    import paper_2509_03024_amd as pk
    csr = workloads.movielens1m_shaped()
    U0, V0 = workloads.init_factors(csr.n_rows, csr.n_cols, K)
    ctx = pk.Context(pk.mf_n16_params(k=K, lr=LR, lam=LAM, rule=2), workloads.CRYPTO_SEED)
    ctx.keygen([])
    m = pk.MF(ctx)
    n_ct = m.encrypt_csr_rows(csr.n_rows, csr.n_cols, csr.row_ptr, csr.col_idx, csr.values)
    print("rating ciphertexts", n_ct, flush=True)
    m.init_factors(U0, V0)
    m.epochs(EPOCHS)
    U, V = m.decrypt_factors()
    rhat = m.decrypt_predictions(0)
    Uf, Vf, rf = mf.train(U0, V0, csr.row_ptr, csr.col_idx, csr.values, LR, LAM, EPOCHS, rule="R2")
    print("max |U-Uf|", np.max(np.abs(U - Uf)), "max |V-Vf|", np.max(np.abs(V - Vf)),
          "max |rhat-rf|", np.max(np.abs(rhat - rf)), flush=True)
    assert np.max(np.abs(U - Uf)) < 1e-4
    assert np.max(np.abs(V - Vf)) < 1e-4
    assert np.max(np.abs(rhat - rf)) < 1e-4
    ctx.close()
