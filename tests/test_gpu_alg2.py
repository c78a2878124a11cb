"""GPU runs of Alg. 2 (user-item batch pairs, Sec. III-D; params.batch_pairs = 1):

* one epoch on the two-pair workload of tests/golden/make_alg2_tiny2.py (the
  second pair starts from the first's user table, the tables are refreshed
  between the pairs): every output ciphertext equals the oracle's, through the
  stored digests;
* three epochs at the MovieLens-100K shape (8 batch pairs per epoch,
  refreshes as the levels run out): decrypted factors and predictions within
  1e-4 of the FP64 Alg. 2 epochs at learning rate 0.001.  The bound is the
  precision of the method's fixed-point masks: the block indicators are
  encoded as integers at scale 2^24 (scatter) and 2^30 (gather), so a masked
  slot is off by about sqrt(N/24)/2^24 (2e-6 at N = 2^15) of the value it
  moves, and over the sequential pairs that error grows with the factor
  magnitudes and the learning rate.
  A cleartext model of the masks and integer weights alone (no encryption)
  gives 1.1e-5 at rate 0.001 and 5e-4 / 1.3e-3 (U / V) at rate 0.005; the
  GPU matched the latter to four digits.
"""
import os

import numpy as np
import pytest

from oracle import ckks, mf, program
import workloads
from tests.golden import make_alg2_tiny2 as gold
from tests.golden.make_ks_n16 import read

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def test_alg2_epoch_bit_exact_against_oracle():
    import paper_2509_03024_amd as pk
    golden = read(os.path.join(HERE, "golden", "alg2_tiny2.txt"))
    prm, csr, U0, V0, lay = gold.setup()
    orc = ckks.Context(prm, workloads.CRYPTO_SEED)          # the oracle's encoder supplies the integers
    pt = gold.plaintexts(orc, lay, csr, U0, V0)
    masks = program.block_masks(orc, gold.K)
    ctx = pk.Context(pk.params(12, 60, 7, 40, 2, 60, 4, 40, k=gold.K, lr=gold.LR, lam=gold.LAM, damp=gold.DAMP,
                               rule=1, refresh_mode=1, batch_pairs=1), workloads.CRYPTO_SEED)
    ctx.keygen([])
    m = pk.MF(ctx)
    assert m.encrypt_csr_rows_int(csr.n_rows, csr.n_cols, csr.row_ptr, csr.col_idx, np.stack(pt["R"])) == lay.n_ct
    m.init_factors_int(np.stack(pt["Utab"]), np.stack(pt["Vtab"]), np.stack(pt["Ug"]), np.stack(pt["Vg"]),
                       masks[program.S_I], masks[program.S_IG], gold.K)
    m.epochs(1)
    assert m.stats()["refreshes"] == 1
    for kind, which in (("utab", 1), ("vtab", 2), ("sdot", 5)):
        hs = m.handles(which)
        for i, h in enumerate(hs):
            got, lvl, scale = ctx.export_ct(h)
            want = golden[(kind, i)]
            assert (lvl, scale) == want[:2], (kind, i)
            assert gold.digest(got[0], got[1]) == want[2], f"{kind} {i} differs from the oracle's"
    ctx.close()


def test_alg2_mf100k_within_1e4_of_fp64():
    import paper_2509_03024_amd as pk
    K, LR, LAM, EP = 10, 0.001, 0.02, 3
    csr = workloads.movielens100k_shaped()
    U0, V0 = workloads.init_factors(csr.n_rows, csr.n_cols, K)
    ctx = pk.Context(pk.params(15, 60, 16, 40, 3, 60, 5, 40, k=K, lr=LR, lam=LAM, damp=0.1, rule=1,
                               refresh_mode=1, batch_pairs=1), workloads.CRYPTO_SEED)
    ctx.keygen([])
    m = pk.MF(ctx)
    m.encrypt_csr_rows(csr.n_rows, csr.n_cols, csr.row_ptr, csr.col_idx, csr.values)
    m.init_factors(U0, V0)
    m.epochs(EP)
    U, V = m.decrypt_factors()
    rhat = m.decrypt_predictions(0)
    D = m.layout()["D"]
    Uf, Vf, rf = mf.train_batch_pairs(U0, V0, csr.row_ptr, csr.col_idx, csr.values, LR, LAM, EP, D, D, damp=0.1)
    print("Alg. 2, 3 epochs: max |U-Uf|", np.max(np.abs(U - Uf)), "max |V-Vf|", np.max(np.abs(V - Vf)),
          "max |rhat-rf|", np.max(np.abs(rhat - rf)), "refreshes", m.stats()["refreshes"])
    assert np.max(np.abs(U - Uf)) < 1e-4
    assert np.max(np.abs(V - Vf)) < 1e-4
    assert np.max(np.abs(rhat - rf)) < 1e-4
    ctx.close()
