"""GPU parity of the encrypted MF program on a degenerate CSR matrix
(workloads.edge_ratings(): empty rows and columns, single-rating rows, a row
of 1030 ratings cut across two ciphertexts, the first and the last item) with
k = 1 at the tiny chain: one epoch (rule R1) gives the oracle's output
ciphertexts bit for bit (digests written by tests/golden/make_mf_edge.py from
the oracle alone), and the decrypted factors are within 1e-4 of FP64 MF, the
factors of users and items without ratings unchanged within that bound."""
import os

import numpy as np
import pytest

from oracle import ckks, mf, program
import workloads
from tests.golden import make_mf_edge as gold

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def test_degenerate_csr_bit_exact_and_within_1e4():
    import paper_2509_03024_amd as pk
    golden = gold.read(os.path.join(HERE, "golden", "mf_edge_n12_k1.txt"))
    prm, csr, U0, V0, lay = gold.setup()
    orc = ckks.Context(prm, workloads.CRYPTO_SEED)          # the oracle's encoder supplies the integers
    pt = gold.plaintexts(orc, lay, csr, U0, V0)
    masks = program.block_masks(orc, gold.K)
    ctx = pk.Context(pk.tiny_params(k=gold.K, lr=gold.LR, lam=gold.LAM, rule=1), workloads.CRYPTO_SEED)
    ctx.keygen([])
    m = pk.MF(ctx)
    assert m.encrypt_csr_rows_int(csr.n_rows, csr.n_cols, csr.row_ptr, csr.col_idx, np.stack(pt["R"])) == 3
    m.init_factors_int(np.stack(pt["Utab"]), np.stack(pt["Vtab"]), np.stack(pt["Ug"]), np.stack(pt["Vg"]),
                       masks[program.S_I], masks[program.S_IG], gold.K)
    m.epochs(1)
    n = 0
    for kind, which in (("utab", 1), ("vtab", 2), ("sdot", 5)):
        for i, h in enumerate(m.handles(which)):
            got, lvl, scale = ctx.export_ct(h)
            want = golden[(kind, i)]
            assert (lvl, scale) == want[:2], (kind, i)
            assert gold.digest(got[0], got[1]) == want[2], f"{kind} {i} differs from the oracle's"
            n += 1
    assert n == len(golden)
    U, V = m.decrypt_factors()
    Uf, Vf, _ = mf.train(U0, V0, csr.row_ptr, csr.col_idx, csr.values, gold.LR, gold.LAM, 1, rule="R1")
    assert np.max(np.abs(U - Uf)) < 1e-4 and np.max(np.abs(V - Vf)) < 1e-4
    empty_users = np.diff(csr.row_ptr) == 0
    empty_items = np.bincount(csr.col_idx, minlength=csr.n_cols) == 0
    assert np.max(np.abs(U[empty_users] - U0[empty_users])) < 1e-4
    assert np.max(np.abs(V[empty_items] - V0[empty_items])) < 1e-4
    ctx.close()
