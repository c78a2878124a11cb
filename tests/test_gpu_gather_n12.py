"""GPU parity of block permutations with large baby steps: encrypted
predictions (both gathers, the product and the windowed sum) of a workload
at N = 2^12 with k = 1 (D = 1024) whose gathers choose G = 128, so babies run
up to beta = 127 in two blocks of 64.  Sampled prediction ciphertexts are
compared with the oracle's digests (tests/golden/make_gather_n12_k1.py), all
predictions are checked against <u_i, v_j> within 1e-4, and the result does
not depend on how many babies the library keeps alive at once (checked at
the MovieLens-100K shape, where the scatters have ~200 sources)."""
import os

import numpy as np
import pytest

from oracle import ckks, program
import workloads
from tests.golden import make_gather_n12_k1 as gold
from tests.golden.make_ks_n16 import read

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _run(budget=None):
    import paper_2509_03024_amd as pk
    prm, csr, U0, V0, lay = gold.setup()
    orc = ckks.Context(prm, workloads.CRYPTO_SEED)      # the oracle's encoder supplies the integers
    S = 2.0 ** 40
    enc = lambda Z: np.stack([orc.encode(z, S) for z in Z])
    masks = program.block_masks(orc, gold.K)
    ctx = pk.Context(pk.tiny_params(k=gold.K), workloads.CRYPTO_SEED)
    ctx.keygen([])
    m = pk.MF(ctx)
    if budget is not None:
        m.set_baby_budget(budget)
    n_ct = m.encrypt_csr_rows_int(csr.n_rows, csr.n_cols, csr.row_ptr, csr.col_idx,
                                  enc(program.slot_vectors(lay, csr.values, which="R")))
    assert n_ct == lay.n_ct == 16
    m.init_factors_int(enc(program.table_vectors(lay, U0, lay.n_utab)), enc(program.table_vectors(lay, V0, lay.n_vtab)),
                       enc(program.slot_vectors(lay, users=U0, which="U")),
                       enc(program.slot_vectors(lay, items=V0, which="V")),
                       masks[program.S_I], masks[program.S_IG], gold.K)
    m.predict()
    return ctx, m, csr, U0, V0


def test_predictions_with_g128_gathers_match_oracle():
    golden = read(os.path.join(HERE, "golden", "gather_n12_k1.txt"))
    ctx, m, csr, U0, V0 = _run()
    hs = m.handles(6)
    for c in gold.SAMPLE_CTS:
        got, lvl, scale = ctx.export_ct(hs[c])
        want = golden[("pred", c)]
        assert (lvl, scale) == want[:2]
        assert gold.digest(got[0], got[1]) == want[2], f"prediction ciphertext {c} differs from the oracle's"
    rhat = m.decrypt_predictions(1)
    rows = np.repeat(np.arange(csr.n_rows), np.diff(csr.row_ptr))
    want = np.sum(U0[rows] * V0[csr.col_idx], axis=1)
    assert np.max(np.abs(rhat - want)) < 1e-4
    ctx.close()


def _mf100k(budget):
    import paper_2509_03024_amd as pk
    csr = workloads.movielens100k_shaped()
    U0, V0 = workloads.init_factors(csr.n_rows, csr.n_cols, 10)
    ctx = pk.Context(pk.mf_n15_params(k=10, lr=0.01, lam=0.02, rule=2), workloads.CRYPTO_SEED)
    ctx.keygen([])
    m = pk.MF(ctx)
    if budget is not None:
        m.set_baby_budget(budget)
    m.encrypt_csr_rows(csr.n_rows, csr.n_cols, csr.row_ptr, csr.col_idx, csr.values)
    m.init_factors(U0, V0)
    m.epochs(1)
    m.predict()
    return ctx, m


def test_baby_budget_does_not_change_bits():
    """At the MovieLens-100K shape, the scatters of an epoch (~200 sources) and
    the gathers of a prediction (G = 128 / 256) run with the default budget
    and with 64 babies alive (many more source chunks): every table and
    prediction ciphertext is the same."""
    ctx1, m1 = _mf100k(None)
    ctx2, m2 = _mf100k(64)
    for which in (1, 2, 6):
        for h1, h2 in zip(m1.handles(which), m2.handles(which)):
            a, l1, s1 = ctx1.export_ct(h1)
            b, l2, s2 = ctx2.export_ct(h2)
            assert (l1, s1) == (l2, s2) and np.array_equal(a, b), which
    ctx1.close()
    ctx2.close()
