"""GPU parity of the encrypted MF program at the tiny configuration (N=2^12,
32 users x 64 items, 205 ratings, k=4, 1 epoch, rule R1): every output
ciphertext is compared bit for bit with the oracle's (same seed, same integer
plaintexts, same serial order), and the decrypted factors and predictions are
checked against FP64 MF within 1e-4."""
import numpy as np
import pytest

from oracle import ckks, mf, params, program
import workloads
from tests.test_oracle_program import run_encrypted_tiny

pytestmark = pytest.mark.gpu


def _same(lib, h, o):
    got, lvl, scale = lib.export_ct(h)
    assert lvl == o.level and scale == o.scale
    assert np.array_equal(got[0], o.c0) and np.array_equal(got[1], o.c1)


@pytest.fixture(scope="module")
def tiny_run():
    import paper_2509_03024_amd as pk
    csr = workloads.tiny_ratings()
    U0, V0 = workloads.init_factors(32, 64, 4)
    prm = params.config_tiny()
    lay = program.make_layout(prm.N, 4, 32, 64, csr.row_ptr, csr.col_idx)
    steps = program.rotation_steps(lay)
    orc = ckks.Context(prm, workloads.CRYPTO_SEED)
    orc.keygen(rot_steps=steps)
    masks = program.block_masks(orc, 4)
    lay, ores, pt = run_encrypted_tiny(orc, csr, U0, V0, masks)

    ctx = pk.Context(pk.tiny_params(k=4, lr=0.01, lam=0.02, rule=1), workloads.CRYPTO_SEED)
    ctx.keygen([])            # the program generates its rotation keys itself
    m = pk.MF(ctx)
    n_ct = m.encrypt_csr_rows_int(32, 64, csr.row_ptr, csr.col_idx, np.stack(pt["R"]))
    assert n_ct == lay.n_ct
    m.init_factors_int(np.stack(pt["Utab"]), np.stack(pt["Vtab"]), np.stack(pt["Ug"]), np.stack(pt["Vg"]),
                       masks[program.S_I], masks[program.S_IG], 4)
    m.epochs(1)
    yield ctx, m, orc, ores, lay, csr, U0, V0
    ctx.close()


def test_layout_matches(tiny_run):
    ctx, m, orc, ores, lay, csr, U0, V0 = tiny_run
    L = m.layout()
    assert (L["n_ct"], L["n_utab"], L["n_vtab"], L["D"], L["B"]) == (lay.n_ct, lay.n_utab, lay.n_vtab, lay.D, lay.B)


def test_tables_bit_exact(tiny_run):
    ctx, m, orc, ores, lay, csr, U0, V0 = tiny_run
    for h, o in zip(m.handles(1), ores.utab):
        _same(ctx, h, o)
    for h, o in zip(m.handles(2), ores.vtab):
        _same(ctx, h, o)


def test_forward_dot_products_bit_exact(tiny_run):
    ctx, m, orc, ores, lay, csr, U0, V0 = tiny_run
    for h, o in zip(m.handles(5), ores.sdot):
        _same(ctx, h, o)


def test_decrypted_within_1e4_of_fp64(tiny_run):
    ctx, m, orc, ores, lay, csr, U0, V0 = tiny_run
    U, V = m.decrypt_factors()
    rhat = m.decrypt_predictions(0)
    Uf, Vf, rf = mf.train(U0, V0, csr.row_ptr, csr.col_idx, csr.values, 0.01, 0.02, 1, rule="R1")
    assert np.max(np.abs(U - Uf)) < 1e-4
    assert np.max(np.abs(V - Vf)) < 1e-4
    assert np.max(np.abs(rhat - rf)) < 1e-4


def test_float_api_end_to_end():
    """The library's own encoder path (encrypt_csr_rows + init_factors):
    decrypted results within 1e-4 of FP64 MF."""
    import paper_2509_03024_amd as pk
    csr = workloads.tiny_ratings()
    U0, V0 = workloads.init_factors(32, 64, 4)
    prm = params.config_tiny()
    lay = program.make_layout(prm.N, 4, 32, 64, csr.row_ptr, csr.col_idx)
    ctx = pk.Context(pk.tiny_params(k=4, lr=0.01, lam=0.02, rule=1), workloads.CRYPTO_SEED)
    ctx.keygen(program.rotation_steps(lay))
    m = pk.MF(ctx)
    m.encrypt_csr_rows(32, 64, csr.row_ptr, csr.col_idx, csr.values)
    m.init_factors(U0, V0)
    m.epochs(1)
    U, V = m.decrypt_factors()
    Uf, Vf, rf = mf.train(U0, V0, csr.row_ptr, csr.col_idx, csr.values, 0.01, 0.02, 1, rule="R1")
    assert np.max(np.abs(U - Uf)) < 1e-4 and np.max(np.abs(V - Vf)) < 1e-4
    assert np.max(np.abs(m.decrypt_predictions(0) - rf)) < 1e-4
    with pytest.raises(pk.CsrmfError) as e:          # no level left for another epoch
        m.epochs(1)
    assert e.value.name == "LEVEL"
    ctx.close()


def test_invalid_csr_rejected():
    import paper_2509_03024_amd as pk
    ctx = pk.Context(pk.tiny_params(k=4), workloads.CRYPTO_SEED)
    ctx.keygen([1])
    m = pk.MF(ctx)
    with pytest.raises(pk.CsrmfError) as e:
        m.encrypt_csr_rows(2, 3, [0, 2, 1], [0, 1, 2], [1.0, 2.0, 3.0])     # row_ptr not monotone
    assert e.value.name == "INVAL"
    with pytest.raises(pk.CsrmfError) as e:
        m.encrypt_csr_rows(2, 3, [0, 2, 3], [1, 0, 2], [1.0, 2.0, 3.0])     # unsorted columns
    assert e.value.name == "INVAL"
    with pytest.raises(pk.CsrmfError) as e:
        m.encrypt_csr_rows(2, 3, [0, 2, 3], [0, 1, 2], [1.0, float("nan"), 3.0])
    assert e.value.name == "INVAL"
    ctx.close()


def _golden_tiny2(name="mf_tiny2_r2_2epochs.txt"):
    import os
    rows = {}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            kind, i, lvl, scale, h = line.split()
            rows[(kind, int(i))] = (int(lvl), float(scale), h)
    return rows


def _check_digests(ctx, m, g, golden):
    n = 0
    for kind, which in (("utab", 1), ("vtab", 2), ("sdot", 5)):
        for i, h in enumerate(m.handles(which)):
            got, lvl, sc = ctx.export_ct(h)
            want = golden[(kind, i)]
            assert (lvl, sc) == want[:2], (kind, i)
            assert g.digest(got[0], got[1]) == want[2], (kind, i)
            n += 1
    assert n == len(golden)


def test_two_epochs_bit_exact_through_a_gather_and_a_refresh():
    """Two epochs (rule R2) on the two-epoch chain, the second from gathered
    factors, then a third call of one epoch that first refreshes the tables
    (level 0) and gathers.  Every output ciphertext equals the oracle's
    (SHA-256 digests written by tests/golden/make_mf_tiny2.py from the oracle
    alone), and the decrypted values are within 1e-4 of FP64 MF."""
    import paper_2509_03024_amd as pk
    from tests.golden import make_mf_tiny2 as g
    prm = params.config_tiny_two_epochs()
    csr = workloads.tiny_ratings()
    U0, V0 = workloads.init_factors(csr.n_rows, csr.n_cols, g.K)
    lay = program.make_layout(prm.N, g.K, csr.n_rows, csr.n_cols, csr.row_ptr, csr.col_idx)
    orc = ckks.Context(prm, workloads.CRYPTO_SEED)          # encoder only
    pt = g.integer_plaintexts(orc, lay, csr, U0, V0)
    masks = program.block_masks(orc, g.K)
    golden = _golden_tiny2()

    ctx = pk.Context(pk.params(12, 60, 7, 40, 2, 60, 4, 40, k=g.K, lr=g.LR, lam=g.LAM, rule=2, refresh_mode=1),
                     workloads.CRYPTO_SEED)
    ctx.keygen([])
    m = pk.MF(ctx)
    assert m.encrypt_csr_rows_int(csr.n_rows, csr.n_cols, csr.row_ptr, csr.col_idx, np.stack(pt["R"])) == lay.n_ct
    m.init_factors_int(np.stack(pt["Utab"]), np.stack(pt["Vtab"]), np.stack(pt["Ug"]), np.stack(pt["Vg"]),
                       masks[program.S_I], masks[program.S_IG], g.K)
    m.epochs(g.EPOCHS)
    _check_digests(ctx, m, g, golden)
    U, V = m.decrypt_factors()
    rhat = m.decrypt_predictions(0)
    Uf, Vf, rf = mf.train(U0, V0, csr.row_ptr, csr.col_idx, csr.values, g.LR, g.LAM, g.EPOCHS, rule=g.RULE)
    assert np.max(np.abs(U - Uf)) < 1e-4 and np.max(np.abs(V - Vf)) < 1e-4
    assert np.max(np.abs(rhat - rf)) < 1e-4
    # third epoch: the tables are at level 0, so the call refreshes them first
    m.epochs(1)
    _check_digests(ctx, m, g, _golden_tiny2("mf_tiny2_r2_refresh.txt"))
    U, V = m.decrypt_factors()
    rhat = m.decrypt_predictions(0)
    Uf, Vf, rf = mf.train(U0, V0, csr.row_ptr, csr.col_idx, csr.values, g.LR, g.LAM, g.EPOCHS + 1, rule=g.RULE)
    assert np.max(np.abs(U - Uf)) < 1e-4 and np.max(np.abs(V - Vf)) < 1e-4
    assert np.max(np.abs(rhat - rf)) < 1e-4
    ctx.close()
