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
    ind = np.zeros(prm.N // 2)
    ind[:4] = 1.0
    mask0 = orc.encode(ind, program.S_I)
    lay, ores, pt = run_encrypted_tiny(orc, csr, U0, V0, mask0)

    ctx = pk.Context(pk.tiny_params(k=4, lr=0.01, lam=0.02, rule=1), workloads.CRYPTO_SEED)
    ctx.keygen([])            # the program generates its rotation keys itself
    m = pk.MF(ctx)
    n_ct = m.encrypt_csr_rows_int(32, 64, csr.row_ptr, csr.col_idx, np.stack(pt["R"]))
    assert n_ct == lay.n_ct
    m.init_factors_int(np.stack(pt["Utab"]), np.stack(pt["Vtab"]), np.stack(pt["Ug"]), np.stack(pt["Vg"]), mask0, 4)
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
