"""Encrypted MF at the MovieLens-100K-shaped workload (943 x 1682, 99,926
ratings, k = 10, N = 2^15, 17 limbs, rule R2):
* decrypted factors and forward predictions after 3 epochs, and after 10
  epochs with two table refreshes, within 1e-4 of the FP64 synchronous
  epochs (oracle.mf);
* the first epoch's forward dot-product ciphertext of a sampled rating
  ciphertexts bit-exact against the oracle (same seed, integer plaintexts and
  serial numbers; those ciphertexts depend only on their own rating block)."""
import numpy as np
import pytest

from oracle import ckks, mf, params, program
import workloads

pytestmark = pytest.mark.gpu

K, LR, LAM = 10, 0.01, 0.02


def test_mf100k_three_epochs_within_1e4_of_fp64():
    import paper_2509_03024_amd as pk
    csr = workloads.movielens100k_shaped()
    U0, V0 = workloads.init_factors(csr.n_rows, csr.n_cols, K)
    ctx = pk.Context(pk.mf_n15_params(k=K, lr=LR, lam=LAM, rule=2), workloads.CRYPTO_SEED)
    ctx.keygen([])
    m = pk.MF(ctx)
    m.encrypt_csr_rows(csr.n_rows, csr.n_cols, csr.row_ptr, csr.col_idx, csr.values)
    m.init_factors(U0, V0)
    m.epochs(3)
    U, V = m.decrypt_factors()
    rhat = m.decrypt_predictions(0)
    Uf, Vf, rf = mf.train(U0, V0, csr.row_ptr, csr.col_idx, csr.values, LR, LAM, 3, rule="R2")
    print("max |U-Uf|", np.max(np.abs(U - Uf)), "max |V-Vf|", np.max(np.abs(V - Vf)),
          "max |rhat-rf|", np.max(np.abs(rhat - rf)))
    assert np.max(np.abs(U - Uf)) < 1e-4
    assert np.max(np.abs(V - Vf)) < 1e-4
    assert np.max(np.abs(rhat - rf)) < 1e-4
    ctx.close()


def test_mf100k_ten_epochs_with_two_refreshes_within_1e4_of_fp64():
    """The workload's full run: 10 epochs on the 16-prime chain, refreshing the
    tables twice (after epochs 4 and 8), within 1e-4 of the FP64 epochs."""
    import paper_2509_03024_amd as pk
    csr = workloads.movielens100k_shaped()
    U0, V0 = workloads.init_factors(csr.n_rows, csr.n_cols, K)
    ctx = pk.Context(pk.mf_n15_params(k=K, lr=LR, lam=LAM, rule=2, refresh_mode=1), workloads.CRYPTO_SEED)
    ctx.keygen([])
    m = pk.MF(ctx)
    m.encrypt_csr_rows(csr.n_rows, csr.n_cols, csr.row_ptr, csr.col_idx, csr.values)
    m.init_factors(U0, V0)
    m.epochs(10)
    st = m.stats()
    assert st["epochs_done"] == 10 and st["refreshes"] == 2
    U, V = m.decrypt_factors()
    rhat = m.decrypt_predictions(0)
    Uf, Vf, rf = mf.train(U0, V0, csr.row_ptr, csr.col_idx, csr.values, LR, LAM, 10, rule="R2")
    print("10 epochs: max |U-Uf|", np.max(np.abs(U - Uf)), "max |V-Vf|", np.max(np.abs(V - Vf)),
          "max |rhat-rf|", np.max(np.abs(rhat - rf)), "refresh s", st["refresh_seconds"])
    assert np.max(np.abs(U - Uf)) < 1e-4
    assert np.max(np.abs(V - Vf)) < 1e-4
    assert np.max(np.abs(rhat - rf)) < 1e-4
    ctx.close()


def test_mf100k_sampled_dot_products_bit_exact():
    import paper_2509_03024_amd as pk
    csr = workloads.movielens100k_shaped()
    U0, V0 = workloads.init_factors(csr.n_rows, csr.n_cols, K)
    prm = params.config_mf_n15()
    lay = program.make_layout(prm.N, K, csr.n_rows, csr.n_cols, csr.row_ptr, csr.col_idx)
    orc = ckks.Context(prm, workloads.CRYPTO_SEED)
    S = 2.0 ** 40
    enc = lambda Z: np.stack([orc.encode(z, S) for z in Z])
    pR = enc(program.slot_vectors(lay, csr.values, which="R"))
    pUt = enc(program.table_vectors(lay, U0, lay.n_utab))
    pVt = enc(program.table_vectors(lay, V0, lay.n_vtab))
    pUg = enc(program.slot_vectors(lay, users=U0, which="U"))
    pVg = enc(program.slot_vectors(lay, items=V0, which="V"))
    masks = program.block_masks(orc, K)

    ctx = pk.Context(pk.mf_n15_params(k=K, lr=LR, lam=LAM, rule=2), workloads.CRYPTO_SEED)
    ctx.keygen([])
    m = pk.MF(ctx)
    assert m.encrypt_csr_rows_int(csr.n_rows, csr.n_cols, csr.row_ptr, csr.col_idx, pR) == lay.n_ct
    m.init_factors_int(pUt, pVt, pUg, pVg, masks[program.S_I], masks[program.S_IG], K)
    m.epochs(1)
    sdot = m.handles(5)

    # oracle: keys for HMult and the windowed sum only, then the sampled ciphertexts
    win = [s for s in program.rotation_steps(lay) if s == -lay.kp or (0 < s < lay.B)]
    print("oracle key generation ...", flush=True)
    orc.keygen(rot_steps=win)
    n_ct, nu, nv = lay.n_ct, lay.n_utab, lay.n_vtab
    for c in (n_ct // 2,):
        print(f"oracle rating ciphertext {c} ...", flush=True)
        orc.serial = c
        R = orc.encrypt_int(pR[c], prm.L, S)
        orc.serial = n_ct + nu + nv + c
        Ug = orc.encrypt_int(pUg[c], prm.L, S)
        orc.serial = n_ct + nu + nv + n_ct + c
        Vg = orc.encrypt_int(pVg[c], prm.L, S)
        P = orc.hmult(Ug, Vg)
        T = P
        s = 1
        while s < lay.B:
            T = orc.add(T, orc.rotate(T, s))
            print(f"  window step {s} done", flush=True)
            s *= 2
        Sd = orc.rotate(T, -lay.kp)
        got, lvl, sc = ctx.export_ct(sdot[c])
        assert lvl == Sd.level and sc == Sd.scale
        assert np.array_equal(got[0], Sd.c0) and np.array_equal(got[1], Sd.c1), c
    ctx.close()
