"""Pins for the encrypted MF program of the oracle.

* ClearBackend: the program's rotations, block masks and weights applied to
  plain slot vectors reproduce the FP64 synchronous epoch exactly (pure index
  algebra: layout, windowed block sum, BlockPermute grouping, self terms).
* CkksBackend at the tiny configuration: decrypted factors and forward
  predictions within 1e-4 of FP64 MF (the value contract).
"""
import numpy as np
import pytest

from oracle import ckks, mf, params, program
import workloads


def _layout_for(csr, N, k):
    return program.make_layout(N, k, csr.n_rows, csr.n_cols, csr.row_ptr, csr.col_idx)


def test_layout_packing_rules():
    # rows of lengths 3, 0, 5, 2 with D = 4 blocks: row 0 -> ct0 blocks 0..2; row 2 is
    # longer than D -> chunks 4 + 1, the first starts ct1 (does not fit in ct0), the
    # second continues in ct2 (ct1 full); row 3 fits after it in ct2.
    row_ptr = np.array([0, 3, 3, 8, 10])
    col_idx = np.array([0, 1, 2, 0, 1, 2, 3, 4, 1, 3])
    lay = program.make_layout(32, 4, 4, 5, row_ptr, col_idx)   # k'=4, B=8, D=32/16=2? -> N/2B
    assert lay.B == 8 and lay.D == 2
    lay = program.make_layout(64, 4, 4, 5, row_ptr, col_idx)
    assert lay.D == 4
    assert list(lay.ct_of) == [0, 0, 0, 1, 1, 1, 1, 2, 2, 2]
    assert list(lay.blk_of) == [0, 1, 2, 0, 1, 2, 3, 0, 1, 2]
    assert lay.n_ct == 3


def _clear_run(csr, N, k, U0, V0, epochs, alpha, lam, rule, damp=0.0):
    lay = _layout_for(csr, N, k)
    q = params.config_tiny().q if N == 4096 else [2 ** 40] * 30
    qchain = [1] + [2 ** 40 + 7] * 29      # scales are irrelevant for the exact back end
    be = program.ClearBackend(N, qchain, lay.B, k)
    L = 4 * epochs + 2
    R = [be.wrap(z, L, 2.0 ** 40) for z in program.slot_vectors(lay, csr.values, which="R")]
    Ug = [be.wrap(z, L, 2.0 ** 40) for z in program.slot_vectors(lay, users=U0, which="U")]
    Vg = [be.wrap(z, L, 2.0 ** 40) for z in program.slot_vectors(lay, items=V0, which="V")]
    Ut = [be.wrap(z, L, 2.0 ** 40) for z in program.table_vectors(lay, U0, lay.n_utab)]
    Vt = [be.wrap(z, L, 2.0 ** 40) for z in program.table_vectors(lay, V0, lay.n_vtab)]
    res = program.run_epochs(be, lay, R, Ug, Vg, Ut, Vt, epochs, alpha, lam, damp=damp, rule=rule,
                             exact_weights=True)
    U = program.decode_tables([v.z for v in res.utab], lay, csr.n_rows)
    V = program.decode_tables([v.z for v in res.vtab], lay, csr.n_cols)
    rhat = program.decode_predictions([v.z for v in res.sdot], lay)
    return U, V, rhat, lay


@pytest.mark.parametrize("rule,epochs", [("R1", 1), ("R1", 3), ("R2", 2)])
def test_clear_program_equals_fp64_epochs(rule, epochs):
    csr = workloads.tiny_ratings()
    U0, V0 = workloads.init_factors(32, 64, 4)
    U, V, rhat, lay = _clear_run(csr, 4096, 4, U0, V0, epochs, 0.01, 0.02, rule, damp=0.1)
    Uf, Vf, rf = mf.train(U0, V0, csr.row_ptr, csr.col_idx, csr.values, 0.01, 0.02, epochs, damp=0.1, rule=rule)
    assert np.max(np.abs(U - Uf)) < 1e-12 and np.max(np.abs(V - Vf)) < 1e-12
    assert np.max(np.abs(rhat - rf)) < 1e-12


def test_clear_program_multi_ciphertext_layout():
    """Small N so the 205 ratings span several rating and table ciphertexts,
    with rows split across ciphertexts, k not a power of two."""
    csr = workloads.tiny_ratings()
    U0, V0 = workloads.init_factors(32, 64, 3, seed=4)
    U, V, rhat, lay = _clear_run(csr, 128, 3, U0, V0, 2, 0.02, 0.05, "R2")
    assert lay.n_ct > 10 and lay.n_utab > 1 and lay.n_vtab > 1
    Uf, Vf, rf = mf.train(U0, V0, csr.row_ptr, csr.col_idx, csr.values, 0.02, 0.05, 2, rule="R2")
    assert np.max(np.abs(U - Uf)) < 1e-12 and np.max(np.abs(V - Vf)) < 1e-12
    assert np.max(np.abs(rhat - rf)) < 1e-12


def run_encrypted_tiny(ctx, csr, U0, V0, masks, epochs=1, alpha=0.01, lam=0.02, rule="R1"):
    """Encrypt the tiny workload with the oracle (serial order: R, Utab, Vtab, Ug, Vg)
    and run the program on CkksBackend; returns (layout, result, plaintexts)."""
    N = ctx.N
    lay = _layout_for(csr, N, U0.shape[1])
    L = ctx.prm.L
    D40 = 2.0 ** 40
    enc = lambda Z: [ctx.encode(z, D40) for z in Z]
    pt = {
        "R": enc(program.slot_vectors(lay, csr.values, which="R")),
        "Utab": enc(program.table_vectors(lay, U0, lay.n_utab)),
        "Vtab": enc(program.table_vectors(lay, V0, lay.n_vtab)),
        "Ug": enc(program.slot_vectors(lay, users=U0, which="U")),
        "Vg": enc(program.slot_vectors(lay, items=V0, which="V")),
    }
    cts = {key: [ctx.encrypt_int(m, L, D40) for m in pt[key]] for key in ["R", "Utab", "Vtab", "Ug", "Vg"]}
    be = program.CkksBackend(ctx, masks)
    res = program.run_epochs(be, lay, cts["R"], cts["Ug"], cts["Vg"], cts["Utab"], cts["Vtab"], epochs,
                             alpha, lam, rule=rule)
    return lay, res, pt


def test_encrypted_program_tiny_within_1e4_of_fp64():
    """The whole program on oracle ciphertexts (every CkksBackend operation but
    refresh, which test_oracle_backend pins): decrypted factors and forward
    predictions within 1e-4 of the FP64 epoch (about 45 s)."""
    prm = params.config_tiny()
    csr = workloads.tiny_ratings()
    U0, V0 = workloads.init_factors(32, 64, 4)
    ctx = ckks.Context(prm, workloads.CRYPTO_SEED)
    lay0 = _layout_for(csr, prm.N, 4)
    ctx.keygen(rot_steps=program.rotation_steps(lay0))
    lay, res, _ = run_encrypted_tiny(ctx, csr, U0, V0, program.block_masks(ctx, 4))
    U = program.decode_tables([ctx.decrypt(c) for c in res.utab], lay, 32)
    V = program.decode_tables([ctx.decrypt(c) for c in res.vtab], lay, 64)
    rhat = program.decode_predictions([ctx.decrypt(c) for c in res.sdot], lay)
    Uf, Vf, rf = mf.train(U0, V0, csr.row_ptr, csr.col_idx, csr.values, 0.01, 0.02, 1, rule="R1")
    assert np.max(np.abs(U - Uf)) < 1e-4
    assert np.max(np.abs(V - Vf)) < 1e-4
    assert np.max(np.abs(rhat - rf)) < 1e-4
    assert res.utab[0].level == 0


@pytest.mark.slow
def test_encrypted_program_two_epochs_matches_golden():
    """Two encrypted epochs (R2) on the two-epoch chain, through a gather:
    within 1e-4 of FP64, and the output ciphertexts match the stored digests."""
    from tests.golden import make_mf_tiny2 as g
    from tests.test_gpu_mf import _golden_tiny2
    prm = params.config_tiny_two_epochs()
    csr = workloads.tiny_ratings()
    U0, V0 = workloads.init_factors(csr.n_rows, csr.n_cols, g.K)
    ctx = ckks.Context(prm, workloads.CRYPTO_SEED)
    lay0 = _layout_for(csr, prm.N, g.K)
    ctx.keygen(rot_steps=program.rotation_steps(lay0))
    lay, res, _ = run_encrypted_tiny(ctx, csr, U0, V0, program.block_masks(ctx, g.K), epochs=g.EPOCHS,
                                     alpha=g.LR, lam=g.LAM, rule=g.RULE)
    U = program.decode_tables([ctx.decrypt(c) for c in res.utab], lay, csr.n_rows)
    V = program.decode_tables([ctx.decrypt(c) for c in res.vtab], lay, csr.n_cols)
    rhat = program.decode_predictions([ctx.decrypt(c) for c in res.sdot], lay)
    Uf, Vf, rf = mf.train(U0, V0, csr.row_ptr, csr.col_idx, csr.values, g.LR, g.LAM, g.EPOCHS, rule=g.RULE)
    assert np.max(np.abs(U - Uf)) < 1e-4 and np.max(np.abs(V - Vf)) < 1e-4
    assert np.max(np.abs(rhat - rf)) < 1e-4
    golden = _golden_tiny2()
    for kind, lst in (("utab", res.utab), ("vtab", res.vtab), ("sdot", res.sdot)):
        for i, c in enumerate(lst):
            assert (c.level, c.scale, g.digest(c.c0, c.c1)) == golden[(kind, i)], (kind, i)


class _MaskNoise(program.ClearBackend):
    """Cleartext program whose masks carry the real rounding error of the
    encoded I_0 (decoded slot values of the integer mask) and whose weights are
    the rounded integers W: the mask and weight error of the reading, without
    ciphertext noise."""

    def __init__(self, N, q, B, k, decoded):
        super().__init__(N, q, B, k)
        self.decoded = decoded           # {mask scale: S_I * (indicator + error)}

    def mask_mul(self, a, terms, scale, mask_scale, const=0):
        m = np.full(self.N // 2, float(const))
        dec = self.decoded[mask_scale]
        for p, W in terms:
            m += W * np.roll(dec, p * self.B)
        return self.V(a.z * m * a.scale / scale, a.level, scale)


@pytest.mark.slow
def test_mask_reading_within_1e4_at_mf100k_shape():
    """The block-mask reading (gather masks at 2^30 with the exact term scale,
    scatter masks at 2^24 into tables held at 2^50, the self term's constant
    split off) keeps three epochs at the MovieLens-100K shape (N = 2^15,
    k = 10, D = 512) within 1e-5 of FP64 (the model gives ~1e-6).  With every
    mask at 2^20 and tables at 2^40 the same model drifts to ~3e-3."""
    K, LR, LAM, EP = 10, 0.01, 0.02, 3
    csr = workloads.movielens100k_shaped()
    U0, V0 = workloads.init_factors(csr.n_rows, csr.n_cols, K)
    prm = params.config_mf_n15()
    lay = program.make_layout(prm.N, K, csr.n_rows, csr.n_cols, csr.row_ptr, csr.col_idx)
    ctx = ckks.Context(prm, workloads.CRYPTO_SEED)
    dec = {s: ctx.decode(m, 1.0) for s, m in program.block_masks(ctx, K).items()}
    be = _MaskNoise(prm.N, prm.q, lay.B, K, dec)
    S = 2.0 ** 40
    w = lambda Z: [be.wrap(z, prm.L, S) for z in Z]
    res = program.run_epochs(be, lay, w(program.slot_vectors(lay, csr.values, which="R")),
                             w(program.slot_vectors(lay, users=U0, which="U")),
                             w(program.slot_vectors(lay, items=V0, which="V")),
                             w(program.table_vectors(lay, U0, lay.n_utab)),
                             w(program.table_vectors(lay, V0, lay.n_vtab)), EP, LR, LAM, rule="R2")
    U = program.decode_tables([x.z for x in res.utab], lay, csr.n_rows)
    V = program.decode_tables([x.z for x in res.vtab], lay, csr.n_cols)
    rhat = program.decode_predictions([x.z for x in res.sdot], lay)
    Uf, Vf, rf = mf.train(U0, V0, csr.row_ptr, csr.col_idx, csr.values, LR, LAM, EP, rule="R2")
    assert np.max(np.abs(U - Uf)) < 1e-5 and np.max(np.abs(V - Vf)) < 1e-5
    assert np.max(np.abs(rhat - rf)) < 1e-5


@pytest.mark.parametrize("G", [1, 2, 16, 128, 256, None])
def test_block_permute_schedule_equals_direct_block_moves(G):
    """BlockPermute's rotation schedule (baby blocks of doubling trees, the
    pairwise giant tree, any baby-step size G including the chosen one) on
    plain slot vectors equals the block moves applied directly: destination
    block b gets the sum of w * (first k slots of source block a)."""
    rng = np.random.default_rng(11)
    N, k = 4096, 3
    lay = program.make_layout(N, k, 1, 1, np.array([0, 0]), np.array([], np.int64))
    D, B = lay.D, lay.B
    assert D == 256 and B == 8
    n_src, n_dst = 3, 4
    be = program.ClearBackend(N, [2 ** 40 + 7] * 8, B, k)
    srcs = [be.wrap(rng.normal(size=N // 2), 7, 2.0 ** 40) for _ in range(n_src)]
    moves = [[] for _ in range(n_dst)]
    want = np.zeros((n_dst, N // 2))
    for _ in range(300):
        c, a, b, d = int(rng.integers(n_src)), int(rng.integers(D)), int(rng.integers(D)), int(rng.integers(n_dst))
        w = float(rng.normal())
        moves[d].append(program.Move(c, a, b, w))
        want[d, b * B: b * B + k] += w * srcs[c].z[a * B: a * B + k]
    out = program.block_permute(be, lay, srcs, moves, None, 7, program.S_I, program.S_TAB,
                                exact_weights=True, G=G)
    for d in range(n_dst):
        assert np.max(np.abs(out[d].z - want[d])) < 1e-12, (G, d)


def test_choose_G_counts():
    """The schedule cost model on hand-made move sets: a gather-like call (one
    source, many destinations) prefers large G, a scatter-like call (many
    sources, one destination) small G; rotation counts of the trees."""
    assert program.baby_rotations(1) == 0 and program.baby_rotations(4) == 3
    assert program.baby_rotations(64) == 63 and program.baby_rotations(65) == 64
    assert program.baby_rotations(130) == 63 + 1 + 63 + 1 + 1
    assert program.giant_rotations({0, 1, 2, 3}, 4) == 3
    assert program.giant_rotations({0}, 8) == 0 and program.giant_rotations({7}, 8) == 3
    D = 64
    gather = [[program.Move(0, 0, b, 1.0) for b in range(D)] for _ in range(8)]
    scatter = [[program.Move(c, b, 0, 1.0) for c in range(32) for b in range(D)]]
    # gather: G=16 costs 15 + 8*3 = 39, G=32 costs 31 + 8*1 = 39 (tie -> smaller), G=64 63
    assert program.choose_G(gather, D) == 16
    # scatter: G=1 costs 0 + 63, G=2 costs 32 + 31 (tie -> smaller), G=4 costs 96 + 15
    assert program.choose_G(scatter, D) == 1


def test_layout_of_the_degenerate_matrix():
    """workloads.edge_ratings() at N = 2^12, k = 1 (B = 2, D = 1024): the
    single rating of user 1 opens ciphertext 0, user 2's 1030 ratings do not
    fit beside it and are cut into a chunk of 1024 (ciphertext 1) and one of 6
    (ciphertext 2, which users 4, 5 and 7 then fill to 12 blocks); empty rows
    take no blocks; one user table, two item tables."""
    csr = workloads.edge_ratings()
    lay = program.make_layout(1 << 12, 1, csr.n_rows, csr.n_cols, csr.row_ptr, csr.col_idx)
    assert (lay.B, lay.D, lay.n_ct, lay.n_utab, lay.n_vtab) == (2, 1024, 3, 1, 2)
    ct = np.asarray(lay.ct_of)
    blk = np.asarray(lay.blk_of)
    assert ct[0] == 0 and blk[0] == 0                                  # user 1
    assert np.all(ct[1:1025] == 1) and np.array_equal(blk[1:1025], np.arange(1024))
    assert np.all(ct[1025:] == 2) and np.array_equal(blk[1025:], np.arange(12))
