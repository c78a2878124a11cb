"""Writes gather_n12_k1.txt: SHA-256 digests of the oracle's encrypted
predictions (gather of both factor tables into the rating layout, the product
and the windowed block sum) for sampled rating ciphertexts of a workload whose
block permutations take large baby steps:

* chain: N = 2^12, q_0 + 3 x 40-bit, 1 x 60-bit special, one limb per digit;
* k = 1, so B = 2 and D = 1024 blocks per ciphertext;
* 1024 users x 1024 items, 16 ratings per user (items uniform without
  replacement, ratings uniform 1..5, numpy PCG64 seed 3): 16 rating
  ciphertexts, one user table and one item table;
* both gathers choose G = 128 (one source, 16 destinations), so the babies of
  a source run up to beta = 127 and are built in two blocks of 64.

The plaintexts are the oracle's encodings (serial order R, Utab, Vtab, Ug, Vg),
so a run of the library on the same integers must give the same bits.  Only
oracle/ and the seeded input generators are used.  Run from the repository
root (about a minute):  python tests/golden/make_gather_n12_k1.py
"""
import hashlib
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ckks, mf, params, program  # noqa: E402
import workloads  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "gather_n12_k1.txt")
K = 1
N_USERS = N_ITEMS = 1024
PER_USER = 16
SAMPLE_CTS = (3, 12)


def ratings():
    """1024 x 1024, 16 distinct items per user, ratings uniform 1..5 (PCG64 seed 3)."""
    rng = np.random.default_rng(3)
    cols = [np.sort(rng.choice(N_ITEMS, size=PER_USER, replace=False)) for _ in range(N_USERS)]
    row_ptr = np.arange(0, PER_USER * (N_USERS + 1), PER_USER, dtype=np.int64)
    col_idx = np.concatenate(cols).astype(np.int32)
    vals = rng.integers(1, 6, size=len(col_idx)).astype(np.float64)
    return workloads.Csr(N_USERS, N_ITEMS, row_ptr, col_idx, vals)


def digest(c0, c1):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(np.asarray(c0, dtype=np.uint64), dtype="<u8").tobytes())
    h.update(np.ascontiguousarray(np.asarray(c1, dtype=np.uint64), dtype="<u8").tobytes())
    return h.hexdigest()


def setup():
    """(params, csr, U0, V0, layout, plaintexts) of the workload."""
    prm = params.config_tiny()
    csr = ratings()
    U0, V0 = workloads.init_factors(N_USERS, N_ITEMS, K)
    lay = program.make_layout(prm.N, K, N_USERS, N_ITEMS, csr.row_ptr, csr.col_idx)
    return prm, csr, U0, V0, lay


def gather_moves(lay, owner):
    """Moves of a gather (table entry -> every rating block of that entity)."""
    moves = [[] for _ in range(lay.n_ct)]
    for r in range(len(owner)):
        a_ct, a = divmod(int(owner[r]), lay.D)
        moves[int(lay.ct_of[r])].append(program.Move(a_ct, a, int(lay.blk_of[r]), 1.0))
    return moves


def main():
    prm, csr, U0, V0, lay = setup()
    assert (lay.n_ct, lay.n_utab, lay.n_vtab, lay.D, lay.B) == (16, 1, 1, 1024, 2)
    ctx = ckks.Context(prm, workloads.CRYPTO_SEED)
    ctx.keygen(rot_steps=program.rotation_steps(lay))
    S = 2.0 ** 40
    ctx.serial = lay.n_ct          # R takes serials 0 .. n_ct-1
    utab = [ctx.encrypt_int(ctx.encode(z, S), prm.L, S) for z in program.table_vectors(lay, U0, lay.n_utab)]
    vtab = [ctx.encrypt_int(ctx.encode(z, S), prm.L, S) for z in program.table_vectors(lay, V0, lay.n_vtab)]
    be = program.CkksBackend(ctx, program.block_masks(ctx, K))
    be.set_block(lay.B)
    mu, mv = gather_moves(lay, lay.rows), gather_moves(lay, lay.cols)
    Gu, Gv = program.choose_G(mu, lay.D), program.choose_G(mv, lay.D)
    assert Gu > 64 and Gv > 64, (Gu, Gv)
    lines = ["# Oracle encrypted predictions (gather of both tables, product, windowed sum) of sampled",
             f"# rating ciphertexts; N = 2^12 tiny chain, k = 1, D = 1024, 1024 x 1024 with 16 ratings per",
             f"# user (seed 3); baby-step sizes: user gather G = {Gu}, item gather G = {Gv}.",
             "# Written by tests/golden/make_gather_n12_k1.py.",
             "# kind index level scale sha256(c0 || c1 as little-endian uint64 [level+1][N])"]
    for c in SAMPLE_CTS:
        gu = program.block_permute(be, lay, utab, [mu[c]], None, prm.L, program.S_IG, program.S_T, unit=True, G=Gu)[0]
        gv = program.block_permute(be, lay, vtab, [mv[c]], None, prm.L, program.S_IG, program.S_T, unit=True, G=Gv)[0]
        P = ctx.hmult(gu, gv)
        T = ctx.add(P, ctx.rotate(P, 1))
        Sd = ctx.rotate(T, -lay.kp)
        z = ctx.decrypt(Sd)
        sel = np.nonzero(lay.ct_of == c)[0]
        want = np.sum(U0[lay.rows[sel]] * V0[lay.cols[sel]], axis=1)
        got = z[lay.blk_of[sel] * lay.B]
        err = float(np.max(np.abs(got - want)))
        assert err < 1e-4, err
        lines.append(f"pred {c} {Sd.level} {Sd.scale!r} {digest(Sd.c0, Sd.c1)}")
        print("ciphertext", c, "max |r_hat - <u, v>|", err, flush=True)
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
