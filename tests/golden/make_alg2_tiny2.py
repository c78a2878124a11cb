"""Writes alg2_tiny2.txt: SHA-256 digests of the oracle's output ciphertexts
for one encrypted epoch of Alg. 2 (user-item batch pairs, Sec. III-D):

* chain: N = 2^12, q_0 + 7 x 40-bit, 2 x 60-bit special primes, dnum 4;
* k = 16 (B = 32, D = 64: a batch is one table ciphertext of 64 profiles);
* 64 users x 128 items, 10% of the cells (uniform without replacement,
  ratings 1..5, numpy PCG64 seed 1): one user table, two item tables, so two
  batch pairs that both update the user table, the second from the first's
  result; a pair costs 4 levels, so the tables are refreshed between them;
* lr 0.05, lambda 0.02, dampening 0.1 (epoch 0).

The plaintexts are the oracle's encodings (serial order R, Utab, Vtab).  Only
oracle/ and the seeded input generators are used.  Run from the repository
root (a few minutes):  python tests/golden/make_alg2_tiny2.py
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
OUT = os.path.join(HERE, "alg2_tiny2.txt")
K, LR, LAM, DAMP = 16, 0.05, 0.02, 0.1
N_USERS, N_ITEMS = 64, 128


def digest(c0, c1):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(np.asarray(c0, dtype=np.uint64), dtype="<u8").tobytes())
    h.update(np.ascontiguousarray(np.asarray(c1, dtype=np.uint64), dtype="<u8").tobytes())
    return h.hexdigest()


def setup():
    prm = params.config_tiny_two_epochs()
    csr = workloads.tiny_ratings(seed=1, n=N_USERS, m=N_ITEMS, density=0.10)
    U0, V0 = workloads.init_factors(N_USERS, N_ITEMS, K)
    lay = program.make_pair_layout(prm.N, K, N_USERS, N_ITEMS, csr.row_ptr, csr.col_idx)
    return prm, csr, U0, V0, lay


def plaintexts(ctx, lay, csr, U0, V0):
    S = 2.0 ** 40
    enc = lambda Z: [ctx.encode(z, S) for z in Z]
    return {"R": enc(program.slot_vectors(lay, csr.values, which="R")),
            "Utab": enc(program.table_vectors(lay, U0, lay.n_utab)),
            "Vtab": enc(program.table_vectors(lay, V0, lay.n_vtab)),
            "Ug": enc(program.slot_vectors(lay, users=U0, which="U")),
            "Vg": enc(program.slot_vectors(lay, items=V0, which="V"))}


def main():
    prm, csr, U0, V0, lay = setup()
    assert (lay.n_utab, lay.n_vtab, len(lay.pairs)) == (1, 2, 2)
    ctx = ckks.Context(prm, workloads.CRYPTO_SEED)
    ctx.keygen(rot_steps=program.rotation_steps(lay))
    pt = plaintexts(ctx, lay, csr, U0, V0)
    cts = {key: [ctx.encrypt_int(m, prm.L, 2.0 ** 40) for m in pt[key]] for key in ["R", "Utab", "Vtab"]}
    be = program.CkksBackend(ctx, program.block_masks(ctx, K))
    res = program.run_pair_epochs(be, lay, cts["R"], cts["Utab"], cts["Vtab"], 1, LR, LAM, damp=DAMP)
    assert res.refresh_round == 1
    U = program.decode_tables([ctx.decrypt(c) for c in res.utab], lay, N_USERS)
    V = program.decode_tables([ctx.decrypt(c) for c in res.vtab], lay, N_ITEMS)
    rhat = program.decode_predictions([ctx.decrypt(c) for c in res.sdot], lay)
    Uf, Vf, rf = mf.train_batch_pairs(U0, V0, csr.row_ptr, csr.col_idx, csr.values, LR, LAM, 1, lay.D, lay.D,
                                      damp=DAMP)
    err = max(np.max(np.abs(U - Uf)), np.max(np.abs(V - Vf)), np.max(np.abs(rhat - rf)))
    assert err < 1e-4, err
    print("max error vs FP64 Alg. 2", err, flush=True)
    lines = ["# Oracle output ciphertexts of one encrypted Alg. 2 epoch (two batch pairs, one refresh),",
             "# N = 2^12, q_0 + 7 x 40-bit, 2 x 60-bit special, dnum 4, k 16, 64 x 128 at 10% (seed 1),",
             "# lr 0.05, lambda 0.02, damp 0.1; written by tests/golden/make_alg2_tiny2.py.",
             "# kind index level scale sha256(c0 || c1 as little-endian uint64 [level+1][N])"]
    for kind, lst in (("utab", res.utab), ("vtab", res.vtab), ("sdot", res.sdot)):
        for i, c in enumerate(lst):
            lines.append(f"{kind} {i} {c.level} {c.scale!r} {digest(c.c0, c.c1)}")
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
