"""Writes mf_edge_n12_k1.txt: SHA-256 digests of the oracle's output
ciphertexts for one encrypted MF epoch (rule R1, lr 0.01, lambda 0.02) on the
degenerate CSR matrix of workloads.edge_ratings() (empty rows and columns,
single-rating rows, a row longer than one ciphertext) at the tiny chain
(N = 2^12, q_0 + 3 x 40-bit, 1 special prime, dnum 4) with k = 1 (block width
2, 1024 blocks per ciphertext: 3 rating ciphertexts, 1 user table, 2 item
tables).  The plaintexts are the oracle's encodings (serial order R, Utab,
Vtab, Ug, Vg).  Only oracle/ and the seeded input generators are used.  Run
from the repository root (a few minutes):  python tests/golden/make_mf_edge.py
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
OUT = os.path.join(HERE, "mf_edge_n12_k1.txt")
K, LR, LAM = 1, 0.01, 0.02


def digest(c0, c1):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(np.asarray(c0, dtype=np.uint64), dtype="<u8").tobytes())
    h.update(np.ascontiguousarray(np.asarray(c1, dtype=np.uint64), dtype="<u8").tobytes())
    return h.hexdigest()


def setup():
    prm = params.config_tiny()
    csr = workloads.edge_ratings()
    U0, V0 = workloads.init_factors(csr.n_rows, csr.n_cols, K)
    lay = program.make_layout(prm.N, K, csr.n_rows, csr.n_cols, csr.row_ptr, csr.col_idx)
    return prm, csr, U0, V0, lay


def plaintexts(ctx, lay, csr, U0, V0):
    S = 2.0 ** 40
    enc = lambda Z: [ctx.encode(z, S) for z in Z]
    return {"R": enc(program.slot_vectors(lay, csr.values, which="R")),
            "Utab": enc(program.table_vectors(lay, U0, lay.n_utab)),
            "Vtab": enc(program.table_vectors(lay, V0, lay.n_vtab)),
            "Ug": enc(program.slot_vectors(lay, users=U0, which="U")),
            "Vg": enc(program.slot_vectors(lay, items=V0, which="V"))}


def read(path):
    rows = {}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            kind, i, lvl, scale, h = line.split()
            rows[(kind, int(i))] = (int(lvl), float(scale), h)
    return rows


def main():
    prm, csr, U0, V0, lay = setup()
    assert (lay.n_ct, lay.n_utab, lay.n_vtab) == (3, 1, 2), (lay.n_ct, lay.n_utab, lay.n_vtab)
    ctx = ckks.Context(prm, workloads.CRYPTO_SEED)
    ctx.keygen(rot_steps=program.rotation_steps(lay))
    pt = plaintexts(ctx, lay, csr, U0, V0)
    keys = ["R", "Utab", "Vtab", "Ug", "Vg"]
    cts = {key: [ctx.encrypt_int(m, prm.L, 2.0 ** 40) for m in pt[key]] for key in keys}
    be = program.CkksBackend(ctx, program.block_masks(ctx, K))
    res = program.run_epochs(be, lay, cts["R"], cts["Ug"], cts["Vg"], cts["Utab"], cts["Vtab"], 1, LR, LAM,
                             rule="R1")
    U = program.decode_tables([ctx.decrypt(c) for c in res.utab], lay, csr.n_rows)
    V = program.decode_tables([ctx.decrypt(c) for c in res.vtab], lay, csr.n_cols)
    Uf, Vf, _ = mf.train(U0, V0, csr.row_ptr, csr.col_idx, csr.values, LR, LAM, 1, rule="R1")
    err = max(np.max(np.abs(U - Uf)), np.max(np.abs(V - Vf)))
    assert err < 1e-4, err
    print("max error vs FP64 MF", err, flush=True)
    lines = ["# Oracle output ciphertexts of one encrypted MF epoch (R1, lr 0.01, lambda 0.02) on",
             "# workloads.edge_ratings() (8 x 1100, empty rows and columns, a row of 1030 ratings), k 1,",
             "# N = 2^12, q_0 + 3 x 40-bit, 1 special, dnum 4; written by tests/golden/make_mf_edge.py.",
             "# kind index level scale sha256(c0 || c1 as little-endian uint64 [level+1][N])"]
    for kind, lst in (("utab", res.utab), ("vtab", res.vtab), ("sdot", res.sdot)):
        for i, c in enumerate(lst):
            lines.append(f"{kind} {i} {c.level} {c.scale!r} {digest(c.c0, c.c1)}")
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
