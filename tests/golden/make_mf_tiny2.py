"""Writes mf_tiny2_r2_2epochs.txt and mf_tiny2_r2_refresh.txt: SHA-256
digests of the oracle's output ciphertexts for encrypted MF epochs (rule R2)
of the tiny workload on the two-epoch chain (N = 2^12, q_0 + 7 x 40-bit,
2 x 60-bit special, dnum 4):
* two epochs; the second starts from gathered factors (pins the gather);
* one more epoch from those tables (at level 0), which refreshes them before
  its gather (pins the refresh).

Only oracle/ and the seeded input generators are used.  Run from the repository
root:  python tests/golden/make_mf_tiny2.py
"""
import hashlib
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ckks, params, program  # noqa: E402
import workloads  # noqa: E402

K, LR, LAM, EPOCHS, RULE = 4, 0.01, 0.02, 2, "R2"
HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "mf_tiny2_r2_2epochs.txt")
OUT_REFRESH = os.path.join(HERE, "mf_tiny2_r2_refresh.txt")


def digest(c0, c1):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(np.asarray(c0, dtype=np.uint64), dtype="<u8").tobytes())
    h.update(np.ascontiguousarray(np.asarray(c1, dtype=np.uint64), dtype="<u8").tobytes())
    return h.hexdigest()


def integer_plaintexts(ctx, lay, csr, U0, V0):
    """Serial order of the encryptions: R, Utab, Vtab, Ug, Vg."""
    S = 2.0 ** 40
    enc = lambda Z: [ctx.encode(z, S) for z in Z]
    return {
        "R": enc(program.slot_vectors(lay, csr.values, which="R")),
        "Utab": enc(program.table_vectors(lay, U0, lay.n_utab)),
        "Vtab": enc(program.table_vectors(lay, V0, lay.n_vtab)),
        "Ug": enc(program.slot_vectors(lay, users=U0, which="U")),
        "Vg": enc(program.slot_vectors(lay, items=V0, which="V")),
    }


def main():
    prm = params.config_tiny_two_epochs()
    csr = workloads.tiny_ratings()
    U0, V0 = workloads.init_factors(csr.n_rows, csr.n_cols, K)
    lay = program.make_layout(prm.N, K, csr.n_rows, csr.n_cols, csr.row_ptr, csr.col_idx)
    ctx = ckks.Context(prm, workloads.CRYPTO_SEED)
    ctx.keygen(rot_steps=program.rotation_steps(lay))
    pt = integer_plaintexts(ctx, lay, csr, U0, V0)
    cts = {key: [ctx.encrypt_int(m, prm.L, 2.0 ** 40) for m in pt[key]] for key in ["R", "Utab", "Vtab", "Ug", "Vg"]}
    be = program.CkksBackend(ctx, program.block_masks(ctx, K))
    res = program.run_epochs(be, lay, cts["R"], cts["Ug"], cts["Vg"], cts["Utab"], cts["Vtab"], EPOCHS, LR, LAM,
                             rule=RULE)
    write(OUT, res, "two encrypted MF epochs")
    res2 = program.run_epochs(be, lay, cts["R"], None, None, res.utab, res.vtab, 1, LR, LAM, rule=RULE,
                              refresh=True, refresh_round=0, epoch0=EPOCHS)
    assert res2.refresh_round == 1
    write(OUT_REFRESH, res2, "a third epoch after a refresh of the tables")


def write(path, res, what):
    lines = [f"# Oracle output ciphertexts, {what} (rule R2, lr 0.01, lambda 0.02, k 4)",
             "# of the tiny workload on the two-epoch chain; written by tests/golden/make_mf_tiny2.py.",
             "# kind index level scale sha256(c0 || c1 as little-endian uint64 [level+1][N])"]
    for kind, lst in (("utab", res.utab), ("vtab", res.vtab), ("sdot", res.sdot)):
        for i, c in enumerate(lst):
            lines.append(f"{kind} {i} {c.level} {c.scale!r} {digest(c.c0, c.c1)}")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
