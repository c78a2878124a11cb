"""Writes ks_kernel_batch_n16.txt and ks_mf_n16.txt: SHA-256 digests of the
oracle's output ciphertexts for key-switching operations at N = 2^16, on
inputs of uniform random residues (the kernel-batch workload's inputs:
ciphertext i is workloads.random_residues(q_0..q_L, N, 2, seed=1000 + i) at the
top level, scale 2^40):

kernel batch chain (q_0 + 24 x 40-bit, 3 x 60-bit special, dnum 3: key-switching
digits of 9, 9 and 7 limbs at the top level):
* hmult i     HMult(ct_i, ct_{i+1})                    (tensor, relinearise, rescale)
* rotate i    Rot(ct_i, 1), non-hoisted
* conj i      conjugation of ct_i
* rotadd i    ct_i + Rot(ct_i, 2^14)
* hoisted r   the hoisted rotations of ct_5 by r = 1, 2, 2^14 (one ModUp)
for i in SAMPLES (two of the 64 ciphertexts a batched call processes);

MF chain at N = 2^16 (q_0 + 24 x 40-bit, 3 x 60-bit special, dnum 7: 4-limb digits):
* hmult 0     HMult(ct_0, ct_1)
* rotate 0    Rot(ct_0, 1)

Only oracle/ and the seeded input generators are used.  Run from the repository
root (each chain takes a few minutes on one core):
    python tests/golden/make_ks_n16.py [kernel_batch|mf_n16]
"""
import hashlib
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ckks, params  # noqa: E402
import workloads  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
SAMPLES = (0, 37)
HOIST_SOURCE = 5
HOIST_STEPS = (1, 2, 1 << 14)
ROT_STEP = 1
ROTADD_STEP = 1 << 14
SCALE = 2.0 ** 40


def digest(c0, c1):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(np.asarray(c0, dtype=np.uint64), dtype="<u8").tobytes())
    h.update(np.ascontiguousarray(np.asarray(c1, dtype=np.uint64), dtype="<u8").tobytes())
    return h.hexdigest()


def input_ct(prm, i):
    x = workloads.random_residues(prm.q, prm.N, 2, seed=1000 + i)
    return ckks.Ciphertext(x[0], x[1], SCALE)


def read(path):
    """{(kind, index): (level, scale, digest)} of a digest file."""
    out = {}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            kind, i, lvl, sc, dg = line.split()
            out[(kind, int(i))] = (int(lvl), float(sc), dg)
    return out


def kernel_batch():
    prm = params.config_kernel_batch()
    orc = ckks.Context(prm, workloads.CRYPTO_SEED)
    orc.keygen(rot_steps=sorted({ROT_STEP, ROTADD_STEP, *HOIST_STEPS}), conj=True)
    rows = []
    for i in SAMPLES:
        a, b = input_ct(prm, i), input_ct(prm, i + 1)
        rows.append(("hmult", i, orc.hmult(a, b)))
        rows.append(("rotate", i, orc.rotate(a, ROT_STEP)))
        rows.append(("conj", i, orc.conjugate(a)))
        rows.append(("rotadd", i, orc.add(a, orc.rotate(a, ROTADD_STEP))))
        print("sample", i, "done", flush=True)
    hs = orc.hoisted_rotations(input_ct(prm, HOIST_SOURCE), list(HOIST_STEPS))
    for r in HOIST_STEPS:
        rows.append(("hoisted", r, hs[r]))
    write(os.path.join(HERE, "ks_kernel_batch_n16.txt"), rows,
          "kernel-batch chain, N = 2^16, q_0 + 24 x 40-bit, 3 x 60-bit special, dnum 3")


def mf_n16():
    prm = params.config_mf_n16()
    orc = ckks.Context(prm, workloads.CRYPTO_SEED)
    orc.keygen(rot_steps=[ROT_STEP])
    a, b = input_ct(prm, 0), input_ct(prm, 1)
    rows = [("hmult", 0, orc.hmult(a, b)), ("rotate", 0, orc.rotate(a, ROT_STEP))]
    write(os.path.join(HERE, "ks_mf_n16.txt"), rows,
          "MF chain, N = 2^16, q_0 + 24 x 40-bit, 3 x 60-bit special, dnum 7")


def write(path, rows, what):
    lines = [f"# Oracle output ciphertexts, {what};",
             "# inputs: uniform residues, ciphertext i = workloads.random_residues(q, N, 2, seed=1000+i), scale 2^40;",
             "# written by tests/golden/make_ks_n16.py.",
             "# kind index level scale sha256(c0 || c1 as little-endian uint64 [level+1][N])"]
    for kind, i, c in rows:
        lines.append(f"{kind} {i} {c.level} {c.scale!r} {digest(c.c0, c.c1)}")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", path, flush=True)


if __name__ == "__main__":
    which = sys.argv[1:] or ["kernel_batch", "mf_n16"]
    for w in which:
        {"kernel_batch": kernel_batch, "mf_n16": mf_n16}[w]()
