"""Writes boot_n12.txt: SHA-256 digests of the oracle's bootstrapped ciphertexts
(oracle.bootstrap) on the N = 2^12 test chain (q_0 60-bit + 18 x 40-bit,
3 x 60-bit special primes, dnum 5: 4-limb digits; scale 2^40).

Inputs: two ciphertexts encrypted at level 0 (serials 0 and 1 after keygen),
slot values V[i] tiled with period N_SLOTS over the N/2 slots, V[i] drawn
uniformly from [-1, 1) by numpy's default_rng(100 + i).  Both are bootstrapped
with n = 4 slots, r = 9 squarings, a degree-11 series, pre-multiplication by
2^12; the file holds the inputs' and the outputs' digests, the outputs' level
and scale, and the largest slot error of the oracle's own decryption.  Edge
case: a third ciphertext (serial 2), one value default_rng(99) in every slot,
encrypted at level 2, bootstrapped with n = 1 (no rotation in CoeffToSlot,
log2(N/2) steps of SubSum) under the same keys.  Arcsine case: a fourth
ciphertext (serial 3, values default_rng(98).uniform(-1, 1, 4) tiled) at
level 0 bootstrapped with the arcsine term, r = 8, a degree-16 series and
2^15 pre-multiplication (18 levels: the whole chain).

Only oracle/ and the seeded inputs below are used.  Run from the repository
root (about eight minutes on one core):
    python tests/golden/make_boot_n12.py
"""
import hashlib
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import bootstrap, ckks, params  # noqa: E402
import workloads  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
N_SLOTS, SQUARINGS, DEGREE, PRE_BITS = 4, 9, 11, 12
N_CT = 2
SCALE = 2.0 ** 40
CHAIN = (12, 60, 18, 40, 3, 60, 5, 40)      # logN, base, L, scale bits, alpha, special bits, dnum, log2 scale


def chain():
    return params.make_params(*CHAIN, name="boot_n12")


def config():
    return bootstrap.BootConfig(n=N_SLOTS, r=SQUARINGS, d=DEGREE, pre_bits=PRE_BITS)


def edge_config():
    return bootstrap.BootConfig(n=1, r=SQUARINGS, d=DEGREE, pre_bits=PRE_BITS)


EDGE_LEVEL = 2


def arcsine_config():
    return bootstrap.BootConfig(n=N_SLOTS, r=8, d=16, pre_bits=15, arcsine=True)


def arcsine_values(N):
    return np.tile(np.random.default_rng(98).uniform(-1.0, 1.0, N_SLOTS), N // 2 // N_SLOTS)


def edge_values(N):
    return np.full(N // 2, np.random.default_rng(99).uniform(-1.0, 1.0))


def values(i, N):
    v = np.random.default_rng(100 + i).uniform(-1.0, 1.0, N_SLOTS)
    return np.tile(v, N // 2 // N_SLOTS)


def digest(c0, c1):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(np.asarray(c0, dtype=np.uint64), dtype="<u8").tobytes())
    h.update(np.ascontiguousarray(np.asarray(c1, dtype=np.uint64), dtype="<u8").tobytes())
    return h.hexdigest()


def read(path):
    """{(kind, index): (level, scale, digest)} and {key: float} of the '#=' lines."""
    out, meta = {}, {}
    with open(path) as f:
        for line in f:
            if line.startswith("#="):
                k, v = line[2:].split()
                meta[k] = float(v)
                continue
            if line.startswith("#") or not line.strip():
                continue
            kind, i, lvl, sc, dg = line.split()
            out[(kind, int(i))] = (int(lvl), float(sc), dg)
    return out, meta


def main():
    prm = chain()
    orc = ckks.Context(prm, workloads.CRYPTO_SEED)
    bootstrap.keygen_for(orc, config())
    print("keys done", flush=True)
    rows, err = [], 0.0
    cts = [orc.encrypt(values(i, prm.N), level=0, scale=SCALE) for i in range(N_CT)]
    for i, ct in enumerate(cts):
        rows.append(("input", i, ct))
    for i, ct in enumerate(cts):
        out = bootstrap.bootstrap(orc, ct, config())
        err = max(err, float(np.max(np.abs(orc.decrypt(out) - values(i, prm.N)))))
        rows.append(("boot", i, out))
        print("bootstrap", i, "done, error so far", err, flush=True)
    edge = orc.encrypt(edge_values(prm.N), level=EDGE_LEVEL, scale=SCALE)
    rows.append(("edge_input", 0, edge))
    out = bootstrap.bootstrap(orc, edge, edge_config())
    edge_err = float(np.max(np.abs(orc.decrypt(out) - edge_values(prm.N))))
    rows.append(("edge_boot", 0, out))
    print("edge bootstrap done, error", edge_err, flush=True)
    asn = orc.encrypt(arcsine_values(prm.N), level=0, scale=SCALE)
    rows.append(("arcsine_input", 0, asn))
    out = bootstrap.bootstrap(orc, asn, arcsine_config())
    asn_err = float(np.max(np.abs(orc.decrypt(out) - arcsine_values(prm.N))))
    rows.append(("arcsine_boot", 0, out))
    print("arcsine bootstrap done, error", asn_err, flush=True)
    lines = ["# Oracle bootstrapping on the N = 2^12 test chain (q_0 + 18 x 40-bit, 3 x 60-bit special, dnum 5);",
             f"# n = {N_SLOTS}, r = {SQUARINGS}, d = {DEGREE}, pre_bits = {PRE_BITS}; inputs encrypted at level 0",
             "# (serials 0, 1), slot values default_rng(100 + i).uniform(-1, 1, n) tiled; written by",
             "# tests/golden/make_boot_n12.py.",
             "# kind index level scale sha256(c0 || c1 as little-endian uint64 [level+1][N])",
             "# edge_*: n = 1, input at level 2 (serial 2), one value in every slot;",
             f"#=max_abs_error {err!r}",
             "# arcsine_*: n = 4, r = 8, d = 16, pre_bits = 15 with the arcsine term (serial 3);",
             f"#=edge_max_abs_error {edge_err!r}",
             f"#=arcsine_max_abs_error {asn_err!r}"]
    for kind, i, c in rows:
        lines.append(f"{kind} {i} {c.level} {c.scale!r} {digest(c.c0, c.c1)}")
    path = os.path.join(HERE, "boot_n12.txt")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
