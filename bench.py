"""Benchmark: batched CKKS key switching at N = 2^16 on one MI355X, with the
encrypted MF workloads beside it.

Default run (one JSON line):
* the kernel-batch workload (the headline metric): 64 ciphertexts of uniform
  random residues at N = 2^16 with q_0 (60-bit) + 24 x 40-bit scale primes,
  3 x 60-bit special primes, dnum = 3.  One step is one pass of the whole
  batched path:
    (i)   forward + inverse NTT of all 64 x 2 x 25 limbs,
    (ii)  64 HMult (tensor, relinearise, rescale) ct_i x ct_{i+1 mod 64},
    (iii) per ciphertext a rotate-and-sum chain over steps 2^0 .. 2^14 plus a
          conjugation: 16 key switches per ciphertext, 1024 per step.
  value = key-switch rotations per second over whole steps (1024 * K / time
  of the K timed steps, phases (i) and (ii) included);
* "mf100k": 10 encrypted MF epochs on the MovieLens-100K-shaped matrix
  (943 x 1682, 99,926 ratings, k = 10, N = 2^15, two table refreshes);
* "tiny": the latency of one encrypted MF epoch at the tiny configuration
  (32 x 64, 205 ratings, k = 4, N = 2^12);
* "bootstrap": bootstrapping a batch of 16 ciphertexts at N = 2^16 (MF chain,
  16-periodic slots, 20 levels) back from level 0, ciphertexts per second;
* "cpu_baseline" legs: the oracle on bounded samples of each workload, run
  in parallel processes after the GPU work.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
       [--no-mf] [--workload ks|mf100k|mf1m|serve|accuracy|boot]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_CT = 64
PLAIN_CT = 8
LOGN = 16
CHAIN = [1 << a for a in range(15)]
HBM_PEAK_GBS = 8000.0
# MI355X: 256 CUs at 2.4 GHz; fp64 vector 78.6 TFLOP/s (FMA = 2), fp32 157.3.
FP64_FMA_PER_S = 78.6e12 / 2
# Modular-multiply rates measured on an MI355X by a register-resident
# microbenchmark (4 independent dependent chains per thread, 8192 x 256
# threads, every result stored; method and figures in the design doc), in
# operations per second (fp64_split_mac: conversion terms of four FMAs).
MODMUL_RATE = {"shoup_u64": 1.927e12, "montgomery_u64": 1.318e12, "fp64_exact": 6.164e12, "mac_64x64_128": 2.301e12,
               "fp64_split_mac": 9.624e12}
# HBM bytes per launch of a kernel in the timed step (average over the step's
# launches), from rocprofv3 FETCH_SIZE + WRITE_SIZE counters scaled by a 512 MiB
# copy (profiles/), with the NTT schedule (rows per pair of passes) and the
# split of the transform's stages between its passes of that run, and the
# algorithmic bytes of its launches; only valid for the kernel code the
# counters were taken on.  Under another number of rows the launches differ in
# size and the measured bytes are scaled by the algorithmic bytes
# (traffic_basis); under another split they were not measured (None).
TRAFFIC = {
    "k_ntt_pass<rows,fwd>": {"bytes": 1.4945e+09, "alg_bytes": 7.355e+08, "schedule": 2048, "split": 7},
    "k_ntt_pass<cols,fwd>": {"bytes": 1.4716e+09, "alg_bytes": 7.356e+08, "schedule": 2048, "split": 7},
    "k_ntt_pass<rows,inv>": {"bytes": 1.0653e+09, "alg_bytes": 5.251e+08, "schedule": 2048, "split": 7},
    "k_ntt_pass<cols,inv>": {"bytes": 1.0506e+09, "alg_bytes": 5.251e+08, "schedule": 2048, "split": 7},
    "k_basis_convert": {"bytes": 1.1746e+09, "alg_bytes": 1.174e+09, "schedule": None},
    "k_ks_combine": {"bytes": 7.7946e+09, "alg_bytes": 8.319e+09, "schedule": None},
    "k_ks_inner": {"bytes": 5.128e+08, "alg_bytes": 5.128e+08, "schedule": None},
}
# Counter bytes (FETCH_SIZE + WRITE_SIZE, scaled as above) of a whole step of
# the kernel-batch workload (transform phase, HMult phase and rotation phase),
# from the same counter runs; None once the kernels have changed.
KS_COUNTER_BYTES_PER_STEP = 575.6e9


def traffic_of(name, schedule, alg_bytes):
    """Measured HBM bytes per launch of kernel `name` under `schedule`
    ((NTT rows per pair of passes, column-pass stages)), with their basis.
    Launches of another size (another schedule, or another workload's batch)
    get the measured bytes scaled by their algorithmic bytes."""
    t = TRAFFIC.get(name)
    if t is None:
        return None, None
    same_size = abs(alg_bytes / t["alg_bytes"] - 1.0) <= 0.01
    if t["schedule"] is None:
        if same_size:
            return t["bytes"], "rocprofv3 counters"
        return round(t["bytes"] / t["alg_bytes"] * alg_bytes), \
            "rocprofv3 counters on the kernel-batch launches, scaled by algorithmic bytes"
    rows, split = schedule
    if split != t["split"]:
        return None, f"not measured at NTT split {split} (counters taken at split {t['split']})"
    if t["schedule"] == rows and same_size:
        return t["bytes"], f"rocprofv3 counters at NTT schedule {rows}"
    return round(t["bytes"] / t["alg_bytes"] * alg_bytes), \
        f"rocprofv3 counters at NTT schedule {t['schedule']}, scaled by algorithmic bytes to launches of " \
        f"{round(alg_bytes / 1e6, 1)} MB at schedule {rows}"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mf", action="store_true", help="default run: skip the MF-100K and tiny sub-objects")
    ap.add_argument("--workload", default="ks", choices=["ks", "mf100k", "mf1m", "serve", "accuracy", "boot"],
                    help="ks: batched key switching with the MF and bootstrapping sub-objects (default); "
                         "mf100k / mf1m: encrypted MF epochs alone; serve: the request stream; boot: "
                         "bootstrapping alone")
    ap.add_argument("--epochs", type=int, default=None, help="MF workloads: epochs (100K: 10, 1M: 5)")
    ap.add_argument("--rates", default="10,20,50,100,200,500", help="serve: Poisson arrival rates (requests/s)")
    ap.add_argument("--requests", type=int, default=2000, help="serve: requests per rate")
    ap.add_argument("--ntt-chunk", type=int, default=None,
                    help="fix the NTT schedule (rows per pair of passes) instead of autotuning (for profiles)")
    ap.add_argument("--ntt-split", type=int, default=None,
                    help="with --ntt-chunk: butterfly stages of the NTT's column pass (default log2 N / 2)")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the HIP-graph replay, so that the timed steps end the run (profiles)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="copy a 512 MiB device buffer once before the timed steps (reference for HBM counters)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------- models of one rotation
def ks_model(N, nl, alpha, dnum_digits, key_share):
    """Algorithmic HBM bytes and modular multiplies of one rotate-and-add
    acc + Rot(a, r) at nl limbs (acc = a, as in the chain): read a (c0, c1) and
    write the result once, plus the key's share (key bytes / ciphertexts that
    use it); multiplies of the hybrid key switch: the transforms (N/2 log2 N
    butterflies per limb), the ModUp and ModDown conversions (one
    multiply-accumulate per source limb and target limb), the inner product
    (digits x extended limbs x 2) and the ModDown scaling."""
    logN = N.bit_length() - 1
    limb = 8 * N
    nr = nl + alpha
    key_bytes = len(dnum_digits) * 2 * nr * limb
    alg_bytes = 4 * nl * limb + key_bytes / key_share
    ntt_limbs = nl + sum(nr - d for d in dnum_digits) + 2 * alpha + 2 * nl
    # limbs of 60-bit primes among them (q_0 and the special primes; the
    # others take the FP64 butterflies): q_0 of c1, the special primes and q_0
    # of every digit that does not hold it, the special primes of ModDown, q_0
    # of both ModDown outputs
    int_limbs = 1 + len(dnum_digits) * alpha + (len(dnum_digits) - 1) + 2 * alpha + 2
    bfly = ntt_limbs * (N // 2) * logN
    conv = N * (sum(d * (nr - d) for d in dnum_digits) + 2 * alpha * nl)
    # conversion terms into 60-bit targets (the special primes in ModUp, q_0 in
    # the digits that do not hold it and in ModDown); the others sum in FP64
    conv_int = N * (sum(d * alpha for d in dnum_digits) + sum(dnum_digits[1:]) + 2 * alpha)
    inner = N * len(dnum_digits) * nr * 2
    scal = N * 2 * nl
    # inner-product and scaling multiplies on 60-bit limbs (the special primes
    # and q_0; the 40-bit limbs use the exact FP64 form)
    inner_int = N * len(dnum_digits) * (alpha + 1) * 2
    scal_int = N * 2
    return {"alg_bytes": alg_bytes, "limb_ntts": ntt_limbs, "int_limb_ntts": int_limbs, "butterflies": bfly,
            "conv_macs": conv, "conv_macs_int": conv_int, "inner_mults": inner, "inner_mults_int": inner_int,
            "scale_mults": scal, "scale_mults_int": scal_int, "modmuls": bfly + conv + inner + scal}


def valu_bound(model, q_is_fp64):
    """Seconds per rotation if only the measured modular-multiply rates
    limited it: butterflies of the 40-bit limbs in the exact FP64 form, the
    60-bit ones with Shoup multiplies, conversion terms into 40-bit targets as
    exact FP64 split sums (four FMAs), into 60-bit targets as 64x64->128-bit
    multiply-accumulates, inner products and scalings in the exact FP64 form on
    the 40-bit limbs and as Montgomery multiplies on the 60-bit ones."""
    r = MODMUL_RATE
    if any(v is None for v in r.values()):
        return None
    f = q_is_fp64
    ci = model["conv_macs_int"]
    mi = model["inner_mults_int"] + model["scale_mults_int"]
    mf = model["inner_mults"] + model["scale_mults"] - mi
    return (model["butterflies"] * f / r["fp64_exact"] + model["butterflies"] * (1 - f) / r["shoup_u64"]
            + (model["conv_macs"] - ci) / r["fp64_split_mac"] + ci / r["mac_64x64_128"]
            + mf / r["fp64_exact"] + mi / r["montgomery_u64"])


# ---------------------------------------------------------------- CPU oracle legs
def _single_thread_env():
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"


def cpu_leg_ks(n_workers):
    """Oracle key switching at the kernel-batch shape: keys once, then one
    non-hoisted rotation of one 25-limb ciphertext in this process, and one
    rotation per worker of a process pool over other ciphertexts."""
    _single_thread_env()
    import multiprocessing as mp
    from oracle import ckks, params
    import workloads
    prm = params.config_kernel_batch()
    orc = ckks.Context(prm, workloads.CRYPTO_SEED)
    t0 = time.perf_counter()
    orc.keygen(rot_steps=[1])
    t_key = time.perf_counter() - t0
    global _POOL_ORC
    _POOL_ORC = orc
    t0 = time.perf_counter()
    _pool_rotation(0)
    t_rot = time.perf_counter() - t0
    pool_rate = None
    if n_workers > 1:
        ctxf = mp.get_context("fork")      # the keys are shared with the workers by fork
        with ctxf.Pool(n_workers) as p:
            t0 = time.perf_counter()
            p.map(_pool_rotation, range(1, n_workers + 1))
            pool_rate = n_workers / (time.perf_counter() - t0)
    return {"value": 1.0 / t_rot, "unit": "key-switch rotations/s", "cores": 1, "kind": "oracle",
            "sample": f"1 non-hoisted rotation of one ciphertext, N=2^16, 25 limbs, dnum=3 ({t_rot:.1f} s; "
                      f"key generation {t_key:.1f} s untimed)",
            "pool": None if pool_rate is None else
            {"value": pool_rate, "cores": n_workers,
             "sample": f"{n_workers} rotations of different ciphertexts in a pool of {n_workers} processes"},
            "host_cpu_count": os.cpu_count()}


_POOL_ORC = None


def _pool_rotation(i):
    from oracle import ckks
    import workloads
    prm = _POOL_ORC.prm
    x = workloads.random_residues(prm.q, prm.N, 2, seed=2000 + i)
    _POOL_ORC.rotate(ckks.Ciphertext(x[0], x[1], 2.0 ** 40), 1)
    return i


def cpu_leg_mf100k(n_ks_per_epoch, epochs):
    """MovieLens-100K shape: the FP64 MF (numpy, all epochs, timed) and the
    oracle on one rotation of one rating-sized ciphertext at N = 2^15 (17
    limbs, dnum 5), extrapolated to the epochs' key switches (the count the
    library performed; the key switches dominate the oracle's time)."""
    _single_thread_env()
    import numpy as np
    from oracle import ckks, mf, params
    import workloads
    csr = workloads.movielens100k_shaped()
    U0, V0 = workloads.init_factors(csr.n_rows, csr.n_cols, 10)
    t0 = time.perf_counter()
    mf.train(U0, V0, csr.row_ptr, csr.col_idx, csr.values, 0.01, 0.02, epochs, rule="R2")
    t_fp64 = time.perf_counter() - t0
    prm = params.config_mf_n15()
    orc = ckks.Context(prm, workloads.CRYPTO_SEED)
    orc.keygen(rot_steps=[1])
    x = workloads.random_residues(prm.q, prm.N, 2, seed=7)
    t0 = time.perf_counter()
    orc.rotate(ckks.Ciphertext(x[0], x[1], 2.0 ** 40), 1)
    t_rot = time.perf_counter() - t0
    t_total = t_rot * n_ks_per_epoch * epochs
    return {"value": csr.nnz * epochs / t_total, "unit": "ratings/s", "cores": 1, "kind": "oracle",
            "sample": f"1 oracle rotation at N=2^15, 17 limbs ({t_rot:.1f} s), extrapolated to the "
                      f"{n_ks_per_epoch} key switches per epoch the library ran, x {epochs} epochs (extrapolated)",
            "fp64_mf": {"ratings_per_s": csr.nnz * epochs / t_fp64, "seconds": t_fp64,
                        "what": f"plaintext FP64 MF (oracle.mf, rule R2), {epochs} epochs"},
            "host_cpu_count": os.cpu_count()}


def cpu_leg_tiny():
    """Config 1: the whole encrypted oracle for one epoch (keys excluded)."""
    _single_thread_env()
    from oracle import ckks, params, program
    import workloads
    from tests.test_oracle_program import run_encrypted_tiny
    csr = workloads.tiny_ratings()
    U0, V0 = workloads.init_factors(32, 64, 4)
    prm = params.config_tiny()
    lay = program.make_layout(prm.N, 4, 32, 64, csr.row_ptr, csr.col_idx)
    orc = ckks.Context(prm, workloads.CRYPTO_SEED)
    orc.keygen(rot_steps=program.rotation_steps(lay))
    t0 = time.perf_counter()
    run_encrypted_tiny(orc, csr, U0, V0, program.block_masks(orc, 4))
    t = time.perf_counter() - t0
    return {"value": t, "unit": "s per epoch", "cores": 1, "kind": "oracle",
            "sample": "the full encrypted oracle, 1 epoch of the tiny workload (encryption included, keys excluded)",
            "host_cpu_count": os.cpu_count()}


def run_cpu_legs(legs):
    """Run the legs {name: (fn, args)} in parallel spawned processes (they
    never touch the GPU); returns {name: result or error}."""
    import concurrent.futures as cf
    import multiprocessing as mp
    out = {}
    with cf.ProcessPoolExecutor(max_workers=len(legs), mp_context=mp.get_context("spawn")) as ex:
        futs = {name: ex.submit(fn, *a) for name, (fn, a) in legs.items()}
        for name, f in futs.items():
            try:
                out[name] = f.result()
            except Exception as e:   # reported, not fatal: the GPU figures stand on their own
                out[name] = {"error": repr(e)}
            log(f"cpu leg {name} done")
    return out


# ---------------------------------------------------------------- accuracy (RMSE per iteration)
ACC_ITERS, ACC_LR, ACC_LAM, ACC_DAMP = 20, 0.001, 0.02, 0.1
ACC_PREC_ITERS, ACC_DELTA_BITS = 15, (26, 32, 40)


def run_accuracy(iters=ACC_ITERS):
    """RMSE (Eq. 10) of the decrypted predictions after every iteration of
    the encrypted MF at the MovieLens-100K shape, without batching (CSR
    rows, synchronous epochs, rule R1, the summed form of Alg. 1) and with
    the user-item batch pairs of Alg. 2 (dampened rate), both at alpha =
    0.001, lambda = 0.02, k = 10, N = 2^15, tables refreshed as the levels
    run out.  The prediction after iteration t is <u_i, v_j> from the
    decrypted factors (decrypted on the host, the last step of Alg. 1)."""
    import numpy as np
    import paper_2509_03024_amd as pk
    import workloads
    csr = workloads.movielens100k_shaped()
    K = 10
    U0, V0 = workloads.init_factors(csr.n_rows, csr.n_cols, K)
    rows = np.repeat(np.arange(csr.n_rows), np.diff(csr.row_ptr))
    cols = np.asarray(csr.col_idx)

    def rmse(U, V):
        return float(np.sqrt(np.mean((np.einsum("ij,ij->i", U[rows], V[cols]) - csr.values) ** 2)))

    out = {"initial_rmse": round(rmse(U0, V0), 5)}
    for name, pairs, rule, damp in (("without_batching", 0, 1, 0.0), ("with_batching_alg2", 1, 1, ACC_DAMP)):
        ctx = pk.Context(pk.params(15, 60, 16, 40, 3, 60, 5, 40, k=K, lr=ACC_LR, lam=ACC_LAM, damp=damp, rule=rule,
                                   refresh_mode=1, batch_pairs=pairs), workloads.CRYPTO_SEED)
        ctx.keygen([])
        m = pk.MF(ctx)
        m.encrypt_csr_rows(csr.n_rows, csr.n_cols, csr.row_ptr, csr.col_idx, csr.values)
        m.init_factors(U0, V0)
        curve, t_ep = [], 0.0
        for it in range(iters):
            t0 = time.perf_counter()
            m.epochs(1)
            t_ep += time.perf_counter() - t0
            U, V = m.decrypt_factors()
            curve.append(round(rmse(U, V), 5))
        log(f"accuracy {name}: RMSE {curve[0]} -> {curve[-1]} over {iters} iterations")
        out[name] = {"rmse": curve, "reduction": round(1 - curve[-1] / out["initial_rmse"], 4),
                     "refreshes": m.stats()["refreshes"], "epoch_s": round(t_ep / iters, 3)}
        ctx.close()
    # iterations each variant needs to reach the RMSE the slower one ends at
    target = max(out["without_batching"]["rmse"][-1], out["with_batching_alg2"]["rmse"][-1])
    for name in ("without_batching", "with_batching_alg2"):
        out[name]["iterations_to_slower_final_rmse"] = next(
            i + 1 for i, x in enumerate(out[name]["rmse"]) if x <= target)
    # precision: the same run without batching at smaller scales Delta (scale
    # primes of log2(Delta) bits; the program's masks scale with Delta)
    prec = {}
    for bits in ACC_DELTA_BITS:
        ctx = pk.Context(pk.params(15, 60, 16, bits, 3, 60, 5, bits, k=K, lr=ACC_LR, lam=ACC_LAM, rule=1,
                                   refresh_mode=1), workloads.CRYPTO_SEED)
        ctx.keygen([])
        m = pk.MF(ctx)
        m.encrypt_csr_rows(csr.n_rows, csr.n_cols, csr.row_ptr, csr.col_idx, csr.values)
        m.init_factors(U0, V0)
        curve = []
        for it in range(ACC_PREC_ITERS):
            m.epochs(1)
            U, V = m.decrypt_factors()
            curve.append(round(rmse(U, V), 6))
        prec[f"delta_2^{bits}"] = {"rmse": curve, "refreshes": m.stats()["refreshes"]}
        log(f"accuracy Delta 2^{bits}: RMSE {curve[0]} -> {curve[-1]}")
        ctx.close()
    out["precision_without_batching"] = prec
    out.update({"metric": "RMSE (Eq. 10) per iteration, encrypted MF", "value": out["without_batching"]["rmse"][-1],
                "unit": "rmse", "higher_is_better": False,
                "config": {"workload": f"encrypted MF, MovieLens-100K-shaped 943 x 1682, {csr.nnz} ratings, k={K}, "
                                       f"N=2^15, alpha={ACC_LR}, lambda={ACC_LAM}, {iters} iterations, without "
                                       f"batching (rule R1) and with Alg. 2 batch pairs (damp {ACC_DAMP})"}})
    return out


def cpu_leg_accuracy(iters=ACC_ITERS):
    """The FP64 MF (oracle.mf) on the same iterations: the reference curves."""
    _single_thread_env()
    import numpy as np
    from oracle import mf
    import workloads
    csr = workloads.movielens100k_shaped()
    U0, V0 = workloads.init_factors(csr.n_rows, csr.n_cols, 10)
    res = {}
    t0 = time.perf_counter()
    for name in ("without_batching", "with_batching_alg2"):
        U, V, curve = U0, V0, []
        for t in range(iters):
            if name == "without_batching":
                U, V, _ = mf.epoch(U, V, csr.row_ptr, csr.col_idx, csr.values, ACC_LR, ACC_LAM, t, 0.0, "R1")
            else:
                U, V, _ = mf.batch_pair_epoch(U, V, csr.row_ptr, csr.col_idx, csr.values, ACC_LR, ACC_LAM,
                                              512, 512, t, ACC_DAMP)
            curve.append(round(mf.rmse(mf.predict(U, V, csr.row_ptr, csr.col_idx), csr.values), 5))
        res[name] = curve
    dt = time.perf_counter() - t0
    return {"value": 2 * iters * csr.nnz / dt, "unit": "ratings/s", "cores": 1, "kind": "oracle",
            "sample": f"FP64 MF (oracle.mf), both variants, {iters} iterations each", "fp64_rmse": res}



# ---------------------------------------------------------------- helpers
def kernel_table(prof):
    return {k: {"launches": v[0], "total_ms": round(v[1], 3), "avg_us": round(1e3 * v[1] / v[0], 2),
                "alg_GBps": round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[1] > 0 else None}
            for k, v in sorted(prof.items(), key=lambda kv: -kv[1][1])}


def dominant_roofline(prof, schedule):
    """Roofline entry of the kernel with the largest total time: algorithmic
    bytes per launch over its average launch duration (HIP events on the
    library's stream), against the HBM peak."""
    name, (launches, total_ms, total_bytes) = max(prof.items(), key=lambda kv: kv[1][1])
    avg_ms = total_ms / launches
    achieved = (total_bytes / launches) / (avg_ms * 1e-3) / 1e9
    traffic, basis = traffic_of(name, schedule, total_bytes / launches)
    return {"kernel": name, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "traffic_unit": "HBM bytes per launch",
            "traffic_basis": basis, "alg_bytes_per_launch": round(total_bytes / launches),
            "avg_launch_us": round(1e3 * avg_ms, 2), "launches_in_timed_steps": launches}


def mac_summary(mac, prof, N):
    """The masked MAC's work in the timed epochs and the rates it ran at.  Source
    rows are read (2 polynomials), accumulator rows read and written (2 x 2),
    and each mask term forms one limb row of mask values from the resident I0
    row (a permuted read, from cache)."""
    _, ms, _ = prof.get("k_mask_mac_tasks", (0, 0.0, 0.0))
    hbm = 8.0 * N * (2 * mac["group_rows"] + 4 * mac["task_rows"])
    out = dict(mac)
    out["terms_per_group"] = round(mac["terms"] / max(1, mac["groups"]), 2)
    if ms > 0:
        s = ms * 1e-3
        out["source_and_accumulator_GBps"] = round(hbm / s / 1e9, 1)
        out["mask_elements_per_s"] = float(f"{mac['term_rows'] * N / s:.4g}")
    return out


# ---------------------------------------------------------------- MF workloads
def run_mf(which, epochs, ntt_chunk=None):
    """Encrypted CSR-MF epochs: ratings processed per second of epoch time."""
    import numpy as np
    import torch
    import paper_2509_03024_amd as pk
    import workloads
    if which == "mf100k":
        csr = workloads.movielens100k_shaped()
        prm, k, name = pk.mf_n15_params(k=10, lr=0.01, lam=0.02, rule=2, refresh_mode=1), 10, \
            "MovieLens-100K-shaped 943 x 1682"
    else:
        csr = workloads.movielens1m_shaped()
        prm, k, name = pk.mf_n16_params(k=16, lr=0.01, lam=0.02, rule=2, refresh_mode=1), 16, \
            "MovieLens-1M-shaped 6040 x 3706"
    U0, V0 = workloads.init_factors(csr.n_rows, csr.n_cols, k)
    t0 = time.perf_counter()
    ctx = pk.Context(prm, workloads.CRYPTO_SEED)
    ctx.keygen([], conj=False)
    m = pk.MF(ctx)
    n_ct = m.encrypt_csr_rows(csr.n_rows, csr.n_cols, csr.row_ptr, csr.col_idx, csr.values)
    m.init_factors(U0, V0)
    # tuned once the program's rotation keys exist, so that the transform
    # schedules are ranked on batched rotations too
    if ntt_chunk is not None:
        ctx.set_ntt_schedule(ntt_chunk)
    else:
        ctx.autotune()
    sched = ctx.schedule()
    ctx.sync()
    log(f"{which}: set-up (keys, encryption of {n_ct} rating ciphertexts) {time.perf_counter() - t0:.1f} s")
    ks0 = ctx.counters()["key_switches"]
    pk.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.epochs(epochs)
    ctx.sync()
    elapsed = time.perf_counter() - t0
    prof = pk.profile_report()
    pk.profile_enable(False)
    n_ks = ctx.counters()["key_switches"] - ks0
    st = m.stats()
    mac = m.mac_counts()
    U, V = m.decrypt_factors()
    rhat = m.decrypt_predictions(0)
    rmse = float(np.sqrt(np.mean((rhat - csr.values) ** 2)))
    out = {
        "metric": "encrypted CSR-MF ratings/s",
        "value": round(csr.nnz * epochs / elapsed, 2),
        "unit": "ratings/s",
        "epochs": epochs,
        "ms_per_epoch": round(1e3 * elapsed / epochs, 3),
        "refreshes": st["refreshes"],
        "refresh_s": round(st["refresh_seconds"], 3),
        "ratings_per_s_excluding_refresh": round(csr.nnz * epochs / (elapsed - st["refresh_seconds"]), 2),
        "key_switches_per_epoch": round(n_ks / epochs),
        "key_switches_per_s": round(n_ks / elapsed, 1),
        # share of the timed kernels' time in the key-switching kernels
        "key_switch_kernel_share": round(sum(v[1] for k, v in prof.items()
                                             if k.startswith(("k_ntt_pass", "k_basis_convert", "k_ks_")))
                                         / max(1e-9, sum(v[1] for v in prof.values())), 3),
        "config": {"workload": f"encrypted MF, {name}, {csr.nnz} ratings, k={k}, N=2^{prm.log2N}, "
                               f"{n_ct} rating ciphertexts, rule R2, {epochs} epochs "
                               f"({st['refreshes']} table refreshes)"},
        "rmse_last_forward": round(rmse, 5),
        "roofline": dominant_roofline(prof, (sched["ntt_chunk_rows"], sched["ntt_split"])),
        "kernels": kernel_table(prof),
        "masked_mac": mac_summary(mac, prof, 1 << prm.log2N),
    }
    ctx.close()
    return out


def run_tiny(reps=3):
    """Latency of one encrypted MF epoch at the tiny configuration (N = 2^12,
    32 x 64, 205 ratings, k = 4, rule R1); the factors are re-encrypted before
    each epoch (the chain holds one epoch)."""
    import numpy as np
    import paper_2509_03024_amd as pk
    from oracle import mf
    import workloads
    csr = workloads.tiny_ratings()
    U0, V0 = workloads.init_factors(32, 64, 4)
    ctx = pk.Context(pk.tiny_params(k=4, lr=0.01, lam=0.02, rule=1), workloads.CRYPTO_SEED)
    ctx.keygen([])
    m = pk.MF(ctx)
    m.encrypt_csr_rows(32, 64, csr.row_ptr, csr.col_idx, csr.values)
    lat = []
    for _ in range(reps + 1):
        m.init_factors(U0, V0)
        ctx.sync()
        t0 = time.perf_counter()
        m.epochs(1)
        ctx.sync()
        lat.append(time.perf_counter() - t0)
    U, V = m.decrypt_factors()
    Uf, Vf, rf = mf.train(U0, V0, csr.row_ptr, csr.col_idx, csr.values, 0.01, 0.02, 1, rule="R1")
    err = float(max(np.max(np.abs(U - Uf)), np.max(np.abs(V - Vf))))
    ctx.close()
    return {"metric": "encrypted MF epoch latency", "value": round(1e3 * float(np.median(lat[1:])), 3),
            "unit": "ms", "first_epoch_ms": round(1e3 * lat[0], 3), "max_abs_error_vs_fp64": err,
            "config": {"workload": "tiny: 32 x 64, 205 ratings, k=4, N=2^12, rule R1, 1 epoch"}}


# ---------------------------------------------------------------- bootstrapping
BOOT_CFG = (16, 10, 16, 15, 1)  # n slots, squarings r, series degree d, pre-multiplication bits, arcsine term
BOOT_BATCH = 16


def boot_cpu_baseline(ks_leg, ks_per_boot):
    """The oracle's bootstrap is its key switches: the measured N = 2^16
    rotation times the key switches one bootstrap ran on the device.  The
    rotation is timed at the top level while the bootstrap's run at levels
    24..4, so this overstates the oracle's time (understates its rate)."""
    return {"value": ks_leg["value"] / ks_per_boot, "unit": "ciphertexts/s", "cores": ks_leg["cores"],
            "kind": "oracle",
            "sample": f"extrapolated: the oracle's N=2^16 rotation ({1.0 / ks_leg['value']:.1f} s) "
                      f"times {ks_per_boot} key switches per bootstrap"}


def run_boot(batch=BOOT_BATCH, reps=3):
    """Bootstrapping at N = 2^16 on the MF chain (q_0 + 24 x 40-bit, 3 x 60-bit
    special, dnum 7): a batch of level-0 ciphertexts with 16-periodic slots back
    to level L - 20, every step on the device; ciphertexts per second over the
    timed batches, the key switches they ran, and the largest slot error of the
    outputs against the inputs."""
    import numpy as np
    import torch
    import paper_2509_03024_amd as pk
    import workloads
    ctx = pk.Context(pk.mf_n16_params(), workloads.CRYPTO_SEED)
    cfg = pk.BootConfig(*BOOT_CFG)
    n = BOOT_CFG[0]
    t0 = time.perf_counter()
    ctx.keygen(ctx.boot_rotation_steps(cfg), conj=True)
    ctx.autotune()
    vals = [np.tile(np.random.default_rng(300 + i).uniform(-1, 1, n), ctx.N // (2 * n)) for i in range(batch)]
    cts = [ctx.encrypt(v, level=0, scale=2.0 ** 40) for v in vals]
    ctx.sync()
    log(f"bootstrap: keys, schedule and inputs {time.perf_counter() - t0:.1f} s")
    for h in ctx.bootstrap(cts, cfg):          # warm-up
        ctx.free(h)
    ctx.sync()
    ks0 = ctx.counters()["key_switches"]
    pk.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = []
    for r in range(reps):
        if outs:
            for h in outs:
                ctx.free(h)
        outs = ctx.bootstrap(cts, cfg)
    ctx.sync()
    elapsed = time.perf_counter() - t0
    prof = pk.profile_report()
    pk.profile_enable(False)
    n_ks = ctx.counters()["key_switches"] - ks0
    err = max(float(np.max(np.abs(ctx.decrypt(h) - v))) for h, v in zip(outs, vals))
    lvl = ctx.info(outs[0])[0]
    sched = ctx.schedule()
    out = {
        "metric": "bootstraps/s", "value": round(batch * reps / elapsed, 2), "unit": "ciphertexts/s",
        "ms_per_batch": round(1e3 * elapsed / reps, 2), "batch": batch,
        "levels_used": pk.boot_levels(cfg), "output_level": lvl,
        "key_switches_per_bootstrap": round(n_ks / (batch * reps), 1),
        "key_switches_per_s": round(n_ks / elapsed, 1),
        "max_abs_error": err,
        "config": {"workload": f"bootstrapping, N=2^16, q_0 + 24 x 40-bit, dnum 7, n={n} slots, "
                               f"r={BOOT_CFG[1]}, degree {BOOT_CFG[2]}, pre-multiplication 2^{BOOT_CFG[3]}, "
                               f"{'with' if BOOT_CFG[4] else 'without'} the arcsine term, "
                               f"batch of {batch}, |values| <= 1"},
        "roofline": dominant_roofline(prof, (sched["ntt_chunk_rows"], sched["ntt_split"])),
        "kernels": kernel_table(prof),
    }
    ctx.close()
    return out


# ---------------------------------------------------------------- serving
def bench_serve(args):
    """Poisson stream of encrypted per-user PREDICT / UPDATE requests (50/50) over the
    MovieLens-1M-shaped tables (6040 x 3706, k = 16): rows of lognormal(4.5, 1) length
    clipped to [5, 2000], items Zipf(1.1); rows of <= 512 items go to the N = 2^15
    server, longer ones to the N = 2^16 server.  Reports p50/p99 latency per rate."""
    import numpy as np
    import torch
    import paper_2509_03024_amd as pk
    import workloads
    k = 16
    U0, V0 = workloads.init_factors(6040, 3706, k)
    t0 = time.perf_counter()
    servers = {}
    free, total = torch.cuda.mem_get_info()
    budget = 0.8 * free / 2            # 0.8 x free HBM at start, split over the two servers
    for name, prm in (("n15", pk.mf_n15_params(k=k, lr=0.01, lam=0.02, rule=2)),
                      ("n16", pk.mf_n16_params(k=k, lr=0.01, lam=0.02, rule=2))):
        ctx = pk.Context(prm, workloads.CRYPTO_SEED)
        ctx.keygen([])
        ctx.autotune()
        servers[name] = (ctx, pk.Server(ctx, U0, V0, hbm_budget_bytes=budget, max_batch=64))
        log(f"server {name} ready ({time.perf_counter() - t0:.1f} s)")
    rng = np.random.default_rng(7)
    weights = np.arange(1, 3707, dtype=np.float64) ** -1.1
    perm = rng.permutation(3706)
    w = np.empty(3706)
    w[perm] = weights
    w /= w.sum()
    results = []
    serial = 0
    for rate in [float(x) for x in args.rates.split(",")]:
        reqs = []
        for _ in range(args.requests):
            d = int(np.clip(np.rint(rng.lognormal(4.5, 1.0)), 5, 2000))
            items = np.sort(rng.choice(3706, size=d, replace=False, p=w)).astype(np.int32)
            r = np.rint(np.clip(rng.normal(3.5, 1.1, d), 1, 5))
            reqs.append((int(rng.integers(0, 6040)), items, r, int(rng.integers(0, 2))))
        gaps = rng.exponential(1.0 / rate, len(reqs))
        ids = []
        t_start = time.perf_counter()
        t_next = t_start
        for (user, items, r, op), g in zip(reqs, gaps):
            t_next += g
            delay = t_next - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            srv = servers["n15" if len(items) <= 512 else "n16"][1]
            serial += 1
            ids.append((srv, srv.submit(op, user, items, r if op else None, client_serial=serial), len(items)))
            if len(ids) % 250 == 0:
                log(f"rate {rate}: {len(ids)} requests submitted")
        lats = []
        n_ratings = 0
        for srv, rid, d in ids:
            st, res, lat = srv.poll(rid, wait=True)
            lats.append(lat)
            n_ratings += d
            for h in res:
                srv.ctx.free(h)
        wall = time.perf_counter() - t_start
        lats = np.array(lats)
        results.append({"rate": rate, "requests": len(ids), "p50_ms": round(1e3 * float(np.percentile(lats, 50)), 2),
                        "p99_ms": round(1e3 * float(np.percentile(lats, 99)), 2),
                        "ratings_per_s": round(n_ratings / wall, 1)})
        log(f"rate {rate}: {results[-1]}")
    stats = {n: s[1].stats() for n, s in servers.items()}
    for ctx, srv in servers.values():
        srv.close()
        ctx.close()
    top = results[-1]
    print(json.dumps({
        "metric": "p99 latency of encrypted per-user requests", "value": top["p99_ms"], "unit": "ms",
        "n_gpus": 1, "steps": len(results), "warmup": 0, "ms_per_step": None, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "serving: Poisson PREDICT/UPDATE requests over 6040 x 3706 tables, k=16, "
                               "N=2^15 (rows <= 512) / 2^16", "hbm_budget_bytes_per_server": budget},
        "sweep": results, "servers": stats}), flush=True)


def graph_replay(ctx, cts, steps, eager_ms):
    """The HMult and rotation phases of a step captured once in a HIP graph and
    replayed `steps` times (the transform phase works on caller memory and
    waits for it, so it stays eager).  Reported, not fatal."""
    try:
        ctx.sync()
        ctx.graph_begin()
        prods = ctx.hmult_batch(cts, cts[1:] + cts[:1])
        for p in prods:
            ctx.free(p)
        cur, owned = list(cts), []
        for r in CHAIN:
            nxt = ctx.rotate_add_batch(cur, cur, r)
            for h in owned:
                ctx.free(h)
            cur = owned = nxt
        for h in ctx.conjugate_batch(cur) + owned:
            ctx.free(h)
        gid = ctx.graph_end()
        ctx.graph_launch(gid)
        ctx.sync()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.graph_launch(gid)
        ctx.sync()
        t_graph = (time.perf_counter() - t0) / steps
        ctx.graph_destroy(gid)
        log(f"graph replay {1e3 * t_graph:.2f} ms vs eager {1e3 * eager_ms:.2f} ms")
        return {"what": "HMult + rotation phases of a step captured in one HIP graph, replayed",
                "ms_per_replay": round(1e3 * t_graph, 3), "eager_ms": round(1e3 * eager_ms, 3),
                "rotations_per_s_incl_hmult": round(N_CT * (len(CHAIN) + 1) / t_graph, 2)}
    except Exception as e:
        return {"error": repr(e)}


# ---------------------------------------------------------------- key switching (the headline)
def bench_ks(args):
    import numpy as np
    import torch
    import paper_2509_03024_amd as pk
    import workloads

    t0 = time.perf_counter()
    ctx = pk.Context(pk.kernel_batch_params(), workloads.CRYPTO_SEED)
    ctx.keygen(CHAIN, conj=True)
    log(f"context + keys {time.perf_counter() - t0:.1f} s")
    if args.ntt_chunk is not None:
        ctx.set_schedule(args.ntt_chunk, 0, 0, args.ntt_split or 0)
        tune = {"fixed": args.ntt_chunk}
    else:
        tune = ctx.autotune()
    sched = ctx.schedule()
    schedule = (sched["ntt_chunk_rows"], sched["ntt_split"])
    log(f"schedule {tune}")
    N = ctx.N
    L = ctx.L
    t0 = time.perf_counter()
    cts = []
    for i in range(N_CT):
        x = workloads.random_residues(ctx.moduli[: L + 1], N, 2, seed=1000 + i)
        cts.append(ctx.import_ct(x, L, 2.0 ** 40))
    rows = np.arange(L + 1, dtype=np.int32)
    ntt_buf = torch.empty((N_CT * 2 * (L + 1), N), dtype=torch.int64, device="cuda")
    for i in range(N_CT):
        x = workloads.random_residues(ctx.moduli[: L + 1], N, 2, seed=1000 + i)
        ntt_buf[i * 2 * (L + 1):(i + 1) * 2 * (L + 1)] = torch.from_numpy(x.reshape(-1, N).view(np.int64))
    torch.cuda.synchronize()
    log(f"inputs resident in HBM {time.perf_counter() - t0:.1f} s")

    phase = {"ntt_intt": 0.0, "hmult": 0.0, "rotations": 0.0}

    def step(timed):
        t = time.perf_counter()
        ctx.ntt_rows(ntt_buf.data_ptr(), ntt_buf.shape[0], rows, inverse=False)
        ctx.ntt_rows(ntt_buf.data_ptr(), ntt_buf.shape[0], rows, inverse=True)
        ctx.sync()
        t1 = time.perf_counter()
        prods = ctx.hmult_batch(cts, cts[1:] + cts[:1])
        ctx.sync()
        t2 = time.perf_counter()
        for p in prods:
            ctx.free(p)
        cur = list(cts)
        owned = []
        for r in CHAIN:
            nxt = ctx.rotate_add_batch(cur, cur, r)   # cur + Rot(cur, r), the add fused into the key switch
            for h in owned:
                ctx.free(h)
            cur = owned = nxt
        conj = ctx.conjugate_batch(cur)
        for h in conj + owned:
            ctx.free(h)
        ctx.sync()
        t3 = time.perf_counter()
        if timed:
            phase["ntt_intt"] += t1 - t
            phase["hmult"] += t2 - t1
            phase["rotations"] += t3 - t2

    if args.calib_copy:
        src = torch.zeros(64 << 20, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("calibration copy of 512 MiB done")
    for w in range(args.warmup):
        step(False)
        log(f"warmup step {w} done")
    # plain GPU path: the same rotate-and-sum chain, one ciphertext per call
    # (every key switch its own sequence of launches), on PLAIN_CT ciphertexts;
    # before the timed steps, so that they end the run (profiles read its last launches)
    ctx.sync()
    t_pl = time.perf_counter()
    for i in range(PLAIN_CT):
        cur, owned = cts[i], None
        for r in CHAIN:
            rot = ctx.rotate(cur, r)
            nxt = ctx.add(cur, rot)
            ctx.free(rot)
            if owned is not None:
                ctx.free(owned)
            cur = owned = nxt
        cj = ctx.conjugate(cur)
        ctx.free(cj)
        ctx.free(owned)
    ctx.sync()
    plain_rate = PLAIN_CT * (len(CHAIN) + 1) / (time.perf_counter() - t_pl)
    log(f"plain path {plain_rate:.1f} rotations/s")
    # hoisted fan-out: one ModUp per source, then its 15 rotations by 2^0..2^14
    # (16 sources, one call each)
    ctx.sync()
    t0 = time.perf_counter()
    fan = []
    for i in range(16):
        fan += ctx.rotate_hoisted(cts[i], CHAIN)
    ctx.sync()
    t_fan = time.perf_counter() - t0
    for h in fan:
        ctx.free(h)
    hoisted = {"what": "16 sources, each rotated by 2^0..2^14 from one ModUp (csrmf_rotate_hoisted)",
               "rotations_per_s": round(len(fan) / t_fan, 2)}
    log(f"hoisted fan-out {hoisted['rotations_per_s']} rotations/s")
    torch.cuda.synchronize()
    ctx.sync()
    pk.profile_enable(True)
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(True)
        log(f"timed step {s} done")
    ctx.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = pk.profile_report()
    pk.profile_enable(False)

    eager_ms = (phase["hmult"] + phase["rotations"]) / args.steps
    graph = {"skipped": "--no-graph"} if args.no_graph else graph_replay(ctx, cts, args.steps, eager_ms)

    n_rot = N_CT * (len(CHAIN) + 1)
    value = n_rot * args.steps / elapsed
    rot_rate = n_rot * args.steps / phase["rotations"]
    # metric-level rooflines of the rotation phase (25 limbs, digits 9, 9, 7)
    g = -(-(L + 1) // 3)
    digits = [min(g, L + 1 - j * g) for j in range(3) if j * g < L + 1]
    model = ks_model(N, L + 1, ctx.alpha, digits, N_CT)
    # the 40-bit limbs (FP64 butterflies) among all transformed limbs
    t_valu = valu_bound(model, 1.0 - model["int_limb_ntts"] / model["limb_ntts"])
    ks_roof = {
        "what": "rotation phase: rotate-and-add at 25 limbs (read c0, c1; write the result; "
                "the key's share over the 64 ciphertexts that use it)",
        "alg_bytes_per_rotation": round(model["alg_bytes"]),
        "rotations_per_s": round(rot_rate, 2),
        "achieved_GBps": round(rot_rate * model["alg_bytes"] / 1e9, 1),
        "hbm_roofline_rotations_per_s": round(HBM_PEAK_GBS * 1e9 / model["alg_bytes"], 1),
        "ks_hbm_frac": round(rot_rate * model["alg_bytes"] / (HBM_PEAK_GBS * 1e9), 4),
        "counter_bytes_per_step": KS_COUNTER_BYTES_PER_STEP,
        "counter_bytes_per_rotation_whole_step": None if KS_COUNTER_BYTES_PER_STEP is None
        else round(KS_COUNTER_BYTES_PER_STEP / n_rot),
        "modmuls_per_rotation": model["modmuls"],
        "limb_ntts_per_rotation": model["limb_ntts"],
        "valu": None if t_valu is None else {
            "bound_rotations_per_s": round(1.0 / t_valu, 1),
            "frac": round(rot_rate * t_valu, 4),
            "modmul_rates_per_s": MODMUL_RATE,
            "basis": "measured modular-multiply rates x this rotation's multiplies by kind"},
    }
    out = {
        "metric": "key-switch rotations/s at N=2^16",
        "value": round(value, 2),
        "unit": "rotations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "kernel batch: 64 ciphertexts, N=2^16, q0 60-bit + 24 x 40-bit, "
                               "3 x 60-bit special primes, dnum=3; per step NTT+INTT of 3200 limbs, "
                               "64 HMult, 64 x 16 rotate-and-sum key switches",
                   "ciphertexts": N_CT, "log2N": LOGN, "limbs": L + 1, "special": ctx.alpha, "dnum": 3},
        "phase_ms_per_step": {k: round(1e3 * v / args.steps, 3) for k, v in phase.items()},
        # the transform phase runs the forward and the inverse transform of every
        # limb of the 64 ciphertexts; the HMult phase 64 HMult + relin + rescale
        "ntt_limbs_per_s": round(2 * ntt_buf.shape[0] * args.steps / phase["ntt_intt"]),
        "hmults_per_s": round(N_CT * args.steps / phase["hmult"], 1),
        "autotune_ms": tune,
        "rotation_phase_rotations_per_s": round(rot_rate, 2),
        "plain_gpu_path": {"rotations_per_s": round(plain_rate, 2), "ciphertexts": PLAIN_CT,
                           "what": "same rotate-and-sum chain, one ciphertext per call",
                           "batched_rotation_phase_speedup": round(rot_rate / plain_rate, 2)},
        "graph_path": graph,
        "hoisted_fan_out": hoisted,
        "roofline": dominant_roofline(prof, schedule),
        "ks_roofline": ks_roof,
        "kernels": kernel_table(prof),
    }
    ctx.close()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only (one MI355X); --gpus must be 1"}))
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    torch.cuda.set_device(0)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "accuracy":
        out = run_accuracy(args.epochs or ACC_ITERS)
        out.update({"n_gpus": 1, "steps": args.epochs or ACC_ITERS, "warmup": 0, "scaling": "weak",
                    "vs_baseline": None, "dtype": "u64", "data": "synthetic"})
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = run_cpu_legs({"acc": (cpu_leg_accuracy, (args.epochs or ACC_ITERS,))})["acc"]
            ref = out["cpu_baseline"].get("fp64_rmse", {})
            for name, curve in ref.items():
                enc = out[name]["rmse"]
                out[name]["max_abs_diff_vs_fp64"] = round(max(abs(a - b) for a, b in zip(enc, curve)), 6)
            for v in out.get("precision_without_batching", {}).values():
                ref0 = ref.get("without_batching", [])
                v["max_abs_diff_vs_fp64"] = round(max(abs(a - b) for a, b in zip(v["rmse"], ref0)), 6)
        print(json.dumps(out), flush=True)
        return
    if args.workload == "boot":
        out = run_boot()
        out.update({"n_gpus": 1, "steps": 3, "warmup": 1, "ms_per_step": out["ms_per_batch"],
                    "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
                    "data": "synthetic"})
        print(json.dumps(out), flush=True)
        return
    if args.workload in ("mf100k", "mf1m"):
        epochs = args.epochs or (10 if args.workload == "mf100k" else 5)
        out = run_mf(args.workload, epochs, args.ntt_chunk)
        out.update({"n_gpus": 1, "steps": epochs, "warmup": 0, "ms_per_step": out["ms_per_epoch"],
                    "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
                    "data": "synthetic"})
        if not args.no_cpu_baseline and args.workload == "mf100k":
            legs = run_cpu_legs({"mf100k": (cpu_leg_mf100k, (out["key_switches_per_epoch"], epochs))})
            out["cpu_baseline"] = legs["mf100k"]
        print(json.dumps(out), flush=True)
        return
    out = bench_ks(args)
    if not args.no_mf:
        log("MF-100K: 10 epochs ...")
        out["mf100k"] = run_mf("mf100k", args.epochs or 10)
        log(f"MF-100K {out['mf100k']['value']} ratings/s")
        out["tiny"] = run_tiny()
        log(f"tiny epoch {out['tiny']['value']} ms")
        log("bootstrapping at N = 2^16 ...")
        out["bootstrap"] = run_boot()
        log(f"bootstrap {out['bootstrap']['value']} ciphertexts/s, error {out['bootstrap']['max_abs_error']:.2e}")
    if not args.no_cpu_baseline:
        log("cpu baselines (oracle, parallel processes) ...")
        legs = {"ks": (cpu_leg_ks, (max(1, min(8, (os.cpu_count() or 2) - 3)),))}
        if not args.no_mf:
            legs["mf100k"] = (cpu_leg_mf100k, (out["mf100k"]["key_switches_per_epoch"], out["mf100k"]["epochs"]))
            legs["tiny"] = (cpu_leg_tiny, ())
        res = run_cpu_legs(legs)
        out["cpu_baseline"] = res["ks"]
        if not args.no_mf:
            out["mf100k"]["cpu_baseline"] = res["mf100k"]
            out["tiny"]["cpu_baseline"] = res["tiny"]
            out["bootstrap"]["cpu_baseline"] = boot_cpu_baseline(res["ks"], out["bootstrap"]["key_switches_per_bootstrap"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
