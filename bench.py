"""Benchmark: batched CKKS key switching at N = 2^16 on one MI355X.

Workload (the kernel-batch configuration): 64 ciphertexts of uniform random
residues at N = 2^16 with q_0 (60-bit) + 24 x 40-bit scale primes, 3 x 60-bit
special primes, dnum = 3.  One step is one pass of the whole batched path:
  (i)   forward + inverse NTT of all 64 x 2 x 25 limbs,
  (ii)  64 HMult (tensor, relinearise, rescale) ct_i x ct_{i+1 mod 64},
  (iii) per ciphertext a rotate-and-sum chain over steps 2^0 .. 2^14 plus a
        conjugation: 16 key switches per ciphertext, 1024 per step.
value = key-switch rotations per second over whole steps (1024 * K / time of
the K timed steps, phases (i) and (ii) included).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
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
# HBM bytes per launch of a kernel in the timed step (average over the step's
# launches), from rocprofv3 FETCH_SIZE (x2.0) + WRITE_SIZE (x1.0) counters, the
# factors read off a 512 MiB copy (profiles/ks_kernel_batch_n16_hbm_counters.md),
# with the NTT schedule (rows per pair of passes) of that run and the
# algorithmic bytes of its launches; only valid for the kernel code the counters
# were taken on.  Under another schedule the launches differ in size and the
# measured bytes are scaled by the algorithmic bytes (traffic_basis says which).
# (schedule None: the kernel's launches do not depend on the NTT schedule.)
TRAFFIC = {"k_ntt_pass<rows,fwd>": {"schedule": 2048, "bytes": 1494.4e6, "alg_bytes": 1471.1e6},
           "k_basis_convert": {"schedule": None, "bytes": 1174.6e6, "alg_bytes": 1174.4e6}}


def traffic_of(name, schedule, alg_bytes):
    t = TRAFFIC.get(name)
    if t is None:
        return None, None
    if t["schedule"] is None:
        return t["bytes"], "rocprofv3 counters"
    if t["schedule"] == schedule:
        return t["bytes"], f"rocprofv3 counters at NTT schedule {schedule}"
    return round(t["bytes"] / t["alg_bytes"] * alg_bytes), \
        f"rocprofv3 counters at NTT schedule {t['schedule']}, scaled by algorithmic bytes to schedule {schedule}"



def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="ks", choices=["ks", "mf100k", "mf1m", "serve"],
                    help="ks: batched key switching (default); mf100k / mf1m: encrypted MF epochs on the "
                         "MovieLens-100K / -1M shaped synthetic matrices")
    ap.add_argument("--epochs", type=int, default=10, help="MF workloads: epochs (the 100K workload refreshes as needed)")
    ap.add_argument("--rates", default="10,25,50,100,200", help="serve: Poisson arrival rates (requests/s)")
    ap.add_argument("--requests", type=int, default=60, help="serve: requests per rate")
    ap.add_argument("--ntt-chunk", type=int, default=None,
                    help="fix the NTT schedule (rows per pair of passes) instead of autotuning (for profiles)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="copy a 512 MiB device buffer once before the timed steps (reference for HBM counters)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline():
    """The oracle (numpy, one host thread) on a bounded sample: one non-hoisted
    rotation of one 25-limb ciphertext at N = 2^16 (key generation untimed)."""
    import numpy as np
    from oracle import ckks, params
    import workloads
    prm = params.config_kernel_batch()
    orc = ckks.Context(prm, workloads.CRYPTO_SEED)
    t0 = time.perf_counter()
    orc.keygen(rot_steps=[1])
    t_key = time.perf_counter() - t0
    x = workloads.random_residues(prm.q, prm.N, 2, seed=99)
    ct = ckks.Ciphertext(x[0], x[1], 2.0 ** 40)
    t0 = time.perf_counter()
    orc.rotate(ct, 1)
    t_rot = time.perf_counter() - t0
    return {"value": 1.0 / t_rot, "unit": "key-switch rotations/s", "cores": 1, "kind": "oracle",
            "sample": f"1 non-hoisted rotation of one ciphertext, N=2^16, 25 limbs, dnum=3 "
                      f"({t_rot:.1f} s; key generation {t_key:.1f} s untimed)"}


def bench_mf(args):
    """Encrypted CSR-MF epochs: value = ratings processed per second of epoch time."""
    import numpy as np
    import torch
    import paper_2509_03024_amd as pk
    import workloads
    if args.workload == "mf100k":
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
    if args.ntt_chunk is not None:
        pk.set_ntt_schedule(args.ntt_chunk)
    else:
        ctx.autotune()
    m = pk.MF(ctx)
    n_ct = m.encrypt_csr_rows(csr.n_rows, csr.n_cols, csr.row_ptr, csr.col_idx, csr.values)
    m.init_factors(U0, V0)
    ctx.sync()
    log(f"MF set-up (keys, encryption of {n_ct} rating ciphertexts) {time.perf_counter() - t0:.1f} s")
    pk.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.epochs(args.epochs)
    ctx.sync()
    elapsed = time.perf_counter() - t0
    prof = pk.profile_report()
    pk.profile_enable(False)
    st = m.stats()
    mac = m.mac_counts()
    U, V = m.decrypt_factors()
    rhat = m.decrypt_predictions(0)
    rmse = float(np.sqrt(np.mean((rhat - csr.values) ** 2)))
    out = {
        "metric": "encrypted CSR-MF ratings/s",
        "value": round(csr.nnz * args.epochs / elapsed, 2),
        "refreshes": st["refreshes"],
        "refresh_s": round(st["refresh_seconds"], 3),
        "ratings_per_s_excluding_refresh": round(csr.nnz * args.epochs / (elapsed - st["refresh_seconds"]), 2),
        "unit": "ratings/s",
        "n_gpus": 1, "steps": args.epochs, "warmup": 0,
        "ms_per_step": round(1e3 * elapsed / args.epochs, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"encrypted MF, {name}, {csr.nnz} ratings, k={k}, N=2^{prm.log2N}, "
                               f"{n_ct} rating ciphertexts, rule R2, {args.epochs} epochs "
                               f"({st['refreshes']} table refreshes)"},
        "rmse_last_forward": round(rmse, 5),
        "kernels": {k2: {"launches": v[0], "total_ms": round(v[1], 3)}
                    for k2, v in sorted(prof.items(), key=lambda kv: -kv[1][1])},
        "masked_mac": mac_summary(mac, prof, 1 << prm.log2N),
    }
    ctx.close()
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """Poisson stream of encrypted per-user PREDICT / UPDATE requests (50/50) over the
    MovieLens-1M-shaped tables (6040 x 3706, k = 16): rows of lognormal(4.5, 1) length
    clipped to [5, 2000], items Zipf(1.1); rows of <= 512 items go to the N = 2^15
    server, longer ones to the N = 2^16 server.  Reports p50/p99 latency per rate."""
    import threading
    import numpy as np
    import paper_2509_03024_amd as pk
    import workloads
    k = 16
    U0, V0 = workloads.init_factors(6040, 3706, k)
    t0 = time.perf_counter()
    servers = {}
    for name, prm in (("n15", pk.mf_n15_params(k=k, lr=0.01, lam=0.02, rule=2)),
                      ("n16", pk.mf_n16_params(k=k, lr=0.01, lam=0.02, rule=2))):
        ctx = pk.Context(prm, workloads.CRYPTO_SEED)
        ctx.keygen([])
        ctx.autotune()
        servers[name] = (ctx, pk.Server(ctx, U0, V0, hbm_budget_bytes=40e9, max_batch=64))
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
                               "N=2^15 (rows <= 512) / 2^16"},
        "sweep": results, "servers": stats}), flush=True)


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


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload != "ks":
        return bench_mf(args)
    import numpy as np
    import torch
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    torch.cuda.set_device(0)
    import paper_2509_03024_amd as pk
    import workloads

    t0 = time.perf_counter()
    ctx = pk.Context(pk.kernel_batch_params(), workloads.CRYPTO_SEED)
    ctx.keygen(CHAIN, conj=True)
    log(f"context + keys {time.perf_counter() - t0:.1f} s")
    if args.ntt_chunk is not None:
        pk.set_ntt_schedule(args.ntt_chunk)
        tune = {"fixed": args.ntt_chunk}
        schedule = args.ntt_chunk
    else:
        tune = ctx.autotune()
        schedule = tune["chosen"]
    log(f"NTT schedule {tune}")
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

    n_rot = N_CT * (len(CHAIN) + 1)
    value = n_rot * args.steps / elapsed
    dom = max(prof.items(), key=lambda kv: kv[1][1])
    name, (launches, total_ms, total_bytes) = dom
    avg_ms = total_ms / launches
    achieved = (total_bytes / launches) / (avg_ms * 1e-3) / 1e9
    traffic, traffic_basis = traffic_of(name, schedule, total_bytes / launches)
    kernel_table = {k: {"launches": v[0], "total_ms": round(v[1], 3), "avg_us": round(1e3 * v[1] / v[0], 2),
                        "alg_GBps": round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[1] > 0 else None}
                    for k, v in sorted(prof.items(), key=lambda kv: -kv[1][1])}
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
        "autotune_ms": tune,
        "rotation_phase_rotations_per_s": round(n_rot * args.steps / phase["rotations"], 2),
        "plain_gpu_path": {"rotations_per_s": round(plain_rate, 2), "ciphertexts": PLAIN_CT,
                           "what": "same rotate-and-sum chain, one ciphertext per call",
                           "batched_rotation_phase_speedup": round(n_rot * args.steps / phase["rotations"] / plain_rate, 2)},
        "roofline": {"kernel": name, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch", "traffic_basis": traffic_basis,
                     "alg_bytes_per_launch": round(total_bytes / launches),
                     "avg_launch_us": round(1e3 * avg_ms, 2), "launches_in_timed_steps": launches},
        "kernels": kernel_table,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline()
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
