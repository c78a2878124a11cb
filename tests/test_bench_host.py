"""Host logic of bench.py (no GPU): the measured-traffic lookup that feeds the
roofline object, the masked-MAC summary of the MF lines, and the one-GPU rule."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


_T = {"k_ntt_pass<rows,fwd>": {"schedule": 2048, "split": 8, "bytes": 1500.0e6, "alg_bytes": 1471.1e6},
      "k_basis_convert": {"schedule": None, "bytes": 1174.6e6, "alg_bytes": 1174.4e6}}


def test_traffic_at_the_measured_schedule_is_the_measurement():
    b = _bench()
    b.TRAFFIC = dict(_T)
    for name, t in b.TRAFFIC.items():
        if t["schedule"] is None:
            val, basis = b.traffic_of(name, (512, 8), t["alg_bytes"])
            assert val == t["bytes"] and basis == "rocprofv3 counters"
        else:
            val, basis = b.traffic_of(name, (t["schedule"], t["split"]), t["alg_bytes"])
            assert val == t["bytes"] and str(t["schedule"]) in basis


def test_traffic_under_another_schedule_scales_with_the_launch():
    b = _bench()
    b.TRAFFIC = dict(_T)
    name, t = next((n, t) for n, t in b.TRAFFIC.items() if t["schedule"] is not None)
    other = 64 if t["schedule"] != 64 else 128
    half = t["alg_bytes"] / 2
    val, basis = b.traffic_of(name, (other, t["split"]), half)
    assert abs(val - t["bytes"] / 2) <= 1.0
    assert "scaled" in basis and str(other) in basis


def test_traffic_of_smaller_launches_is_scaled():
    """Another workload's launches (a smaller batch) at the measured schedule:
    the counters are scaled by the algorithmic bytes, not reported as measured."""
    b = _bench()
    b.TRAFFIC = dict(_T)
    for name, t in b.TRAFFIC.items():
        sched = (512, 8) if t["schedule"] is None else (t["schedule"], t["split"])
        val, basis = b.traffic_of(name, sched, t["alg_bytes"] / 4)
        assert abs(val - t["bytes"] / 4) <= 1.0
        assert "scaled" in basis


def test_traffic_under_another_split_is_not_measured():
    """A different split of the transform's stages changes the passes' access
    pattern: their counters do not carry over."""
    b = _bench()
    b.TRAFFIC = dict(_T)
    t = b.TRAFFIC["k_ntt_pass<rows,fwd>"]
    val, basis = b.traffic_of("k_ntt_pass<rows,fwd>", (t["schedule"], t["split"] + 1), t["alg_bytes"])
    assert val is None and "not measured" in basis


def test_measured_traffic_entries_are_consistent():
    b = _bench()
    for name, t in b.TRAFFIC.items():
        assert t["bytes"] > 0 and t["alg_bytes"] > 0
        assert t["schedule"] is None or (t["schedule"] > 0 and 6 <= t["split"] <= 9)


def test_rotation_model_hand_counts():
    """One rotation at 24 limbs, digits 9, 9, 6, three special primes, key shared
    by 64 ciphertexts: read c0, c1 (24 MiB), write 24 MiB, key 3 x 2 x 27 limbs / 64;
    135 limb transforms (24 inverse + 18 + 18 + 21 forward of ModUp, 6 inverse and
    48 forward of ModDown)."""
    b = _bench()
    m = b.ks_model(1 << 16, 24, 3, [9, 9, 6], 64)
    limb = 8 << 16
    assert m["alg_bytes"] == 96 * limb + 162 * limb / 64        # 51.66 MB
    assert round(m["alg_bytes"] / 1e6, 2) == 51.66
    assert m["limb_ntts"] == 135
    assert m["butterflies"] == 135 * (1 << 15) * 16
    assert m["conv_macs"] == (1 << 16) * (9 * 18 + 9 * 18 + 6 * 21 + 2 * 3 * 24)
    assert m["inner_mults"] == (1 << 16) * 3 * 27 * 2
    # terms into 60-bit targets: every digit into the 3 special primes, digits 1
    # and 2 into q_0, and ModDown's 3 special limbs into q_0 for both polynomials
    assert m["conv_macs_int"] == (1 << 16) * ((9 + 9 + 6) * 3 + (9 + 6) + 2 * 3)
    # inner products on the 3 special limbs and q_0, both key polynomials, 3 digits
    assert m["inner_mults_int"] == (1 << 16) * 3 * 4 * 2
    assert m["scale_mults_int"] == (1 << 16) * 2


def test_traffic_of_an_unmeasured_kernel_is_null():
    b = _bench()
    assert b.traffic_of("k_not_measured", (2048, 8), 1e9) == (None, None)


def test_mac_summary_rates():
    b = _bench()
    N = 1 << 15
    mac = {"tasks": 10, "groups": 40, "terms": 44, "const_terms": 2,
           "task_rows": 100, "group_rows": 400, "term_rows": 440}
    prof = {"k_mask_mac_tasks": (3, 2.0, 0.0)}   # 3 launches, 2 ms
    out = b.mac_summary(mac, prof, N)
    assert out["terms_per_group"] == 1.1
    hbm = 8.0 * N * (2 * 400 + 4 * 100)
    assert abs(out["source_and_accumulator_GBps"] - round(hbm / 2e-3 / 1e9, 1)) < 1e-9
    assert out["mask_elements_per_s"] == float(f"{440 * N / 2e-3:.4g}")
    # without a timed MAC launch only the counts are reported
    out = b.mac_summary(mac, {}, N)
    assert "source_and_accumulator_GBps" not in out and out["groups"] == 40


def test_bootstrap_cpu_baseline_extrapolates_the_rotation():
    b = _bench()
    leg = {"value": 1.0 / 30.0, "unit": "key-switch rotations/s", "cores": 1}
    out = b.boot_cpu_baseline(leg, 56.0)
    assert abs(out["value"] - 1.0 / (30.0 * 56.0)) < 1e-15
    assert out["cores"] == 1 and out["kind"] == "oracle" and "56.0 key switches" in out["sample"]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)
