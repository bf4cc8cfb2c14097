"""bench.py on the host: more than one GPU is refused before anything touches a device; the roofline
arithmetic and the keying of the measured traffic by its sources, on made-up stage times."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""


def _stages(gemm_ms, pa_ms, pb_ms, rows):
    st = {k: {"ms_avg": 0.0, "launches": 0, "ms_total": 0.0} for k in ("pass_a", "pass_b", "match_gemm")}
    st["pass_a"].update(ms_avg=pa_ms, launches=2 * len(rows), ms_total=2 * len(rows) * pa_ms)
    st["pass_b"].update(ms_avg=pb_ms, launches=2 * len(rows), ms_total=2 * len(rows) * pb_ms)
    st["match_gemm"].update(ms_avg=gemm_ms, launches=len(rows), ms_total=len(rows) * gemm_ms)
    st["_rows"] = rows
    return st


def test_roofline_arithmetic_and_traffic_gating():
    """bench.roofline on made-up stage times: the kernel with the most time per step is chosen, achieved =
    algorithmic work / time with the GEMM's flops from each profiled step's own rows, and the measured
    traffic is reported only for the workload and sources it was taken on."""
    sys.path.insert(0, ROOT)
    import bench

    rows = [(6000, 9000), (6400, 9800)]
    st = _stages(0.24, 0.08, 0.065, rows)
    r = bench.roofline(st, 1024, 1024, 4, 6, 6400, 9800, 216)
    flop = sum(2.0 * a * b * 216 for a, b in rows) / len(rows)
    assert r["kernel"] == "match_gemm" and r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert abs(r["achieved"] - flop / 0.24e-3 / 1e12) < 0.01
    assert abs(r["frac"] - r["achieved"] / bench.FP32_MFMA_PEAK_TFLOPS) < 1e-3
    hw = 1024 * 1024
    assert abs(r["other"]["pass_a"]["achieved"] - hw * (8 + 8 * 24) / 0.08e-3 / 1e9) < 0.01
    assert abs(r["other"]["pass_b"]["achieved"] - hw * (8 * 24 + 5) / 0.065e-3 / 1e9) < 0.01
    # the measured traffic is reported at the workload it was taken on while its sources are unchanged ...
    mt = bench.MEASURED_TRAFFIC["match_gemm"]
    fresh = bench.sources_hash(mt["sources"]) == mt["sha"]
    assert r["traffic"] == (mt["bytes"] if fresh else None)
    # ... and not at another size
    assert bench.roofline(st, 2048, 2048, 4, 6, 6400, 9800, 216)["traffic"] is None
    # a filter-dominated step picks the column pass against HBM
    r2 = bench.roofline(_stages(0.05, 0.30, 0.20, rows), 1024, 1024, 4, 6, 6400, 9800, 216)
    assert r2["kernel"] == "pass_a" and r2["bound"] == "hbm" and r2["unit"] == "GB/s"
    # GEMM launches must pair with the profiled steps
    bad = _stages(0.24, 0.08, 0.065, rows)
    bad["match_gemm"]["launches"] = 3
    try:
        bench.roofline(bad, 1024, 1024, 4, 6, 6400, 9800, 216)
    except RuntimeError:
        pass
    else:
        raise AssertionError("mismatched GEMM launches accepted")


def test_traffic_is_keyed_by_the_sources_it_was_taken_on(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench

    # a changed source file changes the key, so traffic taken on other sources is never reported
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    csrc = tmp_path / "paper_2303_00319_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in ("match.hip", "api.hip"):
        (csrc / name).write_text("x")
    h1 = bench.sources_hash(("match.hip", "api.hip"))
    (csrc / "api.hip").write_text("y")
    assert bench.sources_hash(("match.hip", "api.hip")) != h1
