#!/usr/bin/env python3
"""RIFT2 hot path on one MI355X: image pairs/s and per-pair latency.

Workload (the 1024 x 1024 case): seeded synthetic uint8 pairs (200 blobs,
60 rectangles/lines, random rotation + translation, 8-knot nonlinear remap,
Gamma speckle with 4 looks), log-Gabor bank N_s = 4 x N_o = 6, FAST with at
most 5000 keypoints per image, 6x6x6 = 216-d dominant-index descriptors,
exhaustive matching with the 0.9 ratio test.  One step = one pair through
every stage: filter bank / MIM / moments (x2), FAST (x2), descriptors (x2),
matching.  Inputs are resident in HBM before timing; each pair's step is a
replayed HIP graph (the two images' stages on two streams, matching after
both).  The same stages launched directly on the two streams are timed as
well ("other_launch"; --direct reports them as the headline): that form is
sometimes a few per cent faster and sometimes 15 % slower from run to run.  With --pipeline the software-pipelined form is timed as well and
reported under "pipelined": step k runs pair k's image stages while pair
k-1's matching runs on a third stream, on alternating buffer sets; its
p50/p99 are per-pair latencies (a pair spans two consecutive steps).

Two forms are timed: plain FP32 (distance GEMM on FP32 MFMA) -- the
reported `value` -- and mixed (BF16 MFMA on the exact integer counts, the
same distances bit for bit), reported under "mixed".

The paper's comparison is timed beside them under "rift_ring": the same
pairs through RIFT's convolution-sequence ring (N_o descriptors per template
keypoint, N_o-fold matching, no dominant index), with the same detector and
matching precision, and RIFT2's speed-up over it.

Prints one JSON line.  `--gpus` above 1 is rejected: the benchmark runs on
one GPU.
"""
from __future__ import annotations

import argparse
import faulthandler
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0
FP8_MFMA_PEAK_TFLOPS = 5000.0
FP64_PEAK_TFLOPS = 78.6  # vector FP64, FMA counted as two flops

# Per-launch HBM bytes (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, the factors a
# plain copy of known size gives) from two rocprofv3 --pmc runs at 1024 x 1024
# (N_s = 4, N_o = 6, 5000 keypoints), valid only for the sources they were
# taken on (hash of the listed files).
MEASURED_TRAFFIC = {
    "pass_a": {"sources": ("fft.hpp", "filter.hip", "api.hip"), "sha": "11f070d763059bd9", "bytes": 213314167},
    "pass_b": {"sources": ("fft.hpp", "filter.hip", "api.hip"), "sha": "11f070d763059bd9", "bytes": 206928490},
    "match_gemm": {"sources": ("match.hip", "api.hip"), "sha": "735150c34e71c285", "bytes": 419825069},
}


def sources_hash(files):
    import hashlib

    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2303_00319_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--pairs", type=int, default=4, help="distinct resident pairs cycled through")
    ap.add_argument("--config", type=int, default=1, choices=(1, 2, 4),
                    help="workload: 1 = 1024^2 u8 pair, 5000 keypoints (the headline); 2 = 2048^2, 20000 keypoints; "
                         "4 = 4096^2 12-bit u16, N_s=5 N_o=8, 50000 keypoints, 288-d")
    ap.add_argument("--forms", default=None,
                    help="matching precisions to time, first one is `value` (default fp32,bf16; config 4: fp8,bf16)")
    ap.add_argument("--ring-forms", default=None,
                    help="matching precisions of RIFT's ring form to time beside RIFT2 (default fp32,bf16; "
                         "config 4: bf16; '' for none)")
    ap.add_argument("--variants", default="turned,union,batched",
                    help="other forms of the path to time (FP32 matching): turned = descriptor grid turned by the "
                         "dominant index, union = RIFT's corner + edge detector, batched = both images' filter banks "
                         "in shared launches (rift2_filter_mim_batch) instead of one image per stream; '' for none")
    ap.add_argument("--size", type=int, default=0, help="override the image side")
    ap.add_argument("--keypoints", type=int, default=0, help="override the keypoints per image")
    ap.add_argument("--direct", action="store_true",
                    help="report the stages launched directly on their streams as the headline (default: the "
                         "replayed graph of the step, whose timing is stable from run to run; the other form is "
                         "always timed too)")
    ap.add_argument("--no-graph", action="store_true", help="direct launches only (no graph capture at all)")
    ap.add_argument("--pipeline", action="store_true",
                    help="also time the software-pipelined form (pair k's image stages beside pair k-1's matching)")
    ap.add_argument("--serial", action="store_true",
                    help="run both images' stages on one stream, one pair per step (no overlap; per-kernel "
                         "durations for rocprofv3)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--serve", action="store_true",
                    help="serving form instead of the headline: a stream of mixed-size pair requests through the "
                         "continuous-batching engine (prints its own JSON line)")
    ap.add_argument("--requests", type=int, default=256, help="--serve: number of requests")
    ap.add_argument("--rates", default="5,10,20,40,80,0",
                    help="--serve: Poisson arrival rates in pairs/s to sweep (0 = all at once, saturation)")
    ap.add_argument("--budget-gib", type=float, default=32.0, help="--serve: HBM arena for in-flight requests")
    ap.add_argument("--inflight", type=int, default=8, help="--serve: requests running at once (two streams each)")
    ap.add_argument("--pool", type=int, default=4, help="--serve: distinct resident pairs per size")
    ap.add_argument("--serve-sizes", default=None, help="--serve: comma-separated square sizes (default: the mix)")
    ap.add_argument("--serve-keypoints", type=int, default=0, help="--serve: keypoints per image (0: 2e-3 HW)")
    ap.add_argument("--serve-form", default="bf16", choices=("fp32", "bf16", "fp8"), help="--serve: matching form")
    ap.add_argument("--serve-batch", type=int, default=4,
                    help="serving: queued same-size requests admitted together, filter banks in shared launches")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the short serving sweep of the default line (rates 5..80 pairs/s + saturation)")
    ap.add_argument("--sweep-requests", type=int, default=48,
                    help="requests per arrival rate in the default line's serving sweep (saturation: --requests)")
    ap.add_argument("--ransac", type=int, default=0,
                    help="hypotheses of an outlier-removal stage appended to every pair step (0: none)")
    ap.add_argument("--ransac-matches", type=int, default=5000,
                    help="matches of the planted set the standalone outlier-removal timing runs on")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 256 MiB read + 256 MiB write elementwise kernel first (HBM counter scale)")
    return ap.parse_args()


def percentile(xs, q):
    s = sorted(xs)
    if not s:
        return float("nan")
    k = (len(s) - 1) * q / 100.0
    lo, hi = int(math.floor(k)), int(math.ceil(k))
    return s[lo] + (s[hi] - s[lo]) * (k - lo)


def _form_params(r2, args, precision):
    pc, det, dp, mp = r2.defaults()
    pc.n_scales, pc.n_orient = args.n_scales, args.n_orient
    dp.n_orient = args.n_orient
    det.max_keypoints = args.keypoints
    mp.precision = precision
    return pc, det, dp, mp


def _last_pair(pipe):
    return {"keypoints": (int(pipe.a.nk.item()), int(pipe.b.nk.item())),
            "descriptor_rows": (int(pipe.a.nd.item()), int(pipe.b.nd.item())),
            "matches": int(pipe.n_out.item())}


def _ransac_words(torch, n_hyp, seed=0):
    from synth.matches import sample_words

    return torch.from_numpy(sample_words(seed, n_hyp).view("int32").copy()).to(torch.device("cuda:0"))


def time_single(r2, torch, imgs, args, precision, ring=False, variant=None, graph=None):
    """One pair per step, nothing overlapped: a replayed graph per resident pair, or the stages
    launched directly on their streams (graph=False)."""
    if graph is None:
        graph = not (args.direct or args.no_graph)
    pc, det, dp, mp = _form_params(r2, args, precision)
    if variant == "turned":
        dp.mode = r2.DESC_TURNED
    words = _ransac_words(torch, args.ransac) if args.ransac > 0 else None
    pipe = r2.PairPipeline(args.size, args.size, pc, det, dp, mp, serial=args.serial, ransac_words=words, ring=ring,
                           union=variant == "union", batched=variant == "batched")
    graphs = []
    if graph:
        for i, (a, b) in enumerate(imgs):
            print(f"[bench] capture single-pair step {i}", file=sys.stderr, flush=True)
            graphs.append(pipe.capture(a, b))

    def step(k):
        i = k % len(imgs)
        if graphs:
            graphs[i].replay()
        else:
            pipe.run(*imgs[i])

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record()
        step(k)
        ev[k][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = [s.elapsed_time(e) for s, e in ev]
    return {
        "pairs_per_s": args.steps / wall,
        "ms_per_step": 1000.0 * wall / args.steps,
        "p50_ms": percentile(lat, 50),
        "p99_ms": percentile(lat, 99),
        "last_pair": _last_pair(pipe),
        "pipe": pipe,
    }


def time_pipelined(r2, torch, imgs, args, precision):
    """Step k = pair k's image stages beside pair k-1's matching (PipelinedPairs)."""
    if len(imgs) % 2:
        raise SystemExit("--pairs must be even for the pipelined form")
    pc, det, dp, mp = _form_params(r2, args, precision)
    pp = r2.PipelinedPairs(args.size, args.size, pc, det, dp, mp)
    n = len(imgs)
    pp.step(0, *imgs[0])  # fills one buffer set; matches nothing
    graphs = {}
    if not args.no_graph:
        for k in range(1, n + 1):
            print(f"[bench] capture pipelined step {k}", file=sys.stderr, flush=True)
            graphs[k % n] = pp.capture(k, *imgs[k % n])
    # steps continue from n + 1 so that every step's parity matches its graph's
    k0 = n + 1

    def step(k):
        if graphs:
            graphs[k % n].replay()
        else:
            pp.step(k, *imgs[k % n])

    for k in range(k0, k0 + args.warmup):
        step(k)
    torch.cuda.synchronize()
    first = k0 + args.warmup
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for q in range(args.steps):
        ev[q][0].record()
        step(first + q)
        ev[q][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # pair first + q: image stages in step q, matching in step q + 1
    lat = [ev[q][0].elapsed_time(ev[q + 1][1]) for q in range(args.steps - 1)]
    steps_ms = [s.elapsed_time(e) for s, e in ev]
    last = first + args.steps - 1
    return {
        "pairs_per_s": args.steps / wall,
        "ms_per_step": 1000.0 * wall / args.steps,
        "p50_ms": percentile(lat, 50),
        "p99_ms": percentile(lat, 99),
        "step_p50_ms": percentile(steps_ms, 50),
        "last_pair": _last_pair(pp.matched_set(last)),
        "pipe": pp.sets[0],
    }


def time_form(r2, torch, imgs, args, precision):
    single = time_single(r2, torch, imgs, args, precision)
    single["other_launch"] = None
    if not args.no_graph:
        graph = not args.direct
        other = time_single(r2, torch, imgs, args, precision, graph=not graph)
        single["other_launch"] = {"launch": "direct" if graph else "graph replay",
                                  **{k: round(other[k], 4) for k in ("pairs_per_s", "ms_per_step", "p50_ms", "p99_ms")}}
    single["pipelined"] = None
    if args.pipeline and not args.serial:
        res = time_pipelined(r2, torch, imgs, args, precision)
        single["pipelined"] = {k: round(res[k], 4) for k in ("pairs_per_s", "ms_per_step", "p50_ms", "p99_ms")}
    return single


def profile_stages(r2, torch, pipe, imgs, steps):
    """Per-kernel-group GPU time with HIP events recorded on the launch stream.

    The stages run serially on one stream here so that each event pair times
    its own kernels only (the timed loop overlaps the two images' stages).
    """
    r2.profile_read()
    r2.profile_enable(True)
    rows = []
    for k in range(steps):
        a, b = imgs[k % len(imgs)]
        pipe.run_serial(a, b)
        # this step's row counts (device values, copied in stream order before the next step overwrites them)
        rows.append((pipe.a.nd.clone(), pipe.b.nd.clone()))
    torch.cuda.synchronize()
    r2.profile_enable(False)
    raw = r2.profile_read()
    out = {k: {"ms_avg": (v[0] / v[1] if v[1] else 0.0), "launches": v[1], "ms_total": v[0]} for k, v in raw.items()}
    # (n_a, n_b) of every profiled step, for flops summed over exactly the timed launches
    out["_rows"] = [(int(ra.item()), int(rb.item())) for ra, rb in rows]
    return out


def roofline(stages, h, w, n_scales, n_orient, n_a, n_b, d, gemm_peak=None):
    """Roofline of the kernel with the most time per step.

    Algorithmic work per launch: the column pass reads the row spectrum
    (8 B/px) and writes F complex planes; the row pass reads the F planes and
    writes MIM (1 B/px) and M (4 B/px); the distance GEMM does 2 n_a n_b D
    flops on the step's actual descriptor rows.  The two filter passes run
    once per image (twice per step), the GEMM once per step.
    """
    hw = h * w
    f = n_scales * n_orient
    # the GEMM's work: flops of each profiled step's own rows, summed, over the summed launch time
    # (the resident pairs' row counts differ by ~10 %)
    step_rows = stages.get("_rows") or [(n_a, n_b)]
    gemm_flop_avg = sum(2.0 * ra * rb * d for ra, rb in step_rows) / len(step_rows)
    cand = {
        "pass_a": ("hbm", hw * (8 + 8 * f), 2),
        "pass_b": ("hbm", hw * (8 * f + 5), 2),
        "match_gemm": ("mfma", gemm_flop_avg, 1),
    }

    def rate(k):
        bound, work, _ = cand[k]
        sec = stages[k]["ms_avg"] * 1e-3
        return work / sec / (1e9 if bound == "hbm" else 1e12)

    def peak(k):
        return HBM_PEAK_GBS if cand[k][0] == "hbm" else (gemm_peak or FP32_MFMA_PEAK_TFLOPS)

    best = max(cand, key=lambda k: cand[k][2] * stages[k]["ms_avg"])
    if best == "match_gemm" and stages["match_gemm"]["launches"] != len(step_rows):
        raise RuntimeError("GEMM launches and profiled steps differ")
    bound, work, per_step = cand[best]
    achieved = rate(best)
    traffic = None
    mt = MEASURED_TRAFFIC[best]
    if (h == w == 1024 and (n_scales, n_orient) == (4, 6) and mt["bytes"] is not None
            and sources_hash(mt["sources"]) == mt["sha"]):
        traffic = mt["bytes"]
    return {
        "kernel": best,
        "bound": bound,
        "achieved": round(achieved, 2),
        "peak": peak(best),
        "unit": "GB/s" if bound == "hbm" else "TFLOP/s",
        "frac": round(achieved / peak(best), 4),
        "traffic": traffic,
        "traffic_unit": "HBM bytes per launch",
        "algorithmic_per_launch": work,
        "ms_per_launch": round(stages[best]["ms_avg"], 5),
        "launches_per_step": per_step,
        "other": {k: {"achieved": round(rate(k), 2), "unit": "GB/s" if cand[k][0] == "hbm" else "TFLOP/s",
                      "frac": round(rate(k) / peak(k), 4), "ms_per_launch": round(stages[k]["ms_avg"], 5)}
                  for k in cand if k != best},
    }


def time_outliers(r2, torch, args, n_hyp=4096, reps=50):
    """rift2_ransac alone on a planted match set of the headline shape (10 % correct, 4096 hypotheses).

    Work: one FP64 residual test per (hypothesis, match), 6 multiplies and 7
    adds with no fused operations, against the FP64 vector peak; the chip's
    FP64 rate counts an FMA as two flops, so plain multiplies and adds reach
    half of it at most.
    """
    from synth.matches import planted_matches

    dev = torch.device("cuda:0")
    n = args.ransac_matches
    ka, kb, m, _, _ = planted_matches(0, n // 10, n - n // 10, size=args.size)
    mt = torch.from_numpy(m).to(dev)
    nt = torch.tensor([n], dtype=torch.int32, device=dev)
    kat, kbt = torch.from_numpy(ka).to(dev), torch.from_numpy(kb).to(dev)
    words = _ransac_words(torch, n_hyp, seed=1)
    res, mask, counts = r2.ransac(mt, nt, kat, kbt, words)
    ws = torch.empty(r2.ransac_workspace_bytes(n, n_hyp), dtype=torch.uint8, device=dev)
    rp = r2.RansacParams(3.0, 2)
    for _ in range(5):
        r2.ransac_into(mt, nt, kat, kbt, words, rp, counts, mask, res, ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        r2.ransac_into(mt, nt, kat, kbt, words, rp, counts, mask, res, ws)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    f = r2.similarity_fields(res)
    flops = 13.0 * n_hyp * n
    return {"workload": f"{n} matches ({n // 10} planted correct), {n_hyp} hypotheses, similarity model, "
                        f"threshold 3 px, 2 least-squares refits", "ms_per_call": round(ms, 5),
            "tests_per_s": round(n_hyp * n / (ms * 1e-3), 1),
            "fp64": {"bound": "alu", "achieved_tflops": round(flops / (ms * 1e-3) / 1e12, 3),
                     "peak_tflops": FP64_PEAK_TFLOPS, "frac": round(flops / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4)},
            "inliers": f["n_inliers"], "best": f["best"]}


def section4_metrics(r2, torch, pipe, imgs, gts):
    """Section 4's evaluation on the resident pairs: matches whose residual under the pair's ground
    truth is below 3 px are correct (rift2_consensus), the RMSE is over them (20 px for a failed pair)
    and a pair succeeds with at least 10 correct matches."""
    from synth.gen import gt_similarity

    per = []
    for (a, b), gt in zip(imgs, gts):
        pipe.run(a, b)
        model = torch.tensor(gt_similarity(gt), dtype=torch.float64, device=a.device)
        res, _ = r2.consensus(model, pipe.out, pipe.n_out, pipe.a.kpts, pipe.b.kpts, threshold=3.0)
        f = r2.consensus_fields(res)
        n = f["n_inliers"]
        per.append({"matches": int(pipe.n_out.item()), "correct": n,
                    "rmse": round(math.sqrt(f["sum_sq"] / n), 3) if n >= 10 else 20.0,
                    "angle_deg": round(math.degrees(gt["phi"]), 1)})
    ok = [p for p in per if p["correct"] >= 10]
    return {"pairs": per, "success_rate": round(len(ok) / len(per), 3),
            "mean_rmse": round(sum(p["rmse"] for p in per) / len(per), 3)}


def form_agreement(r2, torch, args, forms, prec):
    """Match sets of every matching form on one pair that keeps matches (the workload's scene and a
    translated, inverted copy without rotation or speckle; the workload's own pairs leave no row
    through the ratio test), each against the FP64 oracle matching the same descriptor rows
    (stage-isolated: the precision effect alone, Jaccard of (kp_a, kp_b) sets) and against the first
    form's set.  The oracle's whole pipeline at this size is compared by the full-size GPU tests."""
    import numpy as np

    from oracle import match as oracle_match
    from synth import make_shifted_pair

    a, b, _ = make_shifted_pair(args.config, 0, size=args.size)
    dev = torch.device("cuda:0")
    ta, tb = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    sets, vs_oracle = {}, {}
    for f in forms:
        pc, det, dp, mp = _form_params(r2, args, prec[f])
        pipe = r2.PairPipeline(args.size, args.size, pc, det, dp, mp)
        pipe.run(ta, tb)
        torch.cuda.synchronize()
        n = int(pipe.n_out.item())
        sets[f] = {(int(x), int(y)) for x, y in pipe.out[:n, :2].cpu().tolist()}
        rows = []
        for side in (pipe.a, pipe.b):
            nd = int(side.nd.item())
            rows.append((side.desc[:nd].cpu().numpy().astype(np.uint16), side.dkp[:nd].cpu().numpy()))
        ref = oracle_match.match(rows[0][0], rows[0][1], rows[1][0], rows[1][1], dtype=np.float64)
        want = {(int(x), int(y)) for x, y in zip(ref[0], ref[1])}
        vs_oracle[f] = {"oracle_matches": len(want),
                        "jaccard": round(len(sets[f] & want) / max(1, len(sets[f] | want)), 6)}
        del pipe
    ref = sets[forms[0]]
    return {"workload": f"scene of pair 0, B = A shifted by (5, -3) px, inverted + gamma 0.5, no rotation or speckle, "
                        f"{args.keypoints} kpts",
            "reference_form": forms[0],
            **{f: {"matches": len(sets[f]), "jaccard": round(len(sets[f] & ref) / max(1, len(sets[f] | ref)), 6),
                   "vs_fp64_oracle": vs_oracle[f]}
               for f in forms}}


def _oracle_pair_stages(job):
    """One full pair through the FP64 oracle in this process, single-threaded: seconds per stage
    (filter bank / MIM / moments, FAST, descriptors for both images; matching) and the match count."""
    size, keypoints, index = job
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle
    from oracle import describe, detect, filterbank, match
    from synth import make_pair

    a, b, _ = make_pair(1, index, size=size)
    pc = oracle.PCParams()
    det = oracle.DetectParams(max_keypoints=keypoints)
    dp = oracle.DescParams(patch_size=det.patch_size, n_orient=pc.n_orient)
    sec = {"filter": 0.0, "detect": 0.0, "describe": 0.0, "match": 0.0}
    feats = []
    with threadpool_limits(limits=1):
        for img in (a, b):
            t0 = time.perf_counter()
            fm = filterbank.filter_mim(img, pc)
            t1 = time.perf_counter()
            kpts, _ = detect.detect(fm["M"], det, dtype=np.float64)
            t2 = time.perf_counter()
            counts, kp, _ = describe.describe(fm["mim"], kpts, dp)
            t3 = time.perf_counter()
            sec["filter"] += t1 - t0
            sec["detect"] += t2 - t1
            sec["describe"] += t3 - t2
            feats.append((counts, kp))
        t0 = time.perf_counter()
        m = match.match(feats[0][0], feats[0][1], feats[1][0], feats[1][1], oracle.MatchParams(), dtype=np.float64)
        sec["match"] += time.perf_counter() - t0
    return sec, int(len(m[0]))


def _host_cpu():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "model": model}


def cpu_baseline(size, keypoints, one_thread_pairs=2, max_workers=16):
    """The FP64 oracle on full pairs of the same workload, timed per stage on the host cores.

    All cores: one single-threaded oracle process per core of this process's CPU set (at most
    `max_workers`), one pair each, pairs/s = pairs / wall time.  One thread: `one_thread_pairs`
    pairs in this process.  Runs before anything touches the GPU (the pool's worker processes are
    started fresh, not forked from a process holding a GPU context)."""
    import multiprocessing as mp

    host = _host_cpu()
    workers = max(1, min(max_workers, host["affinity"]))
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_pair_stages, [(size, keypoints, i) for i in range(workers)])
    wall = time.perf_counter() - t0
    stage_all = {k: round(1e3 * sum(r[0][k] for r in res) / len(res), 1) for k in res[0][0]}
    one = [_oracle_pair_stages((size, keypoints, i)) for i in range(one_thread_pairs)]
    t_one = sum(sum(r[0].values()) for r in one)
    stage_one = {k: round(1e3 * sum(r[0][k] for r in one) / len(one), 1) for k in one[0][0]}
    return {"value": round(workers / wall, 5), "unit": "pairs/s", "cores": workers, "kind": "oracle",
            "sample": f"{workers} pairs {size}x{size}, {keypoints} kpts each, FP64 numpy oracle, {workers} "
                      f"single-threaded processes, {wall:.1f} s wall (pool start-up included)",
            "stage_ms_per_pair": stage_all,
            "one_thread": {"pairs_per_s": round(len(one) / t_one, 5), "pairs": len(one),
                           "stage_ms_per_pair": stage_one},
            "host": host,
            "matches": [r[1] for r in res]}


def serve_sweep(args, r2, torch, rates, requests, pool_per_size, saturation_requests=None, serial_saturation=False):
    """Serving form: mixed sizes, Poisson arrivals at each rate (0 = all at once, saturation),
    continuous batching; per rate pairs/s and p50/p99 latency (completion minus arrival).  With
    serial_saturation the saturation run is repeated with one request in flight at a time (no
    overlap between requests): the rate the same requests reach back to back."""
    import numpy as np

    from synth import make_pair
    from synth.gen import serving_sizes

    dev = torch.device("cuda:0")
    sizes = tuple(int(x) for x in args.serve_sizes.split(",")) if args.serve_sizes else serving_sizes()
    pool = {}
    for n in sizes:
        for i in range(pool_per_size):
            a, b, _ = make_pair(3, n * 100 + i, size=n)
            pool[(n, i)] = (torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev))
    torch.cuda.synchronize()
    print(f"[serve] pool of {len(pool)} pairs resident", file=sys.stderr, flush=True)
    pc, det, dp, mp = r2.defaults()
    mp.precision = {"fp32": r2.PREC_FP32, "bf16": r2.PREC_BF16, "fp8": r2.PREC_FP8}[args.serve_form]
    kreq = args.serve_keypoints
    results = []
    runs = [(r, args.inflight, args.serve_batch) for r in rates]
    if serial_saturation:
        # the saturation run again with every request admitted on its own (no shared filter launches),
        # and with one request in flight at a time
        runs += [(0.0, args.inflight, 1), (0.0, 1, 1)]
    for rate, inflight, batch in runs:
        n_req = saturation_requests if (rate <= 0 and saturation_requests) else requests
        # the same seeded draw for runs of the same rate and length (both saturation runs see the same requests)
        rng = np.random.default_rng([1_000_003 * 3, int(rate * 1000), n_req])
        req_size = [int(x) for x in rng.choice(sizes, size=n_req)]
        gaps = rng.exponential(1.0 / rate, size=n_req) if rate > 0 else np.zeros(n_req)
        arrive = np.cumsum(gaps) - gaps[0]
        eng = r2.Engine(int(args.budget_gib * (1 << 30)), max_inflight=inflight, pc=pc, det=det, dp=dp, mp=mp)
        eng.set_batch(batch)
        # warm: two requests of every size on the idle engine.  submit queues a request and the next
        # poll admits it and enqueues all of its launches, so the second request's submit + first
        # poll is the host's admission and launch cost of one request
        submit_s = []
        for j, n in enumerate(sizes):
            for rep in range(2):
                t0 = time.perf_counter()
                eng.submit(-1 - 2 * j - rep, *pool[(n, 0)], max_keypoints=kreq)
                got = eng.poll()
                if rep:
                    submit_s.append(time.perf_counter() - t0)
                got += eng.drain()
        torch.cuda.synchronize()
        eng.close()
        eng = r2.Engine(int(args.budget_gib * (1 << 30)), max_inflight=inflight, pc=pc, det=det, dp=dp, mp=mp)
        eng.set_batch(batch)
        t_epoch = time.perf_counter()
        nxt = 0
        done = []
        arr_ms = {}
        while len(done) < n_req:
            now = time.perf_counter() - t_epoch
            while nxt < n_req and arrive[nxt] <= now:
                n = req_size[nxt]
                a, b = pool[(n, nxt % pool_per_size)]
                eng.submit(nxt, a, b, max_keypoints=kreq)
                arr_ms[nxt] = 1000.0 * arrive[nxt]
                nxt += 1
            got = eng.poll()
            done += got
            if not got and nxt < n_req:
                wait = arrive[nxt] - (time.perf_counter() - t_epoch)
                if wait > 2e-4:
                    time.sleep(min(wait, 1e-3))
        bad = [d for d in done if d["status"] != 0]
        lat = [d["done_ms"] - arr_ms[d["id"]] for d in done]
        span_ms = max(d["done_ms"] for d in done) - min(arr_ms.values())
        matches = sum(int(d["n_out"].item()) for d in done if d["n_out"] is not None)
        res = {"rate": rate if rate > 0 else "saturation", "inflight": inflight, "batch": batch, "requests": n_req,
               "pairs_per_s": round(n_req / (span_ms / 1000.0), 2),
               "p50_ms": round(percentile(lat, 50), 3), "p99_ms": round(percentile(lat, 99), 3),
               "gpu_ms_p50": round(percentile([d["gpu_ms"] for d in done], 50), 3), "failed": len(bad),
               "matches": matches, "host_launch_us": round(1e6 * float(np.median(submit_s)), 1)}
        print(f"[serve] {json.dumps(res)}", file=sys.stderr, flush=True)
        results.append(res)
        eng.close()
    return sizes, results


def serve(args, r2, torch):
    """--serve: the serving form alone, its own JSON line."""
    sizes, results = serve_sweep(args, r2, torch, [float(x) for x in args.rates.split(",")], args.requests,
                                 args.pool)
    kreq = args.serve_keypoints
    sat = [r for r in results if r["rate"] == "saturation" and r["inflight"] == args.inflight
           and r["batch"] == args.serve_batch]
    line = {
        "metric": "serving: image pairs/s + p50/p99 latency, mixed sizes, continuous batching",
        "value": sat[0]["pairs_per_s"] if sat else results[-1]["pairs_per_s"],
        "unit": "pairs/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": f"f32 filter + {args.serve_form} matching",
        "data": "synthetic",
        "config": {"workload": f"{args.requests} pair requests, sizes uniform over {list(sizes)}, keypoints "
                               f"{kreq or '2e-3 HW'}, Poisson arrivals", "budget_gib": args.budget_gib,
                   "inflight": args.inflight, "distinct_pairs_per_size": args.pool},
        "rates": results,
    }
    print(json.dumps(line))


def main():
    faulthandler.enable()
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the path is not sharded across GPUs",
              file=sys.stderr)
        sys.exit(2)
    cpu = None
    if not args.no_cpu and args.config == 1 and not args.serve:
        # the oracle's worker processes start before this process touches the GPU
        print("[bench] cpu oracle baseline", file=sys.stderr, flush=True)
        from synth.gen import CONFIGS as _cfgs

        cpu = cpu_baseline(args.size or _cfgs[1].size, args.keypoints or _cfgs[1].max_keypoints)
    import numpy as np
    import torch

    import paper_2303_00319_amd as r2
    from synth import make_pair

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.serve:
        return serve(args, r2, torch)
    from synth.gen import CONFIGS

    cfg = CONFIGS[args.config]
    args.size = args.size or cfg.size
    args.keypoints = args.keypoints or cfg.max_keypoints
    args.n_scales, args.n_orient = cfg.n_scales, cfg.n_orient
    forms = (args.forms or ("fp8,bf16" if args.config == 4 else "fp32,bf16")).split(",")
    prec = {"fp32": r2.PREC_FP32, "bf16": r2.PREC_BF16, "fp8": r2.PREC_FP8}
    peak = {"fp32": FP32_MFMA_PEAK_TFLOPS, "bf16": BF16_MFMA_PEAK_TFLOPS, "fp8": FP8_MFMA_PEAK_TFLOPS}
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.add(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    imgs, gts = [], []
    for i in range(args.pairs):
        a, b, gt = make_pair(args.config, i, size=args.size)
        imgs.append((torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)))
        gts.append(gt)
    torch.cuda.synchronize()
    in_type = "u16 (12-bit)" if imgs[0][0].dtype != torch.uint8 else "u8"
    print(f"[bench] {args.pairs} pairs {args.size}x{args.size} {in_type} resident", file=sys.stderr, flush=True)
    timed = {}
    for f in forms:
        print(f"[bench] timing {f}", file=sys.stderr, flush=True)
        timed[f] = time_form(r2, torch, imgs, args, prec[f])
        print(f"[bench] {f} {timed[f]['pairs_per_s']:.1f} pairs/s", file=sys.stderr, flush=True)
    ring_forms = [f for f in (args.ring_forms if args.ring_forms is not None else
                              ("bf16" if args.config == 4 else "fp32,bf16")).split(",") if f]
    ring = {}
    for f in ring_forms:
        print(f"[bench] timing RIFT ring {f}", file=sys.stderr, flush=True)
        ring[f] = time_single(r2, torch, imgs, args, prec[f], ring=True)
        print(f"[bench] ring {f} {ring[f]['pairs_per_s']:.1f} pairs/s", file=sys.stderr, flush=True)
    variants = {}
    for v in [v for v in args.variants.split(",") if v]:
        print(f"[bench] timing variant {v}", file=sys.stderr, flush=True)
        variants[v] = time_single(r2, torch, imgs, args, prec["fp32"], variant=v)
        print(f"[bench] {v} {variants[v]['pairs_per_s']:.1f} pairs/s", file=sys.stderr, flush=True)
    print("[bench] profiling stages", file=sys.stderr, flush=True)
    stages = {f: profile_stages(r2, torch, timed[f]["pipe"], imgs, args.profile_steps) for f in forms}
    var_stages = {v: profile_stages(r2, torch, variants[v]["pipe"], imgs, args.profile_steps) for v in variants}
    ring_stages = {f: profile_stages(r2, torch, ring[f]["pipe"], imgs, args.profile_steps) for f in ring_forms}
    main_form = forms[0]
    d = args.n_orient * 36
    n_a, n_b = timed[main_form]["last_pair"]["descriptor_rows"]
    roof = roofline(stages[main_form], args.size, args.size, args.n_scales, args.n_orient, n_a, n_b, d,
                    peak[main_form])
    if roof["kernel"] == "match_gemm" and main_form == "fp32":
        # what the matrix cores sustain on register-only chains of the GEMM's instruction, by waves per SIMD
        # (the GEMM runs 3: three 4-wave blocks per CU)
        print("[bench] FP32 MFMA calibration", file=sys.stderr, flush=True)
        rates = {w: round(r2.mfma_rate(r2.PREC_FP32, w), 2) for w in (1, 2, 3, 4)}
        roof["sustained"] = {"instruction": "v_mfma_f32_32x32x2f32, register operands", "waves_per_simd": 3,
                             "tflops": rates[3], "frac_of_peak": round(rates[3] / FP32_MFMA_PEAK_TFLOPS, 4),
                             "gemm_frac_of_sustained": round(roof["achieved"] / rates[3], 4),
                             "tflops_by_waves_per_simd": rates}
    mfma = {}
    # register-only chains of the GEMMs' instructions at their kernels' occupancy (FP32 3, BF16 4 waves per SIMD)
    calib = {"fp32": (r2.PREC_FP32, 3), "bf16": (r2.PREC_BF16, 4)}
    for f in forms:
        # sum of each profiled step's flops over the summed GEMM time
        flop = sum(2.0 * ra * rb * d for ra, rb in stages[f]["_rows"])
        t = stages[f]["match_gemm"]["ms_total"] * 1e-3
        mfma[f] = {"tflops": round(flop / t / 1e12, 2), "frac": round(flop / t / (peak[f] * 1e12), 4),
                   "peak_tflops": peak[f]}
        if f in calib:
            sus = r2.mfma_rate(*calib[f])
            mfma[f]["sustained_tflops"] = round(sus, 2)
            mfma[f]["frac_of_sustained"] = round(flop / t / 1e12 / sus, 4)
    print("[bench] section 4 metrics", file=sys.stderr, flush=True)
    accuracy = {main_form: section4_metrics(r2, torch, timed[main_form]["pipe"], imgs, gts)}
    for v in variants:
        accuracy[v] = section4_metrics(r2, torch, variants[v]["pipe"], imgs, gts)
    print("[bench] match-set agreement of the forms", file=sys.stderr, flush=True)
    agreement = form_agreement(r2, torch, args, forms, prec)
    print("[bench] outlier removal", file=sys.stderr, flush=True)
    outliers = time_outliers(r2, torch, args)
    serving = None
    if args.config == 1 and not args.no_serve:
        print("[bench] serving sweep", file=sys.stderr, flush=True)
        rates = [5.0, 10.0, 20.0, 40.0, 80.0, 0.0]
        sizes, res = serve_sweep(args, r2, torch, rates, args.sweep_requests, 2, saturation_requests=args.requests,
                                 serial_saturation=True)
        serving = {"workload": f"pair requests of sizes uniform over {list(sizes)} (2 resident pairs per size), "
                               f"keypoints 2e-3 HW, Poisson arrivals, {args.sweep_requests} requests per rate, "
                               f"{args.requests} all at once for saturation; latency = completion - arrival",
                   "form": f"f32 filter + {args.serve_form} matching", "budget_gib": args.budget_gib,
                   "inflight": args.inflight, "batch": args.serve_batch, "rates": res}
    head = timed[main_form]
    metric = ("image pairs/s + p50/p99 latency (1024^2 pair, 5k kpts); mixed vs plain FP32" if args.config == 1 else
              f"image pairs/s + p50/p99 latency ({args.size}^2 pair, {args.keypoints} kpts); " + " vs ".join(forms))
    line = {
        "metric": metric,
        "value": round(head["pairs_per_s"], 2),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "p50_ms": round(head["p50_ms"], 4),
        "p99_ms": round(head["p99_ms"], 4),
        "pipelined": head["pipelined"],
        "other_launch": head["other_launch"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "f32 filter + bf16 matching", "fp8": "f32 filter + fp8 matching"}[main_form],
        "data": "synthetic",
        "config": {
            "workload": f"RIFT2 pair {args.size}x{args.size} {in_type}, N_s={args.n_scales} N_o={args.n_orient}, "
                        f"<= {args.keypoints} FAST kpts/image, {d}-d descriptors, exhaustive NN + ratio 0.9",
            "pairs": args.pairs,
            "launch": "direct" if (args.direct or args.no_graph) else "graph replay",
            "streams_per_pair": 1 if args.serial else 2,
            "last_pair": head["last_pair"],
            "matches_note": "the workload's pairs (uniform rotation angles, speckle) leave (almost) no row through "
                            "the ratio test on every path, the FP64 oracle's included (cpu_baseline.matches); "
                            "the forms' agreement with the oracle is measured on shifted pairs (agreement)",
        },
        "roofline": roof,
        "mfma": mfma,
        "stages_ms": {f: {k: round(v["ms_avg"], 5) for k, v in stages[f].items() if k != "_rows" and v["launches"]}
                      for f in forms},
        "cpu_baseline": cpu,
        "outliers": outliers,
        "serving": serving,
        "accuracy": accuracy,
        "agreement": agreement,
        "rift_ring": None,
        "variants": {v: {"what": {"turned": "descriptor grid turned by the dominant index",
                                  "union": "RIFT's corner + edge detector union",
                                  "batched": "both images' filter banks in shared launches, then their keypoints "
                                             "on two streams"}[v],
                         "pairs_per_s": round(t["pairs_per_s"], 2), "ms_per_step": round(t["ms_per_step"], 4),
                         "p50_ms": round(t["p50_ms"], 4), "last_pair": t["last_pair"],
                         "detect_ms": round(var_stages[v]["detect"]["ms_avg"], 5),
                         "describe_ms": round(var_stages[v]["describe"]["ms_avg"], 5)}
                     for v, t in variants.items()},
    }
    if ring:
        line["rift_ring"] = {
            "workload": "same pairs, detector and precision; template described with all N_o ring members, "
                        "reference with one plain row per keypoint, N_o-fold matching (RIFT, Section 2.3)",
            "paper_ratio_cpu": {"sar_optical": round(29.24 / 10.93, 3), "ir_optical": round(35.82 / 13.24, 3),
                                "note": "RIFT (MATLAB) / RIFT2 (C++) running time per pair, Table 2"},
        }
        for f in ring_forms:
            t = ring[f]
            base = timed.get(f)
            line["rift_ring"][f] = {
                "pairs_per_s": round(t["pairs_per_s"], 2), "ms_per_step": round(t["ms_per_step"], 4),
                "p50_ms": round(t["p50_ms"], 4), "p99_ms": round(t["p99_ms"], 4),
                "descriptor_rows": t["last_pair"]["descriptor_rows"], "matches": t["last_pair"]["matches"],
                "stages_ms": {k: round(v["ms_avg"], 5) for k, v in ring_stages[f].items()
                              if k != "_rows" and v["launches"]},
                "rift2_speedup": round(base["pairs_per_s"] / t["pairs_per_s"], 3) if base else None,
            }
    if args.ransac > 0:
        line["config"]["ransac_hypotheses_in_step"] = args.ransac
    for f in forms[1:]:
        t = timed[f]
        key = "mixed" if (args.config == 1 and f == "bf16") else f
        line[key] = {
            "value": round(t["pairs_per_s"], 2),
            "dtype": {"fp32": "f32", "bf16": "f32 filter + bf16 matching (exact on counts)",
                      "fp8": "f32 filter + fp8 candidates + exact re-rank"}[f],
            "ms_per_step": round(t["ms_per_step"], 4),
            "p50_ms": round(t["p50_ms"], 4),
            "p99_ms": round(t["p99_ms"], 4),
            "pipelined": t["pipelined"],
            "other_launch": t["other_launch"],
            f"speedup_vs_{main_form}": round(t["pairs_per_s"] / head["pairs_per_s"], 4),
        }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
