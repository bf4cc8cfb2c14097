"""Parity at the benchmark workloads' full sizes, in the configuration bench.py times.

The whole pair runs as a replayed graph on resident buffers (PairPipeline,
as in bench.py).  The oracle then checks what it can afford at that size:

* 1024^2 / 5000 keypoints and 2048^2 / 20000 keypoints: the full FP64 filter
  bank / MIM / moments; detection bit-exact on the GPU's own moment map;
  descriptors bit-exact for a seeded sample of 400 keypoints on the GPU's own
  MIM; FP32 and BF16 matches bit-exact for a seeded sample of 300 A keypoints
  (every row of a sampled keypoint against every B row).
* 4096^2 12-bit, N_s = 5, N_o = 8, 50000 keypoints: every filter's amplitude
  |EO_{s,o}|, the amplitude sums and the MIM at 64 x 64 = 4096 sampled pixels
  (64 whole rows of each FP64 response, by a row-restricted inverse DFT),
  detection bit-exact, 400 sampled descriptors bit-exact, and the FP8 form's
  match agreement with the exact decision on 300 sampled keypoints.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from oracle import detect, describe, filterbank, match  # noqa: E402
from synth import make_pair, make_shifted_pair  # noqa: E402
from synth.gen import CONFIGS  # noqa: E402


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_00319_amd as r2

    return r2, torch.device("cuda:0")


_pairs = {}


def _pair(config):
    """Image A of the workload and a shifted, intensity-inverted copy: the descriptor grid is
    axis-aligned, so a rotation-free pair gives many matches to compare."""
    if config not in _pairs:
        a, b, _ = make_shifted_pair(config, 0, shift=(7.0, 4.0))
        _pairs[config] = (a, b)
    return _pairs[config]


def _run_pipeline(r2, dev, config, precision, want_amp=False):
    cfg = CONFIGS[config]
    a, b = _pair(config)
    pc, det, dp, mp = r2.defaults()
    pc.n_scales, pc.n_orient = cfg.n_scales, cfg.n_orient
    dp.n_orient = cfg.n_orient
    det.max_keypoints = cfg.max_keypoints
    mp.precision = precision
    ta, tb = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    pipe = r2.PairPipeline(cfg.size, cfg.size, pc, det, dp, mp)
    g = pipe.capture(ta, tb)
    g.replay()
    torch.cuda.synchronize()
    return a, b, pipe, (pc, det, dp, mp)


def _image_outputs(buf):
    nk = int(buf.nk.item())
    nd = int(buf.nd.item())
    return {
        "M": buf.M.cpu().numpy(),
        "mim": buf.mim.cpu().numpy(),
        "kpts": buf.kpts[:nk].cpu().numpy(),
        "desc": buf.desc[:nd].cpu().numpy().astype(np.uint16),
        "inv": buf.inv[:nd].cpu().numpy(),
        "dkp": buf.dkp[:nd].cpu().numpy(),
    }


def _check_detect(out, k):
    kp_ref, sc_ref = detect.detect(out["M"], oracle.DetectParams(max_keypoints=k), dtype=np.float32)
    got = out["kpts"]
    assert len(got) == len(kp_ref), f"{len(got)} vs {len(kp_ref)} keypoints"
    assert np.array_equal(got[:, :2], kp_ref), "keypoint positions / order differ"
    assert np.array_equal(got[:, 2].view(np.float32), sc_ref.astype(np.float32)), "scores differ"


def _rows_of(out, i, n):
    """GPU rows of keypoint i: its primary row, then its secondary row if any."""
    rows = [i]
    sec = np.nonzero(out["dkp"][n:] == i)[0]
    rows += [n + int(r) for r in sec]
    return rows


def _check_describe(out, n_orient, rng, samples=400):
    n = len(out["kpts"])
    pick = np.sort(rng.choice(n, size=min(samples, n), replace=False))
    c_ref, k_ref, _ = describe.describe(out["mim"], out["kpts"][pick, :2], oracle.DescParams(n_orient=n_orient))
    for r in range(len(c_ref)):
        i = int(pick[k_ref[r]])
        rows = _rows_of(out, i, n)
        which = 0 if r < len(pick) else 1
        assert len(rows) > which, f"keypoint {i}: missing secondary row"
        assert np.array_equal(out["desc"][rows[which]], c_ref[r]), f"keypoint {i}: counts differ"
    n_sec_ref = len(c_ref) - len(pick)
    n_sec_gpu = sum(len(_rows_of(out, int(i), n)) - 1 for i in pick)
    assert n_sec_ref == n_sec_gpu
    inv_ref = match.inv_norms(c_ref, np.float32)
    for r in range(len(pick)):
        assert out["inv"][int(pick[r])] == inv_ref[r]


def _sampled_match(oa, ob, rng, samples=300, dtype=np.float32):
    """Oracle matches of a sample of A keypoints (all their rows) against every B row."""
    n = len(oa["kpts"])
    pick = np.sort(rng.choice(n, size=min(samples, n), replace=False))
    rows = sorted(r for i in pick for r in _rows_of(oa, int(i), n))
    ca = oa["desc"][rows]
    ka = oa["dkp"][rows]
    return set(int(i) for i in pick), match.match(ca, ka, ob["desc"], ob["dkp"], dtype=dtype)


def _gpu_matches(pipe, keys):
    n = int(pipe.n_out.item())
    o = pipe.out[:n].cpu().numpy()
    sel = [r for r in o if int(r[0]) in keys]
    return {(int(r[0]), int(r[1])): int(r[2]) for r in sel}


@pytest.mark.parametrize("config", [1, 2])
def test_full_size_pair(config):
    r2, dev = _gpu()
    cfg = CONFIGS[config]
    print(f"[full size] config {config}: {cfg.size}^2, K={cfg.max_keypoints}", flush=True)
    a, b, pipe, (pc, det, dp, mp) = _run_pipeline(r2, dev, config, r2.PREC_FP32)
    oa, ob = _image_outputs(pipe.a), _image_outputs(pipe.b)
    # filter bank / MIM / moments against the full FP64 oracle
    ref = filterbank.filter_mim(a, oracle.PCParams(), keep_amp=True)
    ra = ref["amp"]
    mim_agree = (oa["mim"] == ref["mim"]).mean()
    srt = np.sort(ra, axis=0)
    gap = (srt[-1] - srt[-2]) / np.maximum(srt[-1], np.sqrt(np.mean(ra * ra)))
    diff = oa["mim"] != ref["mim"]
    gap_top = (srt[-1] - srt[-2]) / np.maximum(srt[-1], 1e-300)
    max_gap = float(gap[diff].max()) if diff.any() else 0.0
    max_gap_top = float(gap_top[diff].max()) if diff.any() else 0.0
    merr = np.abs(oa["M"].astype(np.float64) - ref["M"]).max() / ref["M"].max()
    print(f"  MIM agreement {mim_agree:.6f} ({int(diff.sum())} disagreements, largest top-two gap {max_gap:.2e}, "
          f"relative to A_top alone {max_gap_top:.2e}), max moment rel err {merr:.2e}", flush=True)
    assert mim_agree >= 0.999, mim_agree
    assert max_gap < 1e-5, max_gap
    assert merr <= 2e-3, merr
    for out in (oa, ob):
        _check_detect(out, cfg.max_keypoints)
    rng = np.random.default_rng(config)
    _check_describe(oa, cfg.n_orient, rng)
    keys, ref_m = _sampled_match(oa, ob, rng)
    want = {(int(x), int(y)): int(np.float32(d).view(np.int32)) for x, y, d in zip(*ref_m)}
    got = _gpu_matches(pipe, keys)
    assert len(want) > 20, "too few sampled matches to compare"
    assert got == want, f"FP32 matches differ on the sample ({len(got)} vs {len(want)})"
    # the BF16 form on the same descriptors
    _, _, pipe16, _ = _run_pipeline(r2, dev, config, r2.PREC_BF16)
    assert _gpu_matches(pipe16, keys) == want, "BF16 matches differ on the sample"
    print(f"  detect / describe / match exact; sampled matches {len(want)}", flush=True)


def test_match_set_agreement_1024():
    """Match-set agreement with the FP64 oracle at the headline size (1024^2, 5000 keypoints), every
    descriptor row: (i) stage-isolated, the oracle matching the GPU's own descriptor tables (the pure
    precision effect of each matching form; FP32 and BF16 >= 99.5 %, FP8 >= 98 %), and (ii) end to end,
    the oracle's FP64 pipeline against the GPU pipeline, matches identified by their coordinates."""
    r2, dev = _gpu()
    cfg = CONFIGS[1]
    forms = (("fp32", r2.PREC_FP32, 0.995), ("bf16", r2.PREC_BF16, 0.995), ("fp8", r2.PREC_FP8, 0.98))
    sets = {}
    for name, prec, bar in forms:
        print(f"[agreement] 1024^2 shifted pair, {name} form", flush=True)
        a, b, pipe, _ = _run_pipeline(r2, dev, 1, prec)
        oa, ob = _image_outputs(pipe.a), _image_outputs(pipe.b)
        ref = match.match(oa["desc"], oa["dkp"], ob["desc"], ob["dkp"], dtype=np.float64)
        want = {(int(x), int(y)) for x, y in zip(ref[0], ref[1])}
        n = int(pipe.n_out.item())
        o = pipe.out[:n].cpu().numpy()
        got = {(int(r[0]), int(r[1])) for r in o}
        jac = len(got & want) / max(1, len(got | want))
        print(f"  stage-isolated {name}: rows {len(oa['desc'])} x {len(ob['desc'])}, gpu {len(got)}, "
              f"oracle {len(want)}, Jaccard {jac:.5f}", flush=True)
        assert len(want) > 1000, "too few matches for a meaningful comparison"
        assert jac >= bar, f"{name}: Jaccard {jac}"
        sets[name] = {(tuple(oa["kpts"][i, :2]), tuple(ob["kpts"][j, :2])) for i, j in got}
    assert sets["bf16"] == sets["fp32"], "BF16 and FP32 forms differ on identical descriptors"
    a, b = _pair(1)
    fa, fb, mref = oracle.pipeline.match_pair(a, b, det=oracle.DetectParams(max_keypoints=cfg.max_keypoints))
    want = {(tuple(fa["kpts"][i]), tuple(fb["kpts"][j])) for i, j in zip(mref[0], mref[1])}
    for name in sets:
        jac = len(sets[name] & want) / max(1, len(sets[name] | want))
        print(f"  end-to-end {name}: gpu {len(sets[name])}, oracle {len(want)}, Jaccard {jac:.5f}", flush=True)
        assert jac >= 0.9, f"{name}: end-to-end Jaccard {jac}"


def _responses_on_rows(spec, ys, s, o, p):
    """EO_{s,o} on whole image rows ys: the inverse DFT contracted over the row frequencies for those
    rows only (a matrix product), then an inverse DFT along each row."""
    h, w = spec.shape
    g = filterbank.log_gabor(h, w, s, o, p)
    ey = np.exp(2j * np.pi * np.outer(ys, np.arange(h)) / h)  # (n, H)
    part = ey @ (spec * g)  # (n, W): sum_k SG(k, l) e^{2 pi i k y / H}
    return np.fft.ifft(part, axis=1) / h


def test_full_size_large_fp8():
    r2, dev = _gpu()
    cfg = CONFIGS[4]
    print(f"[full size] config 4: {cfg.size}^2 12-bit, N_s={cfg.n_scales} N_o={cfg.n_orient}, K={cfg.max_keypoints}",
          flush=True)
    a, b, pipe, (pc, det, dp, mp) = _run_pipeline(r2, dev, 4, r2.PREC_FP8)
    # every filter's response at 64 x 64 sampled pixels (64 whole rows of the FP64 oracle's responses)
    ta = torch.from_numpy(a).to(dev)
    fm = r2.filter_mim(ta, pc, want_amp=True)
    rng = np.random.default_rng(4)
    ys = np.sort(rng.choice(cfg.size, size=64, replace=False))
    xs = np.sort(rng.choice(cfg.size, size=64, replace=False))
    yt = torch.from_numpy(ys).to(dev)
    p = oracle.PCParams(n_scales=cfg.n_scales, n_orient=cfg.n_orient)
    spec = filterbank.spectrum(a)
    ws = torch.empty(r2.filter_workspace_bytes(cfg.size, cfg.size, pc), dtype=torch.uint8, device=dev)
    amp_ref = np.zeros((cfg.n_orient, 64, 64))
    worst = 0.0
    for o in range(cfg.n_orient):
        for s in range(cfg.n_scales):
            want = np.abs(_responses_on_rows(spec, ys, s, o, p))[:, xs]
            got = np.abs(r2.debug_response(ta, s, o, pc, workspace=ws)[yt].cpu().numpy().astype(np.complex128))[:, xs]
            scale = np.maximum(want, math.sqrt(float(np.mean(want * want))))
            err = float(np.max(np.abs(got - want) / scale))
            worst = max(worst, err)
            assert err <= 1e-4, f"|EO| s={s} o={o}: {err:.2e}"
            amp_ref[o] += want
        print(f"  orientation {o}: every scale's |EO| at 4096 pixels within {worst:.2e}", flush=True)
    amp_gpu = fm["amp"][:, yt].cpu().numpy()[:, :, xs].astype(np.float64)
    rms = np.sqrt(np.mean(amp_ref * amp_ref))
    aerr = float(np.max(np.abs(amp_gpu - amp_ref) / np.maximum(amp_ref, rms)))
    assert aerr <= 1e-4, f"A_o at sampled pixels: {aerr:.2e}"
    mim_gpu = fm["mim"][yt].cpu().numpy()[:, xs]
    mim_ref = np.argmax(amp_ref, axis=0)
    srt = np.sort(amp_ref, axis=0)
    gap = (srt[-1] - srt[-2]) / np.maximum(srt[-1], rms)
    diff = mim_gpu != mim_ref
    agree = 1.0 - diff.mean()
    print(f"  A_o err {aerr:.2e}; MIM agreement {agree:.5f} over 4096 pixels, "
          f"largest gap at a disagreement {float(gap[diff].max()) if diff.any() else 0.0:.2e}", flush=True)
    assert agree >= 0.999 and (not diff.any() or gap[diff].max() < 1e-5)
    assert np.array_equal(fm["mim"].cpu().numpy(), pipe.a.mim.cpu().numpy())
    oa, ob = _image_outputs(pipe.a), _image_outputs(pipe.b)
    _check_detect(oa, cfg.max_keypoints)
    _check_describe(oa, cfg.n_orient, rng)
    keys, ref_m = _sampled_match(oa, ob, rng, dtype=np.float64)
    want = {(int(x), int(y)) for x, y in zip(ref_m[0], ref_m[1])}
    got = set(_gpu_matches(pipe, keys))
    jac = len(got & want) / max(1, len(got | want))
    print(f"  amplitudes / MIM / detect / describe exact; FP8 sampled matches gpu {len(got)} oracle {len(want)} "
          f"Jaccard {jac:.4f}", flush=True)
    assert len(want) > 20 and jac >= 0.95


def _run_variant(r2, dev, config, **kw):
    cfg = CONFIGS[config]
    a, b = _pair(config)
    pc, det, dp, mp = r2.defaults()
    det.max_keypoints = cfg.max_keypoints
    if kw.pop("turned", False):
        dp.mode = r2.DESC_TURNED
    pipe = r2.PairPipeline(cfg.size, cfg.size, pc, det, dp, mp, **kw)
    g = pipe.capture(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev))
    g.replay()
    torch.cuda.synchronize()
    return pipe


def test_full_size_variants_1024():
    """The corner + edge union, the turned grid and RIFT's ring at 1024^2 / 5000 keypoints, graph
    replayed as bench.py times them: detection bit-exact on the GPU's own moment maps, sampled
    descriptors bit-exact on its own MIM, sampled FP32 matches bit-exact."""
    r2, dev = _gpu()
    cfg = CONFIGS[1]
    rng = np.random.default_rng(11)
    print("[full size] variants at 1024^2: union", flush=True)
    pipe = _run_variant(r2, dev, 1, union=True)
    for buf in (pipe.a, pipe.b):
        nk = int(buf.nk.item())
        ref_pts, ref_sc = detect.detect_union(buf.M.cpu().numpy(), buf.m.cpu().numpy(),
                                              oracle.DetectParams(max_keypoints=cfg.max_keypoints), dtype=np.float32)
        got = buf.kpts[:nk].cpu().numpy()
        assert nk == len(ref_pts) and np.array_equal(got[:, :2], ref_pts)
        assert np.array_equal(got[:, 2].view(np.float32), np.asarray(ref_sc, np.float32))

    print("[full size] variants at 1024^2: turned grid", flush=True)
    pipe = _run_variant(r2, dev, 1, turned=True)
    oa, ob = _image_outputs(pipe.a), _image_outputs(pipe.b)
    n = len(oa["kpts"])
    pick = np.sort(rng.choice(n, size=400, replace=False))
    c_ref, k_ref, _ = describe.describe_rotated(oa["mim"], oa["kpts"][pick, :2], oracle.DescParams())
    for r in range(len(c_ref)):
        i = int(pick[k_ref[r]])
        rows = _rows_of(oa, i, n)
        which = 0 if r < len(pick) else 1
        assert len(rows) > which and np.array_equal(oa["desc"][rows[which]], c_ref[r]), f"keypoint {i}"
    keys, ref_m = _sampled_match(oa, ob, rng)
    want = {(int(x), int(y)): int(np.float32(d).view(np.int32)) for x, y, d in zip(*ref_m)}
    assert _gpu_matches(pipe, keys) == want and len(want) > 20

    print("[full size] variants at 1024^2: RIFT ring", flush=True)
    pipe = _run_variant(r2, dev, 1, ring=True)
    ta = {"mim": pipe.a.mim.cpu().numpy(), "kpts": pipe.a.kpts[:int(pipe.a.nk.item())].cpu().numpy()}
    tb = {"mim": pipe.b.mim.cpu().numpy(), "kpts": pipe.b.kpts[:int(pipe.b.nk.item())].cpu().numpy()}
    nd_a = int(pipe.a.nd.item())
    ring_a = pipe.a.desc[:nd_a].cpu().numpy().astype(np.uint16)
    assert nd_a == 6 * len(ta["kpts"])
    pick = np.sort(rng.choice(len(ta["kpts"]), size=300, replace=False))
    ring_ref, _, _ = describe.describe_ring(ta["mim"], ta["kpts"][pick, :2], oracle.DescParams())
    assert np.array_equal(ring_a.reshape(-1, 6, 216)[pick].reshape(-1, 216), ring_ref)
    # the oracle's ring matching: sampled template keypoints (plain rows) against every reference ring row
    plain_t, _, _ = describe.describe_plain(ta["mim"], ta["kpts"][pick, :2], oracle.DescParams())
    ring_r, kring_r, _ = describe.describe_ring(tb["mim"], tb["kpts"][:, :2], oracle.DescParams())
    ref_m = match.match(plain_t, pick.astype(np.int32), ring_r, kring_r, dtype=np.float32)
    want = {(int(x), int(y)): int(np.float32(d).view(np.int32)) for x, y, d in zip(*ref_m)}
    got = _gpu_matches(pipe, set(int(i) for i in pick))
    print(f"  union, turned and ring exact; sampled ring matches {len(want)}", flush=True)
    assert got == want and len(want) > 20
