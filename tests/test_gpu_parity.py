"""GPU parity of every stage of the HIP path against the CPU oracle.

Tolerances (written here, derived in the design notes):
* amplitude sums A_o and every filter's amplitude |EO_{s,o}|:
  |gpu - oracle| <= 1e-4 * max(A(x), RMS(A)) (FP32 FFT error)
* MIM: >= 99.9 % equal; every disagreement is a near-tie of the oracle's top
  two amplitude sums: gap < 1e-5 relative to max(A_top(x), RMS(A)) (the gap
  relative to A_top(x) alone is printed as well)
* noise threshold: the two middle order statistics of the GPU's own A0 are
  bit-exact against a full sort; T_o is the oracle's threshold of that median
  within 1e-12, and the oracle's end-to-end T_o within 1e-4
* max moment M: |gpu - oracle| <= 2e-3 * max(M)
* FAST keypoints, descriptors, matches: bit-exact when fed the oracle's
  FP32-cast inputs (these stages are integer / correctly-rounded FP32)
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from oracle import filterbank, detect, describe, match  # noqa: E402
from synth import make_pair  # noqa: E402

_cache = {}


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_00319_amd as r2

    return r2, torch.device("cuda:0")


def _ref_fm(key, img, pc=oracle.PCParams()):
    if key not in _cache:
        _cache[key] = filterbank.filter_mim(img, pc)
    return _cache[key]


def _pcparams(r2, n_scales=4, n_orient=6):
    pc = r2.defaults()[0]
    pc.n_scales = n_scales
    pc.n_orient = n_orient
    return pc


def _check_noise(r2, ws, img, ref, pc, tag):
    """Order statistics bit-exact against a full sort of the GPU's own A0; T_o against the oracle."""
    h, w = img.shape
    a0, ostat, t_o = r2.debug_noise(ws, h, w, pc)
    torch.cuda.synchronize()
    a0 = a0.cpu().numpy()
    ostat = ostat.cpu().numpy()
    t_o = t_o.cpu().numpy()
    # the library's parameter record holds FP32 values (mult = fl32(2.1), k = 2): its FP64 threshold
    # arithmetic is checked on exactly those values
    p = oracle.PCParams(n_scales=pc.n_scales, n_orient=pc.n_orient, mult=float(pc.mult), k=float(pc.k))
    hw = h * w
    worst = 0.0
    for o in range(pc.n_orient):
        srt = np.sort(a0[o].ravel())
        assert srt[hw // 2 - 1].view(np.uint32) == ostat[o, 0].view(np.uint32), f"{tag}: order statistic o={o}"
        assert srt[hw // 2].view(np.uint32) == ostat[o, 1].view(np.uint32), f"{tag}: order statistic o={o}"
        own = filterbank.noise_threshold(a0[o].astype(np.float64), p)
        assert abs(t_o[o] - own) <= 1e-12 * own, f"{tag}: T_o arithmetic o={o}"
        worst = max(worst, abs(t_o[o] - ref["T"][o]) / ref["T"][o])
    assert worst <= 1e-4, f"{tag}: T_o vs oracle {worst:.2e}"
    return worst


def _check_responses(r2, dev, img, pc, tag):
    """Every filter's amplitude |EO_{s,o}| against the FP64 oracle's response."""
    t = torch.from_numpy(img).to(dev)
    p = oracle.PCParams(n_scales=pc.n_scales, n_orient=pc.n_orient)
    spec = filterbank.spectrum(img)
    ws = torch.empty(r2.filter_workspace_bytes(img.shape[0], img.shape[1], pc), dtype=torch.uint8, device=dev)
    worst = 0.0
    for o in range(pc.n_orient):
        ref = filterbank.responses(spec, o, p)
        for s in range(pc.n_scales):
            got = np.abs(r2.debug_response(t, s, o, pc, workspace=ws).cpu().numpy().astype(np.complex128))
            want = np.abs(ref[s])
            scale = np.maximum(want, np.sqrt(np.mean(want * want)))
            err = float(np.max(np.abs(got - want) / scale))
            worst = max(worst, err)
            assert err <= 1e-4, f"{tag}: |EO| s={s} o={o} rel err {err:.2e}"
    print(f"  every |EO_so| within {worst:.2e}", flush=True)
    return worst


def _check_filter(r2, dev, img, ref, pc, tag, responses=False):
    print(f"[filter parity] {tag} shape={img.shape} dtype={img.dtype}", flush=True)
    t = torch.from_numpy(img).to(dev)
    ws = torch.empty(r2.filter_workspace_bytes(img.shape[0], img.shape[1], pc), dtype=torch.uint8, device=dev)
    fm = r2.filter_mim(t, pc, want_amp=True, want_min=True, workspace=ws)
    torch.cuda.synchronize()
    t_err = _check_noise(r2, ws, img, ref, pc, tag)
    amp = fm["amp"].cpu().numpy().astype(np.float64)
    ra = ref["amp"]
    scale = np.maximum(ra, np.sqrt(np.mean(ra * ra, axis=(1, 2), keepdims=True)))
    err = np.abs(amp - ra) / scale
    assert err.max() <= 1e-4, f"{tag}: amplitude rel err {err.max():.3e}"
    mim = fm["mim"].cpu().numpy()
    diff = mim != ref["mim"]
    agree = 1.0 - diff.mean()
    srt = np.sort(ra, axis=0)
    gap = (srt[-1] - srt[-2]) / np.maximum(srt[-1], np.sqrt(np.mean(ra * ra)))
    gap_top = (srt[-1] - srt[-2]) / np.maximum(srt[-1], 1e-300)
    assert agree >= 0.999, f"{tag}: MIM agreement {agree}"
    max_gap = float(gap[diff].max()) if diff.any() else 0.0
    max_gap_top = float(gap_top[diff].max()) if diff.any() else 0.0
    print(f"  MIM: {int(diff.sum())} disagreements, largest top-two gap {max_gap:.2e} "
          f"(relative to A_top alone {max_gap_top:.2e}); T_o err {t_err:.2e}", flush=True)
    assert max_gap < 1e-5, f"{tag}: MIM disagreement away from ties (gap {max_gap:.2e})"
    mm = fm["M"].cpu().numpy().astype(np.float64)
    merr = np.abs(mm - ref["M"]).max() / max(ref["M"].max(), 1e-30)
    assert merr <= 2e-3, f"{tag}: max moment rel err {merr:.3e}"
    mn = fm["m"].cpu().numpy().astype(np.float64)
    nerr = np.abs(mn - ref["m"]).max() / max(ref["M"].max(), 1e-30)
    assert nerr <= 2e-3, f"{tag}: min moment rel err {nerr:.3e}"
    print(f"  amp err {err.max():.2e}  MIM agree {agree:.6f}  M err {merr:.2e}  m err {nerr:.2e}", flush=True)
    if responses:
        _check_responses(r2, dev, img, pc, tag)
    return fm


def test_filter_mim_256_pair():
    r2, dev = _gpu()
    a, b, _ = make_pair(0, 0)
    pc = _pcparams(r2)
    _check_filter(r2, dev, a, _ref_fm(("c0", 0, "a"), a), pc, "c0 A", responses=True)
    _check_filter(r2, dev, b, _ref_fm(("c0", 0, "b"), b), pc, "c0 B")


def test_filter_mim_1024():
    r2, dev = _gpu()
    a, _, _ = make_pair(1, 0)
    _check_filter(r2, dev, a, _ref_fm(("c1", 0, "a"), a), _pcparams(r2), "c1 A", responses=True)


@pytest.mark.parametrize("h,w", [(768, 768), (256, 512), (512, 256), (1536, 256), (256, 1536), (1536, 1536)])
def test_filter_mim_mixed_radix_and_rectangular(h, w):
    r2, dev = _gpu()
    a, _, _ = make_pair(1, 3, size=max(h, w))
    img = np.ascontiguousarray(a[:h, :w])
    _check_filter(r2, dev, img, filterbank.filter_mim(img, oracle.PCParams()), _pcparams(r2), f"{h}x{w}")


def test_filter_mim_u16_and_f32_inputs():
    r2, dev = _gpu()
    rng = np.random.default_rng(5)
    a, _, _ = make_pair(0, 1)
    a16 = (a.astype(np.uint16) * 16 + rng.integers(0, 16, size=a.shape)).astype(np.uint16)
    ref = filterbank.filter_mim(a16, oracle.PCParams(n_scales=5, n_orient=8))
    _check_filter(r2, dev, a16.view(np.int16), ref, _pcparams(r2, 5, 8), "u16 5x8")
    f = a.astype(np.float32) / 255.0
    _check_filter(r2, dev, f, filterbank.filter_mim(f, oracle.PCParams()), _pcparams(r2), "f32")


@pytest.mark.parametrize("ns,no", [(4, 8), (5, 6), (5, 8)])
def test_filter_mim_every_built_bank(ns, no):
    """Each instantiated (N_s, N_o) of the row pass against the oracle, every filter included."""
    r2, dev = _gpu()
    a, _, _ = make_pair(0, 4)
    ref = filterbank.filter_mim(a, oracle.PCParams(n_scales=ns, n_orient=no))
    _check_filter(r2, dev, a, ref, _pcparams(r2, ns, no), f"bank {ns}x{no}", responses=True)


def test_filter_mim_constant_image():
    r2, dev = _gpu()
    for val in (0, 91):
        t = torch.full((256, 256), val, dtype=torch.uint8, device=dev)
        fm = r2.filter_mim(t, want_amp=True)
        torch.cuda.synchronize()
        assert float(fm["amp"].abs().max()) < 1e-3
        assert float(fm["M"].abs().max()) < 1e-6
        assert int(fm["mim"].max()) == 0
        kp, n = r2.detect(fm["M"])
        assert int(n.item()) == 0


def test_filter_mim_pitched_rows():
    """A crop of a larger image (row pitch above W, odd byte offsets) gives the outputs of its dense
    copy bit for bit, for every input type and in a batch; views the library cannot read are refused."""
    r2, dev = _gpu()
    pc = _pcparams(r2)
    rng = np.random.default_rng(23)
    for h, w, dt, scale in ((256, 256, np.uint8, 255), (512, 256, np.uint16, 4095), (256, 512, np.float32, 1.0)):
        big = (rng.random((h + 9, w + 37)) * scale).astype(dt)
        big_t = torch.from_numpy(big.view(np.int16) if dt == np.uint16 else big).to(dev)
        crop = big_t[3:3 + h, 5:5 + w]
        assert crop.stride(0) == w + 37 and not crop.is_contiguous()
        print(f"[filter pitched] {h}x{w} {np.dtype(dt).name} pitch {crop.stride(0)}", flush=True)
        got = r2.filter_mim(crop, pc, want_min=True, want_amp=True)
        ref = r2.filter_mim(crop.contiguous(), pc, want_min=True, want_amp=True)
        torch.cuda.synchronize()
        for k in ("mim", "M", "m", "amp"):
            assert torch.equal(got[k], ref[k]), f"{h}x{w} {np.dtype(dt).name}: {k} differs"
        outs = [(torch.empty((h, w), dtype=torch.uint8, device=dev), torch.empty((h, w), dtype=torch.float32, device=dev),
                 None, None, torch.empty(r2.filter_workspace_bytes(h, w, pc), dtype=torch.uint8, device=dev))
                for _ in range(2)]
        r2.filter_mim_batch_into([crop, big_t[4:4 + h, 5:5 + w]], pc, outs)
        torch.cuda.synchronize()
        assert torch.equal(outs[0][0], ref["mim"]) and torch.equal(outs[0][1], ref["M"])
    sq = torch.zeros((256, 256), dtype=torch.uint8, device=dev)
    for bad in (sq.t(), torch.zeros((256, 512), dtype=torch.uint8, device=dev)[:, ::2]):
        with pytest.raises(ValueError):
            r2.filter_mim(bad, pc)
    with pytest.raises(ValueError):
        r2.filter_mim_into(sq, pc, torch.empty((256, 512), dtype=torch.uint8, device=dev)[:, :256],
                           torch.empty((256, 256), dtype=torch.float32, device=dev), None, None,
                           torch.empty(r2.filter_workspace_bytes(256, 256, pc), dtype=torch.uint8, device=dev))


def _check_detect(r2, dev, m32, k, tag):
    print(f"[detect parity] {tag} shape={m32.shape} K={k}", flush=True)
    det = r2.defaults()[1]
    det.max_keypoints = k
    kp_ref, sc_ref = detect.detect(m32, oracle.DetectParams(max_keypoints=k), dtype=np.float32)
    kp, n = r2.detect(torch.from_numpy(m32).to(dev), det)
    n = int(n.item())
    got = kp[:n].cpu().numpy()
    assert n == len(kp_ref), f"{tag}: {n} vs {len(kp_ref)} keypoints"
    assert np.array_equal(got[:, :2], kp_ref), f"{tag}: keypoint positions differ"
    assert np.array_equal(got[:, 2].view(np.float32), sc_ref.astype(np.float32)), f"{tag}: scores differ"
    return kp, n


def test_filter_batch_equals_single_calls():
    """rift2_filter_mim_batch: every image of a batch gets exactly the outputs of its own call."""
    r2, dev = _gpu()
    pc = _pcparams(r2)
    rng = np.random.default_rng(11)
    # the largest batch (8) with 12-bit u16 images, every other image without its optional outputs
    for shape, n, dt, scale in (((256, 256), 3, np.uint8, 255), ((768, 768), 2, np.uint8, 255),
                                ((512, 256), 2, np.float32, 255), ((1024, 1024), 2, np.uint8, 255),
                                ((256, 512), 8, np.uint16, 4095)):
        print(f"[filter batch] {n} x {shape} {np.dtype(dt).name}", flush=True)
        # 16-bit images travel as int16 (same bits): torch's uint16 support is partial
        imgs = [torch.from_numpy((rng.random(shape) * scale).astype(dt).view(np.int16 if dt == np.uint16 else dt))
                .to(dev) for _ in range(n)]
        outs, singles = [], []
        for k, im in enumerate(imgs):
            h, w = shape
            full = n < 8 or k % 2 == 0
            o = (torch.empty((h, w), dtype=torch.uint8, device=dev), torch.empty((h, w), dtype=torch.float32, device=dev),
                 torch.empty((h, w), dtype=torch.float32, device=dev) if full else None,
                 torch.empty((pc.n_orient, h, w), dtype=torch.float32, device=dev) if full else None,
                 torch.empty(r2.filter_workspace_bytes(h, w, pc), dtype=torch.uint8, device=dev))
            outs.append(o)
            singles.append(r2.filter_mim(im, pc, want_min=True, want_amp=True))
        r2.filter_mim_batch_into(imgs, pc, outs)
        torch.cuda.synchronize()
        for o, ref in zip(outs, singles):
            assert torch.equal(o[0], ref["mim"]) and torch.equal(o[1], ref["M"])
            if o[2] is not None:
                assert torch.equal(o[2], ref["m"]) and torch.equal(o[3], ref["amp"])


def test_detect_bitexact_on_oracle_moment():
    r2, dev = _gpu()
    a, b, _ = make_pair(0, 0)
    for key, img in ((("c0", 0, "a"), a), (("c0", 0, "b"), b)):
        m32 = _ref_fm(key, img)["M"].astype(np.float32)
        _check_detect(r2, dev, m32, 500, str(key))
        _check_detect(r2, dev, m32, 37, str(key) + " small K")
        _check_detect(r2, dev, m32, 100000, str(key) + " K above candidates")


def test_detect_bitexact_1024():
    r2, dev = _gpu()
    a, _, _ = make_pair(1, 0)
    m32 = _ref_fm(("c1", 0, "a"), a)["M"].astype(np.float32)
    _check_detect(r2, dev, m32, 5000, "c1 A")


def test_detect_ties_and_random_maps():
    r2, dev = _gpu()
    rng = np.random.default_rng(7)
    m = (rng.integers(0, 6, size=(256, 256)) / 5.0).astype(np.float32)  # many exact score ties
    _check_detect(r2, dev, m, 200, "quantised")
    m = rng.standard_normal((512, 256)).astype(np.float32)  # negative values, non-square
    _check_detect(r2, dev, m, 3000, "gaussian")
    # at 12000 keypoints and more the winners are ranked by a counting sort over score bins: a map
    # with heavy exact ties (whole bins of equal scores, the boundary bin among them) and a smooth one
    m = (rng.integers(0, 6, size=(1024, 1024)) / 5.0).astype(np.float32)
    _check_detect(r2, dev, m, 15000, "quantised, counting sort")
    _check_detect(r2, dev, m, 11999, "quantised, all-pairs ranking")
    m = rng.standard_normal((1024, 768)).astype(np.float32)
    _check_detect(r2, dev, m, 12000, "gaussian, counting sort")


def _check_describe(r2, dev, mim, kpts, tag, n_orient=6, patch=96, grid=6):
    print(f"[describe parity] {tag} n={len(kpts)} patch={patch} grid={grid}", flush=True)
    dp = r2.defaults()[2]
    dp.n_orient = n_orient
    dp.patch_size = patch
    dp.grid = grid
    c_ref, k_ref, _ = describe.describe(mim, kpts, oracle.DescParams(patch_size=patch, grid=grid, n_orient=n_orient))
    kp = np.zeros((max(len(kpts), 1), 3), dtype=np.int32)
    kp[:len(kpts), :2] = kpts
    kp_t = torch.from_numpy(kp).to(dev)
    n_t = torch.tensor([len(kpts)], dtype=torch.int32, device=dev)
    d, inv, dk, nd = r2.describe(torch.from_numpy(mim).to(dev), kp_t, n_t, dp)
    nd = int(nd.item())
    assert nd == len(c_ref), f"{tag}: {nd} vs {len(c_ref)} rows"
    assert np.array_equal(d[:nd].cpu().numpy().astype(np.uint16), c_ref), f"{tag}: counts differ"
    assert np.array_equal(dk[:nd].cpu().numpy(), k_ref), f"{tag}: keypoint index differs"
    inv_ref = match.inv_norms(c_ref, np.float32)
    assert np.array_equal(inv[:nd].cpu().numpy(), inv_ref), f"{tag}: inverse norms differ"
    return c_ref, k_ref


def test_describe_bitexact_on_oracle_mim():
    r2, dev = _gpu()
    a, _, _ = make_pair(0, 0)
    ref = _ref_fm(("c0", 0, "a"), a)
    kp_ref, _ = detect.detect(ref["M"], oracle.DetectParams(max_keypoints=500), dtype=np.float32)
    _check_describe(r2, dev, ref["mim"], kp_ref, "c0 A")
    rng = np.random.default_rng(8)
    mim8 = rng.integers(0, 8, size=(300, 260)).astype(np.uint8)
    pts = np.stack([rng.integers(48, 260 - 48 + 1, 700), rng.integers(48, 300 - 48 + 1, 700)], 1).astype(np.int32)
    _check_describe(r2, dev, mim8, pts, "random N_o=8", n_orient=8)
    # near-uniform values so that many patches carry a second descriptor
    mim6 = (rng.integers(0, 2, size=(200, 200)) * 3).astype(np.uint8)
    pts = np.stack([rng.integers(48, 153, 333), rng.integers(48, 153, 333)], 1).astype(np.int32)
    _check_describe(r2, dev, mim6, pts, "two-valued")


def test_describe_small_patch_build():
    """The 64-pixel patch, 4 x 4 grid build against the oracle, keypoints on the extreme rows and columns
    whose patch still fits (32 <= x <= W - 32) and a near-uniform MIM with many second rows."""
    r2, dev = _gpu()
    rng = np.random.default_rng(19)
    h, w = 150, 230
    uniform = rng.integers(0, 6, size=(h, w)).astype(np.uint8)
    xs = np.concatenate([[32, w - 32, 32, w - 32], rng.integers(32, w - 32 + 1, 296)])
    ys = np.concatenate([[32, 32, h - 32, h - 32], rng.integers(32, h - 32 + 1, 296)])
    pts = np.stack([xs, ys], 1).astype(np.int32)
    # value 2 more likely to the right, 4 to the left, a fifth of the pixels 0: a dominant index in most
    # patches, a second row (43 of 300) where 2 and 4 balance
    mixed = np.where(rng.random((h, w)) < np.linspace(0.0, 1.0, w)[None, :], 2, 4).astype(np.uint8)
    mixed[rng.random((h, w)) < 0.2] = 0
    c_ref, _ = _check_describe(r2, dev, mixed, pts, "patch 64 mixed", patch=64, grid=4)
    assert 300 < len(c_ref) < 600
    _check_describe(r2, dev, uniform, pts, "patch 64 uniform", patch=64, grid=4)


def _check_match(r2, dev, ca, ka, cb, kb, precision, tag, mutual=False):
    print(f"[match parity] {tag} nA={len(ca)} nB={len(cb)} prec={precision} mutual={mutual}", flush=True)
    mp = r2.defaults()[3]
    mp.precision = precision
    mp.mutual = int(mutual)
    ref = match.match(ca, ka, cb, kb, oracle.MatchParams(mutual=mutual), dtype=np.float32)

    def dev_set(c, k):
        cap = len(c) + 5
        ct = torch.zeros((cap, c.shape[1]), dtype=torch.int16, device=dev)
        ct[:len(c)] = torch.from_numpy(c.astype(np.int16)).to(dev)
        inv = torch.zeros(cap, dtype=torch.float32, device=dev)
        inv[:len(c)] = torch.from_numpy(match.inv_norms(c, np.float32)).to(dev)
        kt = torch.zeros(cap, dtype=torch.int32, device=dev)
        kt[:len(c)] = torch.from_numpy(k.astype(np.int32)).to(dev)
        return ct, inv, kt, torch.tensor([len(c)], dtype=torch.int32, device=dev)

    out, n = r2.match(*dev_set(ca, ka), *dev_set(cb, kb), mp)
    n = int(n.item())
    got = out[:n].cpu().numpy()
    assert n == len(ref[0]), f"{tag}: {n} vs {len(ref[0])} matches"
    assert np.array_equal(got[:, 0], ref[0]) and np.array_equal(got[:, 1], ref[1]), f"{tag}: match pairs differ"
    assert np.array_equal(got[:, 2].view(np.float32), ref[2]), f"{tag}: distances differ"
    return n


def test_match_exact_on_oracle_descriptors():
    r2, dev = _gpu()
    import synth.gen as g

    a, _, _ = make_pair(0, 0)
    # translated + intensity-remapped copy of A so that many rows pass the ratio test
    b = g._warp_bilinear(a.astype(np.float64), 0.0, 5.0, -3.0)
    b = np.rint(np.clip(255 * np.power(np.clip((255 - b) / 255, 0, 1), 0.5), 0, 255)).astype(np.uint8)
    fa = oracle.pipeline.image_features(a, det=oracle.DetectParams(max_keypoints=500), dtype=np.float32)
    fb = oracle.pipeline.image_features(b, det=oracle.DetectParams(max_keypoints=500), dtype=np.float32)
    for prec in (r2.PREC_FP32, r2.PREC_BF16):
        n = _check_match(r2, dev, fa["desc"], fa["desc_kp"], fb["desc"], fb["desc_kp"], prec, "c0 shifted")
        assert n > 100
        nm = _check_match(r2, dev, fa["desc"], fa["desc_kp"], fb["desc"], fb["desc_kp"], prec, "c0 shifted",
                          mutual=True)
        assert 50 < nm <= n
    # FP8: approximate candidate choice on the real counts (up to 256), exact re-rank
    jac = _match_agreement(r2, dev, fa["desc"], fa["desc_kp"], fb["desc"], fb["desc_kp"], r2.PREC_FP8, "c0 shifted fp8")
    assert jac >= 0.98


def _match_agreement(r2, dev, ca, ka, cb, kb, precision, tag):
    """Jaccard agreement of the match sets {(kp_a, kp_b)} with the oracle."""
    mp = r2.defaults()[3]
    mp.precision = precision
    ref = match.match(ca, ka, cb, kb, dtype=np.float64)

    def dev_set(c, k):
        ct = torch.from_numpy(c.astype(np.int16)).to(dev)
        inv = torch.from_numpy(match.inv_norms(c, np.float32)).to(dev)
        kt = torch.from_numpy(k.astype(np.int32)).to(dev)
        return ct, inv, kt, torch.tensor([len(c)], dtype=torch.int32, device=dev)

    out, n = r2.match(*dev_set(ca, ka), *dev_set(cb, kb), mp)
    n = int(n.item())
    got = {(int(x), int(y)) for x, y in out[:n, :2].cpu().numpy()}
    want = {(int(x), int(y)) for x, y in zip(ref[0], ref[1])}
    jac = len(got & want) / max(1, len(got | want))
    print(f"[match agreement] {tag}: gpu {len(got)}, oracle {len(want)}, Jaccard {jac:.4f}", flush=True)
    return jac


def test_match_random_sets_with_ties_and_ragged_sizes():
    """Counts below 16 are exact in every precision (FP8 included: power-of-two row scales), so all
    three forms must reproduce the oracle exactly, ties and ragged sizes included."""
    r2, dev = _gpu()
    rng = np.random.default_rng(9)
    for na, nb in ((1, 1), (3, 2), (33, 65), (700, 1111)):
        ca = rng.integers(0, 4, size=(na, 216)).astype(np.uint16)
        cb = rng.integers(0, 4, size=(nb, 216)).astype(np.uint16)
        cb[: min(na, nb) // 2] = ca[: min(na, nb) // 2]
        ka = np.arange(na) // 2
        kb = np.arange(nb) // 2
        for prec in (r2.PREC_FP32, r2.PREC_BF16, r2.PREC_FP8):
            _check_match(r2, dev, ca, ka, cb, kb, prec, f"random {na}x{nb}")
            _check_match(r2, dev, ca, ka, cb, kb, prec, f"random {na}x{nb}", mutual=True)
    # 288-d (N_o = 8) descriptors
    ca = rng.integers(0, 9, size=(300, 288)).astype(np.uint16)
    cb = np.concatenate([ca[:150], rng.integers(0, 9, size=(200, 288)).astype(np.uint16)])
    for prec in (r2.PREC_FP32, r2.PREC_BF16, r2.PREC_FP8):
        _check_match(r2, dev, ca, np.arange(300), cb, np.arange(350), prec, "288-d")
        _check_match(r2, dev, ca, np.arange(300), cb, np.arange(350), prec, "288-d", mutual=True)
    # mutual: two A keypoints whose rows are nearest to the same B row; only the one B picks survives
    ca = rng.integers(0, 4, size=(40, 216)).astype(np.uint16)
    cb = rng.integers(0, 4, size=(50, 216)).astype(np.uint16)
    cb[:20] = ca[:20]
    ca[20:30] = ca[:10]
    ca[20:30, :3] += 1
    for prec in (r2.PREC_FP32, r2.PREC_BF16, r2.PREC_FP8):
        _check_match(r2, dev, ca, np.arange(40), cb, np.arange(50), prec, "shared nearest", mutual=True)


def test_desc_normalize_is_the_correctly_rounded_product():
    r2, dev = _gpu()
    rng = np.random.default_rng(12)
    c = rng.integers(0, 257, size=(333, 216)).astype(np.uint16)
    inv = match.inv_norms(c, np.float32)
    ct = torch.from_numpy(c.astype(np.int16)).to(dev)
    it = torch.from_numpy(inv).to(dev)
    n = torch.tensor([300], dtype=torch.int32, device=dev)
    out = r2.desc_normalize(ct, it, n).cpu().numpy()
    want = (c[:300].astype(np.float32) * inv[:300, None]).astype(np.float32)
    assert np.array_equal(out[:300], want)
    assert not out[300:].any()


def test_end_to_end_pair_agreement():
    """Full GPU pipeline vs the FP64 oracle on a c0 pair: reported agreement."""
    r2, dev = _gpu()
    import synth.gen as g

    a, _, _ = make_pair(0, 2)
    b = g._warp_bilinear(a.astype(np.float64), 0.0, 7.0, 4.0)
    b = np.rint(np.clip(255 * np.power(np.clip((255 - b) / 255, 0, 1), 0.5), 0, 255)).astype(np.uint8)
    det = oracle.DetectParams(max_keypoints=500)
    fa, fb, mref = oracle.pipeline.match_pair(a, b, det=det)
    pc, detp, dp, mp = r2.defaults()
    detp.max_keypoints = 500
    feats = []
    for img in (a, b):
        fm = r2.filter_mim(torch.from_numpy(img).to(dev), pc)
        kp, nk = r2.detect(fm["M"], detp)
        feats.append((kp, nk) + r2.describe(fm["mim"], kp, nk, dp))
    out, n = r2.match(*feats[0][2:6], *feats[1][2:6], mp)
    n = int(n.item())
    ka = feats[0][0].cpu().numpy()
    kb = feats[1][0].cpu().numpy()
    got = {(tuple(ka[i, :2]), tuple(kb[j, :2])) for i, j in out[:n, :2].cpu().numpy()}
    want = {(tuple(fa["kpts"][i]), tuple(fb["kpts"][j])) for i, j in zip(mref[0], mref[1])}
    jac = len(got & want) / max(1, len(got | want))
    print(f"end-to-end: gpu {len(got)} matches, oracle {len(want)}, Jaccard {jac:.4f}", flush=True)
    assert len(want) > 100 and jac > 0.9


@pytest.mark.parametrize("precision,peak", [(0, 157.3), (1, 2500.0)])
def test_mfma_calibration_stays_below_the_peak(precision, peak):
    """rift2_debug_mfma_rate: register-only FP32 / BF16 MFMA chains run at a sizeable fraction of the
    published peak and never above it; more waves per SIMD never run much slower."""
    r2, dev = _gpu()
    rates = [r2.mfma_rate(precision, w, iters=1000, reps=3) for w in (1, 2, 3, 4)]
    print(f"[mfma calibration] precision {precision}: TFLOP/s by waves per SIMD {[round(r, 1) for r in rates]}",
          flush=True)
    for r in rates:
        assert 0.3 * peak < r < 1.01 * peak
    assert rates[3] > 0.9 * rates[0]
