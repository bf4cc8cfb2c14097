"""GPU parity of RIFT's convolution-sequence ring (the baseline variant RIFT2 replaces) against the oracle.

The describe forms (plain rows, N_o ring rows per keypoint) are integer
counts and the ring matching evaluates the same FP32 distances as the plain
matching, so the bar is bit-exact: rows, keypoint indices, inverse norms,
matched pairs and distance bits.  The GPU puts the N_o-fold rows on the
template side (A) and matches them against plain reference rows (B); the
oracle matches plain template rows against reference ring rows, as RIFT
does.  The two are the same dot products, so the results must be identical.
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


def _fm(key, img):
    if key not in _cache:
        _cache[key] = filterbank.filter_mim(img, oracle.PCParams())
    return _cache[key]


def _shifted_pair(index, dx=5.0, dy=-3.0):
    import synth.gen as g

    a, _, _ = make_pair(0, index)
    b = g._warp_bilinear(a.astype(np.float64), 0.0, dx, dy)
    b = np.rint(np.clip(255 * np.power(np.clip((255 - b) / 255, 0, 1), 0.5), 0, 255)).astype(np.uint8)
    return a, b


def _describe_gpu(r2, dev, mim, kpts, mode, n_orient=6):
    dp = r2.defaults()[2]
    dp.n_orient = n_orient
    dp.mode = mode
    kp = np.zeros((max(len(kpts), 1), 3), dtype=np.int32)
    kp[:len(kpts), :2] = kpts
    d, inv, dk, nd = r2.describe(torch.from_numpy(mim).to(dev), torch.from_numpy(kp).to(dev),
                                 torch.tensor([len(kpts)], dtype=torch.int32, device=dev), dp)
    nd = int(nd.item())
    return d[:nd].cpu().numpy().astype(np.uint16), inv[:nd].cpu().numpy(), dk[:nd].cpu().numpy()


@pytest.mark.parametrize("n_orient", [6, 8])
def test_plain_and_ring_rows_bitexact(n_orient):
    r2, dev = _gpu()
    rng = np.random.default_rng(40 + n_orient)
    if n_orient == 6:
        a, _, _ = make_pair(0, 0)
        mim = _fm(("c0", 0), a)["mim"]
        kpts, _ = detect.detect(_fm(("c0", 0), a)["M"], oracle.DetectParams(max_keypoints=500), dtype=np.float32)
    else:
        mim = rng.integers(0, 8, size=(300, 260)).astype(np.uint8)
        kpts = np.stack([rng.integers(48, 213, 301), rng.integers(48, 253, 301)], 1).astype(np.int32)
    p = oracle.DescParams(n_orient=n_orient)
    for mode, form, rows in ((r2.DESC_PLAIN, describe.describe_plain, 1), (r2.DESC_RING, describe.describe_ring,
                                                                           n_orient)):
        print(f"[ring parity] describe mode {mode} N_o={n_orient} n={len(kpts)}", flush=True)
        c_ref, k_ref, _ = form(mim, kpts, p)
        c, inv, k = _describe_gpu(r2, dev, mim, kpts, mode, n_orient)
        assert len(c) == rows * len(kpts) == len(c_ref)
        assert np.array_equal(c, c_ref) and np.array_equal(k, k_ref)
        assert np.array_equal(inv, match.inv_norms(c_ref, np.float32))


def _ring_match_gpu(r2, dev, c_ring_t, k_ring_t, c_plain_r, k_plain_r, n_orient, precision):
    mp = r2.defaults()[3]
    mp.precision = precision
    mp.ring = n_orient

    def dev_set(c, k, extra):
        cap = len(c) + extra
        ct = torch.zeros((cap, c.shape[1]), dtype=torch.int16, device=dev)
        ct[:len(c)] = torch.from_numpy(c.astype(np.int16)).to(dev)
        inv = torch.zeros(cap, dtype=torch.float32, device=dev)
        inv[:len(c)] = torch.from_numpy(match.inv_norms(c, np.float32)).to(dev)
        kt = torch.zeros(cap, dtype=torch.int32, device=dev)
        kt[:len(c)] = torch.from_numpy(k.astype(np.int32)).to(dev)
        return ct, inv, kt, torch.tensor([len(c)], dtype=torch.int32, device=dev)

    out, n = r2.match(*dev_set(c_ring_t, k_ring_t, 3 * n_orient), *dev_set(c_plain_r, k_plain_r, 7), mp)
    n = int(n.item())
    return out[:n].cpu().numpy()


def _assert_same(got, ref, tag):
    assert len(got) == len(ref[0]), f"{tag}: {len(got)} vs {len(ref[0])} matches"
    assert np.array_equal(got[:, 0], ref[0]) and np.array_equal(got[:, 1], ref[1]), f"{tag}: pairs differ"
    assert np.array_equal(got[:, 2].view(np.float32), ref[2]), f"{tag}: distances differ"


def test_ring_matching_bitexact_on_oracle_descriptors():
    """Template A = shifted, intensity-inverted copy's partner; reference ring on B."""
    r2, dev = _gpu()
    a, b = _shifted_pair(0)
    det = oracle.DetectParams(max_keypoints=500)
    fa, fb = _fm(("c0", 0), a), _fm(("c0s", 0), b)
    ka, _ = detect.detect(fa["M"], det, dtype=np.float32)
    kb, _ = detect.detect(fb["M"], det, dtype=np.float32)
    p = oracle.DescParams()
    plain_t, kpt_t, _ = describe.describe_plain(fa["mim"], ka, p)
    ring_t, kring_t, _ = describe.describe_ring(fa["mim"], ka, p)
    plain_r, kpt_r, _ = describe.describe_plain(fb["mim"], kb, p)
    ring_r, kring_r, _ = describe.describe_ring(fb["mim"], kb, p)
    ref = match.match(plain_t, kpt_t, ring_r, kring_r, dtype=np.float32)
    for prec in (r2.PREC_FP32, r2.PREC_BF16):
        print(f"[ring parity] match 500 x 6*500, precision {prec}", flush=True)
        got = _ring_match_gpu(r2, dev, ring_t, kring_t, plain_r, kpt_r, 6, prec)
        _assert_same(got, ref, f"c0 ring prec {prec}")
    assert len(ref[0]) > 100


def test_ring_matching_random_sets_with_ties():
    """Small counts make exact distance ties between ring members and between keypoints common."""
    r2, dev = _gpu()
    rng = np.random.default_rng(44)
    for n_t, n_r, no, top in ((1, 1, 6, 3), (5, 2, 6, 2), (40, 70, 6, 3), (333, 517, 8, 4)):
        d = 36 * no
        base_t = rng.integers(0, top, size=(n_t, 36, no))
        base_r = rng.integers(0, top, size=(n_r, 36, no))
        m = min(n_t, n_r) // 2
        base_r[:m] = np.roll(base_t[:m], 2, axis=2)  # reference copies with rotated values
        plain_t = base_t.reshape(n_t, d).astype(np.uint16)
        ring_t = np.stack([np.roll(base_t[k], -w, axis=1).ravel() for k in range(n_t) for w in range(no)])
        ring_r = np.stack([np.roll(base_r[k], -w, axis=1).ravel() for k in range(n_r) for w in range(no)])
        plain_r = base_r.reshape(n_r, d).astype(np.uint16)
        kt = np.arange(n_t)
        kr = np.arange(n_r)
        ref = match.match(plain_t, kt, ring_r.astype(np.uint16), np.repeat(kr, no), dtype=np.float32)
        for prec in (r2.PREC_FP32, r2.PREC_BF16):
            print(f"[ring parity] random {n_t} x {no}*{n_r}, precision {prec}", flush=True)
            got = _ring_match_gpu(r2, dev, ring_t.astype(np.uint16), np.repeat(kt, no), plain_r, kr, no, prec)
            _assert_same(got, ref, f"random {n_t}x{n_r} N_o={no} prec {prec}")


def test_ring_pipeline_agrees_with_the_oracle_ring_pipeline():
    r2, dev = _gpu()
    a, b = _shifted_pair(3, 7.0, 4.0)
    ft, fr, mref = oracle.pipeline.ring_match_pair(a, b, det=oracle.DetectParams(max_keypoints=500))
    pc, det, dp, mp = r2.defaults()
    det.max_keypoints = 500
    pipe = r2.PairPipeline(256, 256, pc, det, dp, mp, ring=True)
    pipe.run(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev))
    torch.cuda.synchronize()
    assert int(pipe.a.nd.item()) == 6 * int(pipe.a.nk.item())
    assert int(pipe.b.nd.item()) == int(pipe.b.nk.item())
    got_m = pipe.matches().numpy()
    ka, kb = pipe.a.kpts.cpu().numpy(), pipe.b.kpts.cpu().numpy()
    got = {(tuple(ka[i, :2]), tuple(kb[j, :2])) for i, j in got_m[:, :2]}
    want = {(tuple(ft["kpts"][i]), tuple(fr["kpts"][j])) for i, j in zip(mref[0], mref[1])}
    jac = len(got & want) / max(1, len(got | want))
    print(f"ring end-to-end: gpu {len(got)}, oracle {len(want)}, Jaccard {jac:.4f}", flush=True)
    assert len(want) > 100 and jac > 0.9
