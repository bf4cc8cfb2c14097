"""Graph capture and replay of the whole pair step (the form bench.py times).

A captured pair step is replayed several times, with eager work and host
synchronisations between replays, and every replay's keypoints, descriptor
rows and matches must equal those of the eager run.  Two pipelines (two
pairs in flight on two streams) are also replayed concurrently.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from synth import make_pair  # noqa: E402


def _translated_pair(index):
    """Image A of the small case and a shifted, remapped copy (the descriptor grid is axis-aligned, so a
    rotation-free pair has many correct matches)."""
    import synth.gen as g

    a, _, _ = make_pair(0, index)
    b = g._warp_bilinear(a.astype(np.float64), 0.0, 7.0, 4.0)
    b = np.rint(np.clip(255 * np.power(np.clip((255 - b) / 255, 0, 1), 0.5), 0, 255)).astype(np.uint8)
    return a, b


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_00319_amd as r2

    return r2, torch.device("cuda:0")


def _snapshot(pipe):
    torch.cuda.synchronize()
    out = {}
    for name, buf in (("a", pipe.a), ("b", pipe.b)):
        nk = int(buf.nk.item())
        nd = int(buf.nd.item())
        out[name + "_kpts"] = buf.kpts[:nk].cpu().numpy().copy()
        out[name + "_desc"] = buf.desc[:nd].cpu().numpy().copy()
        out[name + "_dkp"] = buf.dkp[:nd].cpu().numpy().copy()
    n = int(pipe.n_out.item())
    out["matches"] = pipe.out[:n].cpu().numpy().copy()
    if getattr(pipe, "ransac_words", None) is not None:
        out["ransac"] = pipe.ransac_result.cpu().numpy().copy()
        out["ransac_mask"] = pipe.ransac_mask.cpu().numpy().copy()
    return out


def _same(x, y, tag):
    assert x.keys() == y.keys()
    for k in x:
        assert x[k].shape == y[k].shape and np.array_equal(x[k], y[k]), f"{tag}: {k} differs"


def _pipeline(r2, size, k, precision, words=None):
    pc, det, dp, mp = r2.defaults()
    det.max_keypoints = k
    mp.precision = precision
    return r2.PairPipeline(size, size, pc, det, dp, mp, ransac_words=words)


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replay_equals_eager(precision):
    r2, dev = _gpu()
    print(f"[graph] 256x256 pair, 500 keypoints, precision {precision}", flush=True)
    a, b = _translated_pair(1)
    ta, tb = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    pipe = _pipeline(r2, 256, 500, precision)
    pipe.run(ta, tb)
    ref = _snapshot(pipe)
    assert len(ref["a_kpts"]) > 0 and len(ref["matches"]) > 0
    g = pipe.capture(ta, tb)
    side = torch.cuda.Stream()
    for rep in range(3):
        junk = torch.ones(1 << 20, device=dev) * rep  # eager work between replays
        with torch.cuda.stream(side):
            g.replay()
        torch.cuda.current_stream().wait_stream(side)
        _same(ref, _snapshot(pipe), f"replay {rep}")
        del junk


def test_graph_replay_with_outlier_removal():
    """The pair step with rift2_ransac appended: every replay equals the eager run, and the
    model moves the image centre by the pair's (7, 4) shift."""
    r2, dev = _gpu()
    from synth.matches import sample_words

    print("[graph] 256x256 pair + RANSAC (512 hypotheses)", flush=True)
    a, b = _translated_pair(8)
    ta, tb = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    words = torch.from_numpy(sample_words(8, 512).view(np.int32).copy()).to(dev)
    pipe = _pipeline(r2, 256, 500, 1, words)
    pipe.run(ta, tb)
    ref = _snapshot(pipe)
    f = r2.similarity_fields(pipe.ransac_result)
    assert f["status"] == 0 and f["n_inliers"] > 50
    a_, b_, tx, ty = f["model"]
    assert abs(a_ - 1) < 1e-2 and abs(b_) < 1e-2
    c = 127.5  # the image centre moves by the shift
    assert abs(a_ * c - b_ * c + tx - (c + 7)) < 1.0 and abs(b_ * c + a_ * c + ty - (c + 4)) < 1.0
    g = pipe.capture(ta, tb)
    for rep in range(3):
        junk = torch.ones(1 << 20, device=dev) * rep
        pipe.ransac_mask.zero_()
        g.replay()
        _same(ref, _snapshot(pipe), f"replay {rep}")
        del junk


def test_two_pairs_in_flight():
    r2, dev = _gpu()
    print("[graph] two 256x256 pairs in flight on two streams", flush=True)
    pairs = []
    for i in (2, 3):
        a, b = _translated_pair(i)
        pairs.append((torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)))
    pipes = [_pipeline(r2, 256, 500, 0) for _ in pairs]
    refs = []
    for pipe, (ta, tb) in zip(pipes, pairs):
        pipe.run(ta, tb)
        refs.append(_snapshot(pipe))
    graphs = [pipe.capture(ta, tb) for pipe, (ta, tb) in zip(pipes, pairs)]
    streams = [torch.cuda.Stream() for _ in pipes]
    for rep in range(3):
        for g, s in zip(graphs, streams):
            with torch.cuda.stream(s):
                g.replay()
        torch.cuda.synchronize()
        for i, pipe in enumerate(pipes):
            _same(refs[i], _snapshot(pipe), f"pair {i} replay {rep}")


@pytest.mark.parametrize("use_graph", [True, False])
def test_pipelined_steps_equal_single_pairs(use_graph):
    """Software-pipelined steps (pair k's image stages beside pair k-1's matching, two
    alternating buffer sets) give every pair the same keypoints, descriptors and matches
    as running it alone."""
    r2, dev = _gpu()
    print(f"[graph] pipelined steps, 4 pairs 256x256, graph={use_graph}", flush=True)
    pairs = []
    for i in (4, 5, 6, 7):
        a, b = _translated_pair(i)
        pairs.append((torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)))
    single = _pipeline(r2, 256, 500, 0)
    refs = []
    for ta, tb in pairs:
        single.run(ta, tb)
        refs.append(_snapshot(single))
        assert len(refs[-1]["matches"]) > 0
    pc, det, dp, mp = r2.defaults()
    det.max_keypoints = 500
    pp = r2.PipelinedPairs(256, 256, pc, det, dp, mp)
    n = len(pairs)
    pp.step(0, *pairs[0])
    graphs = {}
    if use_graph:
        for k in range(1, n + 1):
            graphs[k % n] = pp.capture(k, *pairs[k % n])
    for k in range(n + 1, 3 * n + 1):
        junk = torch.ones(1 << 18, device=dev) * k  # eager work between steps
        if use_graph:
            graphs[k % n].replay()
        else:
            pp.step(k, *pairs[k % n])
        _same(refs[(k - 1) % n], _snapshot(pp.matched_set(k)), f"step {k} (pair {(k - 1) % n})")
        del junk


def test_batched_filter_pipeline_equals_two_streams():
    """Both images' filter banks in shared launches (PairPipeline(batched=True)): eager and captured
    replays equal the two-stream pipeline's keypoints, descriptor rows and matches."""
    r2, dev = _gpu()
    a, b = _translated_pair(1)
    ta, tb = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    pc, det, dp, mp = r2.defaults()
    det.max_keypoints = 400
    mp.precision = r2.PREC_BF16
    ref = r2.PairPipeline(256, 256, pc, det, dp, mp)
    ref.run(ta, tb)
    want = _snapshot(ref)
    assert len(want["matches"]) > 20
    pipe = r2.PairPipeline(256, 256, pc, det, dp, mp, batched=True)
    pipe.run(ta, tb)
    _same(_snapshot(pipe), want, "batched eager")
    pipe.run_serial(ta, tb)
    _same(_snapshot(pipe), want, "batched serial")
    g = pipe.capture(ta, tb)
    for rep in range(3):
        ref.run(tb, ta)  # other work between the replays
        torch.cuda.synchronize()
        g.replay()
        _same(_snapshot(pipe), want, f"batched replay {rep}")


def test_convenience_calls_on_a_side_stream():
    """The allocating calls given a stream allocate and fill their outputs on that stream: with the
    current stream kept busy, every stage's results on a side stream equal those of the same calls on
    the current stream."""
    r2, dev = _gpu()
    a, b = _translated_pair(2)
    ta, tb = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)

    def run(stream):
        outs = []
        for t in (ta, tb):
            fm = r2.filter_mim(t, stream=stream)
            kp, n = r2.detect(fm["M"], stream=stream)
            desc, inv, dkp, nd = r2.describe(fm["mim"], kp, n, stream=stream)
            outs.append((fm["mim"], fm["M"], kp, n, desc, inv, dkp, nd))
        (_, _, kpa, _, da, ia, pa, na), (_, _, kpb, _, db, ib, pb, nb) = outs
        m, nm = r2.match(da, ia, pa, na, db, ib, pb, nb, stream=stream)
        return outs, m, nm

    def host(outs, m, nm):
        res = []
        for mim, M, kp, n, desc, inv, dkp, nd in outs:
            k, d = int(n.item()), int(nd.item())
            res += [mim.cpu().numpy(), M.cpu().numpy(), kp[:k].cpu().numpy(), desc[:d].cpu().numpy(),
                    dkp[:d].cpu().numpy()]
        res.append(m[:int(nm.item())].cpu().numpy())
        return res

    ref = host(*run(None))
    assert len(ref[-1]) > 0
    side = torch.cuda.Stream(device=dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    big = torch.randn((4096, 4096), device=dev)
    for _ in range(6):  # about 0.8 TFLOP queued on the current stream
        big = big @ big / 64.0
    got = run(side)
    side.synchronize()
    for x, y in zip(ref, host(*got)):
        assert x.shape == y.shape and np.array_equal(x, y)
