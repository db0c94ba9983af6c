"""What the trained proposal network gains over the method without it, end to
end: me_estimate in learned-proposal mode (pool, network, decode + exact +-2
refine, fallback list, full search over the list) against the same refine and
fallback fed zero proposals, on held-out sequences (training uses sequence
seeds from 1000 up, the confidence threshold stored with the weights was
chosen on seeds 500-502).

Per sequence and mode: the fraction of blocks that fall back to full search,
the MV-error rate against full search (Euclidean error above 1 packed pixel;
full search is the oracle's result bit for bit by the parity tests) and the
median event time of the motion estimation per pair.

* Background pan (the 4K stress sequence's kind of motion, and a 1080p
  sequence with a pan of (10, -14) packed pixels per frame): a zero proposal
  misses every panned block, the network's proposal lands within the refine
  window for most of them, so fewer blocks fall back and the pair is faster,
  at an MV-error rate of at most 2 %.  Asserted.
* Static background (the 1080p benchmark sequence): most blocks do not move,
  so a zero proposal already accepts them and the network's forward pass is
  pure cost.  Only the MV-error bound is asserted; the times are printed.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

MAX_ERR = 0.02


@pytest.fixture(scope="module")
def dev():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2508_05990_amd import me

    return me


@pytest.fixture(scope="module")
def loaded(dev):
    from paper_2508_05990_amd import train

    params, median, thr = train.load_weights(train.DEFAULT_WEIGHTS)
    ctx = dev.Context(0)
    dev.cnn_set_params(ctx, params, median)
    yield ctx, median, thr
    ctx.close()


def _modes(dev, ctx, frames, R, median, thr, reps=3):
    """Fallback rate, MV-error rate and median ME time per pair (ms) of the
    trained network (confidence fallback at the stored logit threshold, SAD
    fallback) and of zero proposals (SAD fallback: a zero logit carries no
    confidence)."""
    import torch

    fr = [torch.from_numpy(f).cuda() for f in frames]
    H, W = frames[0].shape
    bh, bw = dev.block_grid(H, W, 16)
    zero = torch.zeros((3, bh, bw), dtype=torch.float32, device="cuda")
    p = dev.make_params(16, R, dev.ME_MODE_PROPOSAL, 2, thr, 1.5, median)
    mv = torch.empty((bh, bw, 2), dtype=torch.int16, device="cuda")
    sad = torch.empty((bh, bw), dtype=torch.int32, device="cuda")
    fb = torch.empty((bh, bw), dtype=torch.uint8, device="cuda")
    res = {}
    for mode in ("trained", "zero"):
        fall = err = 0
        times = []
        for t in range(1, len(fr)):
            mv_e, _ = dev.estimate(fr[t - 1], fr[t], 16, R, ctx=ctx)
            for k in range(reps + 1):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                if mode == "trained":
                    dev.estimate(fr[t - 1], fr[t], mv=mv, sad=sad, fallback=fb, params=p, ctx=ctx)
                else:
                    dev.refine(fr[t - 1], fr[t], zero, ctx, 16, R, 2, -1e30, 1.5, median, mv=mv, sad=sad,
                               fallback=fb)
                b.record()
                torch.cuda.synchronize()
                if k > 0:                                   # the first call warms the context's buffers
                    times.append(a.elapsed_time(b))
            d = (mv.int() - mv_e.int()).float()
            err += int(((d[..., 0] ** 2 + d[..., 1] ** 2) > 1.0).sum().item())
            fall += int(fb.sum().item())
        n = (len(fr) - 1) * bh * bw
        res[mode] = {"fallback_rate": fall / n, "mv_err_rate": err / n, "ms_per_pair": float(np.median(times))}
    return res


def _report(name, res):
    for mode, r in res.items():
        print("%s %s: fallback %.4f, MV error %.4f, %.4f ms per pair" % (name, mode, r["fallback_rate"],
                                                                        r["mv_err_rate"], r["ms_per_pair"]),
              flush=True)


@pytest.mark.parametrize("case", ["uhd_pan", "hd_pan"])
def test_trained_network_beats_zero_proposals_under_pan(dev, loaded, case):
    from paper_2508_05990_amd import synth

    ctx, median, thr = loaded
    if case == "uhd_pan":
        seq, R = synth.uhd_sequence(4, n_frames=4), 64
    else:
        seq, R = synth.sequence(3, 1080, 1920, 5, 8, (48, 192), 24, 2.0, pan_max=16), 32
    assert seq.pan != (0, 0)
    res = _modes(dev, ctx, seq.frames, R, median, thr)
    _report(case, res)
    tr, zr = res["trained"], res["zero"]
    assert tr["mv_err_rate"] <= MAX_ERR
    assert zr["mv_err_rate"] <= MAX_ERR
    assert tr["fallback_rate"] < 0.9 * zr["fallback_rate"]
    assert tr["ms_per_pair"] < zr["ms_per_pair"]


def test_static_background_error_bound(dev, loaded):
    from paper_2508_05990_amd import synth

    ctx, median, thr = loaded
    seq = synth.hd_sequence(1, n_frames=5)
    res = _modes(dev, ctx, seq.frames, 32, median, thr)
    _report("hd_static", res)
    assert res["trained"]["mv_err_rate"] <= MAX_ERR
    assert res["zero"]["mv_err_rate"] <= MAX_ERR
