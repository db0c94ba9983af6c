"""What the trained proposal network gains over the method without it (the
same refine + fallback with a zero proposal), on held-out 1080p pairs of the
synthetic generator (training uses sequence seeds from 1000 up; these are
seed 1).  The packaged weights were trained by the library's own kernels
(paper_2508_05990_amd/train.py).

Measured on blocks that move (full-search vector not zero) and that the
proposal path could accept (full-search SAD within the fallback threshold):
the fraction whose decoded proposal lies within +-4 packed pixels of the
full-search vector.  End to end, both modes keep the MV error at zero (the
exact refine and the fallback decide); the proposal quality shows in how many
blocks fall back, which the benchmark reports."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2508_05990_amd import me

    return me


def test_trained_proposals_beat_zero_proposals(dev):
    import torch

    from paper_2508_05990_amd import synth, train

    params, median = train.load_weights(train.DEFAULT_WEIGHTS)
    seq = synth.hd_sequence(1, n_frames=6)
    fr = [torch.from_numpy(f).cuda() for f in seq.frames]
    ctx = dev.Context(0)
    try:
        dev.cnn_set_params(ctx, params, median)
        hit_net = hit_zero = n = 0
        for t in range(1, len(fr)):
            mv, sad = dev.estimate(fr[t - 1], fr[t], 16, 32, ctx=ctx)
            x = dev.cnn_pool(ctx, fr[t - 1], fr[t])
            out = dev.cnn_forward(ctx, x[None])[0]
            torch.cuda.synchronize()
            mv, sad, out = mv.cpu().numpy().astype(np.int64), sad.cpu().numpy(), out.cpu().numpy()
            p = np.clip(np.rint(out[:2].astype(np.float64) * 8.0), -32, 32)
            nsamp = np.full(sad.shape, 4.0 * 16 * 16)
            nsamp[-1] = 4.0 * 12 * 16                    # last block row is 12 packed rows tall
            usable = (sad <= np.floor(1.5 * float(np.float32(median)) * nsamp)) & (mv != 0).any(-1)
            err_net = np.maximum(np.abs(p[0] - mv[..., 0]), np.abs(p[1] - mv[..., 1]))[usable]
            err_zero = np.abs(mv).max(-1)[usable]
            hit_net += int((err_net <= 4).sum())
            hit_zero += int((err_zero <= 4).sum())
            n += int(usable.sum())
        print("moving usable blocks", n, "within +-4: trained", hit_net / n, "zero", hit_zero / n, flush=True)
        assert n > 500
        assert hit_net / n >= 0.2
        assert hit_net >= 1.5 * hit_zero
    finally:
        ctx.close()
