"""GPU parity of the training-set statistics of the learned-proposal mode
(me_sad_median, me_fallback_weight) against the oracle, bit for bit, and
me_sync."""
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


@pytest.mark.parametrize("n,H,W,B,spread", [(1, 2 * 24, 2 * 24, 16, 9), (7, 1080, 1920, 16, 400000),
                                            (64, 2 * 76, 2 * 108, 8, 3), (2, 2 * 200, 2 * 130, 64, 10 ** 9)])
def test_sad_median_and_weight_match_oracle(dev, oracle_mod, n, H, W, B, spread):
    """Random maps (few distinct values for many ties, or values large enough
    for float32 rounding of the SAD itself), partial blocks on both edges."""
    import torch

    bh, bw = dev.block_grid(H, W, B)
    rng = np.random.default_rng(n * 1000 + B)
    sad = rng.integers(0, spread, size=(n, bh, bw)).astype(np.int32)
    ctx = dev.Context(0)
    try:
        st = torch.from_numpy(sad).cuda()
        m = dev.sad_median(ctx, st, B, H, W)
        for ratio in (1.5, 0.7):
            w = dev.fallback_weight(st, B, H, W, ratio, float(m.item()))
            torch.cuda.synchronize()
            m_o = oracle_mod.median_per_sample(sad, H // 2, W // 2, B)
            assert m.item() == m_o
            assert np.array_equal(w.cpu().numpy(), oracle_mod.fallback_weight(sad, H // 2, W // 2, B, ratio, m_o))
    finally:
        ctx.close()


def test_training_median_of_real_searches(dev, oracle_mod):
    """The median of the full-search SADs of two 1080p pairs (the statistic the
    trainer stores with the weights)."""
    import torch

    from paper_2508_05990_amd import synth

    seq = synth.hd_sequence(1, n_frames=3)
    fr = [torch.from_numpy(f).cuda() for f in seq.frames]
    sads = torch.stack([dev.estimate(fr[t - 1], fr[t], 16, 32)[1] for t in (1, 2)])
    ctx = dev.Context(0)
    try:
        m = dev.sad_median(ctx, sads, 16, 1080, 1920)
        torch.cuda.synchronize()
        assert m.item() == oracle_mod.median_per_sample(sads.cpu().numpy(), 540, 960, 16)
    finally:
        ctx.close()


def test_sync_and_bad_sizes(dev):
    import torch

    s = torch.cuda.Stream()
    x = torch.zeros(1 << 20, device="cuda")
    with torch.cuda.stream(s):
        x.add_(1)
    dev.sync(s)
    assert float(x[0].item()) == 1.0
    dev.sync(None)
    ctx = dev.Context(0)
    try:
        bad = torch.zeros((2, 3), dtype=torch.int32, device="cuda")
        with pytest.raises(ValueError):
            dev.sad_median(ctx, bad, 16, 1080, 1920)
    finally:
        ctx.close()
