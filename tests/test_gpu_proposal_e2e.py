"""End-to-end parity of me_estimate in learned-proposal mode (pool, network
forward, decode + exact refine, fallback compaction, full search over the
fallback list, all inside the one call) against the oracle's proposal search.

The oracle is fed the network output that me_cnn_pool + me_cnn_forward give
for the same pair (the network itself is checked layer by layer against the
float64 oracle in test_gpu_cnn.py); from there every decision -- decoded
proposal, refined vector and SAD, each fallback test, the full-search result
of each fallen-back block -- must agree bit for bit."""
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


@pytest.fixture(scope="module")
def loaded(dev):
    from paper_2508_05990_amd import train

    params, median, _ = train.load_weights(train.DEFAULT_WEIGHTS)
    ctx = dev.Context(0)
    dev.cnn_set_params(ctx, params, median)
    yield ctx, median
    ctx.close()


@pytest.fixture(scope="module")
def hd_frames():
    from paper_2508_05990_amd import synth

    return synth.hd_sequence(1, n_frames=3).frames


def _net_output(dev, ctx, r, c):
    import torch

    x = dev.cnn_pool(ctx, r, c)
    out = dev.cnn_forward(ctx, x[None])[0]
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _check(dev, ctx, oracle_mod, f0, f1, R, thr, ratio, median, rr=2, median_arg=0.0):
    import torch

    r, c = torch.from_numpy(f0).cuda(), torch.from_numpy(f1).cuda()
    bh, bw = dev.block_grid(*f1.shape, 16)
    fb = torch.empty((bh, bw), dtype=torch.uint8, device="cuda")
    p = dev.make_params(16, R, dev.ME_MODE_PROPOSAL, rr, thr, ratio, median_arg)
    mv, sad = dev.estimate(r, c, fallback=fb, params=p, ctx=ctx)
    torch.cuda.synchronize()
    out = _net_output(dev, ctx, r, c)
    pred = oracle_mod.decode_proposal(out[:2], R)
    mv_o, sad_o, fb_o = oracle_mod.proposal_search(f0, f1, 16, R, pred, out[2], thr, ratio, median,
                                                   refine_radius=rr)
    mv, sad, fb = mv.cpu().numpy(), sad.cpu().numpy(), fb.cpu().numpy()
    assert np.array_equal(fb, fb_o), np.argwhere(fb != fb_o)[:8]
    assert np.array_equal(sad, sad_o), np.argwhere(sad != sad_o)[:8]
    assert np.array_equal(mv, mv_o)
    return mv, sad, fb


@pytest.mark.parametrize("t", [1, 2])
def test_hd_proposal_mode_bit_exact(dev, loaded, oracle_mod, hd_frames, t):
    """1080p, B=16, R=32, refine +-2, confidence 0.5 and SAD 1.5 x median,
    the median loaded with the weights."""
    ctx, median = loaded
    print("1080p proposal pair", t, flush=True)
    _, _, fb = _check(dev, ctx, oracle_mod, hd_frames[t - 1], hd_frames[t], 32, 0.0, 1.5, median)
    assert 0 < fb.sum() < fb.size


def test_hd_sad_fallback_only(dev, loaded, oracle_mod, hd_frames):
    """Confidence test off (threshold -inf), an explicit median and ratio."""
    ctx, _ = loaded
    _check(dev, ctx, oracle_mod, hd_frames[0], hd_frames[1], 32, -np.inf, 1.2, 1.7, median_arg=1.7)


def test_hd_forced_fallback_equals_full_search(dev, loaded, oracle_mod, hd_frames):
    """Every block fails the confidence test: the result is the full search."""
    ctx, median = loaded
    mv, sad, fb = _check(dev, ctx, oracle_mod, hd_frames[0], hd_frames[1], 32, np.inf, 1.5, median)
    mv_e, sad_e, _ = oracle_mod.full_search(hd_frames[0], hd_frames[1], 16, 32)
    assert fb.all() and np.array_equal(mv, mv_e) and np.array_equal(sad, sad_e)


def test_ragged_proposal_mode_bit_exact(dev, loaded, oracle_mod):
    """A frame whose packed size is not a multiple of the block (partial last
    block row and column), refine radius 3, radius 20."""
    rng = np.random.default_rng(31)
    H, W = 2 * 76, 2 * 108
    base = rng.integers(0, 4096, size=(H + 40, W + 40)).astype(np.uint16)
    f0 = base[10:10 + H, 12:12 + W].copy()
    f1 = base[13:13 + H, 8:8 + W].copy()
    ctx, _ = loaded
    _check(dev, ctx, oracle_mod, f0, f1, 20, -0.25, 1.3, 1500.0, rr=3, median_arg=1500.0)
