"""GPU parity of the learned-proposal refine + fallback step (me_refine)
against the oracle, bit for bit, given the same seeded network outputs."""
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
def ctx(dev):
    c = dev.Context(0)
    yield c
    c.close()


def _net_out(rng, mv_exh, good_frac, noise_px, R):
    """Seeded stand-in for network outputs: for a fraction of blocks a vector
    near the full-search answer, elsewhere a random one; random logits."""
    bh, bw = mv_exh.shape[:2]
    out = np.empty((3, bh, bw), np.float32)
    good = rng.random((bh, bw)) < good_frac
    for c in range(2):
        near = (mv_exh[..., c] + rng.normal(0, noise_px, (bh, bw))) / 8.0
        far = rng.uniform(-R - 8, R + 8, (bh, bw)) / 8.0
        out[c] = np.where(good, near, far)
    out[2] = rng.normal(0.5, 2.0, (bh, bw))
    # a few values exactly on rounding ties (8*o = k + 0.5)
    out[0].flat[:5] = (np.arange(5) + 0.5) / 8.0
    return out


def _run(dev, ctx, oracle_mod, f0, f1, B, R, net, thr, ratio, M, rr=2):
    import torch

    t0 = torch.from_numpy(f0).cuda()
    t1 = torch.from_numpy(f1).cuda()
    nt = torch.from_numpy(net).cuda()
    mv, sad, fb = dev.refine(t0, t1, nt, ctx, B, R, rr, thr, ratio, M)
    torch.cuda.synchronize()
    pred = oracle_mod.decode_proposal(net[:2], R)
    mv_o, sad_o, fb_o = oracle_mod.proposal_search(f0, f1, B, R, pred, net[2], thr, ratio, M, refine_radius=rr)
    mv, sad, fb = mv.cpu().numpy(), sad.cpu().numpy(), fb.cpu().numpy()
    assert np.array_equal(fb, fb_o), np.argwhere(fb != fb_o)[:8]
    assert np.array_equal(sad, sad_o), np.argwhere(sad != sad_o)[:8]
    assert np.array_equal(mv, mv_o)
    return mv, sad, fb


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_small_pair(dev, ctx, oracle_mod, seed):
    from paper_2508_05990_amd import synth

    f0, f1, _ = synth.small_pair(seed)
    B, R = 16, 8
    mv_e, sad_e, _ = oracle_mod.full_search(f0, f1, B, R)
    net = _net_out(np.random.default_rng(seed), mv_e, 0.7, 1.0, R)
    _, _, fb = _run(dev, ctx, oracle_mod, f0, f1, B, R, net, 0.0, 1.5, 1.6)
    assert 0 < fb.sum() < fb.size


def test_hd_pair(dev, ctx, oracle_mod):
    from paper_2508_05990_amd import synth

    seq = synth.hd_sequence(1, n_frames=2)
    f0, f1 = seq.frames
    B, R = 16, 32
    mv_e, sad_e, _ = oracle_mod.full_search(f0, f1, B, R)
    M = float(np.median(sad_e / oracle_mod.block_samples(540, 960, B)))
    net = _net_out(np.random.default_rng(7), mv_e, 0.8, 1.5, R)
    _, _, fb = _run(dev, ctx, oracle_mod, f0, f1, B, R, net, 0.0, 1.5, M)
    assert 0 < fb.sum() < fb.size


def test_forced_fallback_equals_full_search(dev, ctx, oracle_mod):
    from paper_2508_05990_amd import synth

    f0, f1, _ = synth.small_pair(5)
    B, R = 16, 8
    mv_e, sad_e, _ = oracle_mod.full_search(f0, f1, B, R)
    net = _net_out(np.random.default_rng(3), mv_e, 0.5, 1.0, R)
    mv, sad, fb = _run(dev, ctx, oracle_mod, f0, f1, B, R, net, np.inf, 1.5, 1.0)
    assert fb.all() and np.array_equal(mv, mv_e) and np.array_equal(sad, sad_e)


@pytest.mark.parametrize("B,R,rr", [(8, 16, 2), (32, 12, 3), (16, 5, 0), (64, 9, 1)])
def test_ragged_shapes(dev, ctx, oracle_mod, B, R, rr):
    """Partial blocks on both edges, other block sizes and refine radii."""
    rng = np.random.default_rng(B + R)
    H, W = 2 * (3 * B + 5), 2 * (4 * B + 3)
    base = rng.integers(0, 4096, size=(H + 40, W + 40)).astype(np.uint16)
    f0 = base[10:10 + H, 12:12 + W].copy()
    f1 = base[13:13 + H, 8:8 + W].copy()
    mv_e, _, _ = oracle_mod.full_search(f0, f1, B, R)
    net = _net_out(rng, mv_e, 0.6, 1.0, R)
    med = 1500.0
    _run(dev, ctx, oracle_mod, f0, f1, B, R, net, -0.5, 1.2, med, rr=rr)


def test_needs_median(dev, ctx):
    import torch

    f = torch.zeros((64, 64), dtype=torch.uint16, device="cuda")
    net = torch.zeros((3, 2, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(dev.MeError) as e:
        dev.refine(f, f, net, ctx, 16, 8, sad_median_per_sample=0.0)
    assert e.value.status == dev.ME_E_STATE
