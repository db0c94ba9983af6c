"""GPU parity of the strided stage search and the coarse-to-fine pyramid
search (paper Sec. 3.2) against the CPU oracle, bit for bit."""
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


def _to_dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _same(mv_g, sad_g, mv_o, sad_o):
    mv_g, sad_g = mv_g.cpu().numpy(), sad_g.cpu().numpy()
    assert np.array_equal(sad_g, sad_o), np.argwhere(sad_g != sad_o)[:8]
    assert np.array_equal(mv_g, mv_o), np.argwhere((mv_g != mv_o).any(-1))[:8]


@pytest.mark.parametrize("B,R,step,limit,use_pred", [
    (16, 8, 8, 127, False), (32, 8, 8, 127, True), (16, 4, 4, 40, True), (8, 3, 2, 20, True),
    (64, 6, 8, 127, True), (32, 10, 8, 90, False), (16, 2, 5, 9, True), (8, 12, 3, 127, True)])
def test_strided_stage_search(dev, oracle_mod, B, R, step, limit, use_pred):
    """Ragged frame (partial blocks on both edges), random predictors beyond
    the limit so that some candidate sets are clipped or empty."""
    import torch

    rng = np.random.default_rng(B * 100 + R * 10 + step)
    H, W = 2 * 150, 2 * 214
    f0 = rng.integers(0, 4096, size=(H, W)).astype(np.uint16)
    f1 = rng.integers(0, 4096, size=(H, W)).astype(np.uint16)
    bh, bw = dev.block_grid(H, W, B)
    pred = rng.integers(-limit - 10, limit + 11, size=(bh, bw, 2)).astype(np.int16) if use_pred else None
    print("strided stage", B, R, step, limit, use_pred, flush=True)
    mv, sad = dev.stage_search(_to_dev(f0), _to_dev(f1), B, R, pred=None if pred is None else _to_dev(pred),
                               limit=limit, step=step)
    torch.cuda.synchronize()
    rp, cp = oracle_mod.pack_planes(f0), oracle_mod.pack_planes(f1)
    mv_o, sad_o, _, _ = oracle_mod.stage_search(rp, cp, B, R, step, pred=pred, limit=limit)
    _same(mv, sad, mv_o, sad_o)


@pytest.mark.parametrize("blocks,stages,limit", [
    ((32, 16), ((8, 8), (4, 4), (2, 1)), 127),      # the paper's standard setting
    ((32, 16), ((4, 8), (2, 4), (2, 1)), 127),      # mode 1
    ((16,), ((8, 8), (4, 4), (2, 1)), 64),          # one level (mode 3)
    ((64, 32, 16, 8), ((8, 8), (4, 4), (2, 1)), 127),
    ((32, 16), ((8, 8), (4, 4), (2, 1)), 32)])
def test_pyramid_small_frames(dev, ctx, oracle_mod, blocks, stages, limit):
    import torch

    from paper_2508_05990_amd import synth

    for seed in (0, 1):
        f0, f1, _ = synth.small_pair(seed)
        print("pyramid", blocks, stages, limit, seed, flush=True)
        cfg = dev.pyramid_cfg(blocks, stages, limit)
        mv, sad = dev.pyramid(_to_dev(f0), _to_dev(f1), ctx, cfg)
        torch.cuda.synchronize()
        mv_o, sad_o, _, _ = oracle_mod.pyramid_search(f0, f1, blocks, stages, limit)
        _same(mv, sad, mv_o, sad_o)


def test_pyramid_ragged_random(dev, ctx, oracle_mod):
    import torch

    rng = np.random.default_rng(11)
    for H, W in ((2 * 97, 2 * 131), (2 * 40, 2 * 300), (2 * 17, 2 * 23)):
        f0 = rng.integers(0, 4096, size=(H, W)).astype(np.uint16)
        f1 = np.roll(f0, (6, -10), axis=(0, 1)).copy()
        mv, sad = dev.pyramid(_to_dev(f0), _to_dev(f1), ctx)
        torch.cuda.synchronize()
        mv_o, sad_o, _, _ = oracle_mod.pyramid_search(f0, f1)
        _same(mv, sad, mv_o, sad_o)


def test_pyramid_hd_pair(dev, ctx, oracle_mod):
    import torch

    from paper_2508_05990_amd import synth

    seq = synth.hd_sequence(1, n_frames=3)
    f0, f1 = seq.frames[1], seq.frames[2]
    mv, sad = dev.pyramid(_to_dev(f0), _to_dev(f1), ctx)
    torch.cuda.synchronize()
    mv_o, sad_o, _, _ = oracle_mod.pyramid_search(f0, f1)
    _same(mv, sad, mv_o, sad_o)
