"""GPU parity of block matching: the HIP path through the C ABI against the
CPU oracle, bit for bit (motion vectors and SADs are integers)."""
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


def _to_dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _gpu_full(me, ref, cur, B, R, ctx=None):
    import torch

    mv, sad = me.estimate(_to_dev(ref), _to_dev(cur), B, R, ctx=ctx)
    torch.cuda.synchronize()
    return mv.cpu().numpy(), sad.cpu().numpy()


def _assert_same(mv_g, sad_g, mv_o, sad_o, blocks=None):
    if blocks is None:
        assert np.array_equal(sad_g, sad_o), np.argwhere(sad_g != sad_o)[:10]
        assert np.array_equal(mv_g, mv_o), np.argwhere((mv_g != mv_o).any(-1))[:10]
    else:
        assert np.array_equal(sad_g.ravel()[blocks], sad_o.ravel()[blocks])
        assert np.array_equal(mv_g.reshape(-1, 2)[blocks], mv_o.reshape(-1, 2)[blocks])


def test_small_pair_bit_exact(dev, oracle_mod):
    from paper_2508_05990_amd import synth

    for seed in range(3):
        f0, f1, (sx, sy) = synth.small_pair(seed)
        print("small pair seed", seed, flush=True)
        mv_g, sad_g = _gpu_full(dev, f0, f1, 16, 8)
        mv_o, sad_o, _ = oracle_mod.full_search(f0, f1, 16, 8)
        _assert_same(mv_g, sad_g, mv_o, sad_o)
        assert (mv_g[3, 3] == (-sx, -sy)).all()


@pytest.mark.parametrize("B", [8, 16, 32, 64])
@pytest.mark.parametrize("R", [0, 1, 3, 8, 17])
def test_random_shapes_bit_exact(dev, oracle_mod, B, R):
    """Random 12-bit and low-entropy frames, ragged sizes (partial blocks at
    the bottom and right edge), all block sizes, several radii."""
    rng = np.random.default_rng(B * 100 + R)
    for trial in range(3):
        H = 2 * int(rng.integers(B // 2, 3 * B + 5))
        W = 2 * int(rng.integers(B // 2, 3 * B + 5))
        if trial == 2:
            f0 = rng.integers(0, 3, size=(H, W)).astype(np.uint16)      # ties everywhere
            f1 = rng.integers(0, 3, size=(H, W)).astype(np.uint16)
        else:
            f0 = rng.integers(0, 4096, size=(H, W)).astype(np.uint16)
            f1 = rng.integers(0, 4096, size=(H, W)).astype(np.uint16)
        print("random B=%d R=%d %dx%d trial %d" % (B, R, H, W, trial), flush=True)
        mv_g, sad_g = _gpu_full(dev, f0, f1, B, R)
        mv_o, sad_o, _ = oracle_mod.full_search(f0, f1, B, R)
        _assert_same(mv_g, sad_g, mv_o, sad_o)


def test_full_16bit_range(dev, oracle_mod):
    """Samples above 12 bits (the ABI takes any uint16) and B=64: the largest SADs."""
    rng = np.random.default_rng(5)
    f0 = rng.integers(0, 65536, size=(300, 388)).astype(np.uint16)
    f1 = np.where(rng.random((300, 388)) < 0.5, 65535, 0).astype(np.uint16)
    mv_g, sad_g = _gpu_full(dev, f0, f1, 64, 5)
    mv_o, sad_o, _ = oracle_mod.full_search(f0, f1, 64, 5)
    _assert_same(mv_g, sad_g, mv_o, sad_o)


def test_frame_smaller_than_block(dev, oracle_mod):
    rng = np.random.default_rng(6)
    f0 = rng.integers(0, 4096, size=(10, 14)).astype(np.uint16)
    f1 = rng.integers(0, 4096, size=(10, 14)).astype(np.uint16)
    mv_g, sad_g = _gpu_full(dev, f0, f1, 16, 4)
    mv_o, sad_o, _ = oracle_mod.full_search(f0, f1, 16, 4)
    assert mv_g.shape == (1, 1, 2)
    _assert_same(mv_g, sad_g, mv_o, sad_o)


def test_padded_pitch(dev, oracle_mod):
    import torch

    rng = np.random.default_rng(7)
    f0 = rng.integers(0, 4096, size=(96, 136)).astype(np.uint16)
    f1 = rng.integers(0, 4096, size=(96, 136)).astype(np.uint16)
    big0 = np.zeros((96, 200), np.uint16)
    big1 = np.zeros((96, 200), np.uint16)
    big0[:, :136], big1[:, :136] = f0, f1
    t0, t1 = _to_dev(big0)[:, :136], _to_dev(big1)[:, :136]
    mv, sad = dev.estimate(t0, t1, 16, 6)
    torch.cuda.synchronize()
    mv_o, sad_o, _ = oracle_mod.full_search(f0, f1, 16, 6)
    _assert_same(mv.cpu().numpy(), sad.cpu().numpy(), mv_o, sad_o)


@pytest.mark.parametrize("B,R,limit", [(16, 2, 32), (8, 2, 16), (32, 3, 10), (16, 4, 127)])
def test_stage_search_with_predictors(dev, oracle_mod, B, R, limit):
    import torch

    rng = np.random.default_rng(B + R)
    H, W = 2 * 70, 2 * 90
    f0 = rng.integers(0, 4096, size=(H, W)).astype(np.uint16)
    f1 = rng.integers(0, 4096, size=(H, W)).astype(np.uint16)
    bh, bw = (H // 2 + B - 1) // B, (W // 2 + B - 1) // B
    pred = rng.integers(-limit - 3, limit + 4, size=(bh, bw, 2)).astype(np.int16)
    mv, sad = dev.stage_search(_to_dev(f0), _to_dev(f1), B, R, pred=_to_dev(pred), limit=limit)
    torch.cuda.synchronize()
    rp, cp = oracle_mod.pack_planes(f0), oracle_mod.pack_planes(f1)
    mv_o, sad_o, _, _ = oracle_mod.stage_search(rp, cp, B, R, 1, pred=pred, limit=limit)
    _assert_same(mv.cpu().numpy(), sad.cpu().numpy(), mv_o, sad_o)
    assert (sad_o == -1).any() or limit > 20     # some empty candidate sets are exercised


def test_deterministic_repeat(dev):
    import torch

    from paper_2508_05990_amd import synth

    f0, f1, _ = synth.small_pair(9)
    a = _gpu_full(dev, f0, f1, 16, 8)
    b = _gpu_full(dev, f0, f1, 16, 8)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    del torch


@pytest.fixture(scope="module")
def hd_seq():
    from paper_2508_05990_amd import synth

    return synth.hd_sequence(1, n_frames=3)


def test_hd_sequence_pairs_bit_exact(dev, oracle_mod, hd_seq):
    """1080p, B=16, R=32: two full frame pairs, every block."""
    for t in (1, 2):
        print("1080p pair", t, flush=True)
        mv_g, sad_g = _gpu_full(dev, hd_seq.frames[t - 1], hd_seq.frames[t], 16, 32)
        mv_o, sad_o, ops = oracle_mod.full_search(hd_seq.frames[t - 1], hd_seq.frames[t], 16, 32)
        assert ops == 8_171_357_184
        _assert_same(mv_g, sad_g, mv_o, sad_o)


@pytest.fixture(scope="module")
def uhd_seq():
    from paper_2508_05990_amd import synth

    return synth.uhd_sequence(4, n_frames=4)


@pytest.mark.parametrize("t", [1, 2, 3])
def test_uhd_pairs_bit_exact(dev, oracle_mod, uhd_seq, t):
    """4K, B=16, R=64 (the LDS window is processed in dy bands): three pairs
    of the panning 4K sequence, every block of the frame."""
    print("4K pair", t, flush=True)
    mv_g, sad_g = _gpu_full(dev, uhd_seq.frames[t - 1], uhd_seq.frames[t], 16, 64)
    mv_o, sad_o, ops = oracle_mod.full_search(uhd_seq.frames[t - 1], uhd_seq.frames[t], 16, 64)
    assert ops == 130_206_208_000
    _assert_same(mv_g, sad_g, mv_o, sad_o)


@pytest.mark.parametrize("B", [8, 32, 64])
@pytest.mark.parametrize("R", [48, 64])
def test_large_radius_banded_pairs_bit_exact(dev, oracle_mod, B, R):
    """Radius 48 and 64 with the default launch shape, the window staged in
    several dy bands: blocks of 8 and 32 two per workgroup with 4x2 tiles
    within 80 KB (32: rows walked in 16-word chunks); blocks of 64, whose two-
    block window does not fit 80 KB, one per workgroup with 4x4 tiles; uniform
    12-bit frames and a low-entropy pair full of ties."""
    ctx = dev.Context(0)
    try:
        shape, tuned = dev.tuned_shape(ctx, B, R, 256, 384)
        assert not tuned, shape
        if B == 64:
            assert shape[:3] == (4, 4, 1), shape
        else:
            assert shape[:3] == (4, 2, 2) and shape[3] <= 80, shape
    finally:
        ctx.close()
    rng = np.random.default_rng(B * 1000 + R)
    for trial in range(2):
        if trial:
            f0 = rng.integers(0, 3, size=(256, 384)).astype(np.uint16)
            f1 = rng.integers(0, 3, size=(256, 384)).astype(np.uint16)
        else:
            f0 = rng.integers(0, 4096, size=(256, 384)).astype(np.uint16)
            f1 = rng.integers(0, 4096, size=(256, 384)).astype(np.uint16)
        print("banded B=%d R=%d trial %d" % (B, R, trial), flush=True)
        mv_g, sad_g = _gpu_full(dev, f0, f1, B, R)
        mv_o, sad_o, _ = oracle_mod.full_search(f0, f1, B, R)
        _assert_same(mv_g, sad_g, mv_o, sad_o)
