"""Search and warp in one pass (me_estimate_warp): vectors, SADs and the
warped map bit-identical to me_estimate followed by me_warp_features, on the
1080p pair (float32 and bfloat16 maps), ragged frames whose edge blocks take
the generic kernel, other block and cell sizes, a radius served by the
small-radius kernel, and against the oracle on a small pair."""
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


def _both(dev, ctx, f0, f1, z, B, R):
    import torch

    H, W = f0.shape
    mv1, sad1, out1 = dev.estimate_warp(f0, f1, z, B, R, ctx=ctx)
    mv2, sad2 = dev.estimate(f0, f1, B, R, ctx=ctx)
    out2 = dev.warp_features(z, mv2, B, H, W, ctx=ctx)
    torch.cuda.synchronize()
    assert torch.equal(mv1, mv2) and torch.equal(sad1, sad2)
    assert torch.equal(out1.view(torch.int16) if out1.dtype == torch.bfloat16 else out1.view(torch.int32),
                       out2.view(torch.int16) if out2.dtype == torch.bfloat16 else out2.view(torch.int32))
    return mv1, sad1, out1


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_fused_1080p(dev, dtype):
    import torch

    from paper_2508_05990_amd import synth

    seq = synth.hd_sequence(1, n_frames=2)
    f0, f1 = (torch.from_numpy(f).cuda() for f in seq.frames)
    z = torch.from_numpy(synth.features(11, 256, 135, 240)).cuda()
    if dtype == "bf16":
        z = z.to(torch.bfloat16)
    ctx = dev.Context(0)
    try:
        for _ in range(2):
            _both(dev, ctx, f0, f1, z, 16, 32)
    finally:
        ctx.close()


@pytest.mark.parametrize("H,W,B,R,s,C", [(200, 296, 16, 8, 4, 24), (136, 264, 8, 16, 2, 16), (272, 400, 32, 12, 8, 8),
                                         (72, 104, 16, 3, 4, 12), (128, 128, 64, 6, 16, 4)])
def test_fused_ragged_and_oracle(dev, oracle_mod, H, W, B, R, s, C):
    import torch

    rng = np.random.default_rng(H + W + B)
    base = rng.integers(0, 4096, (H + 40, W + 40)).astype(np.uint16)
    f0 = np.ascontiguousarray(base[20:20 + H, 20:20 + W])
    dy, dx = (int(v) for v in rng.integers(0, 30, 2))
    f1 = np.ascontiguousarray(base[dy:dy + H, dx:dx + W])
    Hf, Wf = H // 2 // s, W // 2 // s
    zf = rng.standard_normal((C, Hf, Wf)).astype(np.float32)
    t0, t1, z = torch.from_numpy(f0).cuda(), torch.from_numpy(f1).cuda(), torch.from_numpy(zf).cuda()
    ctx = dev.Context(0)
    try:
        mv, sad, out = _both(dev, ctx, t0, t1, z, B, R)
        mv_o, sad_o, _ = oracle_mod.full_search(f0, f1, B, R)
        assert np.array_equal(mv.cpu().numpy(), mv_o) and np.array_equal(sad.cpu().numpy(), sad_o)
        ref, absterm = oracle_mod.warp_features(zf.astype(np.float64), mv_o, B, H // 2, W // 2)
        err = np.abs(out.cpu().numpy().astype(np.float64) - ref)
        assert (err <= 1e-6 * absterm + 1e-30).all()
    finally:
        ctx.close()
