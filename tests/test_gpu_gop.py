"""GPU parity of the group-of-pictures propagation (paper Sec. 4.1 GOP
protocol, Sec. 4.4): chained vectors bit-exact against the oracle, and each
schedule's propagated features within the warp tolerance of a float64 warp of
the same inputs."""
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


@pytest.mark.parametrize("B,H,W", [(16, 2 * 45, 2 * 61), (8, 2 * 64, 2 * 100), (32, 2 * 200, 2 * 130)])
def test_compose_vectors(dev, oracle_mod, B, H, W):
    import torch

    rng = np.random.default_rng(B)
    bh, bw = dev.block_grid(H, W, B)
    ms = rng.integers(-60, 61, (bh, bw, 2)).astype(np.int16)
    ma = rng.integers(-200, 201, (bh, bw, 2)).astype(np.int16)
    ref = oracle_mod.compose_vectors(ms, ma, B, H // 2, W // 2)
    got = dev.compose_vectors(_to_dev(ms), _to_dev(ma), B, H, W)
    step = _to_dev(ms)
    dev.compose_vectors(step, _to_dev(ma), B, H, W, out=step)        # in place over the step vectors
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), ref)
    assert np.array_equal(step.cpu().numpy(), ref)


@pytest.mark.parametrize("schedule", ["key", "previous", "composed"])
def test_schedules_match_oracle(dev, oracle_mod, schedule):
    import torch

    from paper_2508_05990_amd import gop, synth

    seq = synth.sequence(21, H=256, W=384, n_frames=6, n_rects=3, side=(24, 64), vmax=8)
    H, W = seq.shape
    B, R = 16, 16
    z0 = synth.features(5, 8, H // 8, W // 8)                         # 4 packed pixels per cell
    frames = [_to_dev(f) for f in seq.frames]
    ctx = dev.Context(0)
    try:
        feats, vecs = gop.propagate(ctx, frames, _to_dev(z0), schedule, B, R)
        torch.cuda.synchronize()
        acc = None
        z_prev = z0.astype(np.float64)
        for t in range(1, len(frames)):
            ref = seq.frames[0] if schedule == "key" else seq.frames[t - 1]
            mv, _, _ = oracle_mod.full_search(ref, seq.frames[t], B, R)
            if schedule == "composed":
                mv = mv if acc is None else oracle_mod.compose_vectors(mv, acc, B, H // 2, W // 2)
                acc = mv
            assert np.array_equal(vecs[t - 1].cpu().numpy(), mv), t
            # the recursive schedule warps the GPU's own previous output (float32)
            src = z_prev if schedule == "previous" else z0
            out, absterm = oracle_mod.warp_features(src, mv, B, H // 2, W // 2)
            got = feats[t - 1].cpu().numpy().astype(np.float64)
            err = np.abs(got - out)
            assert (err <= 1e-6 * absterm + 1e-30).all(), (t, err.max())
            z_prev = got
    finally:
        ctx.close()


@pytest.mark.parametrize("schedule", ["key", "previous"])
def test_corrected_propagation_matches_oracle(dev, oracle_mod, schedule):
    """The paper's video path per frame: ME, warp, correction by the residual
    network (Sec. 3.3), against the oracle's full search, float64 warp and
    float64 network (bfloat16 roundings where the kernels store them)."""
    import torch

    from oracle import prnet as P
    from paper_2508_05990_amd import gop, synth

    seq = synth.sequence(23, H=256, W=384, n_frames=4, n_rects=3, side=(24, 64), vmax=8)
    H, W = seq.shape
    B, R = 16, 16
    cfgt = (32, 16, 16, 4, 1)
    cfg = P.Cfg(*cfgt)
    Hf, Wf = P.feature_grid(H // 2, W // 2)
    z0 = synth.features(6, cfg.c_feat, Hf, Wf)
    params = P.init_params(cfg, 4, head_scale=0.2)
    frames = [_to_dev(f) for f in seq.frames]
    ctx = dev.Context(0)
    net = dev.Prnet(ctx, dev.MePrnetCfg(*cfgt))
    try:
        net.set_params(params)
        feats, _ = gop.propagate(ctx, frames, _to_dev(z0), schedule, B, R, net=net)
        torch.cuda.synchronize()
        z_prev = z0.astype(np.float64)
        for t in range(1, len(frames)):
            ref = seq.frames[0] if schedule == "key" else seq.frames[t - 1]
            mv, _, _ = oracle_mod.full_search(ref, seq.frames[t], B, R)
            src = z_prev if schedule == "previous" else z0
            zw, _ = oracle_mod.warp_features(src, mv, B, H // 2, W // 2)
            _, r, zo = P.forward(params, cfg, seq.frames[t], zw[None])
            got = feats[t - 1].cpu().numpy().astype(np.float64)
            rel = np.linalg.norm(got - zo[0]) / np.linalg.norm(zo[0])
            assert rel < 1e-2, (t, rel)
            z_prev = zo[0]
    finally:
        net.close()
        ctx.close()
