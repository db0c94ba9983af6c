"""Stage-by-stage element-wise parity of the residual network's inference pass
(paper Sec. 3.3) against the float64 oracle, through me_prnet_forward_acts.

The inference pass runs fused kernels (the whole encoder in one kernel, each
inverted residual block in one kernel), so their internal activations never
leave the chip.  Each stage is checked element by element on its own, fed the
GPU's output of the stage before it (the projection gets the GPU's encoder
output, block k the GPU's block k-1 output, the head the GPU's last block).

Bound.  Every stored activation is a float32 sum rounded to bfloat16, within
half a bfloat16 step (2^-8 of its magnitude) plus the float32 summation error
(2e-6 of the sum of |terms|) of the exact sum; the oracle's activation is the
exact sum rounded, so the two may differ by a whole step, 2^-7 of the
magnitude, where the sum lies near a rounding boundary (a 1080p frame has tens
of such elements).  Inside a fused stage those roundings compound, so the bound carries
each layer's worst case forward: an input off by d_in moves a 1x1 output by at
most sum |W| d_in and a depthwise output by at most sum over its taps of |W| d_in
(ReLU6 moves nothing further apart).  The bound is first order and worst case,
still a few bfloat16 steps where the sums do not cancel; a wrong weight, tap,
channel or pixel index gives errors of the order of the values themselves."""
import numpy as np
import pytest

from oracle import prnet as P

pytestmark = pytest.mark.gpu

H8 = 2.0 ** -8                                   # half a bfloat16 step, relative
H7 = 2.0 ** -7 * (1 + 2.0 ** -7)                 # a whole step (of the larger of the two magnitudes)


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


def _host(t):
    return t.float().cpu().numpy().astype(np.float64)


def _pw_abs(x, W):
    return np.abs(np.asarray(x, dtype=np.float64)) @ np.abs(np.asarray(W, dtype=np.float64)).T


def _dw_abs(x, W, stride):
    return P.dwconv(np.abs(x), np.abs(W), np.zeros(W.shape[0]), stride)


def _check(got, ref, bound, what):
    err = np.abs(got - ref)
    bad = err > bound
    assert not bad.any(), (what, int(bad.sum()), float(err.max()), np.argwhere(bad)[:3].tolist(),
                           float(np.abs(ref).max()))


def _stages(dev, ctx, cfgt, frames, zp, zdtype, params):
    """Run the inference pass; check every stage; return the worst error / bound ratios."""
    import torch

    cfg = P.Cfg(*cfgt)
    L = P.unpack(params, cfg)
    rnd = P.bf16_round
    net = dev.Prnet(ctx, dev.MePrnetCfg(*cfgt))
    try:
        net.set_params(params)
        cur = torch.from_numpy(frames).cuda()
        z = torch.from_numpy(np.ascontiguousarray(zp, dtype=np.float32)).cuda()
        if zdtype == "bf16":
            z = z.to(torch.bfloat16)
        out, enc, hid = net.forward_acts(cur, z)
        torch.cuda.synchronize()
    finally:
        net.close()
    zin = zp.astype(np.float64) if zdtype == "f32" else rnd(zp)
    ratios = {}

    # encoder: planes -> dw s2 -> 1x1 -> dw s2 -> 1x1, from the mosaic
    A, _, _ = P.forward(params, cfg, frames, zin)
    d1 = H7 * np.abs(A["e1"]) + 2e-6 * _dw_abs(A["a0"], L[0][0], 2)
    W1 = rnd(L[1][0])
    d2 = H7 * np.abs(A["e2"]) + _pw_abs(d1, W1) + 2e-6 * _pw_abs(A["e1"], W1)
    d3 = H7 * np.abs(A["e3"]) + _dw_abs(d2, L[2][0], 2) + 2e-6 * _dw_abs(A["e2"], L[2][0], 2)
    W3 = rnd(L[3][0])
    d4 = H7 * np.abs(A["e4"]) + _pw_abs(d3, W3) + 2e-6 * _pw_abs(A["e3"], W3) + 1e-7
    e4 = _host(enc)
    _check(e4, A["e4"], d4, "encoder")
    ratios["encoder"] = float((np.abs(e4 - A["e4"]) / d4).max())

    # projection of [z_pred, encoder output]
    xc = np.concatenate([rnd(zin.transpose(0, 2, 3, 1)), e4], axis=-1)
    W4 = rnd(L[4][0])
    h_ref = rnd(P.relu6(P.pwconv(xc, W4, L[4][1])))
    h = _host(hid[0])
    bound = H7 * np.abs(h_ref) + 2e-6 * (_pw_abs(xc, W4) + np.abs(L[4][1])) + 1e-7
    _check(h, h_ref, bound, "projection")
    ratios["projection"] = float((np.abs(h - h_ref) / bound).max())

    # inverted residual blocks, each fed the GPU's previous output
    for k in range(cfg.n_blocks):
        (We, be), (Wd, bd), (Wc, bc) = L[5 + 3 * k:8 + 3 * k]
        We, Wc = rnd(We), rnd(Wc)
        u = rnd(P.relu6(P.pwconv(h, We, be)))
        du = H7 * np.abs(u) + 2e-6 * _pw_abs(h, We)
        v = rnd(P.relu6(P.dwconv(u, Wd, bd, 1)))
        dv = H7 * np.abs(v) + _dw_abs(du, Wd, 1) + 2e-6 * _dw_abs(u, Wd, 1)
        h_ref = rnd(P.pwconv(v, Wc, bc) + h)
        bound = H7 * np.abs(h_ref) + _pw_abs(dv, Wc) + 2e-6 * (_pw_abs(v, Wc) + np.abs(h)) + 1e-7
        h = _host(hid[k + 1])
        _check(h, h_ref, bound, "block %d" % k)
        ratios["block %d" % k] = float((np.abs(h - h_ref) / bound).max())

    # head (float32, not rounded) added to z_pred
    Wh = rnd(L[-1][0])
    r = P.pwconv(h, Wh, L[-1][1]).transpose(0, 3, 1, 2)
    ref = zin + r
    terms = _pw_abs(h, Wh).transpose(0, 3, 1, 2) + np.abs(L[-1][1])[None, :, None, None]
    got = _host(out)
    if zdtype == "bf16":                # stored in bfloat16: half a step from the exact (unrounded) sum
        bound = H8 * np.abs(ref) + 2e-6 * (terms + np.abs(zin)) + 1e-7
    else:
        bound = 2.0 ** -23 * np.abs(ref) + 2e-6 * (terms + np.abs(zin)) + 1e-7
    _check(got, ref, bound, "head")
    ratios["head"] = float((np.abs(got - ref) / bound).max())
    return ratios


# default-width blocks (fused block kernel) and the hidden widths the fused
# encoder and blocks accept; float32 and bfloat16 features
@pytest.mark.parametrize("zdtype,cfgt,nimg", [("f32", (32, 16, 16, 4, 2), 2), ("bf16", (48, 16, 16, 4, 1), 3),
                                              ("f32", (64, 16, 96, 2, 1), 2), ("bf16", (32, 16, 128, 1, 1), 2)])
def test_stages_element_wise(dev, ctx, zdtype, cfgt, nimg):
    from paper_2508_05990_amd import synth

    cfg = P.Cfg(*cfgt)
    H, W = 118, 166
    Hf, Wf = P.feature_grid(H // 2, W // 2)
    frames = np.stack(synth.sequence(5, H=H, W=W, n_frames=nimg, n_rects=2, side=(8, 32), vmax=4).frames)
    rng = np.random.default_rng(5)
    zp = rng.normal(size=(nimg, cfg.c_feat, Hf, Wf)).astype(np.float32)
    params = P.init_params(cfg, 3, head_scale=0.5)
    ratios = _stages(dev, ctx, cfgt, frames, zp, zdtype, params)
    print(cfgt, zdtype, {k: round(v, 3) for k, v in ratios.items()}, flush=True)


def test_stages_element_wise_1080p(dev, ctx):
    """The default network on one 1080p frame and the [256, 135, 240] features."""
    from paper_2508_05990_amd import synth

    cfg = P.Cfg()
    frame = synth.hd_sequence(1, n_frames=2).frames[1][None]
    zp = synth.features(4, 256, 135, 240)[None]
    params = P.init_params(cfg, 0, head_scale=0.1)
    cfgt = (cfg.c_feat, cfg.c_enc, cfg.c_hid, cfg.expand, cfg.n_blocks)
    ratios = _stages(dev, ctx, cfgt, frame, zp, "f32", params)
    print("1080p", {k: round(v, 3) for k, v in ratios.items()}, flush=True)
