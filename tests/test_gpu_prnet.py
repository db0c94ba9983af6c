"""GPU parity of the perception residual network (paper Sec. 3.3) against the
float64 oracle, through the C ABI: every layer kernel (depthwise and 1x1
convolutions forward and backward, with their fused bias, ReLU6, added tensor
and derivative mask, channels-last and channels-first, float32 and
bfloat16), the weighted BerHu loss, the whole forward pass (at the 1080p
feature shape too) and a whole training step's gradient and update.

Tolerances.  A layer output is a float32 sum rounded to bfloat16, so it lies
within half a bfloat16 step (2^-8 relative) plus the float32 summation error
(1e-6 of the sum of |terms|) of the exact float64 value.
Whole-network results compound one rounding per stored activation; they are
compared by relative norm here, and stage by stage, element by element, in
test_gpu_prnet_stages.py."""
import numpy as np
import pytest

from oracle import prnet as P

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


def _bf(x):
    """float64 host array -> (bfloat16-rounded float64, device bfloat16 tensor)."""
    import torch

    r = P.bf16_round(x)
    return r, torch.from_numpy(r.astype(np.float32)).cuda().to(torch.bfloat16)


def _f32(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _host(t):
    import torch

    return t.float().cpu().numpy().astype(np.float64) if t.dtype == torch.bfloat16 else t.cpu().numpy().astype(np.float64)


def _close(got, ref, absterm, what):
    err = np.abs(got - ref)
    bound = 2.0 ** -8 * np.abs(ref) + 2e-6 * absterm + 1e-7
    bad = err > bound
    assert not bad.any(), (what, int(bad.sum()), float(err.max()), np.argwhere(bad)[:3].tolist())


@pytest.mark.parametrize("S,n,H,W,C", [(1, 2, 13, 17, 4), (2, 2, 13, 17, 4), (2, 1, 40, 66, 32), (1, 2, 15, 21, 128),
                                       (2, 1, 1, 3, 8), (1, 3, 5, 70, 64)])
def test_dw_forward_backward(dev, ctx, S, n, H, W, C):
    import torch

    rng = np.random.default_rng(S * 1000 + H * 10 + C)
    x, xt = _bf(rng.normal(size=(n, H, W, C)) * 2 + 1)
    w = rng.normal(size=(C, 9)).astype(np.float32).astype(np.float64)
    b = rng.normal(size=C).astype(np.float32).astype(np.float64)
    for relu6 in (False, True):
        y = dev.prnet_dw_forward(ctx, xt, _f32(w), _f32(b), S, relu6=relu6)
        torch.cuda.synchronize()
        ref = P.dwconv(x, w, b, S)
        absterm = P.dwconv(np.abs(x), np.abs(w), np.abs(b), S)
        if relu6:
            ref = P.relu6(ref)
        _close(_host(y), ref, absterm, "dw forward")
    Ho, Wo = y.shape[1:3]
    dy, dyt = _bf(rng.normal(size=(n, Ho, Wo, C)))
    mask, maskt = _bf(rng.uniform(-1, 7, size=x.shape))
    mask[..., 0] = 6.0                                   # boundary values of the derivative rule
    mask[..., -1] = 0.0
    maskt = _bf(mask)[1]
    dx = torch.empty_like(xt)
    grads = torch.empty(C * 10, dtype=torch.float32, device="cuda")
    dev.prnet_dw_backward(ctx, xt, _f32(w), dyt, S, mask=maskt, dx=dx, grads=grads)
    torch.cuda.synchronize()
    rdx, rdw, rdb = P.dw_backward(x, w, dy, S)
    adx = P.dw_backward(x, np.abs(w), np.abs(dy), S)[0]
    _, adw, adb = P.dw_backward(np.abs(x), w, np.abs(dy), S)
    _close(_host(dx), rdx * P.relu6_grad(mask), adx, "dw dgrad")
    g = grads.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(g[:C * 9] - rdw.ravel()) <= 1e-5 * adw.ravel() + 1e-7), "dw wgrad"
    assert np.all(np.abs(g[C * 9:] - rdb) <= 1e-5 * adb + 1e-7), "dw bgrad"
    # input gradient alone, no mask
    dev.prnet_dw_backward(ctx, xt, _f32(w), dyt, S, dx=dx)
    torch.cuda.synchronize()
    _close(_host(dx), rdx, adx, "dw dgrad unmasked")


def _pw_ref(x, W, b, relu6, add, mask):
    y = P.pwconv(x, P.bf16_round(W), b if b is not None else 0.0)
    absterm = P.pwconv(np.abs(x), np.abs(P.bf16_round(W)), np.abs(b) if b is not None else 0.0)
    if relu6:
        y = P.relu6(y)
    if add is not None:
        y = y + add
        absterm = absterm + np.abs(add)
    if mask is not None:
        y = y * P.relu6_grad(mask)
    return y, absterm


# up to 1024 pixel tiles the kernel runs eight waves per workgroup, beyond four
# (2 x 33000 pixels: 1032 tiles)
@pytest.mark.parametrize("n,HW,cin,cout", [(2, 100, 4, 32), (1, 317, 64, 256), (3, 64, 16, 16), (2, 211, 256, 64),
                                           (1, 70, 32, 48), (2, 33000, 64, 64)])
def test_pw_forward_nhwc(dev, ctx, n, HW, cin, cout):
    import torch

    rng = np.random.default_rng(n * 7 + HW + cin)
    x, xt = _bf(rng.normal(size=(n, HW, cin)))
    W = rng.normal(size=(cout, cin)) / np.sqrt(cin)
    b = rng.normal(size=cout).astype(np.float32).astype(np.float64)
    add, addt = _bf(rng.normal(size=(n, HW, cout)))
    mask, maskt = _bf(rng.uniform(-1, 7, size=(n, HW, cout)))
    for relu6, use_add, use_mask, f32 in [(True, False, False, False), (False, True, False, False),
                                          (False, True, True, False), (True, False, False, True)]:
        out = torch.empty((n, HW, cout), dtype=torch.float32 if f32 else torch.bfloat16, device="cuda")
        dev.prnet_pw_forward(ctx, xt, _f32(W), _f32(b), out, relu6=relu6, add=addt if use_add else None,
                             mask=maskt.reshape(-1, cout) if use_mask else None)
        torch.cuda.synchronize()
        ref, absterm = _pw_ref(x, W, b, relu6, add if use_add else None, mask if use_mask else None)
        got = _host(out)
        if f32:
            assert np.all(np.abs(got - ref) <= 1e-6 * absterm + 1e-7), "pw forward f32"
        else:
            _close(got, ref, absterm, (relu6, use_add, use_mask))


@pytest.mark.parametrize("zdtype,Hf,Wf", [("f32", 9, 23), ("bf16", 9, 23), ("f32", 8, 23), ("bf16", 12, 5),
                                          ("f32", 136, 244), ("bf16", 137, 243)])
def test_pw_forward_concat_and_channels_first(dev, ctx, zdtype, Hf, Wf):
    """The projection's input [z_pred (channels-first), encoder (channels-last)]
    and the head's channels-first output with z_pred added (pixels per image a
    multiple of 4 or not: two store paths; the last two shapes have more than
    1024 pixel tiles)."""
    import torch

    rng = np.random.default_rng(5)
    n, Cz, Ce, Ch = 2, 48, 16, 32
    HW = Hf * Wf
    z = rng.normal(size=(n, Cz, HW))
    if zdtype == "bf16":
        z, zt = _bf(z)
    else:
        z = z.astype(np.float32).astype(np.float64)
        zt = _f32(z)
    e4, e4t = _bf(rng.uniform(0, 6, size=(n, HW, Ce)))
    W = rng.normal(size=(Ch, Cz + Ce)) / 8
    b = rng.normal(size=Ch).astype(np.float32).astype(np.float64)
    out = torch.empty((n, HW, Ch), dtype=torch.bfloat16, device="cuda")
    dev.prnet_pw_forward(ctx, zt, _f32(W), _f32(b), out, x2=e4t, relu6=True, x_layout=dev.ME_NCHW)
    torch.cuda.synchronize()
    xc = np.concatenate([P.bf16_round(z.transpose(0, 2, 1)), e4], axis=-1)
    ref, absterm = _pw_ref(xc, W, b, True, None, None)
    _close(_host(out), ref, absterm, "concat projection")
    # head: channels-first output plus z_pred
    h, ht = _bf(rng.normal(size=(n, HW, Ch)))
    Wh = rng.normal(size=(Cz, Ch)) / 6
    bh = rng.normal(size=Cz).astype(np.float32).astype(np.float64)
    zo = torch.empty((n, Cz, HW), dtype=zt.dtype, device="cuda")
    dev.prnet_pw_forward(ctx, ht, _f32(Wh), _f32(bh), zo, add=zt, add_layout=dev.ME_NCHW, out_layout=dev.ME_NCHW)
    torch.cuda.synchronize()
    r, absterm = _pw_ref(h, Wh, bh, False, None, None)
    ref = z + r.transpose(0, 2, 1)
    absterm = np.abs(z) + absterm.transpose(0, 2, 1)
    got = _host(zo)
    if zdtype == "f32":
        assert np.all(np.abs(got - ref) <= 1e-6 * absterm + 1e-7), "head f32"
    else:
        _close(got, ref, absterm, "head bf16")


@pytest.mark.parametrize("n,HW,cin,cout,c0,cnt", [(2, 150, 64, 256, 0, 64), (1, 333, 288, 64, 256, 32),
                                                  (2, 100, 4, 32, 0, 4), (1, 64, 16, 16, 0, 16)])
def test_pw_backward(dev, ctx, n, HW, cin, cout, c0, cnt):
    import torch

    rng = np.random.default_rng(cin + cout + HW)
    x, xt = _bf(rng.normal(size=(n, HW, cin)))
    W = rng.normal(size=(cout, cin)) / np.sqrt(cin)
    dy, dyt = _bf(rng.normal(size=(n, HW, cout)) * 1e-2)
    add, addt = _bf(rng.normal(size=(n, HW, cnt)) * 1e-2)
    mask, maskt = _bf(rng.uniform(-1, 7, size=(n, HW, cnt)))
    dx = torch.empty((n, HW, cnt), dtype=torch.bfloat16, device="cuda")
    grads = torch.empty(cout * cin + cout, dtype=torch.float32, device="cuda")
    dev.prnet_pw_backward(ctx, xt, _f32(W), dyt, dx=dx, dx_c0=c0, dx_count=cnt, add=addt, mask=maskt, grads=grads)
    torch.cuda.synchronize()
    Wb = P.bf16_round(W)
    rdx, rdw, rdb = P.pw_backward(x, Wb, dy)
    adx = np.abs(dy) @ np.abs(Wb)
    ref = (rdx[..., c0:c0 + cnt] + add) * P.relu6_grad(mask)
    _close(_host(dx), ref, adx[..., c0:c0 + cnt] + np.abs(add), "pw dgrad")
    g = grads.cpu().numpy().astype(np.float64)
    adw = np.abs(dy).reshape(-1, cout).T @ np.abs(x).reshape(-1, cin)
    assert np.all(np.abs(g[:cout * cin] - rdw.ravel()) <= 1e-5 * adw.ravel() + 1e-9), "pw wgrad"
    adb = np.abs(dy).reshape(-1, cout).sum(axis=0)
    assert np.all(np.abs(g[cout * cin:] - rdb) <= 1e-5 * adb + 1e-9), "pw bgrad"


@pytest.mark.parametrize("tau", [-1.0, 0.8, 100.0])
def test_loss(dev, ctx, tau):
    import torch

    rng = np.random.default_rng(17)
    n, C, Hf, Wf = 2, 32, 11, 29
    zp = rng.normal(size=(n, C, Hf, Wf)).astype(np.float32)
    zt = (zp + rng.normal(size=zp.shape) * np.where(rng.random((n, 1, Hf, Wf)) < 0.2, 2.0, 0.05)).astype(np.float32)
    r = (rng.normal(size=zp.shape) * 0.5).astype(np.float32)
    dr, loss = dev.prnet_loss(ctx, _f32(r), _f32(zp), _f32(zt), tau=tau)
    torch.cuda.synchronize()
    L, g, c = P.loss_and_grad(r, zp, zt, tau)
    assert float(loss.item()) == pytest.approx(L, rel=1e-5)
    _close(_host(dr), g, np.abs(g), "loss gradient")


CFG_SMALL = (32, 16, 16, 2, 2)


def _net_inputs(seed, n, H, W, cfg):
    from paper_2508_05990_amd import synth

    Hf, Wf = P.feature_grid(H // 2, W // 2)
    frames = np.stack(synth.sequence(seed, H=H, W=W, n_frames=n, n_rects=2, side=(8, 32), vmax=4).frames)
    rng = np.random.default_rng(seed)
    zp = rng.normal(size=(n, cfg.c_feat, Hf, Wf)).astype(np.float32)
    bad = rng.random((n, 1, Hf, Wf)) < 0.25
    zt = (zp + rng.normal(size=zp.shape) * np.where(bad, 1.0, 0.02)).astype(np.float32)
    return frames, zp, zt


# (32, 16, 16, 2, 2): expanded width 32, blocks layer by layer; the others have
# expanded widths that are multiples of 64 and take the fused block kernel
# (hidden widths 32, 16, 96, 128 and 48).
@pytest.mark.parametrize("zdtype,cfgt,nimg", [("f32", CFG_SMALL, 2), ("bf16", CFG_SMALL, 2),
                                              ("f32", (32, 16, 32, 2, 2), 2), ("bf16", (48, 16, 16, 4, 1), 3),
                                              ("f32", (64, 16, 96, 2, 1), 2), ("bf16", (32, 16, 128, 1, 1), 2),
                                              ("f32", (32, 16, 48, 4, 1), 2)])
def test_network_forward(dev, ctx, zdtype, cfgt, nimg):
    import torch

    cfg = P.Cfg(*cfgt)
    frames, zp, _ = _net_inputs(3, nimg, 118, 166, cfg)
    params = P.init_params(cfg, 1)
    net = dev.Prnet(ctx, dev.MePrnetCfg(*cfgt))
    try:
        net.set_params(params)
        assert np.array_equal(net.get_params(), params)
        cur = torch.from_numpy(frames).cuda()
        z = _f32(zp) if zdtype == "f32" else _f32(zp).to(torch.bfloat16)
        out = net.forward(cur, z)
        torch.cuda.synchronize()
        zin = zp.astype(np.float64) if zdtype == "f32" else P.bf16_round(zp)
        _, r, ref = P.forward(params, cfg, frames, zin)
        got = _host(out)
        rel = np.linalg.norm((got - zin) - r) / np.linalg.norm(r)
        assert rel < 2e-2, rel
        # the same pass as a batch of one, frame by frame
        out1 = net.forward(cur[1], z[1])
        torch.cuda.synchronize()
        assert torch.equal(out1, out[1])
    finally:
        net.close()


def test_network_forward_1080p(dev, ctx):
    """The default network (c_feat 256, c_enc 32, c_hid 64, expand 4, 2 blocks)
    on the 1080p feature shape [256, 135, 240] that the warp produces."""
    import torch

    from paper_2508_05990_amd import synth

    cfg = P.Cfg()
    seq = synth.hd_sequence(1, n_frames=2)
    frame = seq.frames[1]
    zp = synth.features(4, 256, 135, 240)[None]
    params = P.init_params(cfg, 0, head_scale=0.1)
    net = dev.Prnet(ctx)
    try:
        net.set_params(params)
        out = net.forward(torch.from_numpy(frame).cuda(), _f32(zp[0]))
        torch.cuda.synchronize()
        _, r, _ = P.forward(params, cfg, frame, zp)
        got = _host(out)[None] - zp
        rel = np.linalg.norm(got - r) / np.linalg.norm(r)
        assert rel < 2e-2, rel
    finally:
        net.close()


@pytest.mark.parametrize("tau", [-1.0, 0.1])
def test_train_step_gradients_and_update(dev, ctx, tau):
    import torch

    from oracle import cnn as C

    cfg = P.Cfg(*CFG_SMALL)
    frames, zp, zt = _net_inputs(7, 2, 118, 166, cfg)
    params = P.init_params(cfg, 2, head_scale=0.3)
    net = dev.Prnet(ctx, dev.MePrnetCfg(*CFG_SMALL))
    try:
        net.set_params(params)
        cur = torch.from_numpy(frames).cuda()
        grads = torch.empty(net.n_params, dtype=torch.float32, device="cuda")
        loss = net.train_step(cur, _f32(zp), _f32(zt), tau=tau, update=False, grads=grads)
        torch.cuda.synchronize()
        A, r, _ = P.forward(params, cfg, frames, zp)
        L, dr, _ = P.loss_and_grad(r, zp, zt, tau)
        g_ref = P.backward(params, cfg, A, dr)
        assert float(loss.item()) == pytest.approx(L, rel=2e-2)
        g = grads.cpu().numpy().astype(np.float64)
        k = 0
        for i, (W, b) in enumerate(P.unpack(params, cfg)):
            for part in (W, b):
                a, bb = g[k:k + part.size], g_ref[k:k + part.size]
                k += part.size
                rel = np.linalg.norm(a - bb) / max(np.linalg.norm(bb), 1e-30)
                cos = a @ bb / max(np.linalg.norm(a) * np.linalg.norm(bb), 1e-30)
                assert rel < 5e-2 and cos > 0.998, (i, rel, cos)
        # determinism: the same step again gives the same bits
        grads2 = torch.empty_like(grads)
        net.train_step(cur, _f32(zp), _f32(zt), tau=tau, update=False, grads=grads2)
        torch.cuda.synchronize()
        assert torch.equal(grads, grads2)
        # one AdamW step: its first update is lr * sign(g) (plus decay), so wherever the
        # oracle's gradient is clearly nonzero the new weights match the oracle's update
        lr = 1e-3
        net.train_step(cur, _f32(zp), _f32(zt), tau=tau, lr=lr, update=True)
        torch.cuda.synchronize()
        w0 = params.astype(np.float64)
        w_ref, _, _ = C.adamw_step(w0, g_ref, np.zeros_like(g_ref), np.zeros_like(g_ref), 1, lr)
        got = net.get_params().astype(np.float64)
        clear = np.abs(g_ref) > 0.5 * np.sqrt(np.mean(g_ref ** 2))
        assert clear.mean() > 0.2
        assert np.all(np.abs(got - w_ref)[clear] <= 1e-6 * np.abs(w_ref[clear]) + 1e-3 * lr)
        assert np.all(np.abs(got - w0) <= lr * (1.0 + 0.01 * np.abs(w0)) * 1.001 + 1e-9)
    finally:
        net.close()


def test_training_reduces_loss(dev, ctx):
    """A few hundred steps on one synthetic batch fit part of the residual:
    the kernels' gradients descend."""
    import torch

    cfg = P.Cfg(*CFG_SMALL)
    frames, zp, _ = _net_inputs(9, 2, 118, 166, cfg)
    M = np.random.default_rng(4).normal(size=(cfg.c_feat, cfg.c_feat)) / np.sqrt(cfg.c_feat)
    zt = (zp + 0.5 * np.einsum("oc,nchw->nohw", M, zp)).astype(np.float32)   # a residual the network can represent
    net = dev.Prnet(ctx, dev.MePrnetCfg(*CFG_SMALL))
    try:
        net.set_params(P.init_params(cfg, 3, head_scale=0.1))
        cur = torch.from_numpy(frames).cuda()
        zpt, ztt = _f32(zp), _f32(zt)
        first = float(net.train_step(cur, zpt, ztt, update=False).item())
        for _ in range(200):
            loss = net.train_step(cur, zpt, ztt, lr=2e-3, update=True)
        torch.cuda.synchronize()
        assert float(loss.item()) < 0.9 * first, (first, float(loss.item()))
    finally:
        net.close()


@pytest.mark.parametrize("cfgt", [(16, 16, 16, 1, 0), (32, 16, 48, 4, 1), (16, 32, 32, 3, 2)])
def test_train_step_other_shapes(dev, ctx, cfgt):
    """No residual block (the head's input gradient carries the projection's
    mask), a fused-width hidden layer of 48 channels, an expansion of 3 (96
    channels, layer by layer at inference): gradients against the oracle;
    frames with a padded pitch and a frame stride larger than the frame."""
    import torch

    cfg = P.Cfg(*cfgt)
    frames, zp, zt = _net_inputs(11, 2, 86, 134, cfg)
    n, H, W = frames.shape
    padded = np.zeros((n, H + 3, W + 10), np.uint16)
    padded[:, :H, :W] = frames
    buf = torch.from_numpy(padded).cuda()
    cur = buf[:, :H, :W]                                   # pitch W + 10, frame stride (H + 3)(W + 10)
    params = P.init_params(cfg, 5, head_scale=0.3)
    net = dev.Prnet(ctx, dev.MePrnetCfg(*cfgt))
    try:
        net.set_params(params)
        grads = torch.empty(net.n_params, dtype=torch.float32, device="cuda")
        loss = net.train_step(cur, _f32(zp), _f32(zt), tau=0.1, update=False, grads=grads)
        out = net.forward(cur, _f32(zp))
        torch.cuda.synchronize()
        A, r, zo = P.forward(params, cfg, frames, zp)
        L, dr, _ = P.loss_and_grad(r, zp, zt, 0.1)
        assert float(loss.item()) == pytest.approx(L, rel=2e-2)
        rel = np.linalg.norm((_host(out) - zp) - r) / np.linalg.norm(r)
        assert rel < 2e-2, rel
        g_ref = P.backward(params, cfg, A, dr)
        g = grads.cpu().numpy().astype(np.float64)
        k = 0
        for i, (W_, b_) in enumerate(P.unpack(params, cfg)):
            for part in (W_, b_):
                a, bb = g[k:k + part.size], g_ref[k:k + part.size]
                k += part.size
                relg = np.linalg.norm(a - bb) / max(np.linalg.norm(bb), 1e-30)
                cos = a @ bb / max(np.linalg.norm(a) * np.linalg.norm(bb), 1e-30)
                assert relg < 5e-2 and cos > 0.998, (i, relg, cos)
    finally:
        net.close()
