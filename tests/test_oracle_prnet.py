"""Pins of the PRNet oracle (paper Sec. 3.3): each convolution against the
library convolution and a loop written from its definition, each backward
against autograd of the library convolution, the whole network's gradient
against finite differences, the loss against closed forms, and the residual
structure against its special cases."""
import numpy as np
import pytest
import torch

from oracle import prnet as P

CFG = P.Cfg(c_feat=16, c_enc=8, c_hid=16, expand=2, n_blocks=2)


def _torch_dw(x, W, b, s):
    xt = torch.from_numpy(x).permute(0, 3, 1, 2)
    C = x.shape[-1]
    y = torch.nn.functional.conv2d(xt, torch.from_numpy(W).reshape(C, 1, 3, 3), torch.from_numpy(b), stride=s,
                                   padding=1, groups=C)
    return y.permute(0, 2, 3, 1).numpy()


@pytest.mark.parametrize("s,H,W", [(1, 7, 9), (2, 7, 9), (2, 8, 10), (1, 1, 1), (2, 1, 3)])
def test_dwconv_matches_library_and_loop(s, H, W):
    rng = np.random.default_rng(s * 100 + H)
    x = rng.normal(size=(2, H, W, 5))
    Wt = rng.normal(size=(5, 9))
    b = rng.normal(size=5)
    y = P.dwconv(x, Wt, b, s)
    np.testing.assert_allclose(y, _torch_dw(x, Wt, b, s), rtol=1e-12, atol=1e-12)
    Ho, Wo = (H - 1) // s + 1, (W - 1) // s + 1
    assert y.shape == (2, Ho, Wo, 5)
    n, i, j, c = 1, Ho - 1, 0, 3                       # one element by the definition
    acc = b[c]
    for ky in range(3):
        for kx in range(3):
            yy, xx = s * i + ky - 1, s * j + kx - 1
            if 0 <= yy < H and 0 <= xx < W:
                acc += Wt[c, 3 * ky + kx] * x[n, yy, xx, c]
    assert abs(y[n, i, j, c] - acc) < 1e-12


def test_pwconv_matches_library_and_loop():
    rng = np.random.default_rng(7)
    x = rng.normal(size=(2, 3, 4, 6))
    Wt = rng.normal(size=(5, 6))
    b = rng.normal(size=5)
    y = P.pwconv(x, Wt, b)
    ref = torch.nn.functional.conv2d(torch.from_numpy(x).permute(0, 3, 1, 2), torch.from_numpy(Wt)[:, :, None, None],
                                     torch.from_numpy(b)).permute(0, 2, 3, 1).numpy()
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-12)
    assert abs(y[1, 2, 3, 4] - (b[4] + sum(Wt[4, i] * x[1, 2, 3, i] for i in range(6)))) < 1e-12


@pytest.mark.parametrize("s", [1, 2])
def test_dw_backward_matches_autograd(s):
    rng = np.random.default_rng(11 + s)
    x = rng.normal(size=(2, 9, 7, 4))
    Wt = rng.normal(size=(4, 9))
    b = rng.normal(size=4)
    y = P.dwconv(x, Wt, b, s)
    dy = rng.normal(size=y.shape)
    dx, dW, db = P.dw_backward(x, Wt, dy, s)
    xt = torch.from_numpy(x).permute(0, 3, 1, 2).requires_grad_(True)
    wt = torch.from_numpy(Wt).reshape(4, 1, 3, 3).requires_grad_(True)
    bt = torch.from_numpy(b).requires_grad_(True)
    yt = torch.nn.functional.conv2d(xt, wt, bt, stride=s, padding=1, groups=4)
    yt.backward(torch.from_numpy(dy).permute(0, 3, 1, 2))
    np.testing.assert_allclose(dx, xt.grad.permute(0, 2, 3, 1).numpy(), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(dW, wt.grad.reshape(4, 9).numpy(), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(db, bt.grad.numpy(), rtol=1e-11, atol=1e-11)


def test_pw_backward_matches_autograd():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(2, 3, 5, 6))
    Wt = rng.normal(size=(4, 6))
    b = rng.normal(size=4)
    dy = rng.normal(size=(2, 3, 5, 4))
    dx, dW, db = P.pw_backward(x, Wt, dy)
    xt = torch.from_numpy(x).permute(0, 3, 1, 2).requires_grad_(True)
    wt = torch.from_numpy(Wt)[:, :, None, None].requires_grad_(True)
    bt = torch.from_numpy(b).requires_grad_(True)
    torch.nn.functional.conv2d(xt, wt, bt).backward(torch.from_numpy(dy).permute(0, 3, 1, 2))
    np.testing.assert_allclose(dx, xt.grad.permute(0, 2, 3, 1).numpy(), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(dW, wt.grad[:, :, 0, 0].numpy(), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(db, bt.grad.numpy(), rtol=1e-11, atol=1e-11)


def _inputs(seed, n=2, H=24, W=40, cfg=CFG, noise=0.3):
    rng = np.random.default_rng(seed)
    m = rng.integers(0, 4096, (n, H, W)).astype(np.uint16)
    Hf, Wf = P.feature_grid(H // 2, W // 2)
    z = rng.normal(size=(n, cfg.c_feat, Hf, Wf))
    zt = z + rng.normal(size=z.shape) * noise
    zt[:, :, : Hf // 2] = z[:, :, : Hf // 2] + 0.01 * rng.normal(size=z[:, :, : Hf // 2].shape)   # well propagated half
    return m, z, zt


@pytest.mark.parametrize("tau", [-1.0, 0.1])
def test_network_gradient_matches_finite_differences(tau):
    m, z, zt = _inputs(0)
    p = P.init_params(CFG, 0).astype(np.float64)
    A, r, _ = P.forward(p, CFG, m, z, rnd=P.identity)
    _, dr, c = P.loss_and_grad(r, z, zt, tau)
    g = P.backward(p, CFG, A, dr, rnd=P.identity)
    specs = P.layer_specs(CFG)
    # two parameters of every layer (first weight and last bias), so no layer's gradient goes untested
    idx, k = [], 0
    for kind, ci, co, _, _ in specs:
        nw = co * 9 if kind == "dw" else co * ci
        idx += [k + nw // 2, k + nw + co - 1]
        k += nw + co
    assert k == p.size == P.n_params(CFG)
    eps = 1e-6
    for i in idx:
        q = p.copy()
        q[i] += eps
        lp = P.loss_and_grad(P.forward(q, CFG, m, z, rnd=P.identity)[1], z, zt, tau, c)[0]
        q[i] -= 2 * eps
        lm = P.loss_and_grad(P.forward(q, CFG, m, z, rnd=P.identity)[1], z, zt, tau, c)[0]
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_loss_closed_forms():
    # one element per position, c = 0.2 max|x|: x = [0.1, 1.0] -> c = 0.2
    r = np.array([0.1, 1.0]).reshape(1, 1, 1, 2)
    z = np.zeros_like(r)
    loss, dr, c = P.loss_and_grad(r, z, z)
    assert c == pytest.approx(0.2)
    assert loss == pytest.approx(0.5 * 0.1 + 0.5 * (1.0 + 0.04) / 0.4)
    np.testing.assert_allclose(dr.ravel(), [0.5 * 1.0, 0.5 * 1.0 / 0.2])
    # continuity of BerHu at |x| = c
    xs = np.array([0.2 - 1e-9, 0.2 + 1e-9, 1.0]).reshape(1, 1, 1, 3)
    loss2, _, _ = P.loss_and_grad(xs, np.zeros_like(xs), np.zeros_like(xs))
    assert np.isfinite(loss2)
    # zero residual error: zero loss and gradient
    l0, d0, c0 = P.loss_and_grad(z, z, z)
    assert l0 == 0.0 and c0 == 0.0 and not d0.any()


def test_loss_region_weights():
    """Two regions each carry half of the loss whatever their sizes; an empty
    region falls back to the plain mean; tau < 0 is the plain mean."""
    C = 3
    t = np.zeros((1, C, 1, 4))
    t[:, :, :, 0] = 2.0                                   # one badly propagated position, three good ones
    r = np.full_like(t, 0.5)                              # predicted residual
    z = np.zeros_like(t)
    x = r - t
    c = 0.2 * np.abs(x).max()
    a = np.abs(x)
    ber = np.where(a <= c, a, (x * x + c * c) / (2 * c))
    loss, dr, _ = P.loss_and_grad(r, z, t, tau=1.0)
    want = 0.5 * ber[:, :, :, 0].mean() + 0.5 * ber[:, :, :, 1:].mean()
    assert loss == pytest.approx(want)
    plain = ber.mean()
    assert P.loss_and_grad(r, z, t, tau=-1.0)[0] == pytest.approx(plain)
    assert P.loss_and_grad(r, z, t, tau=5.0)[0] == pytest.approx(plain)     # no bad position
    assert P.loss_and_grad(r, z, t, tau=0.0)[0] == pytest.approx(want)      # mean |t| = 0 is not above tau = 0
    # the position weights sum to one: with |r - t| = 1 everywhere (c = 0.2), every term is
    # (1 + 0.04) / 0.4 = 2.6, so the loss is 2.6 with or without region weights
    rng = np.random.default_rng(0)
    t2 = rng.normal(size=(2, C, 3, 5)) * np.array([0.01, 3.0])[rng.integers(0, 2, (2, 1, 3, 5))]
    r2 = t2 + np.where(rng.random(t2.shape) < 0.5, 1.0, -1.0)
    for tau in (-1.0, 0.5):
        assert P.loss_and_grad(r2, np.zeros_like(t2), t2, tau=tau)[0] == pytest.approx(2.6)


def test_zero_head_and_identity_blocks():
    m, z, _ = _inputs(1)
    p = P.init_params(CFG, 2)
    layers = P.unpack(p, CFG)
    flat = []
    for i, (W, b) in enumerate(layers):
        W, b = W.copy(), b.copy()
        if i == len(layers) - 1:
            W[:] = 0
        flat += [W.ravel(), b.ravel()]
    q = np.concatenate(flat)
    A, r, zo = P.forward(q, CFG, m, z, rnd=P.identity)
    assert not r.any() and np.array_equal(zo, z)
    # zero compression weights and biases: every block passes its input through
    flat = []
    for i, (W, b) in enumerate(layers):
        W, b = W.copy(), b.copy()
        if i >= 5 and i < len(layers) - 1 and (i - 5) % 3 == 2:
            W[:] = 0
            b[:] = 0
        flat += [W.ravel(), b.ravel()]
    A, r, _ = P.forward(np.concatenate(flat), CFG, m, z)
    for h in A["h"][1:]:
        assert np.array_equal(h, A["h"][0])


def test_relu6_derivative_convention_and_planes():
    y = np.array([0.0, 1e-9, 3.0, 6.0 - 1e-9, 6.0])
    np.testing.assert_array_equal(P.relu6_grad(y), [0, 1, 1, 1, 0])
    m = np.arange(4 * 6, dtype=np.uint16).reshape(4, 6) * 100
    pl = P.planes(m, rnd=P.identity)
    assert pl.shape == (1, 2, 3, 4)
    assert pl[0, 1, 2, 0] == (int(m[2, 4]) - 2048) / 1024 and pl[0, 1, 2, 3] == (int(m[3, 5]) - 2048) / 1024
    assert P.feature_grid(540, 960) == (135, 240)
    assert P.feature_grid(11, 5) == (3, 2)


# ---- rounded backward: float64 autograd with bfloat16 store points ---------
#
# The kernels store activations and the gradients that reach them in
# bfloat16.  This pin rebuilds the network in torch (float64, CPU) from the
# library convolutions and lets autograd derive the whole backward pass; the
# only hand-placed parts are the store points themselves, each a torch
# function whose forward rounds the value (torch's bfloat16 cast) and whose
# backward rounds the gradient that reaches the stored tensor:
#   ReLU6 layers: the gradient at the pre-activation, after the ReLU6 mask
#   read from the stored output; linear block outputs: the total gradient;
#   1x1 weights: rounded in the forward, gradient passed straight through.


def _rb(t):
    return t.to(torch.bfloat16).to(torch.float64)


class _StoreRelu6(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x):
        y = _rb(x.clamp(0.0, 6.0))
        ctx.save_for_backward(y)
        return y

    @staticmethod
    def backward(ctx, g):
        (y,) = ctx.saved_tensors
        return _rb(g * ((y > 0) & (y < 6)).to(g.dtype))


class _StoreLinear(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x):
        return _rb(x)

    @staticmethod
    def backward(ctx, g):
        return _rb(g)


class _WeightRound(torch.autograd.Function):
    @staticmethod
    def forward(ctx, w):
        return _rb(w)

    @staticmethod
    def backward(ctx, g):
        return g


def _torch_rounded_grad(p, cfg, m, z, dr, store=True):
    """Flat parameter gradient of <dr, r> through the network built in torch;
    store=False leaves out every rounding (for the sensitivity check)."""
    F = torch.nn.functional
    sr = _StoreRelu6.apply if store else (lambda x: x.clamp(0.0, 6.0))
    sl = _StoreLinear.apply if store else (lambda x: x)
    wr = _WeightRound.apply if store else (lambda w: w)
    fr = _rb if store else (lambda x: x)
    specs = P.layer_specs(cfg)
    leaves, k = [], 0
    flat = torch.from_numpy(np.asarray(p, dtype=np.float64))
    for kind, ci, co, _, _ in specs:
        nw = co * 9 if kind == "dw" else co * ci
        W = flat[k:k + nw].clone().reshape((co, 1, 3, 3) if kind == "dw" else (co, ci)).requires_grad_(True)
        b = flat[k + nw:k + nw + co].clone().requires_grad_(True)
        leaves.append((W, b))
        k += nw + co

    def dw(x, i, s):                                    # NCHW depthwise, zero padding 1
        W, b = leaves[i]
        return F.conv2d(x, W, b, stride=s, padding=1, groups=x.shape[1])

    def pw(x, i):                                       # NCHW 1x1 on rounded weights
        W, b = leaves[i]
        return torch.einsum("oc,nchw->nohw", wr(W), x) + b[None, :, None, None]

    mt = torch.from_numpy(np.asarray(m, dtype=np.float64))
    planes = torch.stack([mt[:, 0::2, 0::2], mt[:, 0::2, 1::2], mt[:, 1::2, 0::2], mt[:, 1::2, 1::2]], dim=1)
    a0 = fr((planes - 2048.0) / 1024.0)
    e1 = sr(dw(a0, 0, 2))
    e2 = sr(pw(e1, 1))
    e3 = sr(dw(e2, 2, 2))
    e4 = sr(pw(e3, 3))
    xc = torch.cat([fr(torch.from_numpy(np.asarray(z, dtype=np.float64))), e4], dim=1)
    h = sr(pw(xc, 4))
    for blk in range(cfg.n_blocks):
        i = 5 + 3 * blk
        u = sr(pw(h, i))
        v = sr(dw(u, i + 1, 1))
        h = sl(pw(v, i + 2) + h)
    r = pw(h, len(specs) - 1)
    r.backward(fr(torch.from_numpy(np.asarray(dr, dtype=np.float64))))
    parts = []
    for W, b in leaves:
        parts += [W.grad.reshape(-1).numpy(), b.grad.numpy()]
    return np.concatenate(parts)


@pytest.mark.parametrize("seed,tau", [(3, -1.0), (4, 0.1)])
def test_rounded_backward_matches_autograd_with_store_points(seed, tau):
    m, z, zt = _inputs(seed, n=2, H=28, W=44)
    p = P.init_params(CFG, seed).astype(np.float64)
    A, r, _ = P.forward(p, CFG, m, z)                   # bfloat16 store points (the default)
    _, dr, _ = P.loss_and_grad(r, z, zt, tau)
    g = P.backward(p, CFG, A, dr)
    ref = _torch_rounded_grad(p, CFG, m, z, dr)
    scale = np.abs(ref).max()
    np.testing.assert_allclose(g, ref, rtol=1e-9, atol=1e-12 * scale)
    # the pin can tell: without the store points the gradient moves by far more
    # than the tolerance (a misplaced rounding would show)
    plain = _torch_rounded_grad(p, CFG, m, z, dr, store=False)
    assert np.abs(plain - ref).max() > 1e-4 * scale
