"""Pins of the float64 proposal-network oracle (oracle/cnn.py).

Checked against library routines (torch float64 conv2d and autograd, torch's
bfloat16 conversion), a naive loop definition of the convolution, finite
differences of the loss and of the whole network, and closed forms of AdamW
and the cosine schedule."""
import numpy as np
import pytest
import torch

from oracle import cnn


def test_parameter_count():
    assert cnn.NPARAMS == 21699
    p = cnn.init_params(0)
    assert np.array_equal(cnn.pack(cnn.unpack(p)), p.astype(np.float64))


def test_bf16_round_ties_and_library():
    one = 1.0
    assert cnn.bf16_round(one) == 1.0
    assert cnn.bf16_round(1 + 2.0 ** -8) == 1.0                 # tie -> even
    assert cnn.bf16_round(1 + 3 * 2.0 ** -8) == 1 + 2.0 ** -6    # tie -> even (up)
    assert cnn.bf16_round(-(1 + 2.0 ** -7)) == -(1 + 2.0 ** -7)
    x = np.random.default_rng(0).normal(0, 10, 10000)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cnn.bf16_round(x.astype(np.float32)), ref)


def _naive_conv(x, W, b, s):
    C, H, Wd = x.shape
    Ho, Wo = (H - 1) // s + 1, (Wd - 1) // s + 1
    out = np.zeros((W.shape[0], Ho, Wo))
    for o in range(W.shape[0]):
        for y in range(Ho):
            for xx in range(Wo):
                acc = b[o]
                for c in range(C):
                    for ky in range(3):
                        for kx in range(3):
                            iy, ix = s * y + ky - 1, s * xx + kx - 1
                            if 0 <= iy < H and 0 <= ix < Wd:
                                acc += W[o, c, ky, kx] * x[c, iy, ix]
                out[o, y, xx] = acc
    return out


@pytest.mark.parametrize("s", [1, 2])
def test_conv_matches_naive_definition(s):
    rng = np.random.default_rng(s)
    x = rng.normal(size=(3, 7, 9))
    W = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    np.testing.assert_allclose(cnn.conv3x3(x, W, b, s), _naive_conv(x, W, b, s), atol=1e-12)


@pytest.mark.parametrize("s", [1, 2])
def test_conv_matches_library(s):
    rng = np.random.default_rng(10 + s)
    x = rng.normal(size=(8, 27, 31))
    W = rng.normal(size=(5, 8, 3, 3))
    b = rng.normal(size=5)
    ref = torch.nn.functional.conv2d(torch.from_numpy(x)[None], torch.from_numpy(W), torch.from_numpy(b),
                                     stride=s, padding=1)[0].numpy()
    np.testing.assert_allclose(cnn.conv3x3(x, W, b, s), ref, atol=1e-10)
    assert ref.shape[1] == -(-27 // s) and ref.shape[2] == -(-31 // s)


def test_conv_identity_kernel():
    x = np.random.default_rng(3).normal(size=(4, 6, 5))
    W = np.zeros((4, 4, 3, 3))
    for c in range(4):
        W[c, c, 1, 1] = 1.0
    assert np.array_equal(cnn.conv3x3(x, W, np.zeros(4), 1), x)


@pytest.mark.parametrize("s", [1, 2])
def test_conv_grads_match_autograd(s):
    rng = np.random.default_rng(20 + s)
    x = rng.normal(size=(6, 13, 10))
    W = rng.normal(size=(5, 6, 3, 3))
    d = rng.normal(size=(5, -(-13 // s), -(-10 // s)))
    xt = torch.from_numpy(x).requires_grad_(True)
    Wt = torch.from_numpy(W).requires_grad_(True)
    y = torch.nn.functional.conv2d(xt[None], Wt, None, stride=s, padding=1)[0]
    (y * torch.from_numpy(d)).sum().backward()
    np.testing.assert_allclose(cnn.conv_wgrad(x, d, s), Wt.grad.numpy(), atol=1e-10)
    np.testing.assert_allclose(cnn.conv_dgrad(d, W, s, x.shape), xt.grad.numpy(), atol=1e-10)


def _tiny_batch(seed, H=32, W=48):
    rng = np.random.default_rng(seed)
    x = rng.normal(0, 0.5, size=(8, H, W))
    bh, bw = -(-H // 4), -(-W // 4)           # total stride 4
    mv = rng.integers(-6, 7, size=(bh, bw, 2))
    return x, mv


def test_network_gradient_finite_differences():
    """Backward of the whole network (rounding off) against central differences."""
    params = cnn.init_params(1).astype(np.float64)
    params[cnn.NPARAMS - 3:] = [0.1, -0.2, 0.3]
    x, mv = _tiny_batch(2)
    out, acts, pres = cnn.forward(params, x, cnn.identity)
    y = cnn.labels(out, mv, 8, 2)
    _, dout = cnn.loss_and_grad(out, mv, 8, 2, y=y)
    g = cnn.backward(params, acts, pres, dout, cnn.identity)

    def L(p):
        o, _, _ = cnn.forward(p, x, cnn.identity)
        return cnn.loss_and_grad(o, mv, 8, 2, y=y)[0]

    rng = np.random.default_rng(4)
    idx = np.concatenate([rng.choice(cnn.NPARAMS, 40, replace=False), np.arange(cnn.NPARAMS - 3, cnn.NPARAMS)])
    h = 1e-6
    for i in idx:
        pp, pm = params.copy(), params.copy()
        pp[i] += h
        pm[i] -= h
        fd = (L(pp) - L(pm)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-5 * max(1.0, abs(fd)), (i, fd, g[i])


def test_weighted_loss():
    """Per-block weight of the vector term: zero weights leave the mean BCE
    alone; the gradient matches central differences of the weighted loss."""
    rng = np.random.default_rng(9)
    out = rng.normal(0, 1, (3, 4, 5))
    mv = rng.integers(-12, 13, (4, 5, 2))
    y = cnn.labels(out, mv, 16, 2)
    L0, g0 = cnn.loss_and_grad(out, mv, 16, 2, y=y, weight=np.zeros((4, 5)))
    assert L0 == pytest.approx(cnn.bce_logits(out[2], y).mean(), rel=1e-12)
    assert not g0[:2].any()
    w = rng.choice([0.0, 0.5, 1.0, 2.0], (4, 5))
    L1, _ = cnn.loss_and_grad(out, mv, 16, 2, y=y)
    Lw, gw = cnn.loss_and_grad(out, mv, 16, 2, y=y, weight=w)
    ones, _ = cnn.loss_and_grad(out, mv, 16, 2, y=y, weight=np.ones((4, 5)))
    assert ones == L1
    h = 1e-6
    for idx in [(0, 1, 2), (1, 3, 4), (0, 0, 0), (2, 2, 1)]:
        op, om = out.copy(), out.copy()
        op[idx] += h
        om[idx] -= h
        fd = (cnn.loss_and_grad(op, mv, 16, 2, y=y, weight=w)[0] - cnn.loss_and_grad(om, mv, 16, 2, y=y, weight=w)[0]) / (2 * h)
        assert gw[idx] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_berhu_and_bce():
    c = cnn.BERHU_C
    assert cnn.berhu(c) == pytest.approx(c) and cnn.berhu(c + 1e-12) == pytest.approx(c)   # continuous at c
    assert cnn.berhu(2 * c) == pytest.approx(((2 * c) ** 2 + c * c) / (2 * c))
    for x in [-2.5 * c, -0.5 * c, -0.1 * c, 0.05 * c, 0.3 * c, 1.7 * c]:   # both branches
        fd = (cnn.berhu(x + 1e-7) - cnn.berhu(x - 1e-7)) / 2e-7
        assert cnn.berhu_grad(x) == pytest.approx(fd, rel=1e-5)
    for z in [-30.0, -2.0, 0.0, 1.5, 40.0]:
        for y in [0.0, 1.0]:
            ref = -(y * np.log(1 / (1 + np.exp(-z))) + (1 - y) * np.log(1 - 1 / (1 + np.exp(-z)))) \
                if abs(z) < 30 else None
            if ref is not None:
                assert cnn.bce_logits(z, y) == pytest.approx(ref, rel=1e-10)
            fd = (cnn.bce_logits(z + 1e-6, y) - cnn.bce_logits(z - 1e-6, y)) / 2e-6
            assert cnn.sigmoid(z) - y == pytest.approx(fd, abs=1e-6)


def test_labels():
    out = np.zeros((3, 1, 3))
    out[0] = [0.25, 1.0, -4.0]        # decoded 2, 8, -8 (clamped to R = 8)
    out[1] = [0.0, 0.0, 0.0]
    mv = np.array([[[0, 0], [5, 0], [-20, 1]]])
    assert cnn.labels(out, mv, 8, 2).tolist() == [[1.0, 0.0, 0.0]]


def test_adamw_constant_gradient_closed_form():
    """With a constant gradient the bias-corrected moments are exact at every
    step, so each update is lr_t * (g / (|g| + eps) + wd * w)."""
    rng = np.random.default_rng(5)
    w = rng.normal(size=50)
    g = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    for t in range(1, 6):
        lr = cnn.cosine_lr(t - 1, 10)
        w_prev = w.copy()
        w, m, v = cnn.adamw_step(w, g, m, v, t, lr)
        np.testing.assert_allclose(w, w_prev - lr * (g / (np.abs(g) + 1e-8) + 0.01 * w_prev), rtol=1e-12)


def test_cosine_schedule():
    assert cnn.cosine_lr(0, 100) == pytest.approx(1e-4)
    assert cnn.cosine_lr(100, 100) == pytest.approx(1e-6)
    assert cnn.cosine_lr(50, 100) == pytest.approx((1e-4 + 1e-6) / 2)
    assert cnn.cosine_lr(200, 100) == pytest.approx(1e-6)


def test_pool_input():
    P = np.full((4, 8, 12), 3072, np.uint16)
    x = cnn.pool_input(P, P)
    assert x.shape == (8, 2, 3) and np.all(x == 1.0)
    P2 = np.zeros((4, 4, 8), np.uint16)
    P2[:, 0, 0] = 4095
    P2[2, 3, 7] = 1600
    x2 = cnn.pool_input(P2, P2, cnn.identity)
    assert x2.shape == (8, 1, 2)
    assert x2[0, 0, 0] == pytest.approx((4095 / 16 - 2048) / 1024)
    assert x2[1, 0, 1] == pytest.approx(-2.0)
    assert x2[6, 0, 1] == pytest.approx((1600 / 16 - 2048) / 1024)


def test_pool_input_from_mosaic_by_loops():
    """Each input value is the mean of the 16 mosaic samples of its colour in
    an 8x8 mosaic cell, written as loops over the mosaic itself."""
    import oracle

    rng = np.random.default_rng(3)
    m0 = rng.integers(0, 4096, (16, 24), dtype=np.uint16)
    m1 = rng.integers(0, 4096, (16, 24), dtype=np.uint16)
    x = cnn.pool_input(oracle.pack_planes(m0), oracle.pack_planes(m1), cnn.identity)
    assert x.shape == (8, 2, 3)
    for f, m in enumerate((m0, m1)):
        for c in range(4):
            for y in range(2):
                for xx in range(3):
                    s = 0
                    for r in range(8 * y, 8 * y + 8):
                        for q in range(8 * xx, 8 * xx + 8):
                            if r % 2 == c >> 1 and q % 2 == c & 1:
                                s += int(m[r, q])
                    assert x[4 * f + c, y, xx] == pytest.approx((s / 16 - 2048) / 1024, abs=1e-12)


def test_output_grid_matches_block_grid():
    for Hp, Wp in [(540, 960), (1080, 1920), (360, 640), (240, 320)]:
        h, w = Hp // 4, Wp // 4
        for _, _, s in cnn.LAYERS:
            h, w = cnn.out_size(h, s), cnn.out_size(w, s)
        assert (h, w) == (-(-Hp // 16), -(-Wp // 16))
