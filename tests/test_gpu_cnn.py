"""GPU parity of the proposal network against the float64 oracle (oracle/cnn.py).

Each stage is fed oracle-made inputs.  Bounds follow from the arithmetic:
bfloat16 x bfloat16 products are exact in float32, and a float32 sum of N
such terms is within (N-1) * 2^-24 * sum|terms| of the exact sum: at most 288
terms per output of a forward or input-gradient GEMM (bound 2e-5), at most
about 1700 per weight gradient in these tests (bound 1e-4).  A bfloat16 result
adds one rounding, 2^-8 * |value|.  Whole-network checks, where those
roundings feed later layers, compare in aggregate."""
import numpy as np
import pytest

from oracle import cnn

pytestmark = pytest.mark.gpu
U = 2.0 ** -8


@pytest.fixture(scope="module")
def dev():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2508_05990_amd import me

    return me


@pytest.fixture()
def ctx(dev):
    c = dev.Context(0)
    yield c
    c.close()


def _params(seed):
    """He-normal weights with small random biases, float32."""
    p = cnn.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    flat = p.astype(np.float64)
    k = 0
    for ci, co, _ in cnn.LAYERS:
        k += co * ci * 9
        flat[k:k + co] = rng.normal(0, 0.1, co)
        k += co
    return flat.astype(np.float32)


def _bf(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16).cuda()


def _np(t):
    return t.float().cpu().numpy().astype(np.float64)


def _nhwc(a):          # [n, C, H, W] -> [n, H, W, C]
    return np.ascontiguousarray(np.transpose(a, (0, 2, 3, 1)))


def _nchw(a):
    return np.transpose(a, (0, 3, 1, 2))


def test_pool_bit_exact(dev, ctx, oracle_mod):
    import torch

    from paper_2508_05990_amd import synth

    f0, f1, _ = synth.small_pair(3)
    x = dev.cnn_pool(ctx, torch.from_numpy(f0).cuda(), torch.from_numpy(f1).cuda())
    torch.cuda.synchronize()
    ref = cnn.pool_input(oracle_mod.pack_planes(f0), oracle_mod.pack_planes(f1))
    assert np.array_equal(np.transpose(_np(x), (2, 0, 1)), ref)
    # rows not 8-byte aligned (pitch of W + 2 samples; a view starting two samples in,
    # 4-byte aligned as the ABI requires): the per-sample load path gives the same values
    H, W = f0.shape
    for off in (0, 2):
        big0 = np.zeros((H, W + 2), np.uint16)
        big1 = np.zeros((H, W + 2), np.uint16)
        assert off + W <= W + 2
        big0[:, off:off + W], big1[:, off:off + W] = f0, f1
        t0, t1 = torch.from_numpy(big0).cuda(), torch.from_numpy(big1).cuda()
        x = dev.cnn_pool(ctx, t0[:, off:off + W], t1[:, off:off + W])
        torch.cuda.synchronize()
        assert np.array_equal(np.transpose(_np(x), (2, 0, 1)), ref), off


@pytest.mark.parametrize("layer", [0, 1, 2, 3])
def test_layer_forward(dev, ctx, layer):
    import torch

    params = _params(1)
    dev.cnn_set_params(ctx, params, 1.0)
    ci, co, s = cnn.LAYERS[layer]
    n, H, W = 2, 37, 53
    rng = np.random.default_rng(layer)
    x = cnn.bf16_round(rng.normal(0, 1, (n, ci, H, W)))
    if layer > 0:
        x = np.maximum(x, 0)
    Ho, Wo = cnn.out_size(H, s), cnn.out_size(W, s)
    inp = _bf(_nhwc(x))
    if layer < 3:
        out = torch.empty((n, Ho, Wo, co), dtype=torch.bfloat16, device="cuda")
    else:
        out = torch.empty((n, co, Ho, Wo), dtype=torch.float32, device="cuda")
    dev.cnn_layer_forward(ctx, layer, inp, out)
    torch.cuda.synchronize()
    got = _nchw(_np(out)) if layer < 3 else _np(out)
    Wl, bl = cnn.unpack(params)[layer]
    for i in range(n):
        z = cnn.conv3x3(x[i], cnn.bf16_round(Wl), bl, s)
        ab = cnn.conv3x3_abs(x[i], cnn.bf16_round(Wl), bl, s)
        ref = np.maximum(z, 0) if layer < 3 else z
        bound = (U * np.abs(ref) if layer < 3 else 0) + 2e-5 * ab + 1e-30
        assert (np.abs(got[i] - ref) <= bound).all(), np.abs(got[i] - ref).max()


@pytest.mark.parametrize("layer", [0, 1, 2, 3])
def test_layer_backward(dev, ctx, layer):
    import torch

    params = _params(2)
    dev.cnn_set_params(ctx, params, 1.0)
    ci, co, s = cnn.LAYERS[layer]
    coutp = 4 if layer == 3 else co
    n, H, W = 2, 29, 46
    rng = np.random.default_rng(10 + layer)
    x = cnn.bf16_round(np.maximum(rng.normal(0, 1, (n, ci, H, W)), 0) if layer > 0 else rng.normal(0, 1, (n, ci, H, W)))
    Ho, Wo = cnn.out_size(H, s), cnn.out_size(W, s)
    dz = cnn.bf16_round(rng.normal(0, 1e-3, (n, coutp, Ho, Wo)))
    if layer == 3:
        dz[:, 3] = 0.0
    grads = torch.zeros(cnn.NPARAMS, dtype=torch.float32, device="cuda")
    dx = torch.empty((n, H, W, ci), dtype=torch.bfloat16, device="cuda") if layer > 0 else None
    dev.cnn_layer_backward(ctx, layer, _bf(_nhwc(x)), _bf(_nhwc(dz)), dx, grads)
    torch.cuda.synchronize()
    g = grads.cpu().numpy().astype(np.float64)
    Wl, _ = cnn.unpack(params)[layer]
    d = dz[:, :co]
    dW = sum(cnn.conv_wgrad(x[i], d[i], s) for i in range(n))
    dWa = sum(cnn.conv_wgrad(np.abs(x[i]), np.abs(d[i]), s) for i in range(n))
    db = d.sum(axis=(0, 2, 3))
    dba = np.abs(d).sum(axis=(0, 2, 3))
    gl = cnn.unpack(g)[layer]
    assert (np.abs(gl[0] - dW) <= 1e-4 * dWa + 1e-30).all(), np.abs(gl[0] - dW).max()
    assert (np.abs(gl[1] - db) <= 1e-4 * dba + 1e-30).all()
    others = np.ones(cnn.NPARAMS, bool)
    k = sum(c2 * c1 * 9 + c2 for c1, c2, _ in cnn.LAYERS[:layer])
    others[k:k + co * ci * 9 + co] = False
    assert not g[others].any()
    if layer > 0:
        got = _nchw(_np(dx))
        for i in range(n):
            ref = cnn.conv_dgrad(d[i], cnn.bf16_round(Wl), s, x[i].shape) * (x[i] > 0)
            ab = cnn.conv_dgrad(np.abs(d[i]), np.abs(cnn.bf16_round(Wl)), s, x[i].shape)
            assert (np.abs(got[i] - ref) <= U * np.abs(ref) + 2e-5 * ab + 1e-30).all()


@pytest.mark.parametrize("weighted", [False, True])
def test_loss(dev, ctx, weighted):
    import torch

    dev.cnn_set_params(ctx, _params(3), 1.0)
    n, bh, bw, R, rr = 3, 9, 11, 32, 2
    rng = np.random.default_rng(4)
    mv = rng.integers(-R, R + 1, (n, bh, bw, 2)).astype(np.int16)
    out = np.empty((n, 3, bh, bw), np.float32)
    out[:, 0] = (mv[..., 0] + rng.normal(0, 2, (n, bh, bw))) / 8
    out[:, 1] = (mv[..., 1] + rng.normal(0, 2, (n, bh, bw))) / 8
    out[:, 2] = rng.normal(0, 3, (n, bh, bw))
    out[0, 0, 0, :4] = (np.arange(4) + 0.5) / 8         # rounding ties
    dz = torch.empty((n, bh * bw, 4), dtype=torch.bfloat16, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    w = rng.choice(np.array([0.0, 0.5, 1.0, 2.0], np.float32), (n, bh, bw)) if weighted else None
    dev.cnn_loss(ctx, torch.from_numpy(out).cuda(), torch.from_numpy(mv).cuda(), R, rr, dz, loss,
                 weight=None if w is None else torch.from_numpy(w).cuda())
    Ls, Gs = zip(*[cnn.loss_and_grad(out[i].astype(np.float64), mv[i], R, rr, weight=None if w is None else w[i])
                   for i in range(n)])
    assert float(loss.item()) == pytest.approx(np.mean(Ls), rel=1e-5)
    g = np.stack(Gs) / n                                  # gradient of the batch mean
    got = _np(dz).reshape(n, bh, bw, 4)
    for c in range(3):
        assert (np.abs(got[..., c] - g[:, c]) <= U * np.abs(g[:, c]) + 1e-12).all()
    assert not got[..., 3].any()


def test_adamw(dev, ctx):
    import torch

    p0 = _params(5)
    dev.cnn_set_params(ctx, p0, 1.0)
    rng = np.random.default_rng(6)
    w = p0.astype(np.float64)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    lr = 1e-3
    for t in range(1, 4):
        g = rng.normal(0, 1e-2, cnn.NPARAMS).astype(np.float32)
        dev.cnn_adamw(ctx, torch.from_numpy(g).cuda(), lr)
        w, m, v = cnn.adamw_step(w, g.astype(np.float64), m, v, t, lr)
    got, _ = dev.cnn_get_params(ctx)
    assert (np.abs(got - w) <= 1e-6 * np.abs(w) + 3e-3 * lr * 3).all()


def _pair_inputs(dev, ctx, seeds):
    import torch

    import oracle
    from paper_2508_05990_amd import synth

    xs, mvs, xs_o = [], [], []
    for sd in seeds:
        f0, f1, _ = synth.small_pair(sd)
        x = dev.cnn_pool(ctx, torch.from_numpy(f0).cuda(), torch.from_numpy(f1).cuda())
        xs.append(x)
        mv, _, _ = oracle.full_search(f0, f1, 16, 8)
        mvs.append(mv)
        xs_o.append(cnn.pool_input(oracle.pack_planes(f0), oracle.pack_planes(f1)))
    return torch.stack(xs), np.stack(mvs), xs_o


def test_forward_whole_network(dev, ctx):
    import torch

    params = _params(7)
    dev.cnn_set_params(ctx, params, 1.0)
    x, _, xs_o = _pair_inputs(dev, ctx, [0, 1])
    out = dev.cnn_forward(ctx, x)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    for i, xo in enumerate(xs_o):
        ref, _, _ = cnn.forward(params, xo)
        for c in range(3):
            err = np.linalg.norm(got[i, c] - ref[c]) / np.linalg.norm(ref[c])
            assert err < 2e-2, (i, c, err)


@pytest.mark.parametrize("weighted", [False, True])
def test_train_step_gradients(dev, ctx, weighted):
    import torch

    params = _params(8)
    dev.cnn_set_params(ctx, params, 1.0)
    x, mv, xs_o = _pair_inputs(dev, ctx, [2, 3])
    w = np.random.default_rng(5).choice(np.array([0.0, 1.0], np.float32), mv.shape[:3]) if weighted else None
    grads = torch.empty(cnn.NPARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    dev.cnn_train_step(ctx, x, torch.from_numpy(mv).cuda(), radius=8, refine_radius=2, update=False, grads=grads,
                       loss=loss, weight=None if w is None else torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    L, g_ref = cnn.batch_loss_and_grads(params, xs_o, list(mv), 8, 2, weights=w)
    assert float(loss.item()) == pytest.approx(L, rel=2e-2)
    g = grads.cpu().numpy().astype(np.float64)
    for (Wg, bg), (Wr, br) in zip(cnn.unpack(g), cnn.unpack(g_ref)):
        for a, b in ((Wg, Wr), (bg, br)):
            a, b = a.ravel(), b.ravel()
            rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
            cos = a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-30)
            assert rel < 5e-2 and cos > 0.998, (rel, cos)
    after, _ = dev.cnn_get_params(ctx)
    assert np.array_equal(after, params)                  # update=False leaves the weights alone


def test_training_is_deterministic_and_resumable(dev, ctx):
    import torch

    params = _params(9)
    x, mv, _ = _pair_inputs(dev, ctx, [4, 5, 6])
    mv_t = torch.from_numpy(mv).cuda()
    batches = [(x[0:2], mv_t[0:2]), (x[1:3], mv_t[1:3]), (x[0:3:2], mv_t[0:3:2])]

    def run(c, bs):
        for xb, mb in bs:
            dev.cnn_train_step(c, xb.contiguous(), mb.contiguous(), radius=8, lr=1e-3)
        torch.cuda.synchronize()
        return dev.cnn_get_params(c)[0]

    dev.cnn_set_params(ctx, params, 1.0)
    a = run(ctx, batches)
    dev.cnn_set_params(ctx, params, 1.0)
    b = run(ctx, batches)
    assert np.array_equal(a, b) and not np.array_equal(a, params)
    dev.cnn_set_params(ctx, params, 1.0)
    run(ctx, batches[:1])
    blob = dev.cnn_save_state(ctx)
    c2 = dev.Context(0)
    try:
        dev.cnn_load_state(c2, blob)
        r = run(c2, batches[1:])
    finally:
        c2.close()
    assert np.array_equal(r, a)


# Grids the batch-16 1080p training step runs: at 1024 or more 64-pixel tiles
# the forward takes the unsplit kernel (one wave per 16 output pixels), and
# beyond 256 chunks of 64 output pixels each weight-gradient workgroup walks
# several chunks before its partial is reduced.  (layer, n, H, W) below give
# 1148, 1052, 1052 and 1052 forward tiles, and 383, 287, 287 and 287 chunks.
FULL_FWD = [(0, 9, 135, 240), (1, 33, 68, 120), (2, 33, 34, 60), (3, 33, 34, 60)]
FULL_BWD = [(0, 3, 135, 240), (1, 9, 68, 120), (2, 9, 34, 60), (3, 9, 34, 60)]


@pytest.mark.parametrize("layer,n,H,W", FULL_FWD)
def test_layer_forward_full_grid(dev, ctx, layer, n, H, W):
    """Each layer's forward element by element on a grid large enough for the
    unsplit forward kernel, inputs of the 1080p network's shapes."""
    import torch

    params = _params(11)
    dev.cnn_set_params(ctx, params, 1.0)
    ci, co, s = cnn.LAYERS[layer]
    Ho, Wo = cnn.out_size(H, s), cnn.out_size(W, s)
    assert (n * Ho * Wo + 63) // 64 >= 1024
    rng = np.random.default_rng(100 + layer)
    x = cnn.bf16_round(rng.normal(0, 1, (n, ci, H, W)))
    if layer > 0:
        x = np.maximum(x, 0)
    if layer < 3:
        out = torch.empty((n, Ho, Wo, co), dtype=torch.bfloat16, device="cuda")
    else:
        out = torch.empty((n, co, Ho, Wo), dtype=torch.float32, device="cuda")
    print("forward layer %d on %d x %dx%d" % (layer, n, H, W), flush=True)
    dev.cnn_layer_forward(ctx, layer, _bf(_nhwc(x)), out)
    torch.cuda.synchronize()
    got = _nchw(_np(out)) if layer < 3 else _np(out)
    Wl, bl = cnn.unpack(params)[layer]
    Wr = cnn.bf16_round(Wl)
    for i in range(n):
        z = cnn.conv3x3(x[i], Wr, bl, s)
        ab = cnn.conv3x3_abs(x[i], Wr, bl, s)
        ref = np.maximum(z, 0) if layer < 3 else z
        bound = (U * np.abs(ref) if layer < 3 else 0) + 2e-5 * ab + 1e-30
        assert (np.abs(got[i] - ref) <= bound).all(), (i, np.abs(got[i] - ref).max())


@pytest.mark.parametrize("layer,n,H,W", FULL_BWD)
def test_layer_backward_many_chunks(dev, ctx, layer, n, H, W):
    """Weight, bias and input gradients element by element with more than 256
    chunks of output pixels (several per weight-gradient workgroup).  A float32
    sum of the per-chunk products over c chunks per workgroup, then over 256
    workgroups, has at most ~4c + 272 rounding steps: within 1e-4 sum|terms|
    for c up to 5."""
    import torch

    params = _params(12)
    dev.cnn_set_params(ctx, params, 1.0)
    ci, co, s = cnn.LAYERS[layer]
    coutp = 4 if layer == 3 else co
    Ho, Wo = cnn.out_size(H, s), cnn.out_size(W, s)
    assert (n * Ho * Wo + 63) // 64 > 256
    rng = np.random.default_rng(200 + layer)
    x = cnn.bf16_round(np.maximum(rng.normal(0, 1, (n, ci, H, W)), 0) if layer > 0 else rng.normal(0, 1, (n, ci, H, W)))
    dz = cnn.bf16_round(rng.normal(0, 1e-3, (n, coutp, Ho, Wo)))
    if layer == 3:
        dz[:, 3] = 0.0
    grads = torch.zeros(cnn.NPARAMS, dtype=torch.float32, device="cuda")
    dx = torch.empty((n, H, W, ci), dtype=torch.bfloat16, device="cuda") if layer > 0 else None
    print("backward layer %d on %d x %dx%d" % (layer, n, H, W), flush=True)
    dev.cnn_layer_backward(ctx, layer, _bf(_nhwc(x)), _bf(_nhwc(dz)), dx, grads)
    torch.cuda.synchronize()
    g = grads.cpu().numpy().astype(np.float64)
    Wl, _ = cnn.unpack(params)[layer]
    d = dz[:, :co]
    dW = sum(cnn.conv_wgrad(x[i], d[i], s) for i in range(n))
    dWa = sum(cnn.conv_wgrad(np.abs(x[i]), np.abs(d[i]), s) for i in range(n))
    db = d.sum(axis=(0, 2, 3))
    dba = np.abs(d).sum(axis=(0, 2, 3))
    gl = cnn.unpack(g)[layer]
    assert (np.abs(gl[0] - dW) <= 1e-4 * dWa + 1e-30).all(), np.abs(gl[0] - dW).max()
    assert (np.abs(gl[1] - db) <= 1e-4 * dba + 1e-30).all()
    if layer > 0:
        got = _nchw(_np(dx))
        Wr = cnn.bf16_round(Wl)
        for i in range(n):
            ref = cnn.conv_dgrad(d[i], Wr, s, x[i].shape) * (x[i] > 0)
            ab = cnn.conv_dgrad(np.abs(d[i]), np.abs(Wr), s, x[i].shape)
            assert (np.abs(got[i] - ref) <= U * np.abs(ref) + 2e-5 * ab + 1e-30).all(), i


@pytest.mark.parametrize("n,Hq,Wq", [(9, 135, 240), (2, 19, 27), (1, 3, 5), (3, 1, 2)])
def test_fused_forward_each_layer(dev, ctx, n, Hq, Wq):
    """The one-launch forward (me_cnn_forward, the proposal mode's network)
    with its activations stored: each layer element by element against the
    oracle layer fed the kernel's own previous activation, at the bounds of
    test_layer_forward; full tiles, ragged tiles and grids smaller than one
    tile.  At 9 x 135 x 240 layer 0 runs the unsplit layer kernel in the
    layer-by-layer path, and the two paths agree bit for bit there."""
    import torch

    params = _params(13)
    dev.cnn_set_params(ctx, params, 1.0)
    rng = np.random.default_rng(300 + Hq)
    x = cnn.bf16_round(rng.normal(0, 1, (n, 8, Hq, Wq)))
    xt = _bf(_nhwc(x))
    print("fused forward on %d x %dx%d" % (n, Hq, Wq), flush=True)
    out, acts = dev.cnn_forward_acts(ctx, xt)
    plain = dev.cnn_forward(ctx, xt)
    torch.cuda.synchronize()
    assert torch.equal(out, plain)                           # the stores change nothing
    layers = cnn.unpack(params)
    prev = x
    for l in range(4):
        ci, co, s = cnn.LAYERS[l]
        Wl, bl = layers[l]
        Wr = cnn.bf16_round(Wl)
        got = _nchw(_np(acts[l])) if l < 3 else _np(out)
        for i in range(n):
            z = cnn.conv3x3(prev[i], Wr, bl, s)
            ab = cnn.conv3x3_abs(prev[i], Wr, bl, s)
            ref = np.maximum(z, 0) if l < 3 else z
            bound = (U * np.abs(ref) if l < 3 else 0) + 2e-5 * ab + 1e-30
            assert got[i].shape == ref.shape, (l, got[i].shape, ref.shape)
            assert (np.abs(got[i] - ref) <= bound).all(), (l, i, np.abs(got[i] - ref).max())
        prev = got
    if n * ((Hq + 1) // 2) * ((Wq + 1) // 2) >= 1024 * 64:
        a0 = torch.empty_like(acts[0])
        dev.cnn_layer_forward(ctx, 0, xt, a0)
        torch.cuda.synchronize()
        assert torch.equal(a0, acts[0])
