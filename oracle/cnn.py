"""Float64 oracle of the learned proposal network, its loss and optimiser.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The proposal network is an addition to the paper's method: the
paper's learned part corrects propagated features (PRNet, Sec. 3.3), while
here a small CNN proposes one vector per block that an exact search refines.
What the paper fixes and this reuses:

* the loss family -- reverse Huber (BerHu) on the regression target,
  Sec. 3.3 (PRNet supervision);
* the optimiser -- AdamW, learning rate 1e-4 decayed by a cosine schedule to
  1e-6, batch 16 (Sec. 4.1, training details).

The network itself (a project choice, stated here because the paper is
silent): input = 4x4 mean of each of the four packed planes of reference and
current frame (8 channels, the packed frame pair at a quarter of its
resolution per axis), normalised to (v - 2048) / 1024; four 3x3 convolutions
with zero padding 1, strides 2, 2, 1, 1, channels 8 -> 32 -> 32 -> 32 -> 3,
ReLU after the first three; output per block of 16x16 packed pixels:
(mvx, mvy) in units of 8 packed pixels and a confidence logit.  The reverse
Huber threshold is one output unit (8 packed pixels): absolute error below
it, squared beyond.  Weights and activations are bfloat16
(round to nearest even) and biases are used as given (the float32 master
values); sums are exact here; the gradient of a rounding step is taken as 1.
"""
from __future__ import annotations

import numpy as np

LAYERS = ((8, 32, 2), (32, 32, 2), (32, 32, 1), (32, 3, 1))   # (in channels, out channels, stride)
NPARAMS = sum(co * ci * 9 + co for ci, co, _ in LAYERS)          # 21699
BERHU_C = 1.0


def bf16_round(x):
    """Nearest bfloat16 value (ties to even) of each element, as float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    r = u.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(nan, np.nan, r)


def identity(x):
    return np.asarray(x, dtype=np.float64)


def unpack(flat):
    """Flat parameter vector -> [(W [co, ci, 3, 3], b [co]), ...] in layer order."""
    flat = np.asarray(flat, dtype=np.float64)
    if flat.size != NPARAMS:
        raise ValueError("expected %d parameters" % NPARAMS)
    out, k = [], 0
    for ci, co, _ in LAYERS:
        W = flat[k:k + co * ci * 9].reshape(co, ci, 3, 3)
        k += co * ci * 9
        b = flat[k:k + co]
        k += co
        out.append((W, b))
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def init_params(seed):
    """He-normal weights, zero biases, as float32 values (the master copy)."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co, _ in LAYERS:
        parts.append(rng.normal(0.0, np.sqrt(2.0 / (ci * 9)), co * ci * 9))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


def pool_input(ref_planes, cur_planes, rnd=bf16_round):
    """[8, Hp/4, Wp/4]: 4x4 means of the packed planes of ref (channels 0-3) and
    cur (4-7), normalised to (v - 2048) / 1024, then rounded."""
    out = []
    for P in (ref_planes, cur_planes):
        P = np.asarray(P, dtype=np.float64)
        q = sum(P[:, i::4, j::4] for i in range(4) for j in range(4)) / 16.0
        out.append((q - 2048.0) / 1024.0)
    return rnd(np.concatenate(out, axis=0))


def out_size(n, stride):
    return (n - 1) // stride + 1


def conv3x3(x, W, b, stride):
    """Direct 3x3 convolution, zero padding 1:
    out[o, y, x] = b[o] + sum_{c, ky, kx} W[o, c, ky, kx] * x[c, s*y + ky - 1, s*x + kx - 1]."""
    C, H, Wd = x.shape
    Ho, Wo = out_size(H, stride), out_size(Wd, stride)
    xp = np.zeros((C, H + 2, Wd + 2))
    xp[:, 1:-1, 1:-1] = x
    out = np.zeros((W.shape[0], Ho, Wo)) + np.asarray(b, dtype=np.float64)[:, None, None]
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride]
            out += np.tensordot(W[:, :, ky, kx], patch, axes=(1, 0))
    return out


def conv3x3_abs(x, W, b, stride):
    """Sum of |terms| of conv3x3 (scale of its rounding error)."""
    return conv3x3(np.abs(x), np.abs(W), np.abs(b), stride)


def forward(params, x, rnd=bf16_round):
    """Network forward.  Returns (out [3, bh, bw], acts, pres): acts[l] is the
    input of layer l (rounded), pres[l] its pre-activation output."""
    layers = unpack(params)
    acts, pres = [np.asarray(x, dtype=np.float64)], []
    for l, ((W, b), (_, _, s)) in enumerate(zip(layers, LAYERS)):
        z = conv3x3(acts[-1], rnd(W), b, s)
        pres.append(z)
        if l < len(LAYERS) - 1:
            acts.append(rnd(np.maximum(z, 0.0)))
    return pres[-1], acts, pres


def conv_wgrad(x, d, stride):
    """dW[o, c, ky, kx] = sum_{y, x} d[o, y, x] * x_pad[c, s*y + ky, s*x + kx]."""
    C, H, Wd = x.shape
    _, Ho, Wo = d.shape
    xp = np.zeros((C, H + 2, Wd + 2))
    xp[:, 1:-1, 1:-1] = x
    dW = np.zeros((d.shape[0], C, 3, 3))
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride]
            dW[:, :, ky, kx] = np.tensordot(d, patch, axes=((1, 2), (1, 2)))
    return dW


def conv_dgrad(d, W, stride, in_shape):
    """Gradient of conv3x3's output with respect to its input."""
    C, H, Wd = in_shape
    _, Ho, Wo = d.shape
    dxp = np.zeros((C, H + 2, Wd + 2))
    for ky in range(3):
        for kx in range(3):
            dxp[:, ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride] += \
                np.tensordot(W[:, :, ky, kx], d, axes=(0, 0))
    return dxp[:, 1:-1, 1:-1]


def backward(params, acts, pres, dout, rnd=bf16_round):
    """Gradients of a loss with respect to the flat parameters, given dL/d(out)."""
    layers = unpack(params)
    grads = [None] * len(LAYERS)
    d = np.asarray(dout, dtype=np.float64)
    for l in reversed(range(len(LAYERS))):
        W, _ = layers[l]
        s = LAYERS[l][2]
        grads[l] = (conv_wgrad(acts[l], d, s), d.sum(axis=(1, 2)))
        if l > 0:
            d = conv_dgrad(d, rnd(W), s, acts[l].shape) * (pres[l - 1] > 0)
    return pack(grads)


def berhu(x, c=BERHU_C):
    """Reverse Huber: |x| for |x| <= c, (x^2 + c^2) / (2c) beyond."""
    a = np.abs(x)
    return np.where(a <= c, a, (x * x + c * c) / (2 * c))


def berhu_grad(x, c=BERHU_C):
    return np.where(np.abs(x) <= c, np.sign(x), x / c)


def bce_logits(z, y):
    """Binary cross-entropy of a logit z against a 0/1 label, stable form."""
    return np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z)))


def sigmoid(z):
    return np.where(z >= 0, 1.0 / (1.0 + np.exp(-z)), np.exp(z) / (1.0 + np.exp(z)))


def labels(out, mv_exh, R, refine_radius):
    """1 where the full-search vector lies in the refine window of the decoded
    proposal clamp(rint(8 o), -R, R), else 0 (taken on the given output values)."""
    p = np.clip(np.rint(np.asarray(out[:2], dtype=np.float64) * 8.0), -R, R)
    e = np.maximum(np.abs(p[0] - mv_exh[..., 0]), np.abs(p[1] - mv_exh[..., 1]))
    return (e <= refine_radius).astype(np.float64)


def loss_and_grad(out, mv_exh, R, refine_radius=2, y=None, weight=None):
    """Mean over blocks of w * (BerHu(o_x - t_x) + BerHu(o_y - t_y)), t =
    full-search vector / 8, plus mean BCE of the logit against the
    refine-success label; w = per-block weight of the vector term (default 1).
    Returns (loss, dL/d(out) [3, bh, bw])."""
    out = np.asarray(out, dtype=np.float64)
    mv = np.asarray(mv_exh, dtype=np.float64)
    n = out.shape[1] * out.shape[2]
    w = np.ones(out.shape[1:]) if weight is None else np.asarray(weight, dtype=np.float64)
    if y is None:
        y = labels(out, mv, R, refine_radius)
    ex = out[0] - mv[..., 0] / 8.0
    ey = out[1] - mv[..., 1] / 8.0
    loss = ((w * (berhu(ex) + berhu(ey))).sum() + bce_logits(out[2], y).sum()) / n
    g = np.stack([w * berhu_grad(ex), w * berhu_grad(ey), sigmoid(out[2]) - y]) / n
    return loss, g


def batch_loss_and_grads(params, xs, mvs, R, refine_radius=2, rnd=bf16_round, weights=None):
    """Mean loss over a batch of pairs and the gradient of that mean."""
    tot, g = 0.0, np.zeros(NPARAMS)
    for k, (x, mv) in enumerate(zip(xs, mvs)):
        out, acts, pres = forward(params, x, rnd)
        L, dout = loss_and_grad(out, mv, R, refine_radius, weight=None if weights is None else weights[k])
        tot += L
        g += backward(params, acts, pres, dout, rnd)
    return tot / len(xs), g / len(xs)


def cosine_lr(step, total, lr0=1e-4, lr_min=1e-6):
    """Cosine decay from lr0 at step 0 to lr_min at step `total`."""
    t = min(max(step, 0), total) / float(total)
    return lr_min + 0.5 * (lr0 - lr_min) * (1.0 + np.cos(np.pi * t))


def adamw_step(w, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, wd=0.01):
    """One AdamW update (decoupled weight decay), step count t >= 1.
    Returns (w, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    w = w - lr * (mh / (np.sqrt(vh) + eps) + wd * w)
    return w, m, v
