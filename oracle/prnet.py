"""Float64 oracle of the perception residual network (PRNet, paper Sec. 3.3)
on synthetic features: forward, weighted BerHu loss and backward.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What the paper fixes (Sec. 3.3): the network corrects propagated features,
``z_out = z_pred + PRNet(x_C, z_pred)`` with ``z_pred = Warp(z_R, MV)``, and
learns the residual ``z_C - z_pred``.  Its parts, in order: an encoder of
depthwise-separable stride-2 convolutions over the current Bayer frame; the
encoder output concatenated with ``z_pred`` and projected by a 1x1
convolution; a chain of inverted residual blocks (1x1 expansion, depthwise
filtering, 1x1 compression); a 1x1 head predicting the residual.  The loss is
reverse Huber (BerHu) with weights set by region size.

Readings where the paper is silent (a project choice, stated here):

* input: the four packed planes of the current mosaic, ``(v - 2048) / 1024``;
* depthwise-separable block = depthwise 3x3 (zero padding 1, stride s) with
  bias and ReLU6, then 1x1 with bias and ReLU6; two of them with stride 2
  bring the packed planes to the feature grid ``ceil(Hp / 4) x ceil(Wp / 4)``
  (4 packed pixels per feature cell); both output ``c_enc`` channels;
* projection: 1x1 over ``[z_pred, encoder]`` (``c_feat + c_enc`` channels,
  that order) to ``c_hid`` channels, bias, ReLU6;
* inverted residual block (MobileNetV2 form): 1x1 ``c_hid -> expand*c_hid``
  + ReLU6, depthwise 3x3 stride 1 + ReLU6, 1x1 back to ``c_hid`` without
  activation, plus the block's input;
* head: 1x1 ``c_hid -> c_feat`` without activation: the residual ``r``;
* loss: per feature position p, the target residual ``t = z_C - z_pred``;
  p is "incorrectly propagated" when the mean over channels of ``|t|``
  exceeds ``tau``.  Each of the two regions carries half of the loss
  whatever its size (weight ``1 / (2 N_region)`` per position, ``1 / N``
  when one region is empty, plain mean when ``tau < 0``), and the per-element
  term is ``BerHu(r - t) / c_feat`` with the threshold ``c = 0.2 max |r - t|``
  over the batch (the common BerHu choice; ``c`` is held constant in the
  gradient);
* the derivative of ReLU6 is taken from its output: 1 where ``0 < y < 6``;
* precision (what the kernels store): 1x1 weights and activations bfloat16,
  depthwise weights and biases float32, the head output and the loss float32;
  ``rnd`` applies the rounding, ``identity`` turns it off.

Layouts: activations ``[n, H, W, C]``; features ``[n, C, Hf, Wf]``; 1x1
weights ``[c_out, c_in]``; depthwise weights ``[C, 9]`` (tap = 3 ky + kx).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .cnn import bf16_round, identity

__all__ = ["Cfg", "layer_specs", "n_params", "unpack", "init_params", "planes", "dwconv", "pwconv", "relu6",
           "relu6_grad", "dw_backward", "pw_backward", "forward", "loss_and_grad", "backward", "bf16_round",
           "identity"]


@dataclass(frozen=True)
class Cfg:
    c_feat: int = 256
    c_enc: int = 32
    c_hid: int = 64
    expand: int = 4
    n_blocks: int = 2


def layer_specs(cfg: Cfg):
    """Parameterised layers in forward order: (kind, c_in, c_out, stride, act).
    kind "dw" has c_in == c_out; act is "relu6" or None."""
    e, h, x = cfg.c_enc, cfg.c_hid, cfg.c_hid * cfg.expand
    out = [("dw", 4, 4, 2, "relu6"), ("pw", 4, e, 1, "relu6"), ("dw", e, e, 2, "relu6"), ("pw", e, e, 1, "relu6"),
           ("pw", cfg.c_feat + e, h, 1, "relu6")]
    for _ in range(cfg.n_blocks):
        out += [("pw", h, x, 1, "relu6"), ("dw", x, x, 1, "relu6"), ("pw", x, h, 1, None)]
    out.append(("pw", h, cfg.c_feat, 1, None))
    return out


def _sizes(spec):
    kind, ci, co, _, _ = spec
    return (co * 9, co) if kind == "dw" else (co * ci, co)


def n_params(cfg: Cfg) -> int:
    return sum(a + b for a, b in map(_sizes, layer_specs(cfg)))


def unpack(flat, cfg: Cfg):
    """Flat float vector -> [(W, b)] per layer: W [C, 9] (dw) or [c_out, c_in]
    (pw), in the order of ``layer_specs``, each layer's W then b."""
    flat = np.asarray(flat, dtype=np.float64)
    if flat.size != n_params(cfg):
        raise ValueError("expected %d parameters" % n_params(cfg))
    out, k = [], 0
    for spec in layer_specs(cfg):
        nw, nb = _sizes(spec)
        kind, ci, co, _, _ = spec
        W = flat[k:k + nw].reshape((co, 9) if kind == "dw" else (co, ci))
        out.append((W, flat[k + nw:k + nw + nb]))
        k += nw + nb
    return out


def init_params(cfg: Cfg, seed: int, head_scale: float = 1.0):
    """He-normal weights (fan-in 9 for depthwise, c_in for 1x1), biases 0.1 for
    layers followed by ReLU6 and 0 otherwise, as float32 values.  The head's
    weights are multiplied by ``head_scale``."""
    rng = np.random.default_rng(seed)
    specs = layer_specs(cfg)
    parts = []
    for i, (kind, ci, co, _, act) in enumerate(specs):
        fan = 9 if kind == "dw" else ci
        w = rng.normal(0.0, np.sqrt(2.0 / fan), (co * 9) if kind == "dw" else (co * ci))
        if i == len(specs) - 1:
            w = w * head_scale
        parts += [w, np.full(co, 0.1 if act else 0.0)]
    return np.concatenate(parts).astype(np.float32)


def planes(mosaic, rnd=bf16_round):
    """[n, Hp, Wp, 4]: plane c of packed pixel (y, x) = mosaic sample
    (2y + (c >> 1), 2x + (c & 1)) (RGGB packing, Sec. 3.1), normalised."""
    m = np.asarray(mosaic, dtype=np.float64)
    if m.ndim == 2:
        m = m[None]
    p = np.stack([m[:, 0::2, 0::2], m[:, 0::2, 1::2], m[:, 1::2, 0::2], m[:, 1::2, 1::2]], axis=-1)
    return rnd((p - 2048.0) / 1024.0)


def relu6(x):
    return np.clip(x, 0.0, 6.0)


def relu6_grad(y):
    """Derivative of ReLU6 read from its output y."""
    return ((y > 0.0) & (y < 6.0)).astype(np.float64)


def out_size(n, stride):
    return (n - 1) // stride + 1


def dwconv(x, W, b, stride):
    """Depthwise 3x3 convolution, zero padding 1: y[n, i, j, c] = b[c] +
    sum over taps (ky, kx) of W[c, 3 ky + kx] x[n, s i + ky - 1, s j + kx - 1, c]."""
    x = np.asarray(x, dtype=np.float64)
    n, H, Wd, C = x.shape
    Ho, Wo = out_size(H, stride), out_size(Wd, stride)
    xp = np.zeros((n, H + 2, Wd + 2, C))
    xp[:, 1:-1, 1:-1] = x
    y = np.broadcast_to(np.asarray(b, dtype=np.float64), (n, Ho, Wo, C)).copy()
    for ky in range(3):
        for kx in range(3):
            y += W[:, 3 * ky + kx] * xp[:, ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride]
    return y


def pwconv(x, W, b):
    """1x1 convolution: y[..., o] = b[o] + sum_i W[o, i] x[..., i]."""
    return np.asarray(x, dtype=np.float64) @ np.asarray(W, dtype=np.float64).T + b


def dw_backward(x, W, dy, stride):
    """Gradients of ``dwconv`` w.r.t. its input, weights and bias, given the
    gradient dy of its output."""
    x = np.asarray(x, dtype=np.float64)
    dy = np.asarray(dy, dtype=np.float64)
    n, H, Wd, C = x.shape
    Ho, Wo = dy.shape[1:3]
    xp = np.zeros((n, H + 2, Wd + 2, C))
    xp[:, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dW = np.zeros((C, 9))
    for ky in range(3):
        for kx in range(3):
            sl = (slice(None), slice(ky, ky + stride * (Ho - 1) + 1, stride), slice(kx, kx + stride * (Wo - 1) + 1, stride))
            dW[:, 3 * ky + kx] = (dy * xp[sl]).sum(axis=(0, 1, 2))
            dxp[sl] += dy * W[:, 3 * ky + kx]
    return dxp[:, 1:-1, 1:-1], dW, dy.sum(axis=(0, 1, 2))


def pw_backward(x, W, dy):
    """Gradients of ``pwconv``: (dx, dW, db)."""
    x = np.asarray(x, dtype=np.float64)
    dy = np.asarray(dy, dtype=np.float64)
    C = x.shape[-1]
    O = dy.shape[-1]
    return dy @ np.asarray(W, dtype=np.float64), dy.reshape(-1, O).T @ x.reshape(-1, C), dy.reshape(-1, O).sum(axis=0)


def feature_grid(Hp, Wp):
    """Feature grid of a packed frame: two stride-2 layers, ceil(Hp/4) x ceil(Wp/4)."""
    return out_size(out_size(Hp, 2), 2), out_size(out_size(Wp, 2), 2)


def forward(params, cfg: Cfg, mosaic, z_pred, rnd=bf16_round):
    """Returns (acts, r, z_out).  acts: the stored activations, a dict with
    "a0" (input planes), "e1".."e4" (encoder), "xc" (projection input
    [z_pred, e4]), "h" (h0 = projection output, then each block's output),
    "u", "v" (each block's expansion and depthwise outputs); r the head
    output [n, c_feat, Hf, Wf]; z_out = z_pred + r.
    mosaic [n, H, W] (or [H, W]); z_pred [n, c_feat, Hf, Wf] (or without n)."""
    m = np.asarray(mosaic)
    m = m[None] if m.ndim == 2 else m
    z = np.asarray(z_pred, dtype=np.float64)
    z = z[None] if z.ndim == 3 else z
    Hf, Wf = feature_grid(m.shape[1] // 2, m.shape[2] // 2)
    if z.shape != (m.shape[0], cfg.c_feat, Hf, Wf):
        raise ValueError("z_pred must be [%d, %d, %d, %d]" % (m.shape[0], cfg.c_feat, Hf, Wf))
    L = unpack(params, cfg)
    A = {"a0": planes(m, rnd)}
    A["e1"] = rnd(relu6(dwconv(A["a0"], L[0][0], L[0][1], 2)))
    A["e2"] = rnd(relu6(pwconv(A["e1"], rnd(L[1][0]), L[1][1])))
    A["e3"] = rnd(relu6(dwconv(A["e2"], L[2][0], L[2][1], 2)))
    A["e4"] = rnd(relu6(pwconv(A["e3"], rnd(L[3][0]), L[3][1])))
    A["xc"] = np.concatenate([rnd(z.transpose(0, 2, 3, 1)), A["e4"]], axis=-1)
    h = rnd(relu6(pwconv(A["xc"], rnd(L[4][0]), L[4][1])))
    A["h"], A["u"], A["v"] = [h], [], []
    for k in range(cfg.n_blocks):
        (We, be), (Wd, bd), (Wc, bc) = L[5 + 3 * k:8 + 3 * k]
        u = rnd(relu6(pwconv(h, rnd(We), be)))
        v = rnd(relu6(dwconv(u, Wd, bd, 1)))
        h = rnd(pwconv(v, rnd(Wc), bc) + h)
        A["u"].append(u)
        A["v"].append(v)
        A["h"].append(h)
    r = pwconv(h, rnd(L[-1][0]), L[-1][1]).transpose(0, 3, 1, 2)
    return A, r, z + r


def loss_and_grad(r, z_pred, z_target, tau=-1.0, c=None):
    """Weighted BerHu loss of the residual (reading in the module docstring).
    ``c`` overrides the BerHu threshold (default 0.2 max |r - t|).
    Returns (loss, dr, c) with dr = dloss/dr, all float64."""
    r = np.asarray(r, dtype=np.float64)
    t = np.asarray(z_target, dtype=np.float64) - np.asarray(z_pred, dtype=np.float64)
    n, C, Hf, Wf = r.shape
    x = r - t
    if c is None:
        c = 0.2 * np.abs(x).max()
    wpos = np.full((n, Hf, Wf), 1.0 / (n * Hf * Wf))
    if tau >= 0:
        bad = np.abs(t).mean(axis=1) > tau
        nb = int(bad.sum())
        ng = bad.size - nb
        if nb and ng:
            wpos = np.where(bad, 0.5 / nb, 0.5 / ng)
    w = wpos[:, None] / C
    if c == 0.0:
        return 0.0, np.zeros_like(x), c
    a = np.abs(x)
    ber = np.where(a <= c, a, (x * x + c * c) / (2 * c))
    g = np.where(a <= c, np.sign(x), x / c)
    return float((w * ber).sum()), w * g, c


def backward(params, cfg: Cfg, acts, dr, rnd=bf16_round):
    """Gradient of the loss w.r.t. the flat parameter vector, given the stored
    activations of ``forward`` and dr = dloss/dr [n, c_feat, Hf, Wf].  Every
    gradient that reaches a stored activation is rounded as the kernels store
    it (after the ReLU6 derivative of that activation); no gradient flows
    into z_pred or the input planes.  Returns the flat gradient (float64)."""
    L = unpack(params, cfg)
    A = acts
    g = [None] * len(L)
    d = rnd(np.asarray(dr, dtype=np.float64).transpose(0, 2, 3, 1))
    nb = cfg.n_blocks

    def pw(i, x, d, want_dx=True):
        dx, dW, db = pw_backward(x, rnd(L[i][0]), d)
        g[i] = (dW, db)
        return dx

    def dw(i, x, d, s):
        dx, dW, db = dw_backward(x, L[i][0], d, s)
        g[i] = (dW, db)
        return dx

    dh = pw(len(L) - 1, A["h"][-1], d)                  # head: linear, no mask
    for k in range(nb - 1, -1, -1):
        hin = A["h"][k]
        dh_out = rnd(dh) if k == nb - 1 else dh
        dv = rnd(pw(7 + 3 * k, A["v"][k], dh_out) * relu6_grad(A["v"][k]))
        du = rnd(dw(6 + 3 * k, A["u"][k], dv, 1) * relu6_grad(A["u"][k]))
        dh = pw(5 + 3 * k, hin, du) + dh_out           # expansion path + skip
        if k > 0:
            dh = rnd(dh)                                 # block outputs are linear
    dp = rnd(dh * relu6_grad(A["h"][0]))               # h0 = ReLU6(projection)
    dx = pw(4, A["xc"], dp)
    de4 = rnd(dx[..., cfg.c_feat:] * relu6_grad(A["e4"]))
    de3 = rnd(pw(3, A["e3"], de4) * relu6_grad(A["e3"]))
    de2 = rnd(dw(2, A["e2"], de3, 2) * relu6_grad(A["e2"]))
    de1 = rnd(pw(1, A["e1"], de2) * relu6_grad(A["e1"]))
    dw(0, A["a0"], de1, 2)
    return np.concatenate([np.concatenate([np.ravel(W), np.ravel(b)]) for W, b in g])
