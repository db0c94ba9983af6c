"""Propagation of a key frame's features over a group of pictures (paper
Sec. 4.1 GOP test protocol; Sec. 4.4 compares the reference frames).

Three schedules, every step through the library's kernels (the host only
orders the calls):

* ``key``      -- vectors from the key frame to frame t, ``z_t = Warp(z_0, MV_0t)``;
* ``previous`` -- vectors from frame t-1, warped recursively:
  ``z_t = Warp(z_{t-1}, MV_{t-1,t})``;
* ``composed`` -- vectors from frame t-1 chained back to the key frame
  (``me_compose_vectors``), one warp of the key frame's features:
  ``z_t = Warp(z_0, MV_{t-1,t} o ... o MV_01)``.

With a residual network (``net``, paper Sec. 3.3) every propagated map is
corrected with the current frame before it is used or returned:
``z_t = PRNet(x_t, Warp(...))`` -- the paper's video inference path (key
frame through the base model, then ME, warp and correction per frame).
"""
from __future__ import annotations

import torch

from paper_2508_05990_amd import me

SCHEDULES = ("key", "previous", "composed")


def propagate(ctx, frames, z_key, schedule="previous", block=16, radius=32, stream=None, net=None):
    """frames: device mosaics, frames[0] the key frame; z_key: [C, Hf, Wf]
    float32 or bfloat16 features of the key frame; net: an ``me.Prnet`` whose
    c_feat is C and whose feature grid is [Hf, Wf], or None.  Returns the
    propagated (and corrected) features of frames 1.. and the vectors used
    (to the previous frame for ``previous``, to the key frame otherwise)."""
    if schedule not in SCHEDULES:
        raise ValueError("schedule must be one of %s" % (SCHEDULES,))
    H, W = frames[0].shape
    bh, bw = me.block_grid(H, W, block)
    params = me.make_params(block, radius)
    feats, vecs = [], []
    z_prev, acc = z_key, None
    for t in range(1, len(frames)):
        mv = torch.empty((bh, bw, 2), dtype=torch.int16, device=frames[t].device)
        ref = frames[0] if schedule == "key" else frames[t - 1]
        me.estimate(ref, frames[t], mv=mv, params=params, ctx=ctx, stream=stream)
        if schedule == "composed":
            mv = mv if acc is None else me.compose_vectors(mv, acc, block, H, W, stream=stream)
            acc = mv
        src = z_prev if schedule == "previous" else z_key
        z = me.warp_features(src, mv, block, H, W, ctx=ctx, stream=stream)
        if net is not None:
            z = net.forward(frames[t], z, stream=stream)
        feats.append(z)
        vecs.append(mv)
        z_prev = z
    return feats, vecs
