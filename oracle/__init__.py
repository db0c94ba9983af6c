"""CPU oracle for the Bayer motion-estimation + feature-warp path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the HIP
library (it neither imports nor loads it) and is written from the paper:

* block matching with the SAD criterion -- paper Sec. 2.2 ("Definition",
  "Block Matching-based ME") and Sec. 3.2 ("Matching Criterion");
  implemented in plain C (``me_oracle.c``), called through ctypes;
* propagation of reference features by the motion vectors,
  ``z_pred = Warp(z_R, MV)`` -- paper Sec. 3.3 (perception-residual
  formulation); implemented here in float64 numpy;
* the proposal/refine/fallback decisions of the learned-proposal mode, the
  proposal CNN and its training loss/optimiser (``cnn.py``);
* the perception residual network that corrects propagated features, its
  weighted BerHu loss and its gradients (``prnet.py``, paper Sec. 3.3).

Every function names the passage it follows; the readings taken where the
paper is silent are listed in the module docstrings.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_build", "libme_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile me_oracle.c with gcc into oracle/_build/libme_oracle.so."""
    if os.path.exists(_SO) and not force:
        return _SO
    os.makedirs(os.path.dirname(_SO), exist_ok=True)
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           os.path.join(_HERE, "me_oracle.c"), "-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        L.oracle_pack_planes.argtypes = [P, i32, i32, i64, P]
        L.oracle_pack_planes.restype = None
        L.oracle_stage_search.argtypes = [P, P, i32, i32, i32, i32, i32, P, i32, P, i32, P, P, P, P, i32]
        L.oracle_stage_search.restype = i32
        L.oracle_full_search.argtypes = [P, P, i32, i32, i64, i64, i32, i32, P, i32, P, P, P, i32]
        L.oracle_full_search.restype = i32
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def pack_planes(mosaic: np.ndarray) -> np.ndarray:
    """Packed RGGB planes [4, H/2, W/2] of a uint16 mosaic (step A1)."""
    m = np.ascontiguousarray(mosaic, dtype=np.uint16)
    H, W = m.shape
    if H % 2 or W % 2:
        raise ValueError("mosaic height and width must be even")
    out = np.empty((4, H // 2, W // 2), np.uint16)
    lib().oracle_pack_planes(_ptr(m), H, W, W, _ptr(out))
    return out


def block_grid(Hp: int, Wp: int, B: int):
    return (Hp + B - 1) // B, (Wp + B - 1) // B


def stage_search(ref_planes, cur_planes, B, R, step=1, pred=None, limit=None, blocks=None, nthreads=0):
    """One block-matching stage over packed planes (steps A2 + A3).

    Candidates are ``p + step*(u, v)`` with ``u, v`` in ``[-R, R]``; kept when
    the displaced block is inside the reference frame and both components are
    within ``limit`` (default ``R*step`` around zero for ``pred=None``).
    Returns ``(mv [bh,bw,2] int16 (dx,dy), sad [bh,bw] int32, ops_valid, ops_enum)``.
    Blocks with no valid candidate get ``sad = -1``.
    """
    r = np.ascontiguousarray(ref_planes, dtype=np.uint16)
    c = np.ascontiguousarray(cur_planes, dtype=np.uint16)
    _, Hp, Wp = c.shape
    bh, bw = block_grid(Hp, Wp, B)
    if limit is None:
        limit = R * step if pred is None else (1 << 30)
    pr = None if pred is None else np.ascontiguousarray(pred, dtype=np.int16).reshape(bh, bw, 2)
    bl = None if blocks is None else np.ascontiguousarray(blocks, dtype=np.int32)
    mv = np.zeros((bh, bw, 2), np.int16)
    sad = np.full((bh, bw), -1, np.int32)
    ov = ctypes.c_int64(0)
    oe = ctypes.c_int64(0)
    rc = lib().oracle_stage_search(_ptr(r), _ptr(c), Hp, Wp, B, R, step, _ptr(pr), int(limit),
                                   _ptr(bl), 0 if bl is None else len(bl), _ptr(mv), _ptr(sad),
                                   ctypes.byref(ov), ctypes.byref(oe), nthreads)
    if rc != 0:
        raise ValueError("oracle_stage_search failed: %d" % rc)
    return mv, sad, ov.value, oe.value


def full_search(ref, cur, B, R, blocks=None, nthreads=0):
    """Exhaustive block matching on two uint16 RGGB mosaics (paper Sec. 2.2 full search).

    Returns ``(mv [bh,bw,2] int16 (dx,dy), sad [bh,bw] int32, ops_valid)``.
    With ``blocks`` (row-major block indices) only those blocks are computed;
    the others keep ``sad = -1``.
    """
    r = np.ascontiguousarray(ref, dtype=np.uint16)
    c = np.ascontiguousarray(cur, dtype=np.uint16)
    H, W = c.shape
    if r.shape != c.shape:
        raise ValueError("frame shapes differ")
    bh, bw = block_grid(H // 2, W // 2, B)
    bl = None if blocks is None else np.ascontiguousarray(blocks, dtype=np.int32)
    mv = np.zeros((bh, bw, 2), np.int16)
    sad = np.full((bh, bw), -1, np.int32)
    ov = ctypes.c_int64(0)
    rc = lib().oracle_full_search(_ptr(r), _ptr(c), H, W, W, W, B, R, _ptr(bl),
                                  0 if bl is None else len(bl), _ptr(mv), _ptr(sad), ctypes.byref(ov), nthreads)
    if rc != 0:
        raise ValueError("oracle_full_search failed: %d" % rc)
    return mv, sad, ov.value


# Preset of the paper's FME settings table, "Standard" row: blocks of 64 and
# 32 Bayer pixels (32 and 16 packed pixels), stages (range, step) coarse
# (8, 8), intermediate (4, 4), fine (2, 1).
PYRAMID_BLOCKS = (32, 16)
PYRAMID_STAGES = ((8, 8), (4, 4), (2, 1))


def pyramid_search(ref, cur, blocks=PYRAMID_BLOCKS, stages=PYRAMID_STAGES, limit=127, nthreads=0):
    """Coarse-to-fine block matching over a block pyramid (paper Sec. 3.2,
    "Pyramid Block Structure" and "Parallel Coarse-to-fine Block Matching").

    Levels go from the largest block to the smallest; each level runs the
    stages in order (coarse, intermediate, fine), each stage a stage search
    around the previous stage's vectors.  The first stage of the first level
    starts from zero; the first stage of a finer level starts from the vector
    of the coarser block containing each block.  Every candidate keeps
    |dx|, |dy| <= limit.  Returns ``(mv, sad, ops_valid, ops_enum)`` for the
    finest level; the op counts sum over all levels and stages.
    """
    rp, cp = pack_planes(ref), pack_planes(cur)
    _, Hp, Wp = cp.shape
    mv = None
    prev_B = None
    ops_v = ops_e = 0
    for B in blocks:
        bh, bw = block_grid(Hp, Wp, B)
        if mv is None:
            pred = np.zeros((bh, bw, 2), np.int16)
        else:
            r = prev_B // B
            if r * B != prev_B:
                raise ValueError("each level's block size must divide the previous one's")
            pred = mv[np.arange(bh)[:, None] // r, np.arange(bw)[None, :] // r]
        for R, step in stages:
            mv, sad, ov, oe = stage_search(rp, cp, B, R, step, pred=pred, limit=limit, nthreads=nthreads)
            ops_v += ov
            ops_e += oe
            pred = mv
        prev_B = B
    return mv, sad, ops_v, ops_e


def compose_vectors(mv_step, mv_acc, B, Hp, Wp):
    """Chain block vectors over two frame steps (propagation over a group of
    pictures, paper Sec. 4.1 test protocol and Sec. 4.4): ``mv_step`` maps
    the blocks of frame t to frame t-1, ``mv_acc`` the blocks of frame t-1 to
    the key frame.  Reading: block b of frame t, whose centre is
    ``(x0 + w // 2, y0 + h // 2)``, lands at centre + mv_step[b] in frame t-1;
    the block of frame t-1 containing that point (indices clamped to the
    grid) carries it on to the key frame.  Result: mv_step[b] + mv_acc[b'].
    int16 [bh, bw, 2] (dx, dy)."""
    bh, bw = block_grid(Hp, Wp, B)
    ms = np.asarray(mv_step, dtype=np.int64).reshape(bh, bw, 2)
    ma = np.asarray(mv_acc, dtype=np.int64).reshape(bh, bw, 2)
    out = np.empty((bh, bw, 2), np.int64)
    for bi in range(bh):
        y0 = bi * B
        cy = y0 + min(B, Hp - y0) // 2
        for bj in range(bw):
            x0 = bj * B
            cx = x0 + min(B, Wp - x0) // 2
            px, py = cx + ms[bi, bj, 0], cy + ms[bi, bj, 1]
            pi = min(max(py // B, 0), bh - 1)
            pj = min(max(px // B, 0), bw - 1)
            out[bi, bj] = ms[bi, bj] + ma[pi, pj]
    return out.astype(np.int16)


def warp_features(z_ref, mv, block, Hp, Wp):
    """Bilinear propagation of a reference feature map by block motion vectors.

    Paper Sec. 3.3: ``z_pred = Warp(z_R, MV)``.  The paper does not spell the
    warp out; the reading used here: a feature map ``[C, Hf, Wf]`` covers the
    packed frame with ``s = Hp/Hf = Wp/Wf`` packed pixels per cell (``s``
    divides the block size); cell ``(i, j)`` takes the vector ``(dx, dy)`` of
    the block holding it and samples the reference map at
    ``(i + dy/s, j + dx/s)`` bilinearly, with the two row and two column
    indices clamped into the map.  Arithmetic in float64 on the given values.

    Returns ``(out [C,Hf,Wf] float64, absterm [C,Hf,Wf])`` where ``absterm`` is
    the sum of ``|w_k v_k|`` over the four taps, the scale of the rounding
    error any ordering of the four products can make.
    """
    z = np.asarray(z_ref, dtype=np.float64)
    C, Hf, Wf = z.shape
    if Hp % Hf or Wp % Wf or Hp // Hf != Wp // Wf:
        raise ValueError("feature map must cover the packed frame with square integer cells")
    s = Hp // Hf
    if block % s:
        raise ValueError("cell size must divide the block size")
    cells = block // s
    mv = np.asarray(mv)
    i = np.arange(Hf)[:, None]
    j = np.arange(Wf)[None, :]
    dx = mv[i // cells, j // cells, 0].astype(np.int64)
    dy = mv[i // cells, j // cells, 1].astype(np.int64)
    ny = i * s + dy                      # sample row times s, an integer
    nx = j * s + dx
    y0 = np.floor_divide(ny, s)
    x0 = np.floor_divide(nx, s)
    wy = (ny - y0 * s) / float(s)
    wx = (nx - x0 * s) / float(s)
    y0c = np.clip(y0, 0, Hf - 1)
    y1c = np.clip(y0 + 1, 0, Hf - 1)
    x0c = np.clip(x0, 0, Wf - 1)
    x1c = np.clip(x0 + 1, 0, Wf - 1)
    w00 = (1 - wy) * (1 - wx)
    w01 = (1 - wy) * wx
    w10 = wy * (1 - wx)
    w11 = wy * wx
    v00 = z[:, y0c, x0c]
    v01 = z[:, y0c, x1c]
    v10 = z[:, y1c, x0c]
    v11 = z[:, y1c, x1c]
    out = w00 * v00 + w01 * v01 + w10 * v10 + w11 * v11
    absterm = np.abs(w00 * v00) + np.abs(w01 * v01) + np.abs(w10 * v10) + np.abs(w11 * v11)
    return out, absterm


def sad_threshold(sad_ratio, median_per_sample, n_samples):
    """Fallback SAD threshold ``floor(ratio * M * n)`` evaluated left to right in double."""
    return np.floor(np.float64(np.float32(sad_ratio)) * np.float64(np.float32(median_per_sample))
                    * np.asarray(n_samples, dtype=np.float64)).astype(np.int64)


def block_samples(Hp, Wp, B):
    """Number of samples (4 planes x rows x cols) in every block, [bh, bw]."""
    bh, bw = block_grid(Hp, Wp, B)
    hs = np.minimum(B, Hp - np.arange(bh) * B)
    ws = np.minimum(B, Wp - np.arange(bw) * B)
    return 4 * hs[:, None].astype(np.int64) * ws[None, :]


def median_per_sample(sad_maps, Hp, Wp, B):
    """M of the SAD fallback test from full-search SAD maps ``[n, bh, bw]``:
    the lower median (rank ``floor((N-1)/2)`` of the ascending values) of the
    per-sample SAD ``sad / n_samples`` taken in float32."""
    s = np.asarray(sad_maps).reshape(-1, *block_grid(Hp, Wp, B))
    q = s.astype(np.float32) / block_samples(Hp, Wp, B).astype(np.float32)[None]
    v = np.sort(q.ravel())
    return np.float32(v[(v.size - 1) // 2])


def fallback_weight(sad_maps, Hp, Wp, B, sad_ratio, median):
    """1.0 where a block's full-search SAD is within the SAD fallback
    threshold ``floor(ratio * M * n)``, else 0.0 (float32, shape of the maps)."""
    s = np.asarray(sad_maps).reshape(-1, *block_grid(Hp, Wp, B))
    thr = sad_threshold(sad_ratio, median, block_samples(Hp, Wp, B))
    return (s.astype(np.int64) <= thr[None]).astype(np.float32)


def decode_proposal(out_mv, R):
    """Proposal vector ``clamp(rint(8*o), -R, R)`` from the network's (mvx, mvy)
    output ``[2, bh, bw]`` (units of 8 packed pixels), rounding half to even."""
    o = np.asarray(out_mv)
    p = np.clip(np.rint(o.astype(np.float64) * 8.0), -R, R).astype(np.int16)
    return np.stack([p[0], p[1]], axis=-1)


def proposal_search(ref, cur, B, R, pred, logit, conf_logit_thresh, sad_ratio, median_per_sample,
                    refine_radius=2, nthreads=0):
    """Learned-proposal mode given the network outputs (refine + fallback).

    ``pred`` [bh,bw,2] int16 are decoded proposals, ``logit`` [bh,bw] the
    confidence logits.  Refinement is an exact stage search around the
    proposal (radius ``refine_radius``, step 1, both components within ``R``).
    A block falls back to the exhaustive result when its logit is below the
    threshold, when its refined SAD exceeds ``floor(ratio*M*n)`` or when no
    refinement candidate is valid.  Returns ``(mv, sad, fallback uint8)``.
    """
    rp = pack_planes(ref)
    cp = pack_planes(cur)
    _, Hp, Wp = cp.shape
    mv_r, sad_r, _, _ = stage_search(rp, cp, B, refine_radius, 1, pred=pred, limit=R, nthreads=nthreads)
    thr = sad_threshold(sad_ratio, median_per_sample, block_samples(Hp, Wp, B))
    lg = np.asarray(logit, dtype=np.float32)
    fb = (lg < np.float32(conf_logit_thresh)) | (sad_r < 0) | (sad_r.astype(np.int64) > thr)
    mv = mv_r.copy()
    sad = sad_r.copy()
    idx = np.flatnonzero(fb.ravel()).astype(np.int32)
    if idx.size:
        mv_e, sad_e, _ = full_search(ref, cur, B, R, blocks=idx, nthreads=nthreads)
        mv.reshape(-1, 2)[idx] = mv_e.reshape(-1, 2)[idx]
        sad.ravel()[idx] = sad_e.ravel()[idx]
    return mv, sad, fb.astype(np.uint8)


def mv_error_rate(mv, mv_ref, thresh=1.0):
    """Fraction of blocks whose Euclidean vector error exceeds ``thresh`` packed pixels."""
    d = mv.astype(np.int64) - mv_ref.astype(np.int64)
    return float(np.mean((d[..., 0] ** 2 + d[..., 1] ** 2) > thresh * thresh))
