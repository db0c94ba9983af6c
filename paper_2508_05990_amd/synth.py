"""Seeded synthetic Bayer sequences and feature maps.

This module only makes inputs: it holds none of the motion-estimation or warp
arithmetic, and both the HIP path and the CPU oracle take their inputs from
it.  Every generator draws from ``numpy.random.default_rng(seed)`` (PCG64).

The paper measures on Bayer conversions of CamVid, Cityscapes and ImageNet VID
(paper Sec. 4.1); those datasets and the RGB-to-Bayer model are not available,
so these generators stand in for them with the same structure: 12-bit RGGB
mosaics of natural-image-like (1/f spectrum) texture, rigid objects moving by
integer packed-pixel offsets (so the colour-filter phase is preserved), and
Gaussian sensor noise.

Recipe
------
* texture: white N(0,1) field, amplitude spectrum scaled by ``1/max(f, 1/N)``
  (f = radial frequency in cycles/sample, N = larger side), inverse FFT,
  z-scored, mapped to ``2048 + 512 z`` DN;
* colour planes from a luminance texture L and two chroma textures:
  R = 0.8 L + 0.2 Cr, Gr = Gb = L, B = 0.8 L + 0.2 Cb;
* objects: rectangles with their own textures plus a uniform DN offset,
  moving with integer velocities and reflecting off the frame borders; drawn
  in index order over a static or panning background;
* noise: N(0, sigma^2) per sample, then round half to even, clip to
  [0, 4095], stored as uint16.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

DN_MAX = 4095


def texture_1f(rng: np.random.Generator, h: int, w: int) -> np.ndarray:
    """1/f-spectrum texture in DN (float64, unclipped)."""
    n = rng.standard_normal((h, w))
    F = np.fft.rfft2(n)
    fy = np.fft.fftfreq(h)[:, None]
    fx = np.fft.rfftfreq(w)[None, :]
    f = np.sqrt(fy * fy + fx * fx)
    F *= 1.0 / np.maximum(f, 1.0 / max(h, w))
    t = np.fft.irfft2(F, s=(h, w))
    t = (t - t.mean()) / t.std()
    return 2048.0 + 512.0 * t


def colour_planes(rng: np.random.Generator, h: int, w: int) -> np.ndarray:
    """Four RGGB colour planes [4, h, w] (float DN) from one luminance and two chroma textures."""
    L = texture_1f(rng, h, w)
    cr = texture_1f(rng, h, w)
    cb = texture_1f(rng, h, w)
    return np.stack([0.8 * L + 0.2 * cr, L, L, 0.8 * L + 0.2 * cb])


def interleave(planes: np.ndarray) -> np.ndarray:
    """Sensor-order mosaic [2h, 2w] with R at (0,0), Gr at (0,1), Gb at (1,0), B at (1,1)."""
    _, h, w = planes.shape
    m = np.empty((2 * h, 2 * w), planes.dtype)
    m[0::2, 0::2] = planes[0]
    m[0::2, 1::2] = planes[1]
    m[1::2, 0::2] = planes[2]
    m[1::2, 1::2] = planes[3]
    return m


def quantize(mosaic: np.ndarray, rng: np.random.Generator | None, sigma: float) -> np.ndarray:
    """Add N(0, sigma^2) noise (if rng is given), round half to even, clip to 12 bits."""
    x = mosaic
    if rng is not None and sigma > 0:
        x = x + sigma * rng.standard_normal(mosaic.shape)
    return np.clip(np.rint(x), 0, DN_MAX).astype(np.uint16)


def shifted_pair(seed: int = 0, H: int = 256, W: int = 256, max_shift: int = 6, sigma: float = 2.0):
    """Two frames: frame1 is frame0's content translated by a seeded integer
    offset ``(sx, sy)`` in ``[-max_shift, max_shift]^2`` packed pixels, plus
    noise on frame1 only.  Returns ``(frame0, frame1, (sx, sy))``; a block of
    frame1 whose true source lies inside frame0 has vector ``(-sx, -sy)``."""
    rng = np.random.default_rng(seed)
    sx, sy = (int(v) for v in rng.integers(-max_shift, max_shift + 1, size=2))
    Hp, Wp, m = H // 2, W // 2, max_shift
    scene = colour_planes(rng, Hp + 2 * m, Wp + 2 * m)
    p0 = scene[:, m:m + Hp, m:m + Wp]
    p1 = scene[:, m - sy:m - sy + Hp, m - sx:m - sx + Wp]
    f0 = quantize(interleave(p0), None, 0.0)
    f1 = quantize(interleave(p1), rng, sigma)
    return f0, f1, (sx, sy)


@dataclass
class Sequence:
    frames: list                      # uint16 mosaics [H, W]
    rect_boxes: list = field(default_factory=list)   # per frame: list of (y, x, h, w) in packed pixels
    pan: tuple = (0, 0)               # background displacement per frame (dx, dy), packed pixels
    seed: int = 0

    @property
    def shape(self):
        return self.frames[0].shape


def sequence(seed: int, H: int = 1080, W: int = 1920, n_frames: int = 16, n_rects: int = 8,
             side: tuple = (48, 192), vmax: int = 24, sigma: float = 2.0, pan_max: int = 0,
             offset: float = 600.0) -> Sequence:
    """Textured background (static, or panning with a seeded constant integer
    velocity up to ``pan_max`` per component) plus ``n_rects`` textured rigid
    rectangles with integer velocities in ``[-vmax, vmax]^2`` packed pixels per
    frame, reflecting at the borders; fresh noise on every frame."""
    rng = np.random.default_rng(seed)
    Hp, Wp = H // 2, W // 2
    if pan_max > 0:
        pvx, pvy = (int(v) for v in rng.integers(-pan_max, pan_max + 1, size=2))
    else:
        pvx = pvy = 0
    BH = Hp + abs(pvy) * (n_frames - 1)
    BW = Wp + abs(pvx) * (n_frames - 1)
    bg = colour_planes(rng, BH, BW)
    oy = (n_frames - 1) * max(pvy, 0)
    ox = (n_frames - 1) * max(pvx, 0)

    rects = []
    for _ in range(n_rects):
        h = int(rng.integers(side[0], side[1] + 1))
        w = int(rng.integers(side[0], side[1] + 1))
        h, w = min(h, Hp), min(w, Wp)
        tex = colour_planes(rng, h, w) + rng.uniform(-offset, offset)
        vy, vx = (int(v) for v in rng.integers(-vmax, vmax + 1, size=2))
        y = int(rng.integers(0, Hp - h + 1))
        x = int(rng.integers(0, Wp - w + 1))
        rects.append([y, x, h, w, vy, vx, tex])

    frames, boxes = [], []
    for t in range(n_frames):
        if t > 0:
            for r in rects:
                for k, lim in ((0, Hp - r[2]), (1, Wp - r[3])):
                    p = r[k] + r[4 + k]
                    if p < 0:
                        p, r[4 + k] = -p, -r[4 + k]
                    elif p > lim:
                        p, r[4 + k] = 2 * lim - p, -r[4 + k]
                    r[k] = min(max(p, 0), lim)
        y_off, x_off = oy - t * pvy, ox - t * pvx
        planes = bg[:, y_off:y_off + Hp, x_off:x_off + Wp].copy()
        for (y, x, h, w, _, _, tex) in rects:
            planes[:, y:y + h, x:x + w] = tex
        frames.append(quantize(interleave(planes), rng, sigma))
        boxes.append([(r[0], r[1], r[2], r[3]) for r in rects])
    return Sequence(frames=frames, rect_boxes=boxes, pan=(pvx, pvy), seed=seed)


def features(seed: int, C: int, Hf: int, Wf: int) -> np.ndarray:
    """Reference feature map [C, Hf, Wf], float32 N(0, 1)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((C, Hf, Wf), dtype=np.float32)


# --- named workloads -------------------------------------------------------

def small_pair(seed: int = 0):
    """Bayer 256x256 pair, seeded shift in [-6, 6]^2, noise on frame1 (B=16, R=8)."""
    return shifted_pair(seed, 256, 256, 6, 2.0)


def hd_sequence(seed: int = 1, n_frames: int = 16) -> Sequence:
    """16 frames of 1920x1080 Bayer with 8 moving rectangles (|v| <= 24), B=16, R=32."""
    return sequence(seed, 1080, 1920, n_frames, 8, (48, 192), 24, 2.0)


def uhd_sequence(seed: int = 4, n_frames: int = 60) -> Sequence:
    """3840x2160 Bayer with 32 rectangles (|v| <= 48) and a background pan up to 16 per component."""
    return sequence(seed, 2160, 3840, n_frames, 32, (96, 384), 48, 2.0, pan_max=16)


# Stream groups of the batched workload: (count, Bayer width, Bayer height).
STREAM_GROUPS = ((8, 640, 480), (8, 1280, 720), (6, 1920, 1080), (2, 3840, 2160))
STREAM_BR = ((8, 16), (8, 32), (16, 16), (16, 32))


def stream_specs():
    """(H, W, B, R) for each of the 24 streams of the batched workload."""
    out = []
    for count, w, h in STREAM_GROUPS:
        for k in range(count):
            B, R = STREAM_BR[k % 4]
            out.append((h, w, B, R))
    return out


def stream_sequences(seed: int = 2, n_frames: int = 8):
    """24 independent sequences of mixed sizes; object sizes scale with the
    width, object speed is bounded by 3/4 of the stream's search radius."""
    seqs = []
    for k, (H, W, B, R) in enumerate(stream_specs()):
        f = (W // 2) / 960.0
        lo, hi = max(4, int(round(48 * f))), max(8, int(round(192 * f)))
        seqs.append((B, R, sequence(seed * 1000 + k, H, W, n_frames, 8, (lo, hi), (3 * R) // 4, 2.0)))
    return seqs
