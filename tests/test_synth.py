"""Seeded input generators: determinism, value range, and the structure the
workloads promise (integer motion of rigid objects, 12-bit samples)."""
import hashlib

import numpy as np

from paper_2508_05990_amd import synth


def _h(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_small_pair_deterministic():
    a0, a1, s = synth.small_pair(3)
    b0, b1, t = synth.small_pair(3)
    assert s == t and _h(a0) == _h(b0) and _h(a1) == _h(b1)
    c0, _, _ = synth.small_pair(4)
    assert _h(a0) != _h(c0)
    assert a0.dtype == np.uint16 and a0.shape == (256, 256) and a0.max() <= 4095
    assert all(-6 <= v <= 6 for v in s)


def test_sequence_structure():
    seq = synth.sequence(9, 96, 160, n_frames=5, n_rects=3, side=(8, 20), vmax=4)
    assert len(seq.frames) == 5 and seq.shape == (96, 160)
    for f in seq.frames:
        assert f.dtype == np.uint16 and f.max() <= 4095
    for t in range(1, 5):
        for (y0, x0, h0, w0), (y1, x1, h1, w1) in zip(seq.rect_boxes[t - 1], seq.rect_boxes[t]):
            assert (h0, w0) == (h1, w1)
            assert abs(y1 - y0) <= 4 and abs(x1 - x0) <= 4
            assert 0 <= y1 and y1 + h1 <= 48 and 0 <= x1 and x1 + w1 <= 80
    again = synth.sequence(9, 96, 160, n_frames=5, n_rects=3, side=(8, 20), vmax=4)
    assert all(_h(a) == _h(b) for a, b in zip(seq.frames, again.frames))


def test_pan_moves_background():
    seq = synth.sequence(5, 64, 96, n_frames=3, n_rects=0, vmax=0, sigma=0.0, pan_max=3)
    pvx, pvy = seq.pan
    f0 = seq.frames[0].astype(np.int64)
    f1 = seq.frames[1].astype(np.int64)
    # noise-free: frame1 at p equals frame0 at p - pan (in packed pixels = 2 mosaic pixels)
    H, W = f0.shape
    ys = slice(max(0, 2 * pvy), H + min(0, 2 * pvy))
    xs = slice(max(0, 2 * pvx), W + min(0, 2 * pvx))
    ys0 = slice(ys.start - 2 * pvy, ys.stop - 2 * pvy)
    xs0 = slice(xs.start - 2 * pvx, xs.stop - 2 * pvx)
    assert np.array_equal(f1[ys, xs], f0[ys0, xs0])


def test_stream_specs():
    specs = synth.stream_specs()
    assert len(specs) == 24
    assert sum(1 for s in specs if s[:2] == (2160, 3840)) == 2
    assert {(b, r) for (_, _, b, r) in specs} == {(8, 16), (8, 32), (16, 16), (16, 32)}


def test_features():
    z = synth.features(1, 4, 5, 6)
    assert z.dtype == np.float32 and z.shape == (4, 5, 6)
    assert np.array_equal(z, synth.features(1, 4, 5, 6))
