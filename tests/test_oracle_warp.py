"""Pins of the float64 warp oracle (propagation z_pred = Warp(z_R, MV), paper Sec. 3.3).

Closed forms that bilinear sampling must meet: zero vectors give the input
back, whole-cell vectors give a shifted copy, a constant map stays constant,
an affine map a + b*i + c*j is reproduced at the displaced position away from
the clamped border; plus a scalar per-cell implementation on tiny maps.
"""
import math

import numpy as np
import pytest


def _mv_field(rng, bh, bw, lo, hi):
    return rng.integers(lo, hi + 1, size=(bh, bw, 2)).astype(np.int16)


def test_zero_mv_is_identity(oracle_mod):
    rng = np.random.default_rng(0)
    z = rng.standard_normal((3, 12, 20))
    out, _ = oracle_mod.warp_features(z, np.zeros((3, 5, 2), np.int16), 16, 48, 80)
    assert np.array_equal(out, z)


def test_whole_cell_mv_is_shifted_copy(oracle_mod):
    rng = np.random.default_rng(1)
    s, B = 4, 16
    Hf, Wf = 16, 24
    z = rng.standard_normal((2, Hf, Wf))
    mv = np.zeros((Hf * s // B, Wf * s // B, 2), np.int16)
    mv[..., 0] = 8        # two cells right
    mv[..., 1] = -4       # one cell up
    out, _ = oracle_mod.warp_features(z, mv, B, Hf * s, Wf * s)
    i, j = np.meshgrid(np.arange(Hf), np.arange(Wf), indexing="ij")
    ok = (i - 1 >= 0) & (j + 2 < Wf)
    src = z[:, np.clip(i - 1, 0, Hf - 1), np.clip(j + 2, 0, Wf - 1)]
    assert np.array_equal(out[:, ok], src[:, ok])


def test_constant_map(oracle_mod):
    rng = np.random.default_rng(2)
    z = np.full((2, 10, 15), 3.25)
    mv = _mv_field(rng, 5, 8, -9, 9)
    out, _ = oracle_mod.warp_features(z, mv, 8, 40, 60)      # s = 4, 2 cells per block
    assert np.array_equal(out, z)


@pytest.mark.parametrize("s,B", [(4, 16), (2, 8), (1, 4), (3, 12)])
def test_affine_map_reproduced(oracle_mod, s, B):
    rng = np.random.default_rng(3 + s)
    Hf, Wf = 18, 24
    a, b, c = 0.5, -1.25, 0.75
    i, j = np.meshgrid(np.arange(Hf, dtype=np.float64), np.arange(Wf, dtype=np.float64), indexing="ij")
    z = (a + b * i + c * j)[None]
    bh, bw = math.ceil(Hf * s / B), math.ceil(Wf * s / B)
    mv = _mv_field(rng, bh, bw, -2 * s, 2 * s)
    out, _ = oracle_mod.warp_features(z, mv, B, Hf * s, Wf * s)
    cells = B // s
    dx = mv[(i // cells).astype(int), (j // cells).astype(int), 0] / s
    dy = mv[(i // cells).astype(int), (j // cells).astype(int), 1] / s
    y, x = i + dy, j + dx
    inside = (y >= 0) & (y <= Hf - 1) & (x >= 0) & (x <= Wf - 1)
    expect = a + b * y + c * x
    assert inside.sum() > 0.5 * inside.size
    np.testing.assert_allclose(out[0][inside], expect[inside], rtol=0, atol=1e-12)


def _scalar_warp(z, mv, B, s):
    C, Hf, Wf = z.shape
    out = np.zeros_like(z)
    for ch in range(C):
        for i in range(Hf):
            for j in range(Wf):
                dx, dy = int(mv[(i * s) // B][(j * s) // B][0]), int(mv[(i * s) // B][(j * s) // B][1])
                y = i + dy / s
                x = j + dx / s
                yf, xf = math.floor(y), math.floor(x)
                wy, wx = y - yf, x - xf
                acc = 0.0
                for oy, wyk in ((0, 1 - wy), (1, wy)):
                    for ox, wxk in ((0, 1 - wx), (1, wx)):
                        yy = min(max(yf + oy, 0), Hf - 1)
                        xx = min(max(xf + ox, 0), Wf - 1)
                        acc += wyk * wxk * z[ch, yy, xx]
                out[ch, i, j] = acc
    return out


@pytest.mark.parametrize("s,B", [(4, 16), (2, 4), (1, 2)])
def test_matches_scalar_definition(oracle_mod, s, B):
    rng = np.random.default_rng(11 * s)
    Hf, Wf = 9, 13
    z = rng.standard_normal((2, Hf, Wf))
    bh, bw = math.ceil(Hf * s / B), math.ceil(Wf * s / B)
    mv = _mv_field(rng, bh, bw, -5 * s, 5 * s)
    out, absterm = oracle_mod.warp_features(z, mv, B, Hf * s, Wf * s)
    ref = _scalar_warp(z, mv, B, s)
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-12)
    assert (absterm >= np.abs(out) - 1e-12).all()


def test_rejects_bad_geometry(oracle_mod):
    z = np.zeros((1, 10, 10))
    with pytest.raises(ValueError):
        oracle_mod.warp_features(z, np.zeros((3, 3, 2), np.int16), 16, 40, 48)   # Hp/Hf != Wp/Wf
    with pytest.raises(ValueError):
        oracle_mod.warp_features(z, np.zeros((3, 3, 2), np.int16), 6, 40, 40)    # s=4 does not divide 6


# --- vector composition over a group of pictures ----------------------------

def test_compose_zero_and_identity(oracle_mod):
    z = np.zeros((5, 7, 2), np.int16)
    rng = np.random.default_rng(0)
    acc = rng.integers(-40, 41, (5, 7, 2)).astype(np.int16)
    assert np.array_equal(oracle_mod.compose_vectors(z, acc, 16, 80, 112), acc)     # no motion: carry as is
    assert np.array_equal(oracle_mod.compose_vectors(acc * 0, z, 16, 80, 112), z)


def test_compose_global_translation(oracle_mod):
    """Every frame moves by the same d: the chained vector after t steps is
    t * d for blocks whose chain stays inside the grid."""
    d = np.array([5, -3], np.int16)
    bh, bw, B = 8, 10, 16
    step = np.broadcast_to(d, (bh, bw, 2)).copy()
    acc = step.copy()
    for t in range(2, 5):
        acc = oracle_mod.compose_vectors(step, acc, B, bh * B, bw * B)
        inner = acc[2:-2, 2:-2]
        assert (inner == t * d).all()


def test_compose_matches_hand_loop(oracle_mod):
    """Against a loop written from the reading on random vectors, ragged grid."""
    rng = np.random.default_rng(3)
    B, Hp, Wp = 8, 45, 61
    bh, bw = -(-Hp // B), -(-Wp // B)
    ms = rng.integers(-30, 31, (bh, bw, 2))
    ma = rng.integers(-99, 100, (bh, bw, 2))
    got = oracle_mod.compose_vectors(ms, ma, B, Hp, Wp)
    for bi in range(bh):
        for bj in range(bw):
            h = min(B, Hp - bi * B)
            w = min(B, Wp - bj * B)
            x = bj * B + w // 2 + int(ms[bi, bj, 0])
            y = bi * B + h // 2 + int(ms[bi, bj, 1])
            i = int(np.clip(np.floor(y / B), 0, bh - 1))
            j = int(np.clip(np.floor(x / B), 0, bw - 1))
            assert tuple(got[bi, bj]) == (ms[bi, bj, 0] + ma[i, j, 0], ms[bi, bj, 1] + ma[i, j, 1])
