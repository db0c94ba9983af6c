"""GPU parity of the feature warp against the float64 oracle.

Tolerance per element: |gpu - ref64| <= rtol * sum_k |w_k v_k| (the scale of
the rounding error of a four-term weighted sum), rtol = 1e-6 for float32 and
1e-2 for bfloat16 (whose output rounding alone is up to 2^-8 relative); the
bfloat16 reference takes the same bfloat16 inputs widened to float64."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2508_05990_amd import me

    return me


def _check(dev, oracle_mod, z32, mv, B, H, W, bf16):
    import torch

    zt = torch.from_numpy(z32).cuda()
    if bf16:
        zt = zt.to(torch.bfloat16)
    mvt = torch.from_numpy(mv).cuda()
    out = dev.warp_features(zt, mvt, B, H, W)
    torch.cuda.synchronize()
    zin = zt.float().cpu().numpy().astype(np.float64)
    ref, absterm = oracle_mod.warp_features(zin, mv, B, H // 2, W // 2)
    got = out.float().cpu().numpy().astype(np.float64)
    rtol = 1e-2 if bf16 else 1e-6
    err = np.abs(got - ref)
    bad = err > rtol * absterm
    assert not bad.any(), (np.argwhere(bad)[:5], err[bad][:5], absterm[bad][:5])
    return got, ref


@pytest.mark.parametrize("bf16", [False, True])
def test_hd_feature_map(dev, oracle_mod, bf16):
    """[256, 135, 240] features, 1080p frame, B=16 (s = 4) with vectors up to +-32."""
    from paper_2508_05990_amd import synth

    z = synth.features(11, 256, 135, 240)
    rng = np.random.default_rng(3)
    mv = rng.integers(-32, 33, size=(34, 60, 2)).astype(np.int16)
    _check(dev, oracle_mod, z, mv, 16, 1080, 1920, bf16)


@pytest.mark.parametrize("bf16", [False, True])
@pytest.mark.parametrize("s,B,C,Hf,Wf", [(4, 16, 3, 17, 23), (2, 8, 5, 31, 9), (1, 8, 2, 40, 33), (8, 64, 7, 9, 14),
                                         (16, 32, 2, 5, 7), (8, 8, 3, 11, 13), (4, 16, 2, 6, 2)])
def test_ragged_shapes(dev, oracle_mod, bf16, s, B, C, Hf, Wf):
    rng = np.random.default_rng(s * 100 + C)
    z = rng.standard_normal((C, Hf, Wf)).astype(np.float32)
    H, W = 2 * s * Hf, 2 * s * Wf
    bh, bw = (H // 2 + B - 1) // B, (W // 2 + B - 1) // B
    mv = rng.integers(-3 * s - 2, 3 * s + 3, size=(bh, bw, 2)).astype(np.int16)
    _check(dev, oracle_mod, z, mv, B, H, W, bf16)


@pytest.mark.parametrize("bf16", [False, True])
def test_zero_mv_is_exact_copy(dev, oracle_mod, bf16):
    z = np.random.default_rng(1).standard_normal((4, 20, 30)).astype(np.float32)
    mv = np.zeros((5, 8, 2), np.int16)
    got, ref = _check(dev, oracle_mod, z, mv, 16, 160, 240, bf16)
    assert np.array_equal(got, ref)


def test_whole_cell_mv_is_exact_shift(dev, oracle_mod):
    z = np.random.default_rng(2).standard_normal((3, 20, 32)).astype(np.float32)
    mv = np.zeros((5, 8, 2), np.int16)
    mv[..., 0], mv[..., 1] = -8, 12          # two cells left, three down (s = 4)
    got, ref = _check(dev, oracle_mod, z, mv, 16, 160, 256, False)
    assert np.array_equal(got, ref)

