"""Every launch shape of the full-search kernel against the oracle: tile
shapes (kx, ky), blocks per workgroup x waves per block, and the current block
read through scalar loads or staged in LDS, on ragged frames (partial blocks
at the right and bottom edges) for block sizes 8, 16 and 32 and radii that
are and are not multiples of 4.  Results must be the oracle's, bit for bit,
whatever the shape."""
import itertools

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


CASES = [(236, 332, 16, 16, 1), (236, 332, 8, 13, 2), (300, 412, 32, 8, 3), (236, 332, 16, 32, 4)]
SHAPES = [(kx, ky, nb, 158, cl, wpb) for kx, ky, (nb, wpb), cl in
          itertools.product((4, 8), (1, 2, 4), ((1, 4), (2, 4), (2, 2), (4, 2), (1, 8)), (0, 1))]


@pytest.mark.parametrize("H,W,B,R,seed", CASES)
def test_every_shape_matches_oracle(dev, oracle_mod, H, W, B, R, seed):
    import torch

    rng = np.random.default_rng(seed)
    f0 = rng.integers(0, 4096, (H, W)).astype(np.uint16)
    f1 = np.clip(np.roll(f0, (2 * (seed % 3) - 2, 4), (0, 1)).astype(np.int32) +
                 rng.integers(-3, 4, (H, W)), 0, 4095).astype(np.uint16)
    mv_o, sad_o, _ = oracle_mod.full_search(f0, f1, B, R)
    d0, d1 = torch.from_numpy(f0).cuda(), torch.from_numpy(f1).cuda()
    ran = 0
    for shape in SHAPES:
        ctx = dev.Context(0)
        try:
            try:
                dev.set_tuned_shape(ctx, B, R, H, W, shape)
            except dev.MeError:
                continue                                  # not compiled or not plannable for this (B, R)
            mv, sad = dev.estimate(d0, d1, B, R, ctx=ctx)
            torch.cuda.synchronize()
            assert np.array_equal(mv.cpu().numpy(), mv_o), shape
            assert np.array_equal(sad.cpu().numpy(), sad_o), shape
            ran += 1
        finally:
            ctx.close()
    assert ran >= 20, ran
