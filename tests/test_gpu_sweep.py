"""Seeded randomised parity sweeps through the C ABI against the CPU oracle,
bit for bit: full search over random frame sizes, block sizes and radii
(textured shifted pairs, low-entropy frames full of ties, full 16-bit noise),
and the learned-proposal refine + fallback over random network outputs,
thresholds, refine radii (the small-radius kernel and the predictor path)
and SAD medians; and batched submissions of random job mixes (frame sizes,
block sizes, radii) through the persistent per-block-size queue.  Fixed seeds
and case counts: the same cases every run."""
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


@pytest.fixture(scope="module")
def ctx(dev):
    c = dev.Context(0)
    yield c
    c.close()


def _frames(rng, H, W, R, kind):
    from paper_2508_05990_amd import synth

    if kind == 0:
        f0, f1, _ = synth.shifted_pair(int(rng.integers(0, 1 << 30)), H=H, W=W, max_shift=max(1, min(R, 12)))
        return f0, f1
    hi = 3 if kind == 1 else 65536
    return (rng.integers(0, hi, size=(H, W)).astype(np.uint16), rng.integers(0, hi, size=(H, W)).astype(np.uint16))


@pytest.mark.parametrize("seed", range(6))
def test_full_search_sweep(dev, ctx, oracle_mod, seed):
    import torch

    rng = np.random.default_rng(9000 + seed)
    for case in range(25):
        B = int(rng.choice([8, 16, 32, 64]))
        R = int(rng.choice([0, 1, 2, 3, 4, 5, 7, 8, 12, 16, 17, 24, 31, 32, 33, 40, 48, 64]))
        H, W = 2 * int(rng.integers(4, 200)), 2 * int(rng.integers(4, 260))
        kind = int(rng.integers(0, 3))
        f0, f1 = _frames(rng, H, W, R, kind)
        mv, sad = dev.estimate(torch.from_numpy(f0).cuda(), torch.from_numpy(f1).cuda(), B, R, ctx=ctx)
        torch.cuda.synchronize()
        mv_o, sad_o, _ = oracle_mod.full_search(f0, f1, B, R)
        what = (seed, case, H, W, B, R, kind)
        assert np.array_equal(sad.cpu().numpy(), sad_o), what
        assert np.array_equal(mv.cpu().numpy(), mv_o), what


@pytest.mark.parametrize("seed", range(4))
def test_refine_sweep(dev, ctx, oracle_mod, seed):
    import torch

    rng = np.random.default_rng(9100 + seed)
    for case in range(20):
        B = int(rng.choice([8, 16, 32, 64]))
        R = int(rng.choice([4, 8, 16, 32, 48, 64]))
        rr = int(rng.choice([1, 2, 3, 4, 6]))
        H, W = 2 * int(rng.integers(8, 220)), 2 * int(rng.integers(8, 280))
        f0, f1 = _frames(rng, H, W, R, 0)
        mv_e, _, _ = oracle_mod.full_search(f0, f1, B, R)
        bh, bw = mv_e.shape[:2]
        net = np.empty((3, bh, bw), np.float32)
        good = rng.random((bh, bw)) < 0.6
        for c in range(2):
            near = (mv_e[..., c] + rng.normal(0, 2.0, (bh, bw))) / 8.0
            far = rng.uniform(-R - 8, R + 8, (bh, bw)) / 8.0
            net[c] = np.where(good, near, far)
        net[2] = rng.normal(0.5, 2.0, (bh, bw))
        thr = float(rng.choice([-1e30, 0.0, 0.5]))
        ratio = float(rng.choice([1.0, 1.5, 3.0]))
        M = float(rng.uniform(0.5, 200.0))
        mv, sad, fb = dev.refine(torch.from_numpy(f0).cuda(), torch.from_numpy(f1).cuda(),
                                 torch.from_numpy(net).cuda(), ctx, B, R, rr, thr, ratio, M)
        torch.cuda.synchronize()
        pred = oracle_mod.decode_proposal(net[:2], R)
        mv_o, sad_o, fb_o = oracle_mod.proposal_search(f0, f1, B, R, pred, net[2], thr, ratio, M, refine_radius=rr)
        what = (seed, case, H, W, B, R, rr, thr, ratio, M)
        assert np.array_equal(fb.cpu().numpy(), fb_o), what
        assert np.array_equal(sad.cpu().numpy(), sad_o), what
        assert np.array_equal(mv.cpu().numpy(), mv_o), what


@pytest.mark.parametrize("seed", range(4))
def test_batch_sweep(dev, ctx, oracle_mod, seed):
    """Two submissions per seed of 3-10 random jobs each (partial blocks on
    both edges, radii with and without a shared two-block window); every
    job's vectors and SADs against the oracle's full search."""
    import torch

    rng = np.random.default_rng(9200 + seed)
    for sub in range(2):
        jobs = []
        for _ in range(int(rng.integers(3, 11))):
            B = int(rng.choice([8, 16, 32, 64]))
            R = int(rng.choice([3, 5, 8, 12, 16, 17, 24, 32, 33, 40]))
            H, W = 2 * int(rng.integers(8, 200)), 2 * int(rng.integers(8, 260))
            f0, f1 = _frames(rng, H, W, R, int(rng.integers(0, 3)))
            bh, bw = dev.block_grid(H, W, B)
            jobs.append(dict(f0=f0, f1=f1, B=B, R=R, t0=torch.from_numpy(f0).cuda(), t1=torch.from_numpy(f1).cuda(),
                             mv=torch.full((bh, bw, 2), 77, dtype=torch.int16, device="cuda"),
                             sad=torch.full((bh, bw), -7, dtype=torch.int32, device="cuda")))
        print("batch sweep", seed, sub, [(j["f0"].shape, j["B"], j["R"]) for j in jobs], flush=True)
        dev.batch_submit(ctx, [(j["t0"], j["t1"], j["B"], j["R"], j["mv"], j["sad"]) for j in jobs])
        torch.cuda.synchronize()
        for k, j in enumerate(jobs):
            mv_o, sad_o, _ = oracle_mod.full_search(j["f0"], j["f1"], j["B"], j["R"])
            what = (seed, sub, k, j["f0"].shape, j["B"], j["R"])
            assert np.array_equal(j["sad"].cpu().numpy(), sad_o), what
            assert np.array_equal(j["mv"].cpu().numpy(), mv_o), what
