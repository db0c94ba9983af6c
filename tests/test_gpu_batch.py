"""Batched submission (one persistent, graph-captured work-queue launch per
block size over many jobs of mixed sizes and radii, plus a per-shape launch
for blocks cut by the right frame edge) and the launch-shape autotuner:
results must be bit-identical to one me_estimate per job, and to the oracle."""
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


def _jobs(dev, seed):
    """Mixed jobs: sizes with partial blocks, B in {8,16,32}, R in {3,8,16,32}."""
    import torch

    rng = np.random.default_rng(seed)
    specs = [(96, 160, 8, 16), (120, 200, 16, 8), (200, 300, 32, 3), (64, 64, 8, 32), (150, 246, 16, 16),
             (256, 256, 16, 32), (74, 90, 8, 3)]
    out = []
    for H, W, B, R in specs:
        base = rng.integers(0, 4096, (H + 40, W + 40)).astype(np.uint16)
        dy, dx = (int(v) for v in rng.integers(0, 20, 2))
        f0 = np.ascontiguousarray(base[10:10 + H, 10:10 + W])
        f1 = np.ascontiguousarray(base[dy:dy + H, dx:dx + W])
        bh, bw = dev.block_grid(H, W, B)
        out.append(dict(f0=f0, f1=f1, B=B, R=R, t0=torch.from_numpy(f0).cuda(), t1=torch.from_numpy(f1).cuda(),
                        mv=torch.full((bh, bw, 2), 77, dtype=torch.int16, device="cuda"),
                        sad=torch.full((bh, bw), -7, dtype=torch.int32, device="cuda")))
    return out


def test_batch_matches_single_launches_and_oracle(dev, oracle_mod):
    import torch

    ctx = dev.Context(0)
    try:
        for seed in (0, 1):                  # the second submission replays the captured graph
            jobs = _jobs(dev, seed)
            print("batch submission", seed, flush=True)   # seed 1: same shapes, graph replay
            dev.batch_submit(ctx, [(j["t0"], j["t1"], j["B"], j["R"], j["mv"], j["sad"]) for j in jobs])
            torch.cuda.synchronize()
            for k, j in enumerate(jobs):
                mv1, sad1 = dev.estimate(j["t0"], j["t1"], j["B"], j["R"])
                torch.cuda.synchronize()
                assert torch.equal(j["mv"], mv1) and torch.equal(j["sad"], sad1), k
                if k % 3 == seed:
                    mv_o, sad_o, _ = oracle_mod.full_search(j["f0"], j["f1"], j["B"], j["R"])
                    assert np.array_equal(j["mv"].cpu().numpy(), mv_o) and np.array_equal(j["sad"].cpu().numpy(), sad_o)
    finally:
        ctx.close()


def test_batch_of_one_and_reordering(dev):
    import torch

    ctx = dev.Context(0)
    try:
        jobs = _jobs(dev, 3)
        dev.batch_submit(ctx, [(jobs[5]["t0"], jobs[5]["t1"], 16, 32, jobs[5]["mv"], jobs[5]["sad"])])
        torch.cuda.synchronize()
        mv1, sad1 = dev.estimate(jobs[5]["t0"], jobs[5]["t1"], 16, 32)
        assert torch.equal(jobs[5]["mv"], mv1) and torch.equal(jobs[5]["sad"], sad1)
        rev = list(reversed(jobs))
        dev.batch_submit(ctx, [(j["t0"], j["t1"], j["B"], j["R"], j["mv"], j["sad"]) for j in rev])
        torch.cuda.synchronize()
        for j in rev:
            mv1, sad1 = dev.estimate(j["t0"], j["t1"], j["B"], j["R"])
            assert torch.equal(j["mv"], mv1) and torch.equal(j["sad"], sad1)
        # fewer pairs than the pointer table holds: a new graph without regrowth
        j = jobs[1]
        j["mv"].fill_(5)
        j["sad"].fill_(5)
        dev.batch_submit(ctx, dev.make_jobs([(j["t0"], j["t1"], j["B"], j["R"], j["mv"], j["sad"])]))
        torch.cuda.synchronize()
        mv1, sad1 = dev.estimate(j["t0"], j["t1"], j["B"], j["R"])
        assert torch.equal(j["mv"], mv1) and torch.equal(j["sad"], sad1)
    finally:
        ctx.close()


def test_batch_of_mixed_streams(dev):
    """24 streams of four frame sizes up to 3840x2160 and (B, R) in
    {8, 16} x {16, 32}, one pair each: shape groups of one to several pairs
    with partial blocks; bit-identical to one launch per pair, on two
    submissions (the second replays the graph)."""
    import torch

    from paper_2508_05990_amd import synth

    ctx = dev.Context(0)
    try:
        jobs, singles = [], []
        for B, R, seq in synth.stream_sequences(2, n_frames=2):
            f0, f1 = (torch.from_numpy(f).cuda() for f in seq.frames)
            bh, bw = dev.block_grid(*seq.shape, B)
            mk = lambda: (torch.full((bh, bw, 2), 99, dtype=torch.int16, device="cuda"),
                          torch.full((bh, bw), -9, dtype=torch.int32, device="cuda"))
            jobs.append((f0, f1, B, R) + mk())
            singles.append((f0, f1, B, R) + mk())
        for ref, cur, B, R, mv, sad in singles:
            dev.estimate(ref, cur, B, R, mv=mv, sad=sad, ctx=ctx)
        arr = dev.make_jobs(jobs)
        for rep in range(2):
            for j in jobs:
                j[4].fill_(99)
                j[5].fill_(-9)
            print("mixed-stream submission", rep, flush=True)
            dev.batch_submit(ctx, arr)
            torch.cuda.synchronize()
            for k, (j, s) in enumerate(zip(jobs, singles)):
                assert torch.equal(j[4], s[4]) and torch.equal(j[5], s[5]), (rep, k, j[2], j[3], tuple(j[0].shape))
    finally:
        ctx.close()


def test_autotune_keeps_results(dev, oracle_mod):
    import torch

    from paper_2508_05990_amd import synth

    seq = synth.hd_sequence(1, n_frames=2)
    t0, t1 = (torch.from_numpy(f).cuda() for f in seq.frames)
    ctx = dev.Context(0)
    try:
        mv0, sad0 = dev.estimate(t0, t1, 16, 32, ctx=ctx)
        ms = dev.autotune(ctx, t0, t1, 16, 32, iters=2)
        assert 0 < ms < 10
        mv1, sad1 = dev.estimate(t0, t1, 16, 32, ctx=ctx)
        torch.cuda.synchronize()
        assert torch.equal(mv0, mv1) and torch.equal(sad0, sad1)
    finally:
        ctx.close()


def test_autotune_after_batch_recaptures(dev):
    """A batch graph recorded before the autotuner runs is dropped by it; the
    next submission records the tuned launch shapes and gives the same
    vectors and SADs as before tuning."""
    import torch

    from paper_2508_05990_amd import synth

    ctx = dev.Context(0)
    try:
        jobs = []
        for B, R, seq in list(synth.stream_sequences(3, n_frames=2))[:6]:
            f0, f1 = (torch.from_numpy(f).cuda() for f in seq.frames)
            bh, bw = dev.block_grid(*seq.shape, B)
            jobs.append((f0, f1, B, R, torch.full((bh, bw, 2), 99, dtype=torch.int16, device="cuda"),
                         torch.full((bh, bw), -9, dtype=torch.int32, device="cuda")))
        arr = dev.make_jobs(jobs)
        print("submission before tuning", flush=True)
        dev.batch_submit(ctx, arr)
        torch.cuda.synchronize()
        before = [(j[4].clone(), j[5].clone()) for j in jobs]
        seen = set()
        for f0, f1, B, R, _, _ in jobs:
            if (B, R) + tuple(f0.shape) not in seen:
                seen.add((B, R) + tuple(f0.shape))
                print("autotune", B, R, tuple(f0.shape), flush=True)
                dev.autotune(ctx, f0, f1, B, R, iters=1)
        for j in jobs:
            j[4].fill_(99)
            j[5].fill_(-9)
        print("submission after tuning", flush=True)
        dev.batch_submit(ctx, arr)
        torch.cuda.synchronize()
        for k, (j, (mv, sad)) in enumerate(zip(jobs, before)):
            assert torch.equal(j[4], mv) and torch.equal(j[5], sad), (k, j[2], j[3], tuple(j[0].shape))
    finally:
        ctx.close()


def test_tuned_shape_report_and_restore(dev):
    """tuned_shape reports the default (untuned) and then the autotuner's
    choice; set in a second context it reads back unchanged; other shapes set
    explicitly give the same vectors and SADs; a rejected shape leaves the
    recorded one in place."""
    import torch

    from paper_2508_05990_amd import synth

    seq = synth.hd_sequence(1, n_frames=2)
    H, W = seq.shape
    t0, t1 = (torch.from_numpy(f).cuda() for f in seq.frames)
    ctx, ctx2 = dev.Context(0), dev.Context(0)
    try:
        sh0, tuned0 = dev.tuned_shape(ctx, 16, 32, H, W)
        assert not tuned0 and sh0[:3] == (4, 4, 2) and 0 < sh0[3] <= 80
        mv0, sad0 = dev.estimate(t0, t1, 16, 32, ctx=ctx)
        dev.autotune(ctx, t0, t1, 16, 32, iters=1)
        sh1, tuned1 = dev.tuned_shape(ctx, 16, 32, H, W)
        assert tuned1
        dev.set_tuned_shape(ctx2, 16, 32, H, W, sh1)
        assert dev.tuned_shape(ctx2, 16, 32, H, W) == (sh1, True)
        for shape in [(4, 4, 1, 53), (8, 2, 1, 80), (4, 1, 2, 158), (8, 4, 1, 30), sh1]:
            print("shape", shape, flush=True)
            dev.set_tuned_shape(ctx2, 16, 32, H, W, shape)
            mv, sad = dev.estimate(t0, t1, 16, 32, ctx=ctx2)
            torch.cuda.synchronize()
            assert torch.equal(mv, mv0) and torch.equal(sad, sad0), shape
        with pytest.raises(dev.MeError):
            dev.set_tuned_shape(ctx2, 16, 32, H, W, (3, 4, 1, 80))
        assert dev.tuned_shape(ctx2, 16, 32, H, W) == (sh1, True)
    finally:
        ctx.close()
        ctx2.close()
