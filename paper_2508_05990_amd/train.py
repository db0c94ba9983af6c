"""Train the proposal network on synthetic 1080p pairs labelled by full search.

Everything numeric runs in the library's HIP kernels: pooling of the network
input, full search for the labels, forward/backward/AdamW training steps and
the evaluation passes.  The host only generates the seeded frames, orders the
batches and follows the cosine learning-rate schedule (paper Sec. 4.1:
AdamW, 1e-4 decayed to 1e-6, batch 16).

    python -m paper_2508_05990_amd.train --pairs 2000 --epochs 100 \\
        --out paper_2508_05990_amd/weights/proposal_1080p.bin

Weights file: header b"MEPW", uint32 version, uint32 parameter count,
float32 median per-sample SAD, and (version 2) float32 logit threshold of the
confidence fallback chosen on validation sequences; then the float32
parameters, little endian.  Version 1 files have no threshold (0: confidence
0.5).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import struct
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "proposal_1080p.bin")
MAGIC = b"MEPW"


def save_weights(path, params, median, threshold=0.0):
    params = np.ascontiguousarray(params, dtype="<f4")
    with open(path + ".tmp", "wb") as f:
        f.write(MAGIC + struct.pack("<IIff", 2, params.size, float(median), float(threshold)))
        f.write(params.tobytes())
    os.replace(path + ".tmp", path)


def load_weights(path):
    """(float32 parameters, median per-sample SAD, logit threshold)."""
    with open(path, "rb") as f:
        head = f.read(16)
        if head[:4] != MAGIC:
            raise ValueError("%s: not a proposal-network weights file" % path)
        version, n, median = struct.unpack("<IIf", head[4:])
        if version == 1:
            threshold = 0.0
        elif version == 2:
            (threshold,) = struct.unpack("<f", f.read(4))
        else:
            raise ValueError("%s: unknown version %d" % (path, version))
        params = np.frombuffer(f.read(4 * n), dtype="<f4").astype(np.float32)
    if params.size != n:
        raise ValueError("%s: truncated" % path)
    return params, median, threshold


def init_params(seed):
    """He-normal weights, zero biases (float32), layer order of the library."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in ((8, 32), (32, 32), (32, 32), (32, 3)):
        parts.append(rng.normal(0.0, math.sqrt(2.0 / (ci * 9)), co * ci * 9))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


def cosine_lr(step, total, lr0, lr_min):
    t = min(max(step, 0), total) / float(max(total, 1))
    return lr_min + 0.5 * (lr0 - lr_min) * (1.0 + math.cos(math.pi * t))


def _make_sequence(spec):
    """Frames of one training sequence: the 1080p generator (8 rectangles,
    |v| <= 24), with a seeded background pan of up to pan_max packed pixels
    per component per frame when pan_max > 0."""
    from paper_2508_05990_amd import synth

    seed, pan_max = spec
    return synth.sequence(seed, 1080, 1920, 16, 8, (48, 192), 24, 2.0, pan_max=pan_max).frames


def sequence_specs(n_seq, seed0, pan_max, pan_every):
    """(seed, pan_max) per training sequence: every pan_every-th sequence pans
    (pan_every = 0: none does)."""
    return [(seed0 + s, pan_max if pan_max > 0 and pan_every > 0 and s % pan_every == 0 else 0)
            for s in range(n_seq)]


def build_dataset(me, ctx, n_pairs, seed0, workers, log, H=1080, W=1920, pan_max=0, pan_every=0):
    """Pooled inputs [n, H/8, W/8, 8] bf16 and full-search labels and SADs
    [n, bh, bw] on the GPU, and the median per-sample SAD (library call)."""
    import torch

    n_seq = (n_pairs + 14) // 15
    bh, bw = me.block_grid(H, W, 16)
    X = torch.empty((n_pairs, H // 8, W // 8, 8), dtype=torch.bfloat16, device="cuda")
    Y = torch.empty((n_pairs, bh, bw, 2), dtype=torch.int16, device="cuda")
    S = torch.empty((n_pairs, bh, bw), dtype=torch.int32, device="cuda")
    k = 0
    t0 = time.time()
    with ProcessPoolExecutor(max_workers=workers, mp_context=__import__("multiprocessing").get_context("spawn")) as ex:
        for si, frames in enumerate(ex.map(_make_sequence, sequence_specs(n_seq, seed0, pan_max, pan_every))):
            dev_frames = [torch.from_numpy(f).cuda() for f in frames]
            assert dev_frames[0].shape == (H, W)
            for t in range(1, len(dev_frames)):
                if k >= n_pairs:
                    break
                me.cnn_pool(ctx, dev_frames[t - 1], dev_frames[t], x=X[k])
                me.estimate(dev_frames[t - 1], dev_frames[t], 16, 32, mv=Y[k], sad=S[k], ctx=ctx)
                k += 1
            torch.cuda.synchronize()
            if si % 20 == 0:
                log({"event": "data", "sequences": si + 1, "pairs": k, "seconds": round(time.time() - t0, 1)})
    median = float(me.sad_median(ctx, S, 16, H, W).item())
    return X, Y, S, median


def exhaustive_vectors(me, ctx, frames, R):
    """Full-search vectors of consecutive pairs (the reference of the MV error)."""
    return [me.estimate(frames[t - 1], frames[t], 16, R, ctx=ctx)[0] for t in range(1, len(frames))]


def evaluate(me, ctx, frames, mv_exh, use_net, median, R=32, rr=2, conf=0.0):
    """Proposal mode on consecutive pairs: fallback rate, MV-error rate against
    full search (Euclidean error > 1 packed pixel) and median time per pair.
    conf: logit threshold of the confidence fallback (0 = confidence 0.5)."""
    import torch

    fb_sum = err_sum = n = 0
    bh, bw = me.block_grid(frames[0].shape[0], frames[0].shape[1], 16)
    net_zero = torch.zeros((3, bh, bw), dtype=torch.float32, device="cuda")
    p = me.make_params(16, R, me.ME_MODE_PROPOSAL, rr, conf, 1.5, median)
    fb = torch.empty((bh, bw), dtype=torch.uint8, device="cuda")
    times = []
    for t in range(1, len(frames)):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        if use_net:
            mv, sad = me.estimate(frames[t - 1], frames[t], fallback=fb, params=p, ctx=ctx)
        else:
            # a zero logit carries no confidence: zero proposals take the SAD fallback only
            mv, sad, fb = me.refine(frames[t - 1], frames[t], net_zero, ctx, 16, R, rr, -1e30, 1.5, median,
                                    fallback=fb)
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
        d = (mv.int() - mv_exh[t - 1].int()).float()
        err_sum += int(((d[..., 0] ** 2 + d[..., 1] ** 2) > 1.0).sum().item())
        fb_sum += int(fb.sum().item())
        n += bh * bw
    return {"fallback_rate": fb_sum / n, "mv_err_rate": err_sum / n, "ms_per_pair": float(np.median(times))}


# logit thresholds tried on the validation sequences (-1e30: SAD fallback only)
THRESHOLDS = (-1e30, -8.0, -6.0, -4.0, -3.0, -2.0, -1.0, 0.0, 1.0, 2.0)


def validation_sets(seed, n_frames=8, uhd_frames=4):
    """Sequences for choosing the confidence threshold, disjoint from the
    training seeds (1000 up) and from the held-out evaluation (1080p seed 1,
    4K seed 4): a 1080p sequence with a static background, a 1080p sequence
    with a background pan, and (uhd_frames > 1) a panning 4K sequence.
    Returns (name, frames, radius) with frames as host arrays."""
    from paper_2508_05990_amd import synth

    sets = [("hd_static", synth.hd_sequence(seed, n_frames=n_frames).frames, 32),
            ("hd_pan", synth.sequence(seed + 1, 1080, 1920, n_frames, 8, (48, 192), 24, 2.0, pan_max=16).frames, 32)]
    if uhd_frames > 1:
        sets.append(("uhd_pan", synth.uhd_sequence(seed + 2, n_frames=uhd_frames).frames, 64))
    return sets


def select_threshold(me, ctx, sets, median, rr, max_err, log):
    """The logit threshold with the fewest fallbacks over all validation
    sequences among those that keep every sequence's MV-error rate at or
    below max_err (ties: the higher, more cautious threshold)."""
    import torch

    dev_sets = []
    for name, frames, R in sets:
        fr = [torch.from_numpy(f).cuda() for f in frames]
        dev_sets.append((name, fr, exhaustive_vectors(me, ctx, fr, R), R))
    best = None
    table = []
    for thr in THRESHOLDS:
        per = {name: evaluate(me, ctx, fr, mv_exh, True, median, R=R, rr=rr, conf=thr)
               for name, fr, mv_exh, R in dev_sets}
        fall = float(np.mean([r["fallback_rate"] for r in per.values()]))
        ok = all(r["mv_err_rate"] <= max_err for r in per.values())
        table.append({"threshold": thr, "mean_fallback_rate": fall, "ok": ok,
                      **{k: {"fallback_rate": v["fallback_rate"], "mv_err_rate": v["mv_err_rate"]}
                         for k, v in per.items()}})
        if ok and (best is None or fall <= best[1]):
            best = (thr, fall)
    log({"event": "threshold_sweep", "max_err": max_err, "table": table})
    return (0.0 if best is None else best[0]), table


def evaluate_all(me, ctx, median, threshold, rr, eval_seed, uhd_frames, log):
    """Held-out 1080p sequence (R=32) and, if uhd_frames > 1, the first frames
    of the 4K sequence with a background pan (R=64): the trained network with
    the chosen threshold, with the SAD fallback only, and zero proposals."""
    import torch

    from paper_2508_05990_amd import synth

    out = {}
    cases = [("hd", synth.hd_sequence(eval_seed), 32)]
    if uhd_frames > 1:
        cases.append(("uhd", synth.uhd_sequence(4, n_frames=uhd_frames), 64))
    for name, seq, R in cases:
        frames = [torch.from_numpy(f).cuda() for f in seq.frames]
        mv_exh = exhaustive_vectors(me, ctx, frames, R)
        out[name] = {"trained": evaluate(me, ctx, frames, mv_exh, True, median, R=R, rr=rr, conf=threshold),
                     "trained_sad_fallback_only": evaluate(me, ctx, frames, mv_exh, True, median, R=R, rr=rr,
                                                           conf=-1e30),
                     "zero_predictor": evaluate(me, ctx, frames, mv_exh, False, median, R=R, rr=rr)}
        log({"event": "eval", "sequence": name, "threshold": threshold, **out[name]})
        del frames
    return out


def fit(me, ctx, X, Y, Wt, median, epochs, batch, lr0, lr_min, seed, init_seed, refine_radius, log):
    """AdamW with a cosine learning rate over `epochs` passes of shuffled
    batches (the library's training step); returns the float32 parameters."""
    import torch

    me.cnn_set_params(ctx, init_params(init_seed), median)
    n = X.shape[0]
    steps_per_epoch = n // batch
    total = steps_per_epoch * epochs
    rng = np.random.default_rng(seed)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    xb = torch.empty((batch,) + tuple(X.shape[1:]), dtype=X.dtype, device="cuda")
    yb = torch.empty((batch,) + tuple(Y.shape[1:]), dtype=Y.dtype, device="cuda")
    wb = None if Wt is None else torch.empty((batch,) + tuple(Wt.shape[1:]), dtype=Wt.dtype, device="cuda")
    step = 0
    lr = lr0
    t0 = time.time()
    for ep in range(epochs):
        order = torch.from_numpy(rng.permutation(n)).cuda()
        for s in range(steps_per_epoch):
            idx = order[s * batch:(s + 1) * batch]
            torch.index_select(X, 0, idx, out=xb)
            torch.index_select(Y, 0, idx, out=yb)
            if wb is not None:
                torch.index_select(Wt, 0, idx, out=wb)
            lr = cosine_lr(step, total, lr0, lr_min)
            me.cnn_train_step(ctx, xb, yb, radius=32, refine_radius=refine_radius, lr=lr, update=True,
                              loss=loss if s == steps_per_epoch - 1 else None, weight=wb)
            step += 1
        if ep % max(1, epochs // 20) == 0 or ep == epochs - 1:
            log({"event": "epoch", "epoch": ep, "step": step, "lr": lr, "loss": float(loss.item()),
                 "seconds": round(time.time() - t0, 1)})
    torch.cuda.synchronize()
    params, _ = me.cnn_get_params(ctx)
    return params, total, time.time() - t0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--pairs", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=100)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-4)
    ap.add_argument("--lr-min", type=float, default=1e-6)
    ap.add_argument("--seed", type=int, default=1000, help="first sequence seed of the training set")
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--eval-seed", type=int, default=1, help="held-out 1080p sequence")
    ap.add_argument("--eval-uhd-frames", type=int, default=0, help="also evaluate on this many 4K frames (0 = no)")
    ap.add_argument("--val-seed", type=int, default=500,
                    help="first seed of the validation sequences that choose the confidence threshold")
    ap.add_argument("--val-uhd-frames", type=int, default=4, help="frames of the 4K validation sequence (0 = none)")
    ap.add_argument("--max-err", type=float, default=0.02,
                    help="largest MV-error rate a validation sequence may show at the chosen threshold")
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--pan-max", type=int, default=0,
                    help="background pan of up to this many packed pixels per frame in some training sequences")
    ap.add_argument("--pan-every", type=int, default=2, help="every n-th training sequence pans (with --pan-max)")
    ap.add_argument("--refine-radius", type=int, default=2, help="refine window of the confidence labels")
    ap.add_argument("--mask-ratio", type=float, default=1.5,
                    help="drop the vector term of blocks whose full-search SAD per sample exceeds this multiple "
                         "of the median (0 = keep all)")
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--log", default=None, help="JSON-lines log file")
    args = ap.parse_args(argv)

    logf = open(args.log, "a") if args.log else None

    def log(rec):
        line = json.dumps(rec)
        print(line, flush=True)
        if logf:
            logf.write(line + "\n")
            logf.flush()

    from paper_2508_05990_amd import me

    ctx = me.Context(0)
    t_all = time.time()
    X, Y, S, median = build_dataset(me, ctx, args.pairs, args.seed, args.workers, log, pan_max=args.pan_max,
                                    pan_every=args.pan_every)
    # vector-term weight: blocks whose full-search match is worse than the
    # fallback threshold always fall back, so their vectors (occlusions,
    # new content) are left out of the regression
    Wt = None
    if args.mask_ratio > 0:
        Wt = me.fallback_weight(S, 16, X.shape[1] * 8, X.shape[2] * 8, args.mask_ratio, median)
    log({"event": "dataset", "pairs": args.pairs, "median_sad_per_sample": median, "pan_max": args.pan_max,
         "pan_every": args.pan_every,
         "vector_weight_mean": None if Wt is None else float(Wt.mean().item())})
    params, total, train_s = fit(me, ctx, X, Y, Wt, median, args.epochs, args.batch, args.lr, args.lr_min, args.seed,
                                 args.init_seed, args.refine_radius, log)
    del X, Y, S, Wt
    thr, _ = select_threshold(me, ctx, validation_sets(args.val_seed, uhd_frames=args.val_uhd_frames), median,
                              args.refine_radius, args.max_err, log)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    save_weights(args.out, params, median, thr)
    res = evaluate_all(me, ctx, median, thr, args.refine_radius, args.eval_seed, args.eval_uhd_frames, log)
    log({"event": "done", "train_seconds": round(train_s, 1), "total_seconds": round(time.time() - t_all, 1),
         "steps": total, "weights": args.out, "refine_radius": args.refine_radius, "threshold": thr,
         "heldout": res})
    ctx.close()
    return res


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
