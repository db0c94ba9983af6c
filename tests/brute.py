"""Brute-force block matching written straight from the definition, on the mosaic.

Pure Python, for tiny frames only.  It never forms colour planes: a block of
``B`` packed pixels is a ``2B x 2B`` patch of the RGGB mosaic and a packed
displacement ``d`` is a mosaic displacement ``2d`` (even offsets keep the
colour phase).  Agreement with the oracle, which works on packed planes, thus
also checks the packed-plane identity.  Selection is Python's tuple order on
``(SAD, dx^2 + dy^2, dy, dx)`` -- the paper's lowest-SAD rule (Sec. 3.2) with
the tie-break taken here (lowest SAD, then smallest squared length, dy, dx).
"""


def brute_stage(ref, cur, B, R, step=1, pred=None, limit=None):
    H, W = len(cur), len(cur[0])
    bh = (H // 2 + B - 1) // B
    bw = (W // 2 + B - 1) // B
    if limit is None:
        limit = R * step if pred is None else 1 << 30
    out = {}
    for bi in range(bh):
        for bj in range(bw):
            Y0, X0 = 2 * B * bi, 2 * B * bj
            Y1, X1 = min(Y0 + 2 * B, H), min(X0 + 2 * B, W)
            px, py = (0, 0) if pred is None else (int(pred[bi][bj][0]), int(pred[bi][bj][1]))
            best = None
            for v in range(-R, R + 1):
                for u in range(-R, R + 1):
                    dx, dy = px + step * u, py + step * v
                    if abs(dx) > limit or abs(dy) > limit:
                        continue
                    if Y0 + 2 * dy < 0 or Y1 + 2 * dy > H or X0 + 2 * dx < 0 or X1 + 2 * dx > W:
                        continue
                    s = 0
                    for y in range(Y0, Y1):
                        rr, cr = ref[y + 2 * dy], cur[y]
                        for x in range(X0, X1):
                            s += abs(int(cr[x]) - int(rr[x + 2 * dx]))
                    key = (s, dx * dx + dy * dy, dy, dx)
                    if best is None or key < best:
                        best = key
            out[(bi, bj)] = None if best is None else (best[3], best[2], best[0])
    return out


def brute_pyramid(ref, cur, blocks, stages, limit):
    """Coarse-to-fine search by hand: for each block size from the largest,
    each (range, step) stage searches around the previous stage's vector; a
    finer level's first stage starts from the vector of the block of the
    previous level that contains it (block index // ratio)."""
    H, W = len(cur), len(cur[0])
    vec = None
    prevB = None
    res = None
    for B in blocks:
        bh = (H // 2 + B - 1) // B
        bw = (W // 2 + B - 1) // B
        if vec is None:
            pred = [[(0, 0) for _ in range(bw)] for _ in range(bh)]
        else:
            r = prevB // B
            pred = [[vec[(bi // r, bj // r)] for bj in range(bw)] for bi in range(bh)]
        for R, step in stages:
            res = brute_stage(ref, cur, B, R, step, pred, limit)
            vec = {k: (v[0], v[1]) if v is not None else (0, 0) for k, v in res.items()}
            pred = [[vec[(bi, bj)] for bj in range(bw)] for bi in range(bh)]
        prevB = B
    return res
