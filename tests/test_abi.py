"""The C ABI library loads, exports every entry point include/me.h declares,
and rejects bad arguments before any device work (runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "me.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(me_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def me():
    from paper_2508_05990_amd import me as mod

    return mod


def test_header_declares_core_calls():
    names = _declared()
    for n in ["me_estimate", "me_warp_features", "me_batch_submit", "me_stage_search", "me_ctx_create"]:
        assert n in names


def test_every_declared_symbol_is_exported(me):
    lib = ctypes.CDLL(me.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    assert set(me.EXPORTS) <= set(_declared())


def test_status_strings(me):
    assert me._me_status_string(0) == b"ME_OK"
    assert me._me_status_string(2) == b"ME_E_UNSUPPORTED"


def test_default_params(me):
    p = me.default_params()
    assert (p.block, p.radius, p.step, p.mode, p.refine_radius) == (16, 32, 1, 0, 2)
    assert p.sad_ratio == pytest.approx(1.5)


# Fake but non-null, 4-byte aligned "device" addresses: every case below must
# be rejected by validation, so nothing is ever dereferenced or launched.
FAKE = 0x10000


def _frame(me, h=64, w=64, pitch=None, data=FAKE):
    return me.MeFrame(data, h, w, w if pitch is None else pitch)


def _est(me, ref, cur, params, mv=FAKE, sad=FAKE):
    return me._me_estimate(None, ctypes.byref(ref), ctypes.byref(cur), ctypes.byref(params), mv, sad, None, None)


@pytest.mark.parametrize("case,status", [
    ("null_data", 1), ("odd_height", 1), ("odd_width", 1), ("tiny", 1), ("pitch_small", 1), ("pitch_odd", 1),
    ("misaligned", 1), ("size_mismatch", 1), ("bad_block", 2), ("radius_big", 1), ("radius_neg", 1),
    ("step2", 2), ("bad_mode", 1), ("null_mv", 1), ("proposal_no_ctx", 5), ("huge", 2),
])
def test_estimate_validation(me, case, status):
    ref, cur = _frame(me), _frame(me)
    p = me.make_params(16, 8)
    mv, sad = FAKE, FAKE
    if case == "null_data":
        cur = _frame(me, data=0)
    elif case == "odd_height":
        cur = _frame(me, h=63)
        ref = _frame(me, h=63)
    elif case == "odd_width":
        cur = _frame(me, w=63, pitch=64)
    elif case == "tiny":
        cur = _frame(me, h=0)
    elif case == "pitch_small":
        cur = _frame(me, pitch=32)
    elif case == "pitch_odd":
        cur = _frame(me, pitch=65)
    elif case == "misaligned":
        cur = _frame(me, data=FAKE + 2)
    elif case == "size_mismatch":
        cur = _frame(me, h=32)
    elif case == "bad_block":
        p.block = 12
    elif case == "radius_big":
        p.radius = 65
    elif case == "radius_neg":
        p.radius = -1
    elif case == "step2":
        p.step = 2
    elif case == "bad_mode":
        p.mode = 7
    elif case == "null_mv":
        mv = 0
    elif case == "proposal_no_ctx":
        p.mode = me.ME_MODE_PROPOSAL
    elif case == "huge":
        ref = _frame(me, h=70000, w=64)
        cur = _frame(me, h=70000, w=64)
    assert _est(me, ref, cur, p, mv, sad) == status
    assert len(me._me_last_error()) > 0


@pytest.mark.parametrize("case,status", [
    ("null", 1), ("dtype", 1), ("empty", 1), ("nonsquare", 2), ("cell_not_dividing", 2), ("overlap", 1),
    ("bad_block", 2), ("odd_frame", 1),
])
def test_warp_validation(me, case, status):
    args = dict(z=FAKE, out=FAKE + (1 << 30), dt=0, C=4, Hf=135, Wf=240, mv=FAKE, block=16, fh=1080, fw=1920)
    if case == "null":
        args["z"] = 0
    elif case == "dtype":
        args["dt"] = 5
    elif case == "empty":
        args["C"] = 0
    elif case == "nonsquare":
        args["Wf"] = 480
    elif case == "cell_not_dividing":
        args.update(Hf=45, Wf=80, block=8)       # s = 12 does not divide 8
    elif case == "overlap":
        args["out"] = FAKE + 16
    elif case == "bad_block":
        args["block"] = 24
    elif case == "odd_frame":
        args["fh"] = 1081
    r = me._me_warp_features(None, args["z"], args["out"], args["dt"], args["C"], args["Hf"], args["Wf"], args["mv"],
                             args["block"], args["fh"], args["fw"], None)
    assert r == status


def test_stage_search_validation(me):
    f = _frame(me)
    assert me._me_stage_search(None, ctypes.byref(f), ctypes.byref(f), 16, 2, 1, FAKE, 200, FAKE, FAKE, None) == 1
    assert me._me_stage_search(None, ctypes.byref(f), ctypes.byref(f), 16, 70, 1, None, 8, FAKE, FAKE, None) == 1
    assert me._me_stage_search(None, ctypes.byref(f), ctypes.byref(f), 4, 2, 1, None, 8, FAKE, FAKE, None) == 2
    assert me._me_stage_search(None, ctypes.byref(f), ctypes.byref(f), 16, 2, 0, None, 8, FAKE, FAKE, None) == 1
    # window of 64 + 2 * 8 * 16 words exceeds what the strided kernel stages
    assert me._me_stage_search(None, ctypes.byref(f), ctypes.byref(f), 64, 8, 16, None, 127, FAKE, FAKE, None) == 2


def test_pyramid_defaults_and_validation(me):
    c = me._me_default_pyramid()
    assert (c.n_levels, list(c.block[:2]), c.n_stages) == (2, [32, 16], 3)
    assert [(c.radius[k], c.step[k]) for k in range(3)] == [(8, 8), (4, 4), (2, 1)] and c.limit == 127
    f = _frame(me)
    ctx = ctypes.c_void_p(FAKE)
    assert me._me_pyramid(None, ctypes.byref(f), ctypes.byref(f), ctypes.byref(c), FAKE, FAKE, None) == 1
    assert me._me_pyramid(ctx, ctypes.byref(f), ctypes.byref(f), None, FAKE, FAKE, None) == 1
    bad = me.pyramid_cfg(blocks=(16, 32))          # finer block must divide the coarser one
    assert me._me_pyramid(ctx, ctypes.byref(f), ctypes.byref(f), ctypes.byref(bad), FAKE, FAKE, None) == 1
    bad = me.pyramid_cfg(limit=128)
    assert me._me_pyramid(ctx, ctypes.byref(f), ctypes.byref(f), ctypes.byref(bad), FAKE, FAKE, None) == 1
    bad = me.pyramid_cfg(blocks=(64, 32), stages=((8, 16),))
    assert me._me_pyramid(ctx, ctypes.byref(f), ctypes.byref(f), ctypes.byref(bad), FAKE, FAKE, None) == 2
    bad = me.pyramid_cfg(blocks=(32, 12))
    assert me._me_pyramid(ctx, ctypes.byref(f), ctypes.byref(f), ctypes.byref(bad), FAKE, FAKE, None) == 2


def test_batch_validation(me):
    assert me._me_batch_submit(None, None, 0, None) == 1
    job = me.MeJob()
    job.ref = _frame(me)
    job.cur = _frame(me)
    job.params = me.make_params(16, 8)
    job.mv = 0
    job.sad = FAKE
    arr = (me.MeJob * 1)(job)
    # a fake non-null context pointer is never dereferenced before job validation fails
    assert me._me_batch_submit(ctypes.c_void_p(FAKE), arr, 1, None) == 1


def test_ctx_create_null_out(me):
    assert me._me_ctx_create(0, None) == 1


def test_refine_validation(me):
    f = _frame(me)
    p = me.make_params(16, 8, me.ME_MODE_PROPOSAL)
    args = lambda ctx, net: me._me_refine(ctx, ctypes.byref(f), ctypes.byref(f), ctypes.byref(p), net, FAKE, FAKE,
                                          None, None)
    assert args(None, FAKE) == 1                       # needs a context
    assert args(ctypes.c_void_p(FAKE), 0) == 1         # null network output
    p.refine_radius = 9
    assert args(ctypes.c_void_p(FAKE), FAKE) == 1


def test_refine_noalloc_validation(me):
    """The no-allocation refine checks its fixed scratch limit before it looks
    at the context, so the limit is checked here without a GPU."""
    p = me.make_params(8, 8, me.ME_MODE_PROPOSAL)
    call = lambda ctx, f, net: me._me_refine_noalloc(ctx, ctypes.byref(f), ctypes.byref(f), ctypes.byref(p), net,
                                                     FAKE, FAKE, None, None)
    # 4104 x 4096 Bayer at B=8: 257 x 256 = 65,792 blocks > 65,536
    big = _frame(me, 4104, 4096)
    assert call(None, big, FAKE) == 1
    assert b"exceed" in me._me_last_error()
    # 4096 x 4096: exactly 65,536 blocks passes the limit and stops at the null context
    edge = _frame(me, 4096, 4096)
    assert call(None, edge, FAKE) == 1
    assert b"null context" in me._me_last_error()
    f = _frame(me)
    assert call(ctypes.c_void_p(FAKE), f, 0) == 1      # null network output
    p.refine_radius = 9
    assert call(ctypes.c_void_p(FAKE), f, FAKE) == 1


def test_prnet_num_params_and_validation(me):
    from oracle import prnet as P

    for cfg in [(256, 32, 64, 4, 2), (16, 16, 16, 2, 0), (48, 16, 32, 3, 5)]:
        c = me.MePrnetCfg(*cfg)
        assert me.prnet_num_params(c) == P.n_params(P.Cfg(*cfg)), cfg
    for bad in [(250, 32, 64, 4, 2), (256, 0, 64, 4, 2), (256, 32, 64, 0, 2), (256, 32, 64, 4, -1),
                (1024, 32, 64, 4, 2), (256, 32, 512, 4, 1)]:
        assert me._me_prnet_num_params(ctypes.byref(me.MePrnetCfg(*bad))) == -1, bad
    h = ctypes.c_void_p()
    assert me._me_prnet_create(None, ctypes.byref(me.prnet_cfg()), ctypes.byref(h)) == me.ME_E_INVAL
    fr = _frame(me)
    assert me._me_prnet_forward(None, ctypes.byref(fr), 1, 0, FAKE, FAKE, 0, None) == me.ME_E_INVAL
    assert me._me_prnet_train_step(None, ctypes.byref(fr), 1, 0, FAKE, FAKE, 0.0, 0.0, 0, None, FAKE,
                                   None) == me.ME_E_INVAL
    assert me._me_prnet_dw_forward(None, FAKE, FAKE, FAKE, 1, 8, 8, 4, 1, 1, FAKE, None) == me.ME_E_INVAL
    assert me._me_prnet_dw_backward(None, FAKE, FAKE, FAKE, None, 1, 8, 8, 4, 1, FAKE, FAKE, None) == me.ME_E_INVAL
    t = me.MeTensor(FAKE, 16, 0, 1)
    assert me._me_prnet_pw_forward(None, ctypes.byref(t), None, 1, 64, FAKE, None, 16, 0, None, None,
                                   ctypes.byref(t), None) == me.ME_E_INVAL
    assert me._me_prnet_pw_backward(None, ctypes.byref(t), None, ctypes.byref(t), 1, 64, FAKE, 16, 0, 16, None, None,
                                    FAKE, FAKE, None) == me.ME_E_INVAL
    assert me._me_prnet_loss(None, FAKE, FAKE, FAKE, 1, 16, 4, 4, 0.0, FAKE, FAKE, None) == me.ME_E_INVAL
    assert me.feature_grid(1080, 1920) == (135, 240) and me.feature_grid(22, 10) == (3, 2)


def test_prnet_init_params_layout(me):
    """The binding's starting parameters have the library's size and order:
    depthwise weights of fan-in 9, biases 0.1 before ReLU6 (compared with the
    oracle's layer table)."""
    import numpy as np

    from oracle import prnet as P

    cfg = P.Cfg(48, 16, 32, 3, 2)
    p = me.prnet_init_params(me.MePrnetCfg(48, 16, 32, 3, 2), seed=1)
    assert p.size == P.n_params(cfg) and p.dtype == np.float32
    for (W, b), (kind, ci, co, _, act) in zip(P.unpack(p, cfg), P.layer_specs(cfg)):
        assert np.all(b == (np.float32(0.1) if act else 0.0))
        assert W.shape == ((co, 9) if kind == "dw" else (co, ci))


def test_estimate_warp_validation(me):
    p = me.default_params()
    fr = _frame(me)
    args = lambda prm, z=FAKE, o=FAKE + 0x100000, C=4, Hf=8, Wf=8, dt=0: (
        None, ctypes.byref(fr), ctypes.byref(fr), ctypes.byref(prm), FAKE, FAKE, z, o, dt, C, Hf, Wf, None)
    assert me._me_estimate_warp(*args(p, z=None)) == me.ME_E_INVAL
    assert me._me_estimate_warp(*args(p, dt=7)) == me.ME_E_INVAL
    assert me._me_estimate_warp(*args(p, Hf=7)) == me.ME_E_UNSUPPORTED       # cells do not tile the frame
    assert me._me_estimate_warp(*args(p, o=FAKE + 16)) == me.ME_E_INVAL      # output overlaps the map
    q = me.default_params()
    q.mode = me.ME_MODE_PROPOSAL
    assert me._me_estimate_warp(*args(q)) == me.ME_E_UNSUPPORTED
    q = me.default_params()
    q.block = 12
    assert me._me_estimate_warp(*args(q)) == me.ME_E_UNSUPPORTED


def test_tuned_shape_validation(me):
    fake = ctypes.c_void_p(FAKE)
    out = (ctypes.c_int32 * 6)()
    ok_shape = (ctypes.c_int32 * 6)(4, 4, 2, 80, 0, 4)
    get = lambda ctx, b, r, h, w, o: me._me_tuned_shape(ctx, b, r, h, w, o, None)
    assert get(None, 16, 32, 1080, 1920, ctypes.addressof(out)) == 1      # null context
    assert get(fake, 16, 32, 1080, 1920, None) == 1                       # null shape
    assert get(fake, 12, 32, 1080, 1920, ctypes.addressof(out)) == 2      # block size
    assert get(fake, 16, 65, 1080, 1920, ctypes.addressof(out)) == 1      # radius
    assert get(fake, 16, 32, 1081, 1920, ctypes.addressof(out)) == 1      # odd frame
    put = lambda sh, b=16, r=32: me._me_set_tuned_shape(fake, b, r, 1080, 1920, ctypes.addressof(sh))
    assert me._me_set_tuned_shape(None, 16, 32, 1080, 1920, ctypes.addressof(ok_shape)) == 1
    assert put((ctypes.c_int32 * 6)(3, 4, 2, 80, 0, 4)) == 2                    # tile not compiled
    assert put((ctypes.c_int32 * 6)(4, 4, 3, 80, 0, 4)) == 2                    # three blocks per workgroup
    assert put((ctypes.c_int32 * 6)(4, 4, 2, 80, 0, 4), r=30) == 2              # two blocks need radius % 4 == 0
    assert put((ctypes.c_int32 * 6)(4, 4, 1, 0, 0, 4)) == 2                     # no LDS budget
    assert put((ctypes.c_int32 * 6)(4, 4, 1, 159, 0, 4)) == 2                   # beyond the LDS of a workgroup
    assert put((ctypes.c_int32 * 6)(4, 4, 1, 1, 0, 4)) == 2                     # no band fits 1 KB
    assert put((ctypes.c_int32 * 6)(4, 4, 1, 80, 2, 4)) == 1                    # current-block source not 0/1
    assert put((ctypes.c_int32 * 6)(4, 4, 1, 80, 0, 3)) == 1                    # waves per block not 2, 4 or 8
    assert put((ctypes.c_int32 * 6)(4, 4, 2, 80, 0, 8)) == 2                    # 16 waves per workgroup


def test_stats_validation(me):
    fake_ctx = ctypes.c_void_p(FAKE)
    assert me._me_sad_median(None, FAKE, 1, 16, 1080, 1920, FAKE, None) == 1      # needs a context
    assert me._me_sad_median(fake_ctx, 0, 1, 16, 1080, 1920, FAKE, None) == 1     # null sad
    assert me._me_sad_median(fake_ctx, FAKE, 0, 16, 1080, 1920, FAKE, None) == 1  # no maps
    assert me._me_sad_median(fake_ctx, FAKE, 1, 12, 1080, 1920, FAKE, None) == 2  # block size
    assert me._me_sad_median(fake_ctx, FAKE, 1, 16, 1079, 1920, FAKE, None) == 1  # odd frame
    assert me._me_fallback_weight(FAKE, 1, 16, 1080, 1920, 1.5, 1.0, 0, None) == 1
    assert me._me_fallback_weight(FAKE, 1, 16, 1080, 1920, -1.0, 1.0, FAKE, None) == 1
    assert me._me_fallback_weight(FAKE, 1, 16, 1080, 1920, 1.5, float("nan"), FAKE, None) == 1


@pytest.mark.parametrize("H,W", [(1080, 1920), (2160, 3840), (256, 256), (152, 216), (480, 640), (720, 1280)])
def test_network_grid_is_block_grid(me, H, W):
    """The binding's network output grid on the [H/8, W/8] input equals the
    16x16 block grid and the oracle network's output size."""
    from oracle import cnn

    h, w = H // 8, W // 8
    for _, _, s in cnn.LAYERS:
        h, w = cnn.out_size(h, s), cnn.out_size(w, s)
    assert me._out_grid(H // 8, W // 8) == me.block_grid(H, W, 16) == (h, w)
    assert tuple(s for _, _, s in cnn.LAYERS) == me.CNN_STRIDES
