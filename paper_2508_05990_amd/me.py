"""ctypes binding of the HIP library (include/me.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch supplies device memory and streams.  Importing this module
raises if the library has not been built -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libme.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("HIP library not built: %s (run paper_2508_05990_amd/build.py or __graft_entry__.build())"
                      % LIB_PATH)

_lib = ctypes.CDLL(LIB_PATH)

ME_OK, ME_E_INVAL, ME_E_UNSUPPORTED, ME_E_HIP, ME_E_NOMEM, ME_E_STATE = range(6)
ME_MODE_EXHAUSTIVE, ME_MODE_PROPOSAL = 0, 1
ME_F32, ME_BF16 = 0, 1


class MeFrame(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("pitch", ctypes.c_int64)]


class MeParams(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("radius", ctypes.c_int32), ("step", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("refine_radius", ctypes.c_int32),
                ("conf_logit_thresh", ctypes.c_float), ("sad_ratio", ctypes.c_float),
                ("sad_median_per_sample", ctypes.c_float)]


class MeJob(ctypes.Structure):
    _fields_ = [("ref", MeFrame), ("cur", MeFrame), ("params", MeParams), ("mv", ctypes.c_void_p),
                ("sad", ctypes.c_void_p)]


_P = ctypes.c_void_p
_I32 = ctypes.c_int32


def _sig(name, args, res=_I32):
    f = getattr(_lib, name)
    f.argtypes = args
    f.restype = res
    return f


_me_default_params = _sig("me_default_params", [], MeParams)
_me_ctx_create = _sig("me_ctx_create", [_I32, ctypes.POINTER(_P)])
_me_ctx_destroy = _sig("me_ctx_destroy", [_P])
_me_estimate = _sig("me_estimate", [_P, ctypes.POINTER(MeFrame), ctypes.POINTER(MeFrame), ctypes.POINTER(MeParams),
                                    _P, _P, _P, _P])
_me_stage_search = _sig("me_stage_search", [_P, ctypes.POINTER(MeFrame), ctypes.POINTER(MeFrame), _I32, _I32, _I32,
                                            _P, _I32, _P, _P, _P])


class MePyramidCfg(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("block", ctypes.c_int32 * 4), ("n_stages", ctypes.c_int32),
                ("radius", ctypes.c_int32 * 4), ("step", ctypes.c_int32 * 4), ("limit", ctypes.c_int32)]


_me_compose_vectors = _sig("me_compose_vectors", [_P, _P, _P, _I32, _I32, _I32, _P])
_me_estimate_warp = _sig("me_estimate_warp", [_P, ctypes.POINTER(MeFrame), ctypes.POINTER(MeFrame),
                                              ctypes.POINTER(MeParams), _P, _P, _P, _P, _I32, _I32, _I32, _I32, _P])
_me_default_pyramid = _sig("me_default_pyramid", [], MePyramidCfg)
_me_pyramid = _sig("me_pyramid", [_P, ctypes.POINTER(MeFrame), ctypes.POINTER(MeFrame), ctypes.POINTER(MePyramidCfg),
                                  _P, _P, _P])
_me_warp_features = _sig("me_warp_features", [_P, _P, _P, _I32, _I32, _I32, _I32, _P, _I32, _I32, _I32, _P])
_me_batch_submit = _sig("me_batch_submit", [_P, ctypes.POINTER(MeJob), _I32, _P])
_me_refine = _sig("me_refine", [_P, ctypes.POINTER(MeFrame), ctypes.POINTER(MeFrame), ctypes.POINTER(MeParams), _P, _P,
                                _P, _P, _P])
_me_refine_noalloc = _sig("me_refine_noalloc", [_P, ctypes.POINTER(MeFrame), ctypes.POINTER(MeFrame),
                                                ctypes.POINTER(MeParams), _P, _P, _P, _P, _P])
_F = ctypes.c_float
_me_autotune = _sig("me_autotune", [_P, ctypes.POINTER(MeFrame), ctypes.POINTER(MeFrame), _I32, _I32, _I32, _P, _P])
_me_tuned_shape = _sig("me_tuned_shape", [_P, _I32, _I32, _I32, _I32, _P, _P])
_me_set_tuned_shape = _sig("me_set_tuned_shape", [_P, _I32, _I32, _I32, _I32, _P])
_me_cnn_set_params = _sig("me_cnn_set_params", [_P, _P, _I32, _F])
_me_cnn_get_params = _sig("me_cnn_get_params", [_P, _P, _I32, _P])
_me_cnn_pool = _sig("me_cnn_pool", [_P, ctypes.POINTER(MeFrame), ctypes.POINTER(MeFrame), _P, _P])
_me_cnn_forward = _sig("me_cnn_forward", [_P, _P, _I32, _I32, _I32, _P, _P])
_me_cnn_forward_acts = _sig("me_cnn_forward_acts", [_P, _P, _I32, _I32, _I32, _P, _P, _P, _P, _P])
_me_cnn_train_step = _sig("me_cnn_train_step", [_P, _P, _P, _P, _I32, _I32, _I32, _I32, _I32, _F, _I32, _P, _P, _P])
_me_cnn_state_bytes = _sig("me_cnn_state_bytes", [], ctypes.c_int64)
_me_cnn_save_state = _sig("me_cnn_save_state", [_P, _P, ctypes.c_int64])
_me_cnn_load_state = _sig("me_cnn_load_state", [_P, _P, ctypes.c_int64])
_me_cnn_layer_forward = _sig("me_cnn_layer_forward", [_P, _I32, _P, _P, _I32, _I32, _I32, _P])
_me_cnn_layer_backward = _sig("me_cnn_layer_backward", [_P, _I32, _P, _P, _P, _P, _I32, _I32, _I32, _P])
_me_cnn_loss = _sig("me_cnn_loss", [_P, _P, _P, _P, _I32, _I32, _I32, _I32, _P, _P, _P])
_me_cnn_adamw = _sig("me_cnn_adamw", [_P, _P, _F, _P])


class MePrnetCfg(ctypes.Structure):
    _fields_ = [("c_feat", ctypes.c_int32), ("c_enc", ctypes.c_int32), ("c_hid", ctypes.c_int32),
                ("expand", ctypes.c_int32), ("n_blocks", ctypes.c_int32)]


class MeTensor(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("channels", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("dtype", ctypes.c_int32)]


_PT = ctypes.POINTER(MeTensor)
_I64 = ctypes.c_int64
_me_prnet_num_params = _sig("me_prnet_num_params", [ctypes.POINTER(MePrnetCfg)], _I64)
_me_prnet_create = _sig("me_prnet_create", [_P, ctypes.POINTER(MePrnetCfg), ctypes.POINTER(_P)])
_me_prnet_destroy = _sig("me_prnet_destroy", [_P])
_me_prnet_set_params = _sig("me_prnet_set_params", [_P, _P, _I64])
_me_prnet_get_params = _sig("me_prnet_get_params", [_P, _P, _I64])
_me_prnet_forward = _sig("me_prnet_forward", [_P, ctypes.POINTER(MeFrame), _I32, _I64, _P, _P, _I32, _P])
_me_prnet_forward_acts = _sig("me_prnet_forward_acts",
                              [_P, ctypes.POINTER(MeFrame), _I32, _I64, _P, _P, _I32, _P, _P, _P])
_me_prnet_train_step = _sig("me_prnet_train_step", [_P, ctypes.POINTER(MeFrame), _I32, _I64, _P, _P, _F, _F, _I32,
                                                    _P, _P, _P])
_me_prnet_dw_forward = _sig("me_prnet_dw_forward", [_P, _P, _P, _P, _I32, _I32, _I32, _I32, _I32, _I32, _P, _P])
_me_prnet_dw_backward = _sig("me_prnet_dw_backward", [_P, _P, _P, _P, _P, _I32, _I32, _I32, _I32, _I32, _P, _P, _P])
_me_prnet_pw_forward = _sig("me_prnet_pw_forward", [_P, _PT, _PT, _I32, _I32, _P, _P, _I32, _I32, _PT, _P, _PT, _P])
_me_prnet_pw_backward = _sig("me_prnet_pw_backward", [_P, _PT, _PT, _PT, _I32, _I32, _P, _I32, _I32, _I32, _P, _P, _P,
                                                      _P, _P])
_me_prnet_loss = _sig("me_prnet_loss", [_P, _P, _P, _P, _I32, _I32, _I32, _I32, _F, _P, _P, _P])
_me_sync = _sig("me_sync", [_P])
_me_sad_median = _sig("me_sad_median", [_P, _P, _I32, _I32, _I32, _I32, _P, _P])
_me_fallback_weight = _sig("me_fallback_weight", [_P, _I32, _I32, _I32, _I32, _F, _F, _P, _P])
_me_status_string = _sig("me_status_string", [_I32], ctypes.c_char_p)
_me_last_error = _sig("me_last_error", [], ctypes.c_char_p)

EXPORTS = ["me_default_params", "me_ctx_create", "me_ctx_destroy", "me_estimate", "me_stage_search",
           "me_warp_features", "me_batch_submit", "me_refine", "me_status_string", "me_last_error",
           "me_cnn_set_params", "me_cnn_get_params", "me_cnn_pool", "me_cnn_forward", "me_cnn_train_step",
           "me_cnn_state_bytes", "me_cnn_save_state", "me_cnn_load_state", "me_cnn_layer_forward",
           "me_cnn_layer_backward", "me_cnn_loss", "me_cnn_adamw", "me_autotune", "me_tuned_shape",
           "me_set_tuned_shape", "me_pyramid",
           "me_default_pyramid", "me_compose_vectors", "me_estimate_warp", "me_prnet_num_params", "me_prnet_create", "me_prnet_destroy",
           "me_prnet_set_params", "me_prnet_get_params", "me_prnet_forward", "me_prnet_train_step",
           "me_prnet_dw_forward", "me_prnet_dw_backward", "me_prnet_pw_forward", "me_prnet_pw_backward",
           "me_prnet_loss", "me_sync", "me_sad_median", "me_fallback_weight", "me_refine_noalloc"]
ME_NHWC, ME_NCHW = 0, 1
ME_CNN_NPARAMS = 21699


class MeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_me_status_string(status).decode(), msg))
        self.status = status


def _check(status):
    if status != ME_OK:
        raise MeError(status, _me_last_error().decode())


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def frame_of(t: torch.Tensor) -> MeFrame:
    """Describe a 2-D uint16/int16 device tensor (Bayer mosaic) as an me_frame."""
    if t.dim() != 2 or t.element_size() != 2:
        raise ValueError("a frame is a 2-D tensor of 16-bit samples")
    if t.stride(1) != 1:
        raise ValueError("frame rows must be contiguous")
    return MeFrame(t.data_ptr(), t.shape[0], t.shape[1], t.stride(0))


def block_grid(H, W, block):
    return (H // 2 + block - 1) // block, (W // 2 + block - 1) // block


def default_params() -> MeParams:
    return _me_default_params()


def make_params(block=16, radius=32, mode=ME_MODE_EXHAUSTIVE, refine_radius=2, conf_logit_thresh=0.0,
                sad_ratio=1.5, sad_median_per_sample=0.0) -> MeParams:
    p = default_params()
    p.block, p.radius, p.step, p.mode = block, radius, 1, mode
    p.refine_radius = refine_radius
    p.conf_logit_thresh = conf_logit_thresh
    p.sad_ratio = sad_ratio
    p.sad_median_per_sample = sad_median_per_sample
    return p


class Context:
    """Owner of an me_ctx (scratch buffers, tuned launch shapes, weights, graphs)."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(_me_ctx_create(device, ctypes.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            _check(_me_ctx_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ctx_handle(ctx):
    return None if ctx is None else ctx.handle


def estimate(ref: torch.Tensor, cur: torch.Tensor, block: int = 16, radius: int = 32, mv=None, sad=None,
             fallback=None, params: MeParams | None = None, ctx: Context | None = None, stream=None):
    """MV = ME(F_R, F_C) on two device Bayer mosaics; returns (mv [bh,bw,2] int16, sad [bh,bw] int32)."""
    H, W = cur.shape
    if params is None:
        params = make_params(block, radius)
    bh, bw = block_grid(H, W, params.block)
    if mv is None:
        mv = torch.empty((bh, bw, 2), dtype=torch.int16, device=cur.device)
    if sad is None:
        sad = torch.empty((bh, bw), dtype=torch.int32, device=cur.device)
    fr, fc = frame_of(ref), frame_of(cur)
    _check(_me_estimate(_ctx_handle(ctx), ctypes.byref(fr), ctypes.byref(fc), ctypes.byref(params), mv.data_ptr(),
                        sad.data_ptr(), None if fallback is None else fallback.data_ptr(), _stream_handle(stream)))
    return mv, sad


def stage_search(ref, cur, block, radius, pred=None, limit=None, mv=None, sad=None, ctx=None, stream=None, step=1):
    """One matching stage, candidates pred + step * (u, v), |u|, |v| <= radius
    (full search when pred is None and step is 1)."""
    H, W = cur.shape
    bh, bw = block_grid(H, W, block)
    if limit is None:
        limit = radius * step
    if mv is None:
        mv = torch.empty((bh, bw, 2), dtype=torch.int16, device=cur.device)
    if sad is None:
        sad = torch.empty((bh, bw), dtype=torch.int32, device=cur.device)
    fr, fc = frame_of(ref), frame_of(cur)
    _check(_me_stage_search(_ctx_handle(ctx), ctypes.byref(fr), ctypes.byref(fc), block, radius, step,
                            None if pred is None else pred.data_ptr(), limit, mv.data_ptr(), sad.data_ptr(),
                            _stream_handle(stream)))
    return mv, sad


def estimate_warp(ref, cur, z_ref, block=16, radius=32, mv=None, sad=None, out=None, params=None, ctx=None,
                  stream=None):
    """Full search and warp in one pass (me_estimate_warp): returns (mv, sad, z_out)."""
    fr, fc = frame_of(ref), frame_of(cur)
    p = params if params is not None else make_params(block, radius)
    bh, bw = block_grid(ref.shape[0], ref.shape[1], p.block)
    if mv is None:
        mv = torch.empty((bh, bw, 2), dtype=torch.int16, device=ref.device)
    if sad is None:
        sad = torch.empty((bh, bw), dtype=torch.int32, device=ref.device)
    if out is None:
        out = torch.empty_like(z_ref)
    C, Hf, Wf = z_ref.shape
    dt = ME_BF16 if z_ref.dtype == torch.bfloat16 else ME_F32
    _check(_me_estimate_warp(_ctx_handle(ctx), ctypes.byref(fr), ctypes.byref(fc), ctypes.byref(p), mv.data_ptr(),
                             sad.data_ptr(), z_ref.data_ptr(), out.data_ptr(), dt, C, Hf, Wf, _stream_handle(stream)))
    return mv, sad, out


def compose_vectors(mv_step, mv_acc, block, frame_h, frame_w, out=None, stream=None):
    """Chain block vectors over a group of pictures: frame t -> t-1 (mv_step)
    then t-1 -> key frame (mv_acc); returns the vectors frame t -> key frame."""
    if out is None:
        out = torch.empty_like(mv_step)
    _check(_me_compose_vectors(mv_step.data_ptr(), mv_acc.data_ptr(), out.data_ptr(), block, frame_h, frame_w,
                               _stream_handle(stream)))
    return out


def pyramid_cfg(blocks=(32, 16), stages=((8, 8), (4, 4), (2, 1)), limit=127) -> MePyramidCfg:
    """Block pyramid (coarse to fine) and (radius, step) stages for pyramid()."""
    c = MePyramidCfg()
    c.n_levels = len(blocks)
    for i, b in enumerate(blocks):
        c.block[i] = b
    c.n_stages = len(stages)
    for i, (r, st) in enumerate(stages):
        c.radius[i] = r
        c.step[i] = st
    c.limit = limit
    return c


def pyramid(ref, cur, ctx: Context, cfg: MePyramidCfg | None = None, mv=None, sad=None, stream=None):
    """Coarse-to-fine pyramid block matching; vectors on the finest level's block grid."""
    if cfg is None:
        cfg = _me_default_pyramid()
    H, W = cur.shape
    B = cfg.block[cfg.n_levels - 1]
    bh, bw = block_grid(H, W, B)
    if mv is None:
        mv = torch.empty((bh, bw, 2), dtype=torch.int16, device=cur.device)
    if sad is None:
        sad = torch.empty((bh, bw), dtype=torch.int32, device=cur.device)
    fr, fc = frame_of(ref), frame_of(cur)
    _check(_me_pyramid(ctx.handle, ctypes.byref(fr), ctypes.byref(fc), ctypes.byref(cfg), mv.data_ptr(),
                       sad.data_ptr(), _stream_handle(stream)))
    return mv, sad


def refine(ref, cur, net_out, ctx: Context, block=16, radius=32, refine_radius=2, conf_logit_thresh=0.0,
           sad_ratio=1.5, sad_median_per_sample=0.0, mv=None, sad=None, fallback=None, stream=None, noalloc=False):
    """Learned-proposal refine + fallback given the network output [3, bh, bw] float32.
    Returns (mv, sad, fallback).  noalloc: call me_refine_noalloc (the step's
    scratch in the library's fixed device array instead of context buffers)."""
    H, W = cur.shape
    bh, bw = block_grid(H, W, block)
    if tuple(net_out.shape) != (3, bh, bw) or net_out.dtype != torch.float32 or not net_out.is_contiguous():
        raise ValueError("net_out must be a contiguous float32 [3, %d, %d] tensor" % (bh, bw))
    p = make_params(block, radius, ME_MODE_PROPOSAL, refine_radius, conf_logit_thresh, sad_ratio,
                    sad_median_per_sample)
    if mv is None:
        mv = torch.empty((bh, bw, 2), dtype=torch.int16, device=cur.device)
    if sad is None:
        sad = torch.empty((bh, bw), dtype=torch.int32, device=cur.device)
    if fallback is None:
        fallback = torch.empty((bh, bw), dtype=torch.uint8, device=cur.device)
    fr, fc = frame_of(ref), frame_of(cur)
    fn = _me_refine_noalloc if noalloc else _me_refine
    _check(fn(ctx.handle, ctypes.byref(fr), ctypes.byref(fc), ctypes.byref(p), net_out.data_ptr(),
              mv.data_ptr(), sad.data_ptr(), fallback.data_ptr(), _stream_handle(stream)))
    return mv, sad, fallback


def warp_features(z_ref: torch.Tensor, mv: torch.Tensor, block: int, frame_h: int, frame_w: int, out=None,
                  ctx=None, stream=None):
    """z_pred = Warp(z_R, MV); z_ref is [C, Hf, Wf] float32 or bfloat16 on the device."""
    if z_ref.dtype == torch.float32:
        dt = ME_F32
    elif z_ref.dtype == torch.bfloat16:
        dt = ME_BF16
    else:
        raise ValueError("features must be float32 or bfloat16")
    if not z_ref.is_contiguous():
        raise ValueError("features must be contiguous")
    C, Hf, Wf = z_ref.shape
    if out is None:
        out = torch.empty_like(z_ref)
    _check(_me_warp_features(_ctx_handle(ctx), z_ref.data_ptr(), out.data_ptr(), dt, C, Hf, Wf, mv.data_ptr(), block,
                             frame_h, frame_w, _stream_handle(stream)))
    return out


def autotune(ctx: Context, ref, cur, block=16, radius=32, iters=3, stream=None) -> float:
    """Pick the fastest launch shape for (block, radius, frame size); returns its time in ms."""
    ms = ctypes.c_float()
    fr, fc = frame_of(ref), frame_of(cur)
    _check(_me_autotune(ctx.handle, ctypes.byref(fr), ctypes.byref(fc), block, radius, iters, ctypes.addressof(ms),
                        _stream_handle(stream)))
    return ms.value


def tuned_shape(ctx: Context, block, radius, height, width):
    """The launch shape used for (block, radius, height x width Bayer frames):
    ((kx, ky, blocks per workgroup, LDS KB, current block in LDS, waves per
    block), tuned) with tuned True when it was recorded by autotune or
    set_tuned_shape."""
    shape = (ctypes.c_int32 * 6)()
    tuned = ctypes.c_int32()
    _check(_me_tuned_shape(ctx.handle, block, radius, height, width, ctypes.addressof(shape), ctypes.addressof(tuned)))
    return tuple(shape), bool(tuned.value)


def set_tuned_shape(ctx: Context, block, radius, height, width, shape):
    """Record a launch shape (kx, ky, blocks per workgroup, LDS budget in KB,
    current block in LDS 0/1, waves per block; missing trailing entries mean
    0 and 4) for (block, radius, frame size), e.g. one reported by
    tuned_shape."""
    vals = [int(v) for v in shape]
    if not 4 <= len(vals) <= 6:
        raise ValueError("shape has 4 to 6 entries")
    vals += [0, 4][len(vals) - 4:]
    arr = (ctypes.c_int32 * 6)(*vals)
    _check(_me_set_tuned_shape(ctx.handle, block, radius, height, width, ctypes.addressof(arr)))


def make_jobs(jobs):
    """Host job array for batch_submit from (ref, cur, block, radius, mv, sad) tuples."""
    arr = (MeJob * len(jobs))()
    for k, (ref, cur, block, radius, mv, sad) in enumerate(jobs):
        arr[k].ref = frame_of(ref)
        arr[k].cur = frame_of(cur)
        arr[k].params = make_params(block, radius)
        arr[k].mv = mv.data_ptr()
        arr[k].sad = sad.data_ptr()
    return arr


def batch_submit(ctx: Context, jobs, stream=None):
    """One submission of many pairs: a list of (ref, cur, block, radius, mv,
    sad) device tensors, or an array made by make_jobs (the tensors must stay
    alive until the work is done)."""
    arr = jobs if isinstance(jobs, ctypes.Array) else make_jobs(jobs)
    _check(_me_batch_submit(ctx.handle, arr, len(arr), _stream_handle(stream)))


def sync(stream=None):
    """Wait for the stream's work; raises MeError (ME_E_HIP) if it failed."""
    _check(_me_sync(_stream_handle(stream)))


# --- proposal network ---------------------------------------------------------

def _sad_maps(sad, block, frame_h, frame_w):
    bh, bw = block_grid(frame_h, frame_w, block)
    if sad.dtype != torch.int32 or not sad.is_contiguous() or sad.numel() % (bh * bw) or sad.numel() == 0:
        raise ValueError("sad must be a contiguous int32 tensor of whole [%d, %d] maps" % (bh, bw))
    return sad.numel() // (bh * bw)


def sad_median(ctx: Context, sad, block, frame_h, frame_w, out=None, stream=None):
    """Lower median of the per-sample full-search SAD over [n, bh, bw] maps
    (device float32 scalar tensor, the M of the SAD fallback test)."""
    n = _sad_maps(sad, block, frame_h, frame_w)
    if out is None:
        out = torch.empty((), dtype=torch.float32, device=sad.device)
    _check(_me_sad_median(ctx.handle, sad.data_ptr(), n, block, frame_h, frame_w, out.data_ptr(),
                          _stream_handle(stream)))
    return out


def fallback_weight(sad, block, frame_h, frame_w, sad_ratio, median_per_sample, out=None, stream=None):
    """0/1 float32 weights [n, bh, bw]: 1 where the full-search SAD is within
    the SAD fallback threshold floor(ratio * M * n_samples)."""
    n = _sad_maps(sad, block, frame_h, frame_w)
    if out is None:
        out = torch.empty(sad.shape, dtype=torch.float32, device=sad.device)
    _check(_me_fallback_weight(sad.data_ptr(), n, block, frame_h, frame_w, sad_ratio, median_per_sample,
                               out.data_ptr(), _stream_handle(stream)))
    return out


def _p(t):
    return None if t is None else t.data_ptr()


def cnn_set_params(ctx: Context, params, median_per_sample: float):
    import numpy as np

    a = np.ascontiguousarray(params, dtype=np.float32)
    _check(_me_cnn_set_params(ctx.handle, a.ctypes.data, a.size, median_per_sample))


def cnn_get_params(ctx: Context):
    import numpy as np

    a = np.empty(ME_CNN_NPARAMS, np.float32)
    m = ctypes.c_float()
    _check(_me_cnn_get_params(ctx.handle, a.ctypes.data, a.size, ctypes.addressof(m)))
    return a, m.value


def cnn_pool(ctx, ref, cur, x=None, stream=None):
    """Network input [H/8, W/8, 8] bfloat16 of one frame pair."""
    H, W = cur.shape
    if x is None:
        x = torch.empty((H // 8, W // 8, 8), dtype=torch.bfloat16, device=cur.device)
    fr, fc = frame_of(ref), frame_of(cur)
    _check(_me_cnn_pool(_ctx_handle(ctx), ctypes.byref(fr), ctypes.byref(fc), x.data_ptr(), _stream_handle(stream)))
    return x


CNN_STRIDES = (2, 2, 1, 1)


def _out_grid(Hq, Wq):
    """Output grid of the proposal network on a [Hq, Wq] input."""
    for s in CNN_STRIDES:
        Hq, Wq = -(-Hq // s), -(-Wq // s)
    return Hq, Wq


def cnn_forward(ctx, x, out=None, stream=None):
    """x: [n, Hq, Wq, 8] bfloat16 -> [n, 3, bh, bw] float32."""
    n, Hq, Wq, _ = x.shape
    bh, bw = _out_grid(Hq, Wq)
    if out is None:
        out = torch.empty((n, 3, bh, bw), dtype=torch.float32, device=x.device)
    _check(_me_cnn_forward(ctx.handle, x.data_ptr(), n, Hq, Wq, out.data_ptr(), _stream_handle(stream)))
    return out


def cnn_forward_acts(ctx, x, stream=None):
    """Whole-network forward that also returns the layer 0-2 activations:
    (out [n, 3, bh, bw] float32, [a0 [n, h1, w1, 32], a1, a2] bfloat16)."""
    n, Hq, Wq, _ = x.shape
    h1, w1 = -(-Hq // 2), -(-Wq // 2)
    h2, w2 = -(-h1 // 2), -(-w1 // 2)
    out = torch.empty((n, 3, h2, w2), dtype=torch.float32, device=x.device)
    acts = [torch.empty((n, h, w, 32), dtype=torch.bfloat16, device=x.device) for h, w in ((h1, w1), (h2, w2), (h2, w2))]
    _check(_me_cnn_forward_acts(ctx.handle, x.data_ptr(), n, Hq, Wq, out.data_ptr(), acts[0].data_ptr(),
                                acts[1].data_ptr(), acts[2].data_ptr(), _stream_handle(stream)))
    return out, acts


def cnn_train_step(ctx, x, mv, radius=32, refine_radius=2, lr=1e-4, update=True, grads=None, loss=None,
                   weight=None, stream=None):
    """weight: optional float32 [n, bh, bw] weight of each block's vector term."""
    n, Hq, Wq, _ = x.shape
    _check(_me_cnn_train_step(ctx.handle, x.data_ptr(), mv.data_ptr(), _p(weight), n, Hq, Wq, radius, refine_radius,
                              lr, 1 if update else 0, _p(grads), _p(loss), _stream_handle(stream)))


def cnn_save_state(ctx) -> bytes:
    nb = _me_cnn_state_bytes()
    buf = ctypes.create_string_buffer(nb)
    _check(_me_cnn_save_state(ctx.handle, ctypes.addressof(buf), nb))
    return buf.raw


def cnn_load_state(ctx, blob: bytes):
    buf = ctypes.create_string_buffer(blob, len(blob))
    _check(_me_cnn_load_state(ctx.handle, ctypes.addressof(buf), len(blob)))


def cnn_layer_forward(ctx, layer, inp, out, stream=None):
    n, H, W, _ = inp.shape
    _check(_me_cnn_layer_forward(ctx.handle, layer, inp.data_ptr(), out.data_ptr(), n, H, W, _stream_handle(stream)))


def cnn_layer_backward(ctx, layer, x, dz, dx, grads, stream=None):
    n, H, W, _ = x.shape
    _check(_me_cnn_layer_backward(ctx.handle, layer, x.data_ptr(), dz.data_ptr(), _p(dx), grads.data_ptr(), n, H, W,
                                  _stream_handle(stream)))


def cnn_loss(ctx, out, mv, radius, refine_radius, dz, loss, weight=None, stream=None):
    n, _, bh, bw = out.shape
    _check(_me_cnn_loss(ctx.handle, out.data_ptr(), mv.data_ptr(), _p(weight), n, bh * bw, radius, refine_radius,
                        dz.data_ptr(), loss.data_ptr(), _stream_handle(stream)))


def cnn_adamw(ctx, grads, lr, stream=None):
    _check(_me_cnn_adamw(ctx.handle, grads.data_ptr(), lr, _stream_handle(stream)))


# ------------------------------------------------- perception residual network --

def prnet_cfg(c_feat=256, c_enc=32, c_hid=64, expand=4, n_blocks=2) -> MePrnetCfg:
    return MePrnetCfg(c_feat, c_enc, c_hid, expand, n_blocks)


def prnet_num_params(cfg: MePrnetCfg) -> int:
    n = _me_prnet_num_params(ctypes.byref(cfg))
    if n < 0:
        raise MeError(ME_E_INVAL, "invalid network configuration")
    return n


def feature_grid(frame_h, frame_w):
    """Feature grid of the network for a Bayer frame: ceil(Hp/4) x ceil(Wp/4)."""
    hp, wp = frame_h // 2, frame_w // 2
    return (((hp - 1) // 2) // 2 + 1, ((wp - 1) // 2) // 2 + 1)


def prnet_init_params(cfg: MePrnetCfg, seed: int = 0, head_scale: float = 1.0):
    """Seeded starting parameters in the library's order: He-normal weights
    (fan-in 9 for depthwise layers, c_in for 1x1 layers), biases 0.1 before a
    ReLU6 and 0 otherwise, the head's weights scaled by head_scale."""
    import numpy as np

    e, h, x = cfg.c_enc, cfg.c_hid, cfg.c_hid * cfg.expand
    layers = [(9, 4, True), (4, e, True), (9, e, True), (e, e, True), (cfg.c_feat + e, h, True)]
    for _ in range(cfg.n_blocks):
        layers += [(h, x, True), (9, x, True), (x, h, False)]
    layers.append((h, cfg.c_feat, False))
    rng = np.random.default_rng(seed)
    parts = []
    for i, (fan, co, relu) in enumerate(layers):
        w = rng.normal(0.0, np.sqrt(2.0 / fan), co * fan)
        parts += [w * (head_scale if i == len(layers) - 1 else 1.0), np.full(co, 0.1 if relu else 0.0)]
    return np.concatenate(parts).astype(np.float32)


class Prnet:
    """A network object of the library (me_prnet_*)."""

    def __init__(self, ctx: Context, cfg: MePrnetCfg | None = None):
        self.cfg = cfg or prnet_cfg()
        self.n_params = prnet_num_params(self.cfg)
        h = _P()
        _check(_me_prnet_create(ctx.handle, ctypes.byref(self.cfg), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            _check(_me_prnet_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        import numpy as np

        a = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        _check(_me_prnet_set_params(self.handle, a.ctypes.data, a.size))

    def get_params(self):
        import numpy as np

        a = np.empty(self.n_params, np.float32)
        _check(_me_prnet_get_params(self.handle, a.ctypes.data, a.size))
        return a

    def forward(self, cur: torch.Tensor, z_pred: torch.Tensor, out=None, stream=None):
        """cur: [n, H, W] (or [H, W]) uint16 mosaics; z_pred [n, c_feat, Hf, Wf] float32 or bfloat16."""
        c = cur if cur.dim() == 3 else cur[None]
        z = z_pred if z_pred.dim() == 4 else z_pred[None]
        if out is None:
            out = torch.empty_like(z)
        dt = ME_BF16 if z.dtype == torch.bfloat16 else ME_F32
        fr = frame_of(c[0])
        _check(_me_prnet_forward(self.handle, ctypes.byref(fr), c.shape[0], c.stride(0), z.data_ptr(), out.data_ptr(),
                                 dt, _stream_handle(stream)))
        return out if z_pred.dim() == 4 else out[0]

    def forward_acts(self, cur: torch.Tensor, z_pred: torch.Tensor, stream=None):
        """forward() on [n, H, W] mosaics and [n, c_feat, Hf, Wf] features that also returns the stage
        outputs: (z_out, enc [n, Hf, Wf, c_enc] bfloat16, hid [n_blocks + 1, n, Hf, Wf, c_hid] bfloat16)."""
        n, Hf, Wf = z_pred.shape[0], z_pred.shape[2], z_pred.shape[3]
        out = torch.empty_like(z_pred)
        enc = torch.empty((n, Hf, Wf, self.cfg.c_enc), dtype=torch.bfloat16, device=z_pred.device)
        hid = torch.empty((self.cfg.n_blocks + 1, n, Hf, Wf, self.cfg.c_hid), dtype=torch.bfloat16,
                          device=z_pred.device)
        dt = ME_BF16 if z_pred.dtype == torch.bfloat16 else ME_F32
        fr = frame_of(cur[0])
        _check(_me_prnet_forward_acts(self.handle, ctypes.byref(fr), n, cur.stride(0), z_pred.data_ptr(),
                                      out.data_ptr(), dt, enc.data_ptr(), hid.data_ptr(), _stream_handle(stream)))
        return out, enc, hid

    def train_step(self, cur, z_pred, z_target, tau=-1.0, lr=1e-3, update=True, grads=None, loss=None, stream=None):
        c = cur if cur.dim() == 3 else cur[None]
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=c.device)
        fr = frame_of(c[0])
        _check(_me_prnet_train_step(self.handle, ctypes.byref(fr), c.shape[0], c.stride(0), z_pred.data_ptr(),
                                    z_target.data_ptr(), tau, lr, 1 if update else 0, _p(grads), loss.data_ptr(),
                                    _stream_handle(stream)))
        return loss


def _tensor(t, layout=ME_NHWC):
    if t is None:
        return None
    dt = {torch.float32: ME_F32, torch.bfloat16: ME_BF16}[t.dtype]
    ch = t.shape[-1] if layout == ME_NHWC else t.shape[1]
    return MeTensor(t.data_ptr(), ch, layout, dt)


def _tp(m):
    return ctypes.byref(m) if m is not None else None


def prnet_dw_forward(ctx, x, w, b, stride, relu6=True, y=None, stream=None):
    """x bfloat16 [n, H, W, C]; w float32 [C, 9]; b [C]."""
    n, H, W, C = x.shape
    if y is None:
        y = torch.empty((n, (H - 1) // stride + 1, (W - 1) // stride + 1, C), dtype=torch.bfloat16, device=x.device)
    _check(_me_prnet_dw_forward(ctx.handle, x.data_ptr(), w.data_ptr(), b.data_ptr(), n, H, W, C, stride,
                                1 if relu6 else 0, y.data_ptr(), _stream_handle(stream)))
    return y


def prnet_dw_backward(ctx, x, w, dy, stride, mask=None, dx=None, grads=None, stream=None):
    n, H, W, C = x.shape
    _check(_me_prnet_dw_backward(ctx.handle, x.data_ptr(), w.data_ptr(), dy.data_ptr(), _p(mask), n, H, W, C, stride,
                                 _p(dx), _p(grads), _stream_handle(stream)))


def prnet_pw_forward(ctx, x, w, b, out, x2=None, relu6=False, add=None, mask=None, hw=None, x_layout=ME_NHWC,
                     add_layout=ME_NHWC, out_layout=ME_NHWC, stream=None):
    """1x1 convolution over n images of hw pixels; tensors in the given layouts
    ([n, hw, C] or [n, C, hw] views); x2 is channels-last bfloat16."""
    n = x.shape[0]
    hw = hw if hw is not None else (x.shape[1] if x_layout == ME_NHWC else x.shape[2])
    tx, tx2, ta, to = _tensor(x, x_layout), _tensor(x2), _tensor(add, add_layout), _tensor(out, out_layout)
    _check(_me_prnet_pw_forward(ctx.handle, ctypes.byref(tx), _tp(tx2), n, hw, w.data_ptr(), _p(b), w.shape[0],
                                1 if relu6 else 0, _tp(ta), _p(mask), ctypes.byref(to), _stream_handle(stream)))
    return out


def prnet_pw_backward(ctx, x, w, dy, x2=None, dx=None, dx_c0=0, dx_count=None, add=None, mask=None, grads=None,
                      hw=None, x_layout=ME_NHWC, dy_layout=ME_NHWC, stream=None):
    n = x.shape[0]
    hw = hw if hw is not None else (x.shape[1] if x_layout == ME_NHWC else x.shape[2])
    cin = w.shape[1]
    dx_count = cin - dx_c0 if dx_count is None else dx_count
    tx, tx2, td = _tensor(x, x_layout), _tensor(x2), _tensor(dy, dy_layout)
    _check(_me_prnet_pw_backward(ctx.handle, ctypes.byref(tx), _tp(tx2), ctypes.byref(td), n, hw, w.data_ptr(),
                                 w.shape[0], dx_c0, dx_count, _p(add), _p(mask), _p(dx), _p(grads),
                                 _stream_handle(stream)))


def prnet_loss(ctx, r, z_pred, z_target, tau=-1.0, dr=None, loss=None, stream=None):
    n, C, Hf, Wf = r.shape
    dr = torch.empty(r.shape, dtype=torch.bfloat16, device=r.device) if dr is None else dr
    loss = torch.empty(1, dtype=torch.float32, device=r.device) if loss is None else loss
    _check(_me_prnet_loss(ctx.handle, r.data_ptr(), z_pred.data_ptr(), z_target.data_ptr(), n, C, Hf, Wf, tau,
                          dr.data_ptr(), loss.data_ptr(), _stream_handle(stream)))
    return dr, loss
