"""Direct filter-bank operations over whole streams and their autograd
Function.  Marshalling only: prune_fb_forward / prune_fb_backward run the HIP
kernels; torch supplies device memory and the current stream.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from ._lib import call


def make_desc(n_streams, stream_len, Kmax, bank_L, n_frames, max_frame_len):
    d = L.FbDesc()
    d.n_streams = n_streams
    d.n_frames = n_frames
    d.stream_len = stream_len
    d.n_banks = len(bank_L)
    d.Kmax = Kmax
    for i, v in enumerate(bank_L):
        d.L[i] = int(v)
    d.max_frame_len = int(max_frame_len)
    return d


def frames_from_side(side, Kmax, routed):
    """Frame rows (stream, t0, n, mask, route) of a batch of streams from the
    configuration actor's side-information [S, F, 4] (K, n, bank, route),
    using the library's own configuration mapping (prune_rule_config_token).
    Routed streams run every branch on filter-bank frames."""
    side = np.asarray(side, dtype=np.uint32)
    S, F, _ = side.shape
    rows = []
    tok = L.CtrlToken()
    for s_ in range(S):
        t0 = 0
        for f in range(F):
            K, n, bank, route = (int(v) for v in side[s_, f])
            if routed:
                mask, r = 0xFFFFFFFF, route
            else:
                si = L.SideInfo(K, n, bank, route)
                call("prune_rule_config_token", L.CONFIG_PREFIX, Kmax, C.byref(si), C.byref(tok))
                mask, r = tok.mask, 0
            rows.append((s_, t0, n, mask, r))
            t0 += n
    return rows


def frame_table(frames, device="cuda"):
    """frames: array [F, 5] of (stream, t0, n, mask, route) -> device table of
    prune_fb_frame records (8 x uint32)."""
    fr = np.zeros((len(frames), 8), dtype=np.uint32)
    fr[:, :5] = np.asarray(frames, dtype=np.int64).astype(np.uint32)
    return torch.from_numpy(fr).to(device)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def fb_forward(x, taps, frames_dev, Kmax, bank_L, max_frame_len, y=None):
    """x: complex64 [S, N] (cuda); taps: complex64 [S, n_banks, Kmax, Lmax];
    frames_dev: frame_table(...).  Returns y [S, N]."""
    S, N = x.shape
    x = x.contiguous()
    taps = taps.contiguous()
    if y is None:
        y = torch.empty_like(x)
    d = make_desc(S, N, Kmax, bank_L, frames_dev.shape[0], max_frame_len)
    call("prune_fb_forward", C.byref(d), C.c_void_p(x.data_ptr()), C.c_void_p(taps.data_ptr()),
         C.c_void_p(frames_dev.data_ptr()), C.c_void_p(y.data_ptr()), _stream())
    return y


def fb_forward_noalloc(x, taps, frames_dev, Kmax, bank_L, max_frame_len, y):
    """fb_forward through prune_fb_forward_noalloc: the library allocates
    nothing (its work list lives in a fixed device array), so y must be
    given."""
    S, N = x.shape
    assert x.is_contiguous() and taps.is_contiguous() and y.is_contiguous()
    d = make_desc(S, N, Kmax, bank_L, frames_dev.shape[0], max_frame_len)
    call("prune_fb_forward_noalloc", C.byref(d), C.c_void_p(x.data_ptr()),
         C.c_void_p(taps.data_ptr()), C.c_void_p(frames_dev.data_ptr()), C.c_void_p(y.data_ptr()),
         _stream())
    return y


def check_frames(frames_dev, n_streams, stream_len, Kmax, bank_L, max_frame_len):
    """Number of frames the filter-bank operations would skip or that break
    the required order (sorted by stream, then t0, no overlap)."""
    d = make_desc(n_streams, stream_len, Kmax, bank_L, frames_dev.shape[0], max_frame_len)
    bad = C.c_uint32()
    call("prune_fb_check_frames", C.byref(d), C.c_void_p(frames_dev.data_ptr()), C.byref(bad),
         _stream())
    return bad.value


def workspace_bytes(S, N, Kmax, bank_L, n_frames, max_frame_len):
    d = make_desc(S, N, Kmax, bank_L, n_frames, max_frame_len)
    ws = C.c_size_t()
    call("prune_fb_workspace_bytes", C.byref(d), C.byref(ws))
    return ws.value


def fb_backward(x, taps, frames_dev, gy, Kmax, bank_L, max_frame_len, gx=None, gt=None, work=None,
                want_gx=True, want_gt=True):
    """Adjoint of fb_forward: (grad_x, grad_taps); a gradient not wanted is
    not computed and returned as None."""
    S, N = x.shape
    x = x.contiguous()
    taps = taps.contiguous()
    gy = gy.contiguous()
    d = make_desc(S, N, Kmax, bank_L, frames_dev.shape[0], max_frame_len)
    ws = C.c_size_t()
    call("prune_fb_workspace_bytes", C.byref(d), C.byref(ws))
    if work is None or work.numel() < ws.value:
        work = torch.empty(max(1, ws.value), dtype=torch.uint8, device=x.device)
    if gx is None and want_gx:
        gx = torch.empty_like(x)
    if gt is None and want_gt:
        gt = torch.empty_like(taps)
    if not want_gx:
        gx = None
    if not want_gt:
        gt = None
    call("prune_fb_backward", C.byref(d), C.c_void_p(x.data_ptr()), C.c_void_p(taps.data_ptr()),
         C.c_void_p(frames_dev.data_ptr()), C.c_void_p(gy.data_ptr()),
         C.c_void_p(gx.data_ptr() if gx is not None else None),
         C.c_void_p(gt.data_ptr() if gt is not None else None), C.c_void_p(work.data_ptr()), ws.value,
         _stream())
    return gx, gt


class FilterBankFn(torch.autograd.Function):
    """y = filter bank(x; taps) over whole streams; gradients w.r.t. x and taps
    come from the hand-written adjoint kernels (the |x|^p basis is recomputed
    in the backward, not stored)."""

    @staticmethod
    def forward(ctx, x, taps, frames_dev, Kmax, bank_L, max_frame_len):
        ctx.save_for_backward(x, taps, frames_dev)
        ctx.cfg = (Kmax, tuple(bank_L), max_frame_len)
        return fb_forward(x, taps, frames_dev, Kmax, bank_L, max_frame_len)

    @staticmethod
    def backward(ctx, gy):
        x, taps, frames_dev = ctx.saved_tensors
        Kmax, bank_L, mfl = ctx.cfg
        want_gx, want_gt = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (want_gx or want_gt):
            return None, None, None, None, None, None
        gx, gt = fb_backward(x, taps, frames_dev, gy, Kmax, bank_L, mfl, want_gx=want_gx, want_gt=want_gt)
        return gx, gt, None, None, None, None


def filter_bank(x, taps, frames_dev, Kmax, bank_L, max_frame_len):
    return FilterBankFn.apply(x, taps, frames_dev, Kmax, bank_L, max_frame_len)


def set_variant(v):
    call("prune_set_fb_variant", int(v))


def variant_names():
    n = L.lib().prune_fb_variant_count()
    return [L.lib().prune_fb_variant_name(v).decode() for v in range(1, n + 1)]


def autotuned_variant(L, K, n):
    """Forward variant the autotuner picks for this shape class (1-based)."""
    v = C.c_int()
    call("prune_autotune_fb", int(L), int(K), int(n), C.byref(v))
    return v.value


def tuned_variant(x, frames_dev, Kmax, bank_L, max_frame_len):
    """Forward variant fb_forward uses for this shape class (1-based; 0 when
    not tuned yet)."""
    S, N = x.shape
    d = make_desc(S, N, Kmax, bank_L, frames_dev.shape[0], max_frame_len)
    v = C.c_int()
    call("prune_fb_tuned_variant", C.byref(d), C.byref(v))
    return v.value


def set_bwd_variant(v):
    """0: autotuned, 1: vector kernel, 2: matrix-core kernels."""
    call("prune_set_bwd_variant", int(v))


def bwd_variant_name(v):
    return L.lib().prune_bwd_variant_name(int(v)).decode()


def autotuned_bwd_variant(L_, K, n):
    v = C.c_int()
    call("prune_autotune_bwd", int(L_), int(K), int(n), C.byref(v))
    return v.value


def set_batch_pipeline(on=True):
    """Bookkeeping of the next batch on a side stream (default on)."""
    call("prune_set_batch_pipeline", int(on))


def timing_enable(on=True):
    call("prune_timing_enable", int(on))


def last_fb_kernel_ms():
    ms = C.c_float()
    n = C.c_uint32()
    call("prune_last_fb_kernel_ms", C.byref(ms), C.byref(n))
    return ms.value, n.value
