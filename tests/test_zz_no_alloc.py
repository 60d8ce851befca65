"""GPU parity of prune_fb_forward_noalloc (the forward with its work list in
the library's fixed device array) against prune_fb_forward, on two calls in a
row, the second with a smaller input, plus its capacity check."""
import numpy as np
import pytest
import torch

import synth
from oracle.filterbank import fb_stream
from oracle.graphs import stream_frames
from paper_1802_06625_amd import _lib as L
from paper_1802_06625_amd import ops

from gpu_util import TOL, announce, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _inputs(wl):
    rows = [(s, t0, n, m, r) for s in range(wl.n_streams) for (t0, n, m, r) in stream_frames(wl, s)]
    return (ops.frame_table(rows), torch.from_numpy(wl.x).cuda(), torch.from_numpy(wl.taps).cuda(),
            int(wl.side[:, :, 1].max()))


def _both(wl):
    fr, x, t, mfl = _inputs(wl)
    y_ref = ops.fb_forward(x, t, fr, wl.Kmax, wl.bank_L, mfl)
    # NaN fill: a sample the entry point should write but does not shows up
    y = torch.full_like(x, complex(float("nan"), float("nan")))
    ops.fb_forward_noalloc(x, t, fr, wl.Kmax, wl.bank_L, mfl, y)
    torch.cuda.synchronize()
    return y.cpu().numpy(), y_ref.cpu().numpy()


def _check(wl, y, y_ref, what):
    for s in range(wl.n_streams):
        assert np.all(np.isfinite(y[s])), (what, s)
        assert rel_l2(y[s], y_ref[s]) <= TOL, (what, s, rel_l2(y[s], y_ref[s]))
        ref = fb_stream(wl.x[s], stream_frames(wl, s), wl.taps[s], wl.bank_L, wl.Kmax)
        assert rel_l2(y[s], ref) <= TOL, (what, s, rel_l2(y[s], ref))


def test_noalloc_matches_forward_twice_shrinking():
    # first call: three streams with passthrough frames, 64 taps; second call:
    # one stream of uneven frames over three banks, fewer frames and tiles
    announce("no-alloc forward: wide multi-stream batch, then a smaller uneven batch")
    big = synth.scaled("C5")
    y, y_ref = _both(big)
    _check(big, y, y_ref, "first call")
    small = synth.scaled("C3", n_frames=9, n_max=3000)
    assert small.x.size < big.x.size
    y, y_ref = _both(small)
    _check(small, y, y_ref, "second call")


def test_noalloc_every_variant_then_smaller():
    announce("no-alloc forward: each forced variant, large then small")
    big = synth.scaled("C2")
    small = synth.scaled("C1", n_frames=5)
    for v in range(1, len(ops.variant_names()) + 1):
        ops.set_variant(v)
        try:
            for wl in (big, small):
                y, y_ref = _both(wl)
                _check(wl, y, y_ref, f"variant {v}")
        finally:
            ops.set_variant(0)


def test_noalloc_rejects_beyond_capacity():
    # rejected on the host before any launch: too many frames, too many tiles
    announce("no-alloc forward: capacity limits")
    x = torch.zeros((1, 16), dtype=torch.complex64, device="cuda")
    t = torch.zeros((1, 1, 1, 8), dtype=torch.complex64, device="cuda")
    y = torch.zeros_like(x)
    fr = ops.frame_table([(0, 0, 16, 1, 0)])
    for n_frames, mfl in ((8193, 16), (1, 1 << 31)):
        d = ops.make_desc(1, 16, 1, [8], n_frames, mfl)
        st = L.lib().prune_fb_forward_noalloc(
            L.C.byref(d), L.C.c_void_p(x.data_ptr()), L.C.c_void_p(t.data_ptr()),
            L.C.c_void_p(fr.data_ptr()), L.C.c_void_p(y.data_ptr()), ops._stream())
        assert st == L.E_CAPACITY, (n_frames, mfl, st)
        assert b"fixed workspace" in L.lib().prune_last_error()
    torch.cuda.synchronize()
    assert torch.all(y == 0)
