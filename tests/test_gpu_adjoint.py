"""GPU parity of the hand-written adjoint (prune_fb_backward) and its
autograd Function against the FP64 closed-form adjoint of the oracle, and of
a short tap fit against the oracle's Adam."""
import numpy as np
import pytest
import torch

import synth
from oracle import fit
from oracle.filterbank import fb_stream_adjoint
from oracle.graphs import stream_frames
from paper_1802_06625_amd import ops

from gpu_util import TOL, announce, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _rows(wl):
    return [(s, t0, n, m, r) for s in range(wl.n_streams) for (t0, n, m, r) in stream_frames(wl, s)]


@pytest.mark.parametrize("name", ["C1", "C3", "C4", "C5"])
def test_backward_parity(name):
    announce(f"backward {name}")
    wl = synth.scaled(name, cotangent=True) if name != "C1" else synth.make("C1", cotangent=True)
    rows = _rows(wl)
    fr = ops.frame_table(rows)
    x = torch.from_numpy(wl.x).cuda()
    t = torch.from_numpy(wl.taps).cuda()
    gy = torch.from_numpy(wl.gy).cuda()
    gx, gt = ops.fb_backward(x, t, fr, gy, wl.Kmax, wl.bank_L, int(wl.side[:, :, 1].max()))
    gx, gt = gx.cpu().numpy(), gt.cpu().numpy()
    for s in range(wl.n_streams):
        rx, rt = fb_stream_adjoint(wl.x[s], stream_frames(wl, s), wl.taps[s], wl.bank_L, wl.Kmax,
                                   wl.gy[s])
        assert rel_l2(gx[s], rx) <= TOL, (name, s, rel_l2(gx[s], rx))
        assert rel_l2(gt[s], rt) <= TOL, (name, s, rel_l2(gt[s], rt))
        # entries beyond each bank's L are exact zeros
        for b, L in enumerate(wl.bank_L):
            assert np.all(gt[s, b, :, L:] == 0)


def test_backward_edge_frames():
    """Short frames (< L-1), empty masks, passthrough frames, several banks."""
    announce("backward edge frames")
    wl = synth.make("C3", n_frames=10, n_max=300, cotangent=True)
    lens = [3, 50, 7, 300, 1, 31, 2, 129, 64, 11]
    N = sum(lens)
    wl.x, wl.gy = wl.x[:, :N].copy(), wl.gy[:, :N].copy()
    masks = [1, 0x3FF, 0x3FF << 10, (1 << 30) - 1, 5, 0x201, 0, 1 << 25, 0x7 | (0x7 << 20), 2]
    routes = [0, 0, 1, 0, 0, 0, 0, 1, 0, 0]
    rows, t0 = [], 0
    for n, m, r in zip(lens, masks, routes):
        rows.append((0, t0, n, m, r))
        t0 += n
    fr = ops.frame_table(rows)
    gx, gt = ops.fb_backward(torch.from_numpy(wl.x).cuda(), torch.from_numpy(wl.taps).cuda(), fr,
                             torch.from_numpy(wl.gy).cuda(), wl.Kmax, wl.bank_L, max(lens))
    ref = [(t, n, m, r) for (_, t, n, m, r) in rows]
    rx, rt = fb_stream_adjoint(wl.x[0], ref, wl.taps[0], wl.bank_L, wl.Kmax, wl.gy[0])
    assert rel_l2(gx.cpu().numpy()[0], rx) <= TOL
    assert rel_l2(gt.cpu().numpy()[0], rt) <= TOL


def test_autograd_function_matches_oracle():
    announce("autograd FilterBankFn")
    wl = synth.scaled("C4", cotangent=True)
    rows = _rows(wl)
    fr = ops.frame_table(rows)
    x = torch.from_numpy(wl.x).cuda().requires_grad_(True)
    t = torch.from_numpy(wl.taps).cuda().requires_grad_(True)
    y = ops.filter_bank(x, t, fr, wl.Kmax, wl.bank_L, int(wl.side[:, :, 1].max()))
    loss = torch.real(torch.sum(torch.conj(torch.from_numpy(wl.gy).cuda()) * y))
    loss.backward()
    rx, rt = fb_stream_adjoint(wl.x[0], stream_frames(wl, 0), wl.taps[0], wl.bank_L, wl.Kmax, wl.gy[0])
    assert rel_l2(x.grad.cpu().numpy()[0], rx) <= TOL
    assert rel_l2(t.grad.cpu().numpy()[0], rt) <= TOL


def test_fit_tracks_oracle_adam():
    """A short Adam fit of the taps to the amplifier target: the GPU loss curve
    (fp32 kernels, torch.optim.Adam) follows the FP64 oracle's."""
    announce("fit vs oracle adam")
    wl = synth.scaled("C4")
    frames = stream_frames(wl)
    steps = 20
    ref_losses, _ = fit.adam_fit(wl.x[0], wl.target[0], frames, wl.taps[0], wl.bank_L, wl.Kmax,
                                 steps=steps, lr=1e-2)
    fr = ops.frame_table([(0,) + f for f in frames])
    x = torch.from_numpy(wl.x).cuda()
    target = torch.from_numpy(wl.target).cuda()
    taps = torch.nn.Parameter(torch.from_numpy(wl.taps).cuda().clone())
    opt = torch.optim.Adam([taps], lr=1e-2)
    losses = []
    for _ in range(steps):
        y = ops.filter_bank(x, taps, fr, wl.Kmax, wl.bank_L, int(wl.side[:, :, 1].max()))
        e = y - target
        loss = torch.mean(e.real ** 2 + e.imag ** 2)
        losses.append(loss.item())
        opt.zero_grad()
        loss.backward()
        opt.step()
    losses = np.array(losses)
    np.testing.assert_allclose(losses, ref_losses[:steps], rtol=1e-3)
    assert losses[-1] < 0.5 * losses[0]
