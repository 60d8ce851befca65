"""Pins of the fit oracle (least squares and Adam)."""
import numpy as np
import torch

import synth
from oracle import fit
from oracle.graphs import stream_frames


def _small_c4(noise):
    wl = synth.make("C4", n_frames=4, frame_len=600)
    x = wl.x[0]
    xd = x.astype(complex)
    a2 = np.abs(xd) ** 2
    target = xd * (1 - 0.15 * a2 + 0.02 * a2 * a2)
    if noise:
        target = wl.target[0].astype(complex)
    return wl, x, target


def test_lsq_recovers_amplifier_exactly():
    """Noise-free target = u_1 - 0.15 u_3 + 0.02 u_5 at tap 0: least squares
    returns exactly those taps and zero loss."""
    wl, x, target = _small_c4(noise=False)
    taps, loss = fit.lsq_taps(x, target, stream_frames(wl), wl.bank_L, wl.Kmax)
    expect = np.zeros_like(taps)
    expect[0, 0, 0], expect[0, 2, 0], expect[0, 4, 0] = 1.0, -0.15, 0.02
    np.testing.assert_allclose(taps, expect, atol=2e-6)
    assert loss < 1e-12


def test_lsq_floor_with_noise():
    wl, x, target = _small_c4(noise=True)
    taps, loss = fit.lsq_taps(x, target, stream_frames(wl), wl.bank_L, wl.Kmax)
    # noise variance per complex sample is 2e-4; 128 fitted parameters on 2400
    # samples take away a share of it
    assert 1.5e-4 < loss < 2.3e-4


def test_adam_matches_torch_adam():
    rng = np.random.default_rng(0)
    p0 = rng.standard_normal((2, 3)) + 1j * rng.standard_normal((2, 3))
    grads = [rng.standard_normal((2, 3)) + 1j * rng.standard_normal((2, 3)) for _ in range(5)]
    ours = fit.Adam(p0.shape, lr=1e-2)
    p = p0.copy()
    tp = torch.tensor(p0, dtype=torch.complex128, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2)
    for gr in grads:
        p = ours.step(p, gr)
        opt.zero_grad()
        tp.grad = torch.tensor(gr)
        opt.step()
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_adam_fit_descends():
    wl, x, target = _small_c4(noise=True)
    losses, taps = fit.adam_fit(x, target, stream_frames(wl), wl.taps[0], wl.bank_L, wl.Kmax,
                                steps=25, lr=1e-2)
    assert losses[-1] < 0.5 * losses[0]
    assert np.all(np.isfinite(losses))
