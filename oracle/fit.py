"""Tap fitting oracle: float64 Adam and the least-squares optimum.

The filter bank is linear in its taps, so the mean-squared-error fit of the
taps to a target has a closed-form optimum (normal equations over the basis
columns u_b(x[n-l])).  Adam follows the update of torch.optim.Adam with
default options (no weight decay, no amsgrad), applied to the real and
imaginary parts of each complex tap separately.

Loss: L = (1/N) sum_n |yhat[n] - t[n]|^2 over complex samples, so
grad_yhat = 2 (yhat - t) / N in the grad = dL/dRe + i dL/dIm convention.

Parity: pinned by tests/test_oracle_fit.py (noise-free target recovered
exactly by least squares; Adam step equal to an independent torch.optim.Adam
run in float64; loss decreases toward the least-squares floor).
"""
from __future__ import annotations

import numpy as np

from .filterbank import fb_stream, fb_stream_adjoint, basis


def mse(yhat, t):
    e = np.asarray(yhat, np.complex128) - np.asarray(t, np.complex128)
    return float(np.mean(e.real ** 2 + e.imag ** 2))


def design_matrix_columns(x, frames, bank_L, Kmax):
    """Yields (bank, p, l, column) with column[n] = u_p(x[n-l]) on frames where
    branch (bank, p) is active and 0 elsewhere (zero history)."""
    x = np.asarray(x, np.complex128)
    N = x.shape[0]
    for bank, L in enumerate(bank_L):
        for p in range(Kmax):
            d = bank * Kmax + p
            act = np.zeros(N, bool)
            for (t0, n, mask, route) in frames:
                if not route and (int(mask) >> d) & 1:
                    act[t0:t0 + n] = True
            if not act.any():
                continue
            u = basis(x, p)
            for l in range(int(L)):
                col = np.zeros(N, np.complex128)
                col[l:] = u[:N - l]
                col[~act] = 0
                yield bank, p, l, col


def lsq_taps(x, target, frames, bank_L, Kmax, chunk=1 << 18):
    """Least-squares taps via the normal equations, Gram matrix accumulated in
    float64 chunks.  Returns (taps [n_banks, Kmax, Lmax], loss at the optimum)."""
    cols = list(design_matrix_columns(x, frames, bank_L, Kmax))
    idx = [(b, p, l) for (b, p, l, _) in cols]
    A = np.stack([c for (_, _, _, c) in cols], axis=1)       # N x P
    t = np.asarray(target, np.complex128)
    P = A.shape[1]
    G = np.zeros((P, P), np.complex128)
    rhs = np.zeros(P, np.complex128)
    for s in range(0, A.shape[0], chunk):
        As = A[s:s + chunk]
        G += As.conj().T @ As
        rhs += As.conj().T @ t[s:s + chunk]
    theta = np.linalg.solve(G, rhs)
    taps = np.zeros((len(bank_L), Kmax, max(bank_L)), np.complex128)
    for (b, p, l), v in zip(idx, theta):
        taps[b, p, l] = v
    return taps, mse(A @ theta, t)


class Adam:
    """torch.optim.Adam (defaults) on the real view of complex parameters."""

    def __init__(self, shape, lr=1e-2, betas=(0.9, 0.999), eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, betas[0], betas[1], eps
        self.m = np.zeros(shape + (2,), np.float64)
        self.v = np.zeros(shape + (2,), np.float64)
        self.t = 0

    def step(self, param, grad):
        p = np.stack([param.real, param.imag], axis=-1).astype(np.float64)
        g = np.stack([grad.real, grad.imag], axis=-1).astype(np.float64)
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        bc1 = 1 - self.b1 ** self.t
        bc2 = 1 - self.b2 ** self.t
        denom = np.sqrt(self.v) / np.sqrt(bc2) + self.eps
        p = p - (self.lr / bc1) * self.m / denom
        return p[..., 0] + 1j * p[..., 1]


def adam_fit(x, target, frames, taps0, bank_L, Kmax, steps=200, lr=1e-2):
    """Full-batch Adam on the taps; returns (losses[steps+1], taps)."""
    taps = np.asarray(taps0, np.complex128).copy()
    opt = Adam(taps.shape, lr=lr)
    t = np.asarray(target, np.complex128)
    N = t.shape[0]
    losses = []
    for _ in range(steps):
        y = fb_stream(x, frames, taps, bank_L, Kmax)
        losses.append(mse(y, t))
        g = 2.0 * (y - t) / N
        _, gt = fb_stream_adjoint(x, frames, taps, bank_L, Kmax, g)
        taps = opt.step(taps, gt)
    losses.append(mse(fb_stream(x, frames, taps, bank_L, Kmax), t))
    return np.array(losses), taps
