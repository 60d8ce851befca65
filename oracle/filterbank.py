"""Filter-bank actor of the DPD application, float64 direct definition.

The DPD workload (Sec. VII-A, "Dynamic Predistortion Filtering") is a set of
parallel complex FIR filters over a polynomial basis, with a configuration
actor choosing per firing which filters are active.  Branch d of a bank uses
the basis u_p(x) = |x|^p * x with p = d mod Kmax (branch b = p + 1), so

    y[n] = sum_{d active} sum_{l < L_d} h_d[l] * |x[n-l]|^{p_d} * x[n-l]

with x[t] = 0 before the start of the stream and the L-1 samples before a
frame taken from the stream's past (frames are cut from one continuous
stream).  Everything is computed in complex128 from the complex64 inputs.

Parity: pinned by tests/test_oracle_filterbank.py (impulse responses equal
the taps, Vandermonde recovery of all branches, equality with numpy's
convolution at K=1, linearity in the taps, phase equivariance, per-branch
homogeneity, frame-split invariance).
"""
from __future__ import annotations

import numpy as np


def _abs(z: np.ndarray) -> np.ndarray:
    # |z| = sqrt(re^2 + im^2), computed explicitly in float64.
    return np.sqrt(z.real * z.real + z.imag * z.imag)


def basis(z: np.ndarray, p: int) -> np.ndarray:
    """u_p(z) = |z|^p * z (|z|^0 = 1, so u_0 = z even at z = 0)."""
    z = np.asarray(z, dtype=np.complex128)
    if p == 0:
        return z.copy()
    return _abs(z) ** p * z


def fb_frame(window: np.ndarray, halo: int, taps: np.ndarray, bank_L, Kmax: int,
             mask: int) -> np.ndarray:
    """One firing of the filter bank.

    window : the ``halo`` stream samples that precede the frame, then the
             frame's n samples (complex).
    taps   : [n_banks, Kmax, Lmax] complex; bank j uses taps[j, :, :L_j].
    mask   : bit d set -> branch d = bank*Kmax + (b-1) is active.
    Returns y[0..n) in complex128.
    """
    w = np.asarray(window, dtype=np.complex128)
    n = w.shape[0] - halo
    y = np.zeros(n, dtype=np.complex128)
    n_banks = len(bank_L)
    for d in range(n_banks * Kmax):
        if not (mask >> d) & 1:
            continue
        bank, p = divmod(d, Kmax)
        L = int(bank_L[bank])
        if L - 1 > halo:
            raise ValueError("window holds fewer past samples than the filter needs")
        u = basis(w, p)
        h = np.asarray(taps[bank, p, :L], dtype=np.complex128)
        # Causal convolution written as a sum over taps: y[n] += h[l] u[n-l].
        for l in range(L):
            y += h[l] * u[halo - l: halo - l + n]
    return y


def fb_stream(x: np.ndarray, frames, taps: np.ndarray, bank_L, Kmax: int,
              history=None) -> np.ndarray:
    """Whole-stream semantics of the graph path on one stream.

    frames : iterable of (t0, n, mask, route); frames tile the stream in order.
             route 0 = filter bank, route 1 = passthrough (y = x).
    history: the Lmax-1 samples before t=0 (zeros when None).
    """
    x = np.asarray(x, dtype=np.complex128)
    H = max(int(L) for L in bank_L) - 1
    past = np.zeros(H, np.complex128) if history is None else np.asarray(history, np.complex128)
    xp = np.concatenate([past, x])
    y = np.zeros_like(x)
    for (t0, n, mask, route) in frames:
        t0, n = int(t0), int(n)
        if route:
            y[t0:t0 + n] = x[t0:t0 + n]
        else:
            y[t0:t0 + n] = fb_frame(xp[t0:t0 + H + n], H, taps, bank_L, Kmax, int(mask))
    return y


def fb_stream_adjoint(x: np.ndarray, frames, taps: np.ndarray, bank_L, Kmax: int,
                      g: np.ndarray):
    """Closed-form adjoint of ``fb_stream`` (zero history).

    For a real loss and the convention grad_z = dL/dRe z + i dL/dIm z, with
    g = grad_y, p = b-1, r = |x|:

      grad_h_d[l] = sum_{frames f active in d} sum_{n in f} g[n] conj(u_p(x[n-l]))
      G_d[m]      = sum_l conj(h_d[l]) g[m+l] [frame(m+l) has d active]
      grad_x[m]   = sum_d (p/2+1) r^p G_d[m] + (p/2) r^(p-2) x^2 conj(G_d[m])
                    (+ g[m] for passthrough frames)

    The second term vanishes for p = 0 and at r = 0 (its magnitude is
    (p/2) r^p |G|).  Returns (grad_x, grad_taps) in complex128.
    """
    x = np.asarray(x, dtype=np.complex128)
    g = np.asarray(g, dtype=np.complex128)
    N = x.shape[0]
    H = max(int(L) for L in bank_L) - 1
    xp = np.concatenate([np.zeros(H, np.complex128), x])
    r = _abs(xp)
    n_banks = len(bank_L)
    gt = np.zeros(taps.shape, dtype=np.complex128)
    gx_p = np.zeros(N + H, dtype=np.complex128)     # gradient w.r.t. xp
    for (t0, n, mask, route) in frames:
        t0, n = int(t0), int(n)
        if route:
            gx_p[H + t0:H + t0 + n] += g[t0:t0 + n]
            continue
        gf = g[t0:t0 + n]
        for d in range(n_banks * Kmax):
            if not (int(mask) >> d) & 1:
                continue
            bank, p = divmod(d, Kmax)
            L = int(bank_L[bank])
            h = np.asarray(taps[bank, p, :L], dtype=np.complex128)
            lo = H + t0 - (L - 1)
            w = xp[lo:H + t0 + n]                   # window of the frame's inputs
            u = basis(w, p)
            rw = r[lo:H + t0 + n]
            G = np.zeros(w.shape[0], np.complex128)  # grad w.r.t. u over the window
            for l in range(L):
                # output n' = i uses input window index i + (L-1) - l
                gt[bank, p, l] += np.sum(gf * np.conj(u[L - 1 - l: L - 1 - l + n]))
                G[L - 1 - l: L - 1 - l + n] += np.conj(h[l]) * gf
            a = (p / 2.0 + 1.0) * rw ** p
            gx_w = a * G
            if p >= 1:
                wz = w * w
                safe = rw > 0
                coef = np.zeros_like(rw)
                coef[safe] = (p / 2.0) * rw[safe] ** (p - 2)
                gx_w = gx_w + coef * wz * np.conj(G)
            gx_p[lo:H + t0 + n] += gx_w
    return gx_p[H:], gt
