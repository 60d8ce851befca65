"""Pins of the oracle filter bank and its adjoint (no GPU)."""
import numpy as np
import pytest
import torch

import synth
from oracle.filterbank import fb_frame, fb_stream, fb_stream_adjoint, basis


def _rand_taps(rng, nb, K, L):
    return (rng.standard_normal((nb, K, L)) + 1j * rng.standard_normal((nb, K, L))) / 3


def _frames(N, cuts, masks, routes=None):
    out, t = [], 0
    for i, c in enumerate(cuts):
        out.append((t, c, masks[i], 0 if routes is None else routes[i]))
        t += c
    assert t == N
    return out


# ---------------------------------------------------------------- P4 impulse
@pytest.mark.parametrize("L", [1, 8, 32])
def test_impulse_response_is_taps(L):
    rng = np.random.default_rng(L)
    taps = _rand_taps(rng, 1, 4, L)
    a = 0.7 - 0.2j
    x = np.zeros(3 * L + 5, complex)
    x[0] = a
    y = fb_stream(x, [(0, len(x), 0b1, 0)], taps, [L], 4)
    np.testing.assert_allclose(y[:L], a * taps[0, 0], rtol=1e-14, atol=1e-15)
    assert np.all(y[L:] == 0)


def test_vandermonde_recovers_all_branches():
    """Impulses of Kmax distinct amplitudes: y_a[l] = sum_b a|a|^(b-1) h_b[l];
    solving the Vandermonde system in |a| gives back every branch's taps."""
    K, L = 5, 6
    rng = np.random.default_rng(3)
    taps = _rand_taps(rng, 1, K, L)
    amps = np.array([0.3, 0.6, 0.9, 1.3, 1.7])
    Y = []
    for a in amps:
        x = np.zeros(L + 3, complex)
        x[0] = a
        Y.append(fb_stream(x, [(0, len(x), (1 << K) - 1, 0)], taps, [L], K)[:L])
    V = np.array([[a * a ** b for b in range(K)] for a in amps])     # real a > 0
    H = np.linalg.solve(V, np.array(Y))
    np.testing.assert_allclose(H, taps[0], rtol=1e-9, atol=1e-11)


# ---------------------------------------------------------------- P5 textbook FIR
def test_k1_equals_numpy_convolve():
    wl = synth.make("C1", n_frames=3, frame_len=500)
    x = wl.x[0].astype(complex)
    h = wl.taps[0, 0, 0].astype(complex)
    frames = _frames(len(x), [500] * 3, [1] * 3)
    y = fb_stream(x, frames, wl.taps[0].astype(complex), wl.bank_L, wl.Kmax)
    np.testing.assert_allclose(y, np.convolve(x, h)[:len(x)], rtol=1e-12, atol=1e-13)


# ---------------------------------------------------------------- P6 invariants
def test_linearity_in_taps():
    rng = np.random.default_rng(5)
    x = rng.standard_normal(400) + 1j * rng.standard_normal(400)
    t1, t2 = _rand_taps(rng, 2, 4, 8), _rand_taps(rng, 2, 4, 8)
    fr = _frames(400, [150, 250], [0b1011, 0b1111 << 4])
    al, be = 0.3 - 1.1j, -2.0 + 0.5j
    y = fb_stream(x, fr, al * t1 + be * t2, [8, 5], 4)
    y1 = fb_stream(x, fr, t1, [8, 5], 4)
    y2 = fb_stream(x, fr, t2, [8, 5], 4)
    np.testing.assert_allclose(y, al * y1 + be * y2, rtol=1e-12, atol=1e-12)


def test_phase_equivariance():
    rng = np.random.default_rng(6)
    x = rng.standard_normal(300) + 1j * rng.standard_normal(300)
    taps = _rand_taps(rng, 1, 6, 7)
    fr = _frames(300, [300], [0b111111])
    ph = np.exp(1j * 0.77)
    np.testing.assert_allclose(fb_stream(ph * x, fr, taps, [7], 6),
                               ph * fb_stream(x, fr, taps, [7], 6), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("b", [1, 2, 3, 6])
def test_branch_homogeneity(b):
    """A single active branch b is homogeneous of degree b for real s > 0."""
    rng = np.random.default_rng(b)
    x = rng.standard_normal(200) + 1j * rng.standard_normal(200)
    taps = _rand_taps(rng, 1, 6, 5)
    fr = _frames(200, [200], [1 << (b - 1)])
    s = 1.7
    np.testing.assert_allclose(fb_stream(s * x, fr, taps, [5], 6),
                               s ** b * fb_stream(x, fr, taps, [5], 6), rtol=1e-11, atol=1e-12)


def test_basis_zero_and_power_zero():
    z = np.array([0.0 + 0.0j, 3.0 + 4.0j])
    np.testing.assert_array_equal(basis(z, 0), z)
    np.testing.assert_allclose(basis(z, 2), np.array([0, 25 * (3 + 4j)]))


def test_frame_boundary_uses_stream_history():
    """The second frame sees the last L-1 samples of the first (A5 reading)."""
    rng = np.random.default_rng(9)
    x = rng.standard_normal(40) + 1j * rng.standard_normal(40)
    taps = _rand_taps(rng, 1, 2, 8)
    y_one = fb_stream(x, [(0, 40, 0b11, 0)], taps, [8], 2)
    y_two = fb_stream(x, [(0, 13, 0b11, 0), (13, 27, 0b11, 0)], taps, [8], 2)
    np.testing.assert_allclose(y_two, y_one, rtol=0, atol=1e-14)


# ---------------------------------------------------------------- P10 gradients
def _torch_forward(x, taps, frames, bank_L, Kmax):
    """Plain torch (complex128, CPU) restatement used only to let torch.autograd
    derive the gradient independently of the closed form."""
    N = x.shape[0]
    H = max(bank_L) - 1
    xp = torch.cat([torch.zeros(H, dtype=x.dtype), x])
    ys = []
    for (t0, n, mask, route) in frames:
        if route:
            ys.append(x[t0:t0 + n])
            continue
        w = xp[t0:t0 + H + n]
        y = torch.zeros(n, dtype=x.dtype)
        for d in range(len(bank_L) * Kmax):
            if not (mask >> d) & 1:
                continue
            bank, p = divmod(d, Kmax)
            u = w if p == 0 else torch.abs(w) ** p * w
            for l in range(bank_L[bank]):
                y = y + taps[bank, p, l] * u[H - l:H - l + n]
        ys.append(y)
    return torch.cat(ys)


def _case(seed=0):
    rng = np.random.default_rng(seed)
    N = 90
    x = (rng.standard_normal(N) + 1j * rng.standard_normal(N)) * 0.6
    bank_L, K = [6, 4], 4
    taps = np.zeros((2, K, 6), complex)
    taps[0] = _rand_taps(rng, 1, K, 6)[0]
    taps[1, :, :4] = _rand_taps(rng, 1, K, 4)[0]
    frames = _frames(N, [30, 25, 35], [0b0111, 0b1111 << 4, 0b1101], routes=[0, 0, 0])
    g = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    return x, taps, bank_L, K, frames, g


def test_adjoint_matches_torch_autograd():
    x, taps, bank_L, K, frames, g = _case(1)
    gx, gt = fb_stream_adjoint(x, frames, taps, bank_L, K, g)
    xt = torch.tensor(x, requires_grad=True)
    tt = torch.tensor(taps, requires_grad=True)
    y = _torch_forward(xt, tt, frames, bank_L, K)
    loss = torch.real(torch.sum(torch.conj(torch.tensor(g)) * y))
    loss.backward()
    np.testing.assert_allclose(gx, xt.grad.numpy(), rtol=1e-10, atol=1e-12)
    mask = np.zeros_like(taps, bool)
    mask[0, :, :6] = True
    mask[1, :, :4] = True
    np.testing.assert_allclose(gt[mask], tt.grad.numpy()[mask], rtol=1e-10, atol=1e-12)


def test_adjoint_matches_finite_differences():
    x, taps, bank_L, K, frames, g = _case(2)
    gx, gt = fb_stream_adjoint(x, frames, taps, bank_L, K, g)

    def loss(xv, tv):
        return float(np.real(np.sum(np.conj(g) * fb_stream(xv, frames, tv, bank_L, K))))
    rng = np.random.default_rng(0)
    for m in rng.choice(len(x), 12, replace=False):
        for comp, unit in ((0, 1.0), (1, 1j)):
            h = 1e-6 * max(1.0, abs(x[m]))
            xp, xm = x.copy(), x.copy()
            xp[m] += unit * h
            xm[m] -= unit * h
            fd = (loss(xp, taps) - loss(xm, taps)) / (2 * h)
            an = gx[m].real if comp == 0 else gx[m].imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
    for (b, p, l) in [(0, 0, 0), (0, 2, 5), (1, 3, 3), (0, 1, 2), (1, 0, 1)]:
        for comp, unit in ((0, 1.0), (1, 1j)):
            h = 1e-6 * max(1.0, abs(taps[b, p, l]))
            tp, tm = taps.copy(), taps.copy()
            tp[b, p, l] += unit * h
            tm[b, p, l] -= unit * h
            fd = (loss(x, tp) - loss(x, tm)) / (2 * h)
            an = gt[b, p, l].real if comp == 0 else gt[b, p, l].imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))


def test_adjoint_k1_closed_form():
    """K=1: grad_h[l] = sum_n g[n] conj(x[n-l]), grad_x[m] = sum_l conj(h[l]) g[m+l]."""
    rng = np.random.default_rng(4)
    N, L = 64, 7
    x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    g = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    taps = _rand_taps(rng, 1, 1, L)
    gx, gt = fb_stream_adjoint(x, [(0, N, 1, 0)], taps, [L], 1, g)
    h = taps[0, 0]
    gh_ref = np.array([np.sum(g[l:] * np.conj(x[:N - l])) for l in range(L)])
    gx_ref = np.array([sum(np.conj(h[l]) * g[m + l] for l in range(L) if m + l < N) for m in range(N)])
    np.testing.assert_allclose(gt[0, 0], gh_ref, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(gx, gx_ref, rtol=1e-12, atol=1e-12)


def test_adjoint_at_zero_input():
    """|x| = 0 inputs: the Wirtinger term vanishes, no NaN (b = 2 branch)."""
    x = np.array([0, 0.5 + 0.1j, 0, -0.3j, 0.2, 0], complex)
    g = np.ones(6, complex) * (0.3 - 0.4j)
    taps = np.zeros((1, 3, 2), complex)
    taps[0] = [[1, 0.5], [0.7j, -0.2], [0.1, 0.3 + 0.1j]]
    gx, gt = fb_stream_adjoint(x, [(0, 6, 0b111, 0)], taps, [2], 3, g)
    assert np.all(np.isfinite(gx)) and np.all(np.isfinite(gt))
    xt = torch.tensor(x, requires_grad=True)
    y = _torch_forward(xt, torch.tensor(taps), [(0, 6, 0b111, 0)], [2], 3)
    torch.real(torch.sum(torch.conj(torch.tensor(g)) * y)).backward()
    nz = np.abs(x) > 0
    np.testing.assert_allclose(gx[nz], xt.grad.numpy()[nz], rtol=1e-10, atol=1e-12)


def test_adjoint_passthrough_frames():
    x, taps, bank_L, K, frames, g = _case(3)
    frames = [(t, n, m, 1 if i == 1 else 0) for i, (t, n, m, _) in enumerate(frames)]
    gx, gt = fb_stream_adjoint(x, frames, taps, bank_L, K, g)
    xt = torch.tensor(x, requires_grad=True)
    y = _torch_forward(xt, torch.tensor(taps), frames, bank_L, K)
    torch.real(torch.sum(torch.conj(torch.tensor(g)) * y)).backward()
    np.testing.assert_allclose(gx, xt.grad.numpy(), rtol=1e-10, atol=1e-12)
