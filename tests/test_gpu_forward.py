"""GPU parity of the direct filter-bank forward (prune_fb_forward) against
the FP64 oracle on every workload recipe, at parity sizes and, by sampled
frames, at full size."""
import numpy as np
import pytest
import torch

import synth
from oracle.filterbank import fb_stream, fb_frame
from oracle.graphs import stream_frames
from paper_1802_06625_amd import ops

from gpu_util import TOL, announce, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _frames(wl):
    rows = []
    for s in range(wl.n_streams):
        for (t0, n, mask, route) in stream_frames(wl, s):
            rows.append((s, t0, n, mask, route))
    return rows


def _device_forward(wl, variant=0):
    ops.set_variant(variant)
    try:
        rows = _frames(wl)
        fr = ops.frame_table(rows)
        x = torch.from_numpy(wl.x).cuda()
        t = torch.from_numpy(wl.taps).cuda()
        y = ops.fb_forward(x, t, fr, wl.Kmax, wl.bank_L, int(wl.side[:, :, 1].max()))
        torch.cuda.synchronize()
        return y.cpu().numpy(), rows
    finally:
        ops.set_variant(0)


def _oracle(wl):
    return np.stack([fb_stream(wl.x[s], stream_frames(wl, s), wl.taps[s], wl.bank_L, wl.Kmax)
                     for s in range(wl.n_streams)])


@pytest.mark.parametrize("name", ["C1", "C2", "C3", "C4", "C5"])
def test_forward_parity_scaled(name):
    announce(f"direct forward {name}")
    wl = synth.scaled(name) if name != "C1" else synth.make("C1")
    y, _ = _device_forward(wl)
    ref = _oracle(wl)
    for s in range(wl.n_streams):
        assert rel_l2(y[s], ref[s]) <= TOL, (name, s, rel_l2(y[s], ref[s]))


N_VARIANTS = 8          # 1-5 vector Horner kernels, 6-8 matrix-core block-Toeplitz
MFMA_VARIANTS = [6, 7, 8]


def test_variant_names():
    names = ops.variant_names()
    assert len(names) == N_VARIANTS
    assert all(names[v - 1].startswith("mfma") for v in MFMA_VARIANTS)


@pytest.mark.parametrize("name", ["C3", "C5"])
@pytest.mark.parametrize("variant", list(range(1, N_VARIANTS + 1)))
def test_every_variant(variant, name):
    """Three banks of L = 8/16/32 with log-uniform frame lengths (C3), and
    L = 64 over routed multi-stream frames (C5)."""
    announce(f"forward variant {variant} {name}")
    wl = synth.scaled(name)
    y, _ = _device_forward(wl, variant)
    ref = _oracle(wl)
    for s in range(wl.n_streams):
        assert rel_l2(y[s], ref[s]) <= TOL, (s, rel_l2(y[s], ref[s]))


@pytest.mark.parametrize("L", [1, 5, 17, 63, 64])
@pytest.mark.parametrize("variant", MFMA_VARIANTS)
def test_mfma_tap_counts(variant, L):
    """Block-Toeplitz kernels at tap counts that are not multiples of the
    step of 4, with every branch, and frames that end inside a tile."""
    announce(f"mfma variant {variant} L={L}")
    wl = synth.make("C4", n_frames=6, frame_len=5000)
    rng = np.random.default_rng(L)
    taps = (rng.standard_normal((1, 1, 10, L)) + 1j * rng.standard_normal((1, 1, 10, L))
            ).astype(np.complex64) / (4 * L)
    lens = [5000, 1, 4500, 9000 - 4501, 700, 3000]
    rows, t0 = [], 0
    for n, m in zip(lens, [0x3FF, 0x3FF, 0x155, 1, 0x3FF, 0x2AA]):
        rows.append((0, t0, n, m, 0))
        t0 += n
    x = wl.x[:, :t0].copy()
    ops.set_variant(variant)
    try:
        y = ops.fb_forward(torch.from_numpy(x).cuda(), torch.from_numpy(taps).cuda(),
                           ops.frame_table(rows), 10, (L,), max(lens)).cpu().numpy()
    finally:
        ops.set_variant(0)
    ref = fb_stream(x[0], [(a, n, m, r) for (_, a, n, m, r) in rows], taps[0], (L,), 10)
    assert rel_l2(y[0], ref) <= TOL, rel_l2(y[0], ref)


@pytest.mark.parametrize("variant", [0, 1, 5, 6, 8])
def test_forward_edge_frames(variant):
    """Empty-mask frames, frames of 1 sample, frames shorter than the filter,
    passthrough frames, and masks mixing two banks."""
    announce(f"forward edge frames variant {variant}")
    wl = synth.make("C3", n_frames=12, n_max=300)
    lens = [1, 3, 50, 7, 300, 1, 31, 2, 129, 64, 5, 11]
    N = sum(lens)
    wl.x = wl.x[:, :N].copy()
    rows, t = [], 0
    masks = [0, 1, 0x3FF, 0x3FF << 10, (1 << 30) - 1, 5, 0x201, 0, 1 << 25, 0x7 | (0x7 << 20), 2, 1]
    routes = [0, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0]
    for n, m, r in zip(lens, masks, routes):
        rows.append((0, t, n, m, r))
        t += n
    fr = ops.frame_table(rows)
    x = torch.from_numpy(wl.x).cuda()
    taps = torch.from_numpy(wl.taps).cuda()
    ops.set_variant(variant)
    try:
        y = ops.fb_forward(x, taps, fr, wl.Kmax, wl.bank_L, max(lens)).cpu().numpy()
    finally:
        ops.set_variant(0)
    ref = fb_stream(wl.x[0], [(t0, n, m, r) for (_, t0, n, m, r) in rows], wl.taps[0], wl.bank_L,
                    wl.Kmax)
    assert rel_l2(y[0], ref) <= TOL
    # exact zeros for empty masks, exact copies for passthrough frames
    for (_, t0, n, m, r) in rows:
        if r:
            np.testing.assert_array_equal(y[0, t0:t0 + n], wl.x[0, t0:t0 + n])
        elif m == 0:
            assert np.all(y[0, t0:t0 + n] == 0)


def test_full_size_c2_sampled_frames():
    """C2 at full size (4096 x 16384, L=32): sampled frames against the
    oracle computed frame by frame from the stream's true history."""
    announce("full-size C2 sampled frames")
    wl = synth.make("C2")
    y, rows = _device_forward(wl)
    x = wl.x[0]
    H = max(wl.bank_L) - 1
    rng = np.random.default_rng(0)
    for f in sorted(rng.choice(len(rows), 6, replace=False).tolist() + [0, len(rows) - 1]):
        _, t0, n, m, r = rows[f]
        past = x[max(0, t0 - H):t0]
        win = np.concatenate([np.zeros(H - len(past), np.complex64), past, x[t0:t0 + n]])
        ref = fb_frame(win, H, wl.taps[0], wl.bank_L, wl.Kmax, m)
        assert rel_l2(y[0, t0:t0 + n], ref) <= TOL, f


def _sampled_frames(wl, y, rows, k, seed=0):
    H = max(wl.bank_L) - 1
    rng = np.random.default_rng(seed)
    for f in sorted(rng.choice(len(rows), k, replace=False).tolist() + [0, len(rows) - 1]):
        s_, t0, n, m, r = rows[f]
        x = wl.x[s_]
        if r:
            np.testing.assert_array_equal(y[s_, t0:t0 + n], x[t0:t0 + n])
            continue
        past = x[max(0, t0 - H):t0]
        win = np.concatenate([np.zeros(H - len(past), np.complex64), past, x[t0:t0 + n]])
        ref = fb_frame(win, H, wl.taps[s_], wl.bank_L, wl.Kmax, m)
        assert rel_l2(y[s_, t0:t0 + n], ref) <= TOL, (f, rel_l2(y[s_, t0:t0 + n], ref))


@pytest.mark.parametrize("variant", [0, 6])
def test_full_size_c5_sampled_frames(variant):
    """C5 at full size (64 streams x 16 x 32768, K=7, L=64, routed frames) in
    the launch configuration of the measured run: sampled frames against the
    oracle, frame by frame."""
    announce(f"full-size C5 sampled frames variant {variant}")
    wl = synth.make("C5")
    y, rows = _device_forward(wl, variant)
    _sampled_frames(wl, y, rows, 8)


def test_check_frames_counts_violations():
    """prune_fb_check_frames: valid tables report 0; each out-of-range or
    out-of-order frame counts once."""
    announce("check frames")
    S, N, mfl = 2, 1000, 300
    good = [(0, 0, 300, 1, 0), (0, 300, 200, 1, 0), (0, 600, 100, 1, 1), (1, 5, 300, 3, 0)]
    assert ops.check_frames(ops.frame_table(good), S, N, 4, (8,), mfl) == 0
    bad = [(0, 0, 300, 1, 0),
           (0, 250, 100, 1, 0),    # overlaps the previous frame of its stream
           (2, 0, 10, 1, 0),       # stream out of range
           (1, 950, 100, 1, 0),    # runs past the stream end
           (1, 0, 301, 1, 0),      # longer than max_frame_len, and before the previous frame
           (0, 700, 10, 1, 0)]     # a lower stream after a higher one
    assert ops.check_frames(ops.frame_table(bad), S, N, 4, (8,), mfl) == 5
    for name in ["C3", "C5"]:
        wl = synth.scaled(name)
        rows = _frames(wl)
        assert ops.check_frames(ops.frame_table(rows), wl.n_streams, wl.x.shape[1], wl.Kmax,
                                wl.bank_L, int(wl.side[:, :, 1].max())) == 0


@pytest.mark.parametrize("variant", [1, 2, 5])
@pytest.mark.parametrize("rounds", [1, 2, 3])
def test_work_list_round_boundaries(variant, rounds):
    """Tile counts around whole rounds of the persistent grid (each
    workgroup's first two tiles are by index, later ones by ticket): the
    grid's multiples minus one, exact and plus one, for the residency the
    grid can have (2, 3 or 4 workgroups per CU), one tile per frame (the
    frames are shorter than any variant's tile)."""
    name = ops.variant_names()[variant - 1]
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    announce(f"forward round boundaries variant {name} rounds {rounds}")
    rng = np.random.default_rng(1000 * variant + rounds)
    Kmax, bank_L = 2, (3,)
    for res in (2, 3, 4):
        for dn in (-1, 0, 1):
            F = rounds * ncu * res + dn
            lens = rng.integers(1, 65, size=F)   # short frames: one tile each, little oracle work
            t0 = np.concatenate([[0], np.cumsum(lens)[:-1]])
            N = int(lens.sum())
            rows = [(0, int(a), int(n), int(rng.integers(1, 4)), 0) for a, n in zip(t0, lens)]
            x = ((rng.standard_normal(N) + 1j * rng.standard_normal(N)) * 0.3).astype(np.complex64)[None]
            taps = ((rng.standard_normal((1, 1, Kmax, 3)) + 1j * rng.standard_normal((1, 1, Kmax, 3))) / 4
                    ).astype(np.complex64)
            ops.set_variant(variant)
            try:
                y = ops.fb_forward(torch.from_numpy(x).cuda(), torch.from_numpy(taps).cuda(),
                                   ops.frame_table(rows), Kmax, bank_L, 64).cpu().numpy()
            finally:
                ops.set_variant(0)
            ref = fb_stream(x[0], [(a, n, m, r) for (_, a, n, m, r) in rows], taps[0], bank_L, Kmax)
            assert rel_l2(y[0], ref) <= TOL, (res, dn, rel_l2(y[0], ref))
