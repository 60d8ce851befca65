"""Seeded synthetic inputs for the filter-bank dataflow workloads.

This module only draws random inputs (frame side-information, complex64
samples, complex64 taps, cotangents and the fit target).  It holds none of
the method's arithmetic: control-token construction, rate decoding, FIFO
indexing and the filter bank itself live in the oracle and in the HIP
library, separately.  Both sides consume the exact bytes produced here.

Draw order (fixed, so a workload is reproducible from its seed):
``SeedSequence(seed).spawn(4)`` gives PCG64 generators for
(ctrl, taps, x, noise).

* ctrl: per stream, per frame, the varying fields in the order
  K, then n, then bank, then route.
* taps: per stream, per bank, real parts then imaginary parts of a
  (Kmax, L_bank) standard-normal array; branch b (1-based) is divided by
  b*L_bank (complex N(0,1) scaled by 1/(k*L)).
* x: the real parts of all samples, then the imaginary parts, N(0, 0.3^2).
* noise: cotangents / fit noise.

Side-information record per frame: uint32 [K, n, bank, route]; route 0
sends the frame through the filter bank, route 1 through the passthrough
branch of a switch/select pair.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = ["Workload", "SPECS", "make", "scaled"]


@dataclasses.dataclass(frozen=True)
class Spec:
    name: str
    n_streams: int
    frames_per_stream: int
    frame_len: int            # fixed frame length (0 -> log-uniform draw)
    n_min: int                # log-uniform bounds when frame_len == 0
    n_max: int
    Kmax: int                 # branches per bank
    K_fixed: int              # 0 -> K ~ U{1..Kmax}
    bank_L: tuple             # taps per branch for each bank
    pass_prob: float          # probability a frame is routed to passthrough
    description: str
    K_min: int = 1            # K ~ U{K_min..Kmax} when K_fixed == 0


SPECS = {
    # Plain graph src -> control -> filter bank -> sink (parity size).
    "C1": Spec("C1", 1, 64, 1024, 0, 0, 4, 0, (8,), 0.0,
               "64 frames x 1024 complex64, K~U{1..4}, L=8"),
    # Plain single-stream graph at scale.
    "C2": Spec("C2", 1, 4096, 16384, 0, 0, 10, 0, (32,), 0.0,
               "4096 frames x 16384 complex64, K~U{1..10}, L=32"),
    # Batched uneven frames over three tap banks.
    "C3": Spec("C3", 1, 2048, 0, 256, 65536, 10, 0, (8, 16, 32), 0.0,
               "2048 frames, n log-uniform [256,65536], K~U{1..10}, L in {8,16,32}"),
    # Differentiation / fit workload.
    "C4": Spec("C4", 1, 256, 8192, 0, 0, 8, 8, (16,), 0.0,
               "256 frames x 8192, K=8, L=16, amplifier-fit target"),
    # Wide multi-stream graph with passthrough routing.
    "C5": Spec("C5", 64, 16, 32768, 0, 0, 7, 7, (64,), 0.3,
               "64 streams x 16 frames x 32768, K=7, L=64, ~30% passthrough"),
    # The shape of the paper's DPD run (Sec. VII-A/C): ten 10-tap branches,
    # a reconfiguration every 65536 samples with 2..10 active branches (the
    # distribution is not given: uniform here), 2^26 samples in all.
    "P": Spec("P", 1, 1024, 65536, 0, 0, 10, 0, (10,), 0.0,
              "1024 frames x 65536 complex64, K~U{2..10}, L=10 (the paper's DPD shape)", K_min=2),
}


@dataclasses.dataclass
class Workload:
    spec: Spec
    side: np.ndarray      # uint32 [S, F, 4]: K, n, bank, route
    x: np.ndarray         # complex64 [S, N]: concatenated frames of each stream
    taps: np.ndarray      # complex64 [S, n_banks, Kmax, Lmax], zero beyond L_bank
    gy: Optional[np.ndarray] = None       # complex64 [S, N] cotangent
    target: Optional[np.ndarray] = None   # complex64 [S, N] fit target (C4)

    @property
    def n_streams(self):
        return self.side.shape[0]

    @property
    def n_frames(self):
        return self.side.shape[1]

    @property
    def Kmax(self):
        return self.spec.Kmax

    @property
    def bank_L(self):
        return self.spec.bank_L

    @property
    def Lmax(self):
        return max(self.spec.bank_L)

    def frame_offsets(self, s=0):
        n = self.side[s, :, 1].astype(np.int64)
        return np.concatenate([[0], np.cumsum(n)])

    @property
    def total_samples(self):
        return int(self.side[:, :, 1].astype(np.int64).sum())


def _draw_side(spec: Spec, g: np.random.Generator, S: int, F: int,
               frame_len: int) -> np.ndarray:
    side = np.zeros((S, F, 4), dtype=np.uint32)
    lo, hi = math.log(spec.n_min or 1), math.log(spec.n_max or 1)
    for s in range(S):
        for f in range(F):
            K = spec.K_fixed if spec.K_fixed else int(g.integers(spec.K_min, spec.Kmax + 1))
            if spec.frame_len == 0 and frame_len == 0:
                n = int(np.rint(math.exp(g.uniform(lo, hi))))
                n = min(max(n, spec.n_min), spec.n_max)
            else:
                n = frame_len or spec.frame_len
            bank = int(g.integers(0, len(spec.bank_L))) if len(spec.bank_L) > 1 else 0
            route = int(g.random() < spec.pass_prob) if spec.pass_prob > 0 else 0
            side[s, f] = (K, n, bank, route)
    return side


def _draw_taps(spec: Spec, g: np.random.Generator, S: int) -> np.ndarray:
    Lmax = max(spec.bank_L)
    taps = np.zeros((S, len(spec.bank_L), spec.Kmax, Lmax), dtype=np.complex64)
    for s in range(S):
        for j, L in enumerate(spec.bank_L):
            re = g.normal(0.0, 1.0, (spec.Kmax, L))
            im = g.normal(0.0, 1.0, (spec.Kmax, L))
            scale = (np.arange(1, spec.Kmax + 1, dtype=np.float64) * L)[:, None]
            taps[s, j, :, :L] = ((re + 1j * im) / scale).astype(np.complex64)
    return taps


def _draw_complex(g: np.random.Generator, shape, sigma: float) -> np.ndarray:
    n = int(np.prod(shape))
    re = g.normal(0.0, sigma, n)
    im = g.normal(0.0, sigma, n)
    return (re + 1j * im).astype(np.complex64).reshape(shape)


def make(name: str, seed: int = 0, n_frames: Optional[int] = None,
         frame_len: int = 0, n_streams: Optional[int] = None,
         cotangent: bool = False, n_max: Optional[int] = None) -> Workload:
    """Draw a workload.  ``n_frames``/``frame_len``/``n_streams``/``n_max``
    shrink it for parity tests while keeping the recipe (the draws of the
    shrunk workload are a different sequence, not a prefix)."""
    spec = SPECS[name]
    if n_max is not None:
        spec = dataclasses.replace(spec, n_max=n_max, n_min=min(spec.n_min, n_max))
    S = n_streams or spec.n_streams
    F = n_frames or spec.frames_per_stream
    g_ctrl, g_taps, g_x, g_noise = [np.random.Generator(np.random.PCG64(s))
                                    for s in np.random.SeedSequence(seed).spawn(4)]
    side = _draw_side(spec, g_ctrl, S, F, frame_len)
    taps = _draw_taps(spec, g_taps, S)
    N = int(side[:, :, 1].astype(np.int64).sum(axis=1).max())
    lens = side[:, :, 1].astype(np.int64).sum(axis=1)
    assert np.all(lens == N), "every stream carries the same number of samples"
    x = _draw_complex(g_x, (S, N), 0.3)
    wl = Workload(spec, side, x, taps)
    if name == "C4":
        wl.target = amplifier_target(x, g_noise)
    if cotangent:
        wl.gy = _draw_complex(g_noise, (S, N), 1.0)
    return wl


def amplifier_target(x: np.ndarray, g_noise: np.random.Generator,
                     noise_sigma: float = 0.01) -> np.ndarray:
    """Synthetic power-amplifier output the C4 fit regresses onto:
    x*(1 - 0.15|x|^2 + 0.02|x|^4) plus complex noise with per-component
    variance 1e-4.  Computed in float64, stored as complex64."""
    xd = x.astype(np.complex128)
    a2 = xd.real ** 2 + xd.imag ** 2
    y = xd * (1.0 - 0.15 * a2 + 0.02 * a2 * a2)
    if noise_sigma > 0:
        y = y + _draw_complex(g_noise, x.shape, noise_sigma).astype(np.complex128)
    return y.astype(np.complex64)


def scaled(name: str, seed: int = 0, **kw) -> Workload:
    """Small parity-size variants of each workload (same recipe)."""
    small = {
        "C1": dict(),
        "C2": dict(n_frames=12, frame_len=3000),
        "C3": dict(n_frames=24, n_max=6000),
        "C4": dict(n_frames=6, frame_len=1500),
        "C5": dict(n_streams=3, n_frames=5, frame_len=1200),
        "P": dict(n_frames=6, frame_len=2500),
    }[name]
    small.update(kw)
    return make(name, seed=seed, **small)


def make_video(n_frames: int, width: int = 1920, height: int = 1080, seed: int = 0,
               n_objects: int = 4) -> np.ndarray:
    """Synthetic 8-bit grayscale video standing in for the 1080p sequence
    of the paper's Motion Detection run: a static textured background (a
    sum of a few random planar cosines), bright or dark rectangles moving
    at constant random velocities, and per-frame Gaussian noise (sigma 3).
    Returns uint8 [n_frames, height, width].  Draw order: background
    waves, then objects (size, position, velocity, level), then noise per
    frame."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed + 1000)))
    yy, xx = np.mgrid[0:height, 0:width].astype(np.float32)
    bg = np.full((height, width), 120.0, np.float32)
    for _ in range(3):
        fx, fy = g.uniform(0.002, 0.02, size=2)
        ph = g.uniform(0, 2 * np.pi)
        bg += g.uniform(10, 30) * np.cos(2 * np.pi * (fx * xx + fy * yy) + ph).astype(np.float32)
    objs = []
    for _ in range(n_objects):
        w = int(g.integers(width // 20, width // 6))
        h = int(g.integers(height // 20, height // 6))
        x0 = float(g.uniform(0, width - w))
        y0 = float(g.uniform(0, height - h))
        vx, vy = g.uniform(-12, 12, size=2)
        level = float(g.choice([-1.0, 1.0]) * g.uniform(40, 80))
        objs.append((w, h, x0, y0, vx, vy, level))
    out = np.empty((n_frames, height, width), np.uint8)
    for f in range(n_frames):
        fr = bg.copy()
        for (w, h, x0, y0, vx, vy, level) in objs:
            x = int(round(x0 + vx * f)) % (width - w)
            y = int(round(y0 + vy * f)) % (height - h)
            fr[y:y + h, x:x + w] += level
        fr += g.normal(0.0, 3.0, size=fr.shape).astype(np.float32)
        out[f] = np.clip(np.rint(fr), 0, 255).astype(np.uint8)
    return out
