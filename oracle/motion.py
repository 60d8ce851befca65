"""Motion Detection actors (oracle, test infrastructure only).

Sec. VII-A describes the graph src -> Gauss -> Thres -> Med -> sink on 8-bit
grayscale 1920x1080 frames: Gauss is a 5x5 Gaussian filter that skips the
two pixel rows at the top and at the bottom of the frame; Thres subtracts
consecutive frames (the previous one arrives through a FIFO with a
one-frame delay) and compares with a fixed constant; Med is a 5-pixel
median filter.

Readings where the paper is silent (each is listed with its reason in the
design notes):
* Gauss weights: the binomial 5-tap kernel [1 4 6 4 1] in both directions,
  integer sum rounded: (sum w_y w_x p + 128) >> 8.  Rows 2..H-3 are
  filtered; the two rows at each end are copied.  Columns beyond the frame
  edge repeat the edge pixel.
* Thres: 255 where |cur - prev| > T, else 0, with T = 20.  The delay token
  (the "previous" frame of the first firing) is a zero frame.
* Med: the median of the pixel and its four neighbours (up, down, left,
  right); rows 0 and H-1 are copied; columns beyond the edge repeat it.

Parity: pinned by tests/test_oracle_motion.py (constant frames, the
impulse response against the binomial kernel, border rows, edge columns,
threshold semantics, outlier removal, the median against numpy's median,
and the graph against the direct composition of the three filters).
"""
from __future__ import annotations

import numpy as np

GAUSS_W = np.array([1, 4, 6, 4, 1], dtype=np.int64)
THRESHOLD = 20


def _clamped_cols(W, dx):
    return np.clip(np.arange(W) + dx, 0, W - 1)


def gauss5(frame: np.ndarray) -> np.ndarray:
    f = np.asarray(frame, dtype=np.int64)
    H, W = f.shape
    out = f.copy()
    if H >= 5:
        acc = np.zeros((H - 4, W), dtype=np.int64)
        for dy in range(-2, 3):
            rows = f[2 + dy:H - 2 + dy]
            for dx in range(-2, 3):
                acc += GAUSS_W[dy + 2] * GAUSS_W[dx + 2] * rows[:, _clamped_cols(W, dx)]
        out[2:H - 2] = (acc + 128) >> 8
    return out.astype(np.uint8)


def thres(cur: np.ndarray, prev: np.ndarray, T: int = THRESHOLD) -> np.ndarray:
    d = np.abs(np.asarray(cur, np.int64) - np.asarray(prev, np.int64))
    return np.where(d > T, 255, 0).astype(np.uint8)


def med5(frame: np.ndarray) -> np.ndarray:
    f = np.asarray(frame, dtype=np.int64)
    H, W = f.shape
    out = f.copy()
    if H >= 3:
        mid = f[1:H - 1]
        stack = np.stack([mid, f[0:H - 2], f[2:H], mid[:, _clamped_cols(W, -1)],
                          mid[:, _clamped_cols(W, 1)]])
        out[1:H - 1] = np.median(stack, axis=0).astype(np.int64)
    return out.astype(np.uint8)


def motion_stream(frames: np.ndarray, T: int = THRESHOLD) -> np.ndarray:
    """The graph's output for a frame sequence, composed directly:
    med5(thres(gauss5(f_k), gauss5(f_{k-1}))) with a zero frame before f_0."""
    out = np.empty_like(frames)
    prev = np.zeros(frames.shape[1:], np.uint8)
    for k, fr in enumerate(frames):
        g = gauss5(fr)
        out[k] = med5(thres(g, prev, T))
        prev = g
    return out
