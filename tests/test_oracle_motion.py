"""Pins of the oracle's Motion Detection actors (Sec. VII-A) against
closed forms, special cases and the direct composition of the filters."""
import numpy as np
import pytest

import synth
from oracle import graphs
from oracle import motion as mo
from oracle import moc


def test_gauss_constant_and_impulse():
    f = np.full((9, 11), 77, np.uint8)
    assert np.array_equal(mo.gauss5(f), f)          # weights sum to 256
    f = np.zeros((9, 11), np.uint8)
    f[4, 5] = 256 - 1
    g = mo.gauss5(f).astype(np.int64)
    w = np.outer([1, 4, 6, 4, 1], [1, 4, 6, 4, 1])
    expect = (w * 255 + 128) >> 8                    # the binomial kernel, rounded
    assert np.array_equal(g[2:7, 3:8], expect)
    assert g.sum() == expect.sum()


def test_gauss_border_rows_and_edge_columns():
    rng = np.random.default_rng(0)
    f = rng.integers(0, 256, size=(8, 6), dtype=np.uint8)
    g = mo.gauss5(f)
    assert np.array_equal(g[:2], f[:2]) and np.array_equal(g[-2:], f[-2:])
    # a frame constant along each row is left unchanged horizontally, so
    # edge replication makes column 0 equal column 3
    rows = np.repeat(rng.integers(0, 256, size=(8, 1)), 6, axis=1).astype(np.uint8)
    gr = mo.gauss5(rows)
    assert np.all(gr == gr[:, :1])
    # brute force at one interior pixel next to the left edge
    y, x = 4, 0
    acc = sum(int(a) * int(b) * int(f[y + dy, min(max(x + dx, 0), 5)])
              for dy, a in zip(range(-2, 3), [1, 4, 6, 4, 1])
              for dx, b in zip(range(-2, 3), [1, 4, 6, 4, 1]))
    assert g[y, x] == (acc + 128) >> 8


def test_threshold():
    a = np.array([[0, 10, 200, 100]], np.uint8)
    b = np.array([[21, 31, 179, 100]], np.uint8)
    assert mo.thres(a, b, 20).tolist() == [[255, 255, 255, 0]]
    assert np.array_equal(mo.thres(a, b), mo.thres(b, a))


def test_median_cross():
    f = np.full((7, 7), 50, np.uint8)
    f[3, 3] = 255                                    # isolated outlier
    assert np.array_equal(mo.med5(f), np.full((7, 7), 50, np.uint8))
    rng = np.random.default_rng(1)
    f = rng.integers(0, 256, size=(6, 5), dtype=np.uint8)
    m = mo.med5(f)
    for y in range(1, 5):
        for x in range(5):
            vals = [f[y, x], f[y - 1, x], f[y + 1, x], f[y, max(x - 1, 0)], f[y, min(x + 1, 4)]]
            assert m[y, x] == int(np.median(vals))
    assert np.array_equal(m[0], f[0]) and np.array_equal(m[-1], f[-1])


@pytest.mark.parametrize("C", [2, 3])
def test_motion_graph_equals_composition(C):
    """The graph with its one-frame delay FIFO equals the direct composition;
    the first frame is compared with the zero delay token."""
    v = synth.make_video(5, width=40, height=24)
    maps, logs, g, ids = graphs.run_motion(v, C=C)
    assert np.array_equal(maps, mo.motion_stream(v))
    first = mo.med5(mo.thres(mo.gauss5(v[0]), np.zeros_like(v[0])))
    assert np.array_equal(maps[0], first)
    # the delayed FIFO ends holding one frame: the last Gauss output
    delayed = [f for f, (s, d, r, q) in enumerate(g.fifos) if q][0]
    st = logs["fifos"][delayed]
    assert st["tokens_written"] - st["tokens_read"] == 0 and st["capacity"] >= 24 * 40


def test_moving_object_is_detected():
    v = synth.make_video(3, width=320, height=180)
    maps = mo.motion_stream(v)
    # frame 0 sees everything (difference with zeros); later frames see the
    # moving objects only: a small, nonzero fraction of the pixels
    frac = (maps[1:] == 255).mean()
    assert 0.001 < frac < 0.3


def test_motion_graph_analysis():
    """Static graph with a delay: consistent, and the delayed FIFO's buffer
    bound is two frames (the delay token plus the frame written before the
    difference reads)."""
    from oracle import analysis as an
    g, ids = graphs.build_motion(16, 8, 2)
    rep = an.analyze(g)
    assert rep["violations"] == [] and rep["dpgs"] == []
    delayed = [f for f, (s, d, r, q) in enumerate(g.fifos) if q][0]
    assert rep["beta"][delayed] == 2 * 16 * 8
