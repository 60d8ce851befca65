"""Pins of the oracle's model of computation against what the paper fixes."""
import itertools
import json
import os

import numpy as np
import pytest

import synth
import stopcases
from oracle import moc
from oracle.moc import (Graph, PruneError, IN, OUT, SRP, DRP, CPORT, SOURCE, CONFIG,
                        FILTERBANK, SWITCH, SELECT, PASSTHROUGH, SINK)
from oracle import graphs

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- Eq. 2 / Fig. 6
def test_fig6_worked_example():
    g = _gold("fig6_fifo.json")
    r, Q, C = g["r"], g["Q"], g["C"]
    assert moc.fifo_capacity(r, Q, C) == g["capacity_tokens"]
    f = moc.FifoState(0, r, Q, C, np.float64, False)
    # Delay token D sits in slot 0: mark it.
    f.buf[g["delay_slot"]] = -1.0
    seq = 0
    for j, slots in enumerate(g["write_slots"][:3]):
        assert f.can_write()
        data = np.arange(seq, seq + r, dtype=np.float64) + 100
        seq += r
        f.write(data, j)
        assert list(range(f.log_w[-1][2], f.log_w[-1][2] + r)) == slots
        if j == g["copy_back_after_write"]:
            # slot 12 copied to slot 0
            assert f.buf[g["copy_back"]["to"][0]] == f.buf[g["copy_back"]["from"][0]]
        if j == 0:
            out = f.read(0)
            assert list(range(f.log_r[-1][2], f.log_r[-1][2] + r)) == g["read_slots"][0]
            assert out[0] == -1.0           # the delay token comes out first
    assert [moc.fifo_write_slot(r, Q, C, j) for j in range(4)] == [s[0] for s in g["write_slots"]]
    assert [moc.fifo_read_slot(r, Q, C, i) for i in range(4)] == [s[0] for s in g["read_slots"]]


@pytest.mark.parametrize("r,Q,C", [(4, 0, 3), (4, 8, 3), (4, 16, 3), (4, 1, 3), (4, 5, 2),
                                   (3, 2, 2), (1, 0, 1), (7, 3, 1), (4, 12, 3), (5, 13, 3)])
def test_eq2_closed_form(r, Q, C):
    expect = r * C + Q if Q % r else max(r * C, Q)
    assert moc.fifo_capacity(r, Q, C) == expect


@pytest.mark.parametrize("r,Q,C", [(4, 1, 3), (4, 0, 3), (4, 8, 3), (3, 2, 2), (5, 3, 3),
                                   (4, 12, 2), (2, 1, 1), (6, 6, 2), (4, 16, 3)])
def test_fifo_preserves_order_with_delay(r, Q, C):
    """Any interleaving the blocking rules allow delivers Q zeros then the
    written stream, and occupancy never exceeds Eq. 2's capacity."""
    if Q % r and (Q >= r * C or (Q < r and Q + r > r * C)):
        with pytest.raises(PruneError):
            moc.FifoState(0, r, Q, C, np.float64, False)
        return
    rng = np.random.default_rng(r * 100 + Q * 10 + C)
    f = moc.FifoState(0, r, Q, C, np.float64, False)
    n_blocks = 40
    stream = rng.standard_normal(n_blocks * r)
    out = []
    w = 0
    while len(out) < (n_blocks * r + Q) // r * r and (w < n_blocks or f.can_read()):
        choices = []
        if w < n_blocks and f.can_write():
            choices.append("w")
        if f.can_read():
            choices.append("r")
        if not choices:
            break
        c = choices[rng.integers(len(choices))]
        if c == "w":
            f.write(stream[w * r:(w + 1) * r], w)
            w += 1
        else:
            out.extend(f.read(0))
        assert f.occupancy <= f.capacity
    expect = np.concatenate([np.zeros(Q), stream])[:len(out)]
    assert len(out) >= n_blocks * r - r * C
    np.testing.assert_array_equal(np.array(out), expect)


def test_unaligned_delay_rejected():
    with pytest.raises(PruneError) as e:
        moc.FifoState(0, 4, 13, 3, np.float64, False)
    assert e.value.code == moc.E_DELAY


# ---------------------------------------------------------------- Eq. 1 / table
def _fig1_graph(tokens, n_src):
    """Fig. 1 shape: dynamic actor x with control port p1 (rate 1), DRP input
    p2 (atr 1, itr 0) and an SRP output p3."""
    g = Graph()
    src = g.actor(SOURCE)
    cfg = g.actor(CONFIG, mode="route", n_elements=3)
    x = g.actor(SELECT)
    snk = g.actor(SINK)
    ps = g.port(src, OUT, SRP, 1)
    pc = g.port(cfg, OUT, SRP, 1)
    p1 = g.port(x, IN, CPORT, 1)
    p2 = g.port(x, IN, DRP, 1)
    p3 = g.port(x, OUT, SRP, 1)
    pk = g.port(snk, IN, SRP, 1)
    g.connect(ps, p2, 1)
    g.connect(pc, p1, 1)
    g.connect(p3, pk, 1)
    # T[pc][p2] = 3: the third element of the control value controls p2.
    g.control(pc, p2, 3)
    g.finalize(3)
    g.push(src, [np.array([1.0 + k]) for k in range(n_src)])
    g.push(cfg, [(0, 1, 0, t) for t in tokens])   # route field sets bit `t`
    return g, x, src, snk


def test_eq1_control_table_element():
    gold = _gold("control_table.json")
    # route=2 -> mask bit 2 = element 3 -> p2 active; other bits -> inactive.
    tokens = [2, 0, 2, 1, 2]
    g, x, src, snk = _fig1_graph(tokens, n_src=tokens.count(2))
    g.run()
    log = g.actors[x].log
    assert [bm for (_, _, _, bm) in log] == [1 if t == gold["element_example"]["mask_bit"] else 0
                                             for t in tokens]
    # p2 reads atr (1) tokens when active, itr (0) otherwise; p3 always writes.
    fin = g.fstate[0]
    assert fin.tokens_read == tokens.count(2) * gold["fig1"]["drp_atr"]
    out = g.sink_output(snk)
    np.testing.assert_array_equal(out.real, [1.0, 0.0, 2.0, 0.0, 3.0])


def test_eq1_rejects_elements_beyond_value():
    g = Graph()
    cfg = g.actor(CONFIG, mode="route", n_elements=2)
    src = g.actor(SOURCE)
    x = g.actor(SELECT)
    pc = g.port(cfg, OUT, SRP, 1)
    ps = g.port(src, OUT, SRP, 1)
    p1 = g.port(x, IN, CPORT, 1)
    p2 = g.port(x, IN, DRP, 1)
    p3 = g.port(x, OUT, SRP, 1)
    snk = g.actor(SINK)
    pk = g.port(snk, IN, SRP, 1)
    g.connect(ps, p2, 1); g.connect(pc, p1, 1); g.connect(p3, pk, 1)
    g.control(pc, p2, 1)
    g.finalize(2)
    g.push(cfg, [(0, 1, 0, 5)])     # bit 5 beyond a 2-element control value
    g.push(src, [np.array([1.0])])
    with pytest.raises(PruneError) as e:
        g.run()
    assert e.value.code == moc.E_TOKEN


# ---------------------------------------------------------------- validation
def _mini(kind_mid=PASSTHROUGH, rates=(4, 4, 4, 4), C=3, delay=0):
    g = Graph()
    src = g.actor(SOURCE); mid = g.actor(kind_mid); snk = g.actor(SINK)
    a = g.port(src, OUT, SRP, rates[0]); b = g.port(mid, IN, SRP, rates[1])
    c = g.port(mid, OUT, SRP, rates[2]); d = g.port(snk, IN, SRP, rates[3])
    g.connect(a, b, rates[0], delay); g.connect(c, d, rates[2])
    return g


def test_validation_rate_mismatch():
    g = _mini(rates=(4, 3, 4, 4))
    with pytest.raises(PruneError) as e:
        g.finalize(3)
    assert e.value.code == moc.E_RATE_MISMATCH


def test_validation_control_port_rate():
    g = Graph()
    cfg = g.actor(CONFIG)
    x = g.actor(SWITCH)
    pc = g.port(cfg, OUT, SRP, 1)
    p1 = g.port(x, IN, CPORT, 2)
    with pytest.raises(PruneError) as e:
        g.connect(pc, p1, 1)
        g.finalize(3)
    assert e.value.code in (moc.E_PORT_KIND, moc.E_RATE_MISMATCH, moc.E_CONNECT)


def test_validation_drp_on_static_actor():
    g = Graph()
    src = g.actor(SOURCE); mid = g.actor(PASSTHROUGH); snk = g.actor(SINK)
    a = g.port(src, OUT, SRP, 4); b = g.port(mid, IN, DRP, 4)
    c = g.port(mid, OUT, SRP, 4); d = g.port(snk, IN, SRP, 4)
    g.connect(a, b, 4); g.connect(c, d, 4)
    with pytest.raises(PruneError) as e:
        g.finalize(3)
    assert e.value.code == moc.E_PORT_KIND


def test_validation_rule4():
    g = Graph()
    cfg = g.actor(CONFIG, n_elements=2)
    src = g.actor(SOURCE)
    x = g.actor(SELECT)
    snk = g.actor(SINK)
    pc = g.port(cfg, OUT, SRP, 1)
    ps = g.port(src, OUT, SRP, 4)
    p1 = g.port(x, IN, CPORT, 1)
    p2 = g.port(x, IN, DRP, 4)
    p3 = g.port(x, OUT, DRP, 4)
    pk = g.port(snk, IN, SRP, 4)
    g.connect(pc, p1, 1); g.connect(ps, p2, 4); g.connect(p3, pk, 4)
    g.control(pc, p2, 1); g.control(pc, p3, 1)
    with pytest.raises(PruneError) as e:
        g.finalize(3)
    assert e.value.code in (moc.E_RULE4, moc.E_ARG)


def test_validation_unconnected_input():
    g = Graph()
    mid = g.actor(PASSTHROUGH)
    g.port(mid, IN, SRP, 4)
    with pytest.raises(PruneError) as e:
        g.finalize(3)
    assert e.value.code == moc.E_CONNECT


def test_validation_unaligned_delay():
    g = _mini(delay=13)
    with pytest.raises(PruneError) as e:
        g.finalize(3)
    assert e.value.code == moc.E_DELAY


def test_validation_edit_after_finalize():
    g = _mini()
    g.finalize(3)
    with pytest.raises(PruneError) as e:
        g.actor(SINK)
    assert e.value.code == moc.E_STATE


# ---------------------------------------------------------------- conservation
@pytest.mark.parametrize("C", [1, 2, 3])
def test_token_conservation_plain(C):
    wl = synth.make("C1", n_frames=12)
    y, logs, g, ids = graphs.run_plain(wl, C=C)
    fb = logs["actors"][ids["fb"]]
    masks = [m for (_, m, _, _) in fb["control"]]
    D = wl.Kmax
    for d in range(D):
        active = sum((m >> d) & 1 for m in masks)
        assert fb["branch_firings"][d] == active
        assert fb["branch_tokens"][d] == active * 1024
    for fid, f in logs["fifos"].items():
        assert f["tokens_written"] == f["tokens_read"]
        assert f["max_occ"] <= f["capacity"]
    assert logs["actors"][ids["snk"]]["tokens"] == wl.total_samples


def test_delay_fifo_in_graph():
    """A delayed channel shifts the stream by Q zeros (the z^-1 operator); at
    the end the channel holds exactly its Q initial tokens, which is a normal
    end of the run, not a deadlock."""
    r, Q = 4, 1
    g = _mini(delay=Q)
    g.finalize(3)
    data = np.arange(1, 4 * 5 + 1, dtype=np.float64)
    g.push(0, [data[i * r:(i + 1) * r] for i in range(5)])
    g.run()
    out = g.sink_output(2).real
    np.testing.assert_array_equal(out, np.concatenate([[0.0], data])[:20])
    assert g.fstate[0].occupancy == Q


# ---------------------------------------------------------------- fused == unfused
def test_fused_equals_unfused():
    wl = synth.make("C1", n_frames=10, frame_len=64)
    y_f, logs_f, gf, idf = graphs.run_plain(wl, C=3)
    g, ids = graphs.build_unfused(wl.taps[0], wl.bank_L, wl.Kmax, 64, 3)
    off = wl.frame_offsets(0)
    g.push(ids["src"], [wl.x[0, off[f]:off[f + 1]] for f in range(wl.n_frames)])
    g.push(ids["cfg"], wl.side[0])
    g.run()
    y_u = g.sink_output(ids["snk"])
    np.testing.assert_allclose(y_u, y_f, rtol=0, atol=1e-12)
    fb = logs_f["actors"][idf["fb"]]
    for b, fir in enumerate(ids["firs"]):
        assert g.actors[fir].firings == fb["branch_firings"][b]
        assert g.actors[fir].state["tokens"] == fb["branch_tokens"][b]


# ---------------------------------------------------------------- schedule independence
def _canon(logs):
    return {k: (v["writes"], v["reads"], v["tokens_written"], v["firings_w"])
            for k, v in logs["fifos"].items()}


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_schedule_independence(seed):
    wl = synth.make("C1", n_frames=8, frame_len=128)
    y0, l0, _, _ = graphs.run_plain(wl, C=3)
    y1, l1, _, _ = graphs.run_plain(wl, C=3, policy="random", rng=np.random.default_rng(seed))
    np.testing.assert_array_equal(y0, y1)
    assert _canon(l0) == _canon(l1)


def test_routed_schedule_independence():
    wl = synth.scaled("C5")
    y0, l0, _, _ = graphs.run_routed(wl, C=2)
    y1, l1, _, _ = graphs.run_routed(wl, C=2, policy="random", rng=np.random.default_rng(7))
    np.testing.assert_array_equal(y0, y1)
    assert _canon(l0) == _canon(l1)


# ---------------------------------------------------------------- decidability consequences
def _tiny_dpg(C, Q, tokens_sw, tokens_sel, n_frames, r=2):
    """Switch/select DPG with two passthrough DCs.  With one control stream
    (Rule 1/2 satisfied) it must never deadlock; with different control
    streams for x and y it deadlocks (the linked-DRP example of Sec. V)."""
    g = Graph()
    src = g.actor(SOURCE)
    q1 = g.actor(CONFIG, mode="route", n_elements=2)
    q2 = g.actor(CONFIG, mode="route", n_elements=2) if tokens_sel is not None else None
    x = g.actor(SWITCH); a1 = g.actor(PASSTHROUGH); a2 = g.actor(PASSTHROUGH)
    y = g.actor(SELECT); snk = g.actor(SINK)
    ps = g.port(src, OUT, SRP, r)
    pq1 = g.port(q1, OUT, SRP, 1)
    pq2 = g.port(q2, OUT, SRP, 1) if q2 is not None else pq1
    xc = g.port(x, IN, CPORT, 1); xi = g.port(x, IN, SRP, r)
    xo = [g.port(x, OUT, DRP, r), g.port(x, OUT, DRP, r)]
    ai = [g.port(a, IN, SRP, r) for a in (a1, a2)]
    ao = [g.port(a, OUT, SRP, r) for a in (a1, a2)]
    yc = g.port(y, IN, CPORT, 1)
    yi = [g.port(y, IN, DRP, r), g.port(y, IN, DRP, r)]
    yo = g.port(y, OUT, SRP, r)
    pk = g.port(snk, IN, SRP, r)
    g.connect(ps, xi, r, Q)
    g.connect(pq1, xc, 1)
    g.connect(pq2, yc, 1)
    for k in range(2):
        g.connect(xo[k], ai[k], r)
        g.connect(ao[k], yi[k], r)
        g.control(pq1, xo[k], k + 1)
        g.control(pq2, yi[k], k + 1)
    g.connect(yo, pk, r)
    g.finalize(C)
    g.push(src, [np.full(r, f + 1.0) for f in range(n_frames)])
    g.push(q1, [(0, r, 0, t) for t in tokens_sw])
    if q2 is not None:
        g.push(q2, [(0, r, 0, t) for t in tokens_sel])
    return g


@pytest.mark.parametrize("C", [1, 2, 3])
@pytest.mark.parametrize("Q", [0, 1])
def test_bruteforce_no_deadlock(C, Q):
    """All control sequences of length <= 4 over a valid two-DC DPG."""
    for n in range(1, 5):
        for toks in itertools.product([0, 1], repeat=n):
            g = _tiny_dpg(C, Q * 2, list(toks), None, n)
            g.run()   # raises on deadlock
            for f in g.fstate:
                assert f.max_occ <= f.capacity


def test_mismatched_control_streams_deadlock():
    g = _tiny_dpg(3, 0, [0, 0, 1, 0], [1, 1, 1, 1], 4)
    with pytest.raises(PruneError) as e:
        g.run()
    assert e.value.code == moc.E_DEADLOCK


# ---------------------------------------------------------------- end of a finite run
@pytest.mark.parametrize("name", sorted(stopcases.cases()))
def test_stop_classification(name):
    """Wait-for classification of the stop (blocking reads and writes,
    Sec. III-A; linked DRPs, Sec. V): a normal end iff every actor that cannot
    fire waits, through the FIFOs it blocks on, on external input that ran
    out."""
    d = stopcases.cases()[name]
    status, g = stopcases.run_oracle(d)
    assert status == d.expect
    for f in g.fstate:
        assert f.max_occ <= f.capacity
        assert f.occupancy == f.Q + f.tokens_written - f.tokens_read


def test_undelayed_cycle_stalls_with_input_unread():
    """THRES needs MED's previous output and MED needs THRES's: nothing fires,
    both frames stay in THRES's input FIFO, the sink gets nothing."""
    d = stopcases.thres_med_cycle(0, 2)
    status, g = stopcases.run_oracle(d)
    assert status == "deadlock"
    stuck, linked = g.stop_classification()
    assert stuck == [d.names["thres"], d.names["med"], d.names["snk"]] and linked == []
    assert g.fstate[0].occupancy == 2 * 64
    assert len(g.sink_output(d.names["snk"])) == 0


def test_delayed_cycle_runs_every_frame():
    """The one-frame delay on MED -> THRES breaks the cycle (the z^-1 of
    Sec. III-D): every frame reaches the sink and the delayed FIFO ends
    holding one frame, its delay."""
    d = stopcases.thres_med_cycle(1, 4)
    status, g = stopcases.run_oracle(d)
    assert status == "normal"
    assert len(g.sink_output(d.names["snk"])) == 4 * 64
    assert g.fstate[2].occupancy == 64


def test_mismatched_tokens_flag_the_select():
    """Sec. V: x routes its first frame to a1 while y's first token demands
    a2; x has fired the firing linked to y's, so y is reported."""
    d = stopcases.switch_select([0], [1], 1)
    status, g = stopcases.run_oracle(d)
    stuck, linked = g.stop_classification()
    assert status == "deadlock" and stuck == [] and linked == [d.names["y"]]


# ---------------------------------------------------------------- frame-split invariance
def test_frame_split_invariance():
    """With a fixed mask, re-cutting a stream into different frame lengths
    leaves the output unchanged (history carries across firings)."""
    wl = synth.make("C3", n_frames=6, n_max=700)
    x = wl.x[0]
    N = x.shape[0]
    D = len(wl.bank_L) * wl.Kmax
    outs = []
    for cuts in ([N], [100, N - 100], [37, 300, N - 337]):
        g, ids = graphs.build_plain(wl.taps[0], wl.bank_L, wl.Kmax, max(cuts), 3, param=True)
        frames, side, t = [], [], 0
        for c in cuts:
            frames.append(x[t:t + c]); side.append((10, c, 2, 0)); t += c
        g.push(ids["src"], frames)
        g.push(ids["cfg"], side)
        g.run()
        outs.append(g.sink_output(ids["snk"]))
    np.testing.assert_allclose(outs[1], outs[0], rtol=0, atol=1e-12)
    np.testing.assert_allclose(outs[2], outs[0], rtol=0, atol=1e-12)


def test_plain_graph_matches_stream_semantics():
    wl = synth.make("C3", n_frames=8, n_max=900)
    y, logs, g, ids = graphs.run_plain(wl, C=2)
    from oracle.filterbank import fb_stream
    ys = fb_stream(wl.x[0], graphs.stream_frames(wl), wl.taps[0], wl.bank_L, wl.Kmax)
    np.testing.assert_allclose(y, ys, rtol=0, atol=1e-12)


def test_routed_graph_matches_stream_semantics():
    wl = synth.scaled("C5")
    ys, logs, g, ids = graphs.run_routed(wl, C=3)
    from oracle.filterbank import fb_stream
    for s in range(wl.n_streams):
        fr = graphs.stream_frames(wl, s)
        ref = fb_stream(wl.x[s], fr, wl.taps[s], wl.bank_L, wl.Kmax)
        np.testing.assert_allclose(ys[s], ref, rtol=0, atol=1e-12)
        # passthrough frames are exact copies
        for (t0, n, m, route) in fr:
            if route:
                np.testing.assert_array_equal(ys[s][t0:t0 + n], wl.x[s, t0:t0 + n])


def test_mask_zero_outputs_zeros():
    wl = synth.make("C1", n_frames=4, frame_len=32)
    wl.side[0, :, 0] = [0, 2, 0, 1]
    y, logs, g, ids = graphs.run_plain(wl, C=3)
    assert np.all(y[:32] == 0) and np.all(y[64:96] == 0)
    assert np.any(y[32:64] != 0)


# ---------------------------------------------------------------- arbitrary branch sets
def test_mask_mode_branch_sets_add_up():
    """Configuration mode "mask": any set of branches, not only a prefix.
    The filter bank is linear in its branch set, so a frame's output under a
    set equals the sum of its outputs under each single branch, and a prefix
    set reproduces the prefix mode."""
    wl = synth.make("C1", n_frames=6, frame_len=96)
    rng = np.random.default_rng(3)
    sets = [int(v) for v in rng.integers(1, 1 << wl.Kmax, size=wl.n_frames)]
    def run(masks):
        w = synth.make("C1", n_frames=6, frame_len=96)
        w.side[0, :, 0] = masks
        y, _, _, _ = graphs.run_plain(w, C=3, cfg_mode="mask")
        return y
    y = run(sets)
    parts = sum(run([m & (1 << b) for m in sets]) for b in range(wl.Kmax))
    np.testing.assert_allclose(y, parts, rtol=0, atol=1e-12)
    pre = [(1 << k) - 1 for k in wl.side[0, :, 0]]
    y_prefix, _, _, _ = graphs.run_plain(wl, C=3)
    np.testing.assert_allclose(run(pre), y_prefix, rtol=0, atol=0)
