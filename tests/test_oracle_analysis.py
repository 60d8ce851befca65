"""Pins of the oracle's compile-time analysis against what the paper fixes:
the Sec. V example, the rule illustrations of Sec. IV, the deadlock that
mismatched control elements cause in the executor, liveness of cycles
(textbook SDF: a period with unit repetitions completes iff every directed
cycle holds a FIFO with at least one firing's worth of initial tokens) and
the paper's unfused DPD graph."""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import analysis as an
from oracle import graphs, moc
from oracle.moc import (Graph, PruneError, IN, OUT, SRP, DRP, CPORT, SOURCE, CONFIG,
                        SWITCH, SELECT, PASSTHROUGH, SINK)

GOLD = os.path.join(os.path.dirname(__file__), "golden")


class B:
    """Small named-graph builder over the oracle's Graph."""

    def __init__(self):
        self.g = Graph()
        self.a, self.p, self.f = {}, {}, {}
        self.qport = {}

    def act(self, name, kind, **kw):
        self.a[name] = self.g.actor(kind, **kw)
        return self.a[name]

    def link(self, src, dst, ks=SRP, kd=SRP, r=4, delay=0, ps=None, pd=None, name=None):
        a = self.g.port(self.a[src], OUT, ks, r) if ps is None or ps not in self.p else self.p[ps]
        b = self.g.port(self.a[dst], IN, kd, r)
        if ps is not None:
            self.p[ps] = a
        if pd is not None:
            self.p[pd] = b
        f = self.g.connect(a, b, r, delay)
        if name:
            self.f[name] = f
        return f

    def ctl(self, q, x, delay=0, name=None):
        if q not in self.qport:
            self.qport[q] = self.g.port(self.a[q], OUT, SRP, 1)
        c = self.g.port(self.a[x], IN, CPORT, 1)
        f = self.g.connect(self.qport[q], c, 1, delay)
        if name:
            self.f[name] = f
        return f

    def T(self, q, drp, e):
        self.g.control(self.qport[q], self.p[drp], e)

    def codes(self):
        return {v[0] for v in an.analyze(self.g)["violations"]}


def _dpg(el_y=(1, 2), two_q=False, r=2, Q=0):
    """src -> x (switch) -> {a1, a2} -> y (select) -> snk; q -> x, y."""
    b = B()
    b.act("src", SOURCE); b.act("q", CONFIG, mode="route", n_elements=2)
    if two_q:
        b.act("q2", CONFIG, mode="route", n_elements=2)
    b.act("x", SWITCH); b.act("a1", PASSTHROUGH); b.act("a2", PASSTHROUGH)
    b.act("y", SELECT); b.act("snk", SINK)
    b.link("src", "x", r=r, delay=Q)
    b.ctl("q", "x")
    b.ctl("q2" if two_q else "q", "y")
    for k, a in enumerate(("a1", "a2")):
        b.link("x", a, ks=DRP, r=r, ps=f"px{k + 1}")
        b.link(a, "y", kd=DRP, r=r, pd=f"py{k + 1}")
    b.link("y", "snk", r=r)
    for k in range(2):
        b.T("q", f"px{k + 1}", k + 1)
        b.T("q2" if two_q else "q", f"py{k + 1}", el_y[k])
    return b


# ---------------------------------------------------------------- Sec. V example
def _sec5():
    b = B()
    for n, k in (("src", SOURCE), ("q", CONFIG), ("x", SWITCH), ("a1", PASSTHROUGH),
                 ("a2", PASSTHROUGH), ("a3", PASSTHROUGH), ("a4", PASSTHROUGH),
                 ("y", SELECT), ("snk", SINK)):
        b.act(n, k, **({"mode": "route", "n_elements": 3} if k == CONFIG else {}))
    b.link("src", "x")
    b.ctl("q", "x"); b.ctl("q", "y")
    b.link("x", "a1", ks=DRP, ps="px1")
    b.link("x", "a2", ks=DRP, ps="px2")
    b.link("a1", "a3"); b.link("a2", "a3")
    b.link("a3", "y", kd=DRP, pd="py1")
    b.link("x", "a4", ks=DRP, ps="px3")
    b.link("a4", "y", kd=DRP, pd="py2")
    b.link("x", "y", ks=DRP, kd=DRP, ps="px4", pd="py3", name="direct")
    b.link("y", "snk")
    for p, e in (("px1", 1), ("px2", 1), ("py1", 1), ("px3", 2), ("py2", 2), ("px4", 3), ("py3", 3)):
        b.T("q", p, e)
    return b


def test_sec5_example_linked_drps_and_dcs():
    gold = json.load(open(os.path.join(GOLD, "sec5_dc_example.json")))
    b = _sec5()
    rep = an.analyze(b.g)
    name_of_port = {v: k for k, v in b.p.items()}
    name_of_actor = {v: k for k, v in b.a.items()}
    linked = sorted(tuple(sorted((name_of_port[p], name_of_port[p2]))) for p, p2 in rep["linked"])
    assert linked == sorted(tuple(x) for x in gold["linked"])
    assert rep["violations"] == []
    assert rep["dpgs"] == [(b.a["q"], b.a["x"], b.a["y"], b.qport["q"])]
    dcs = []
    for (dpg, el, acts, f) in rep["dcs"]:
        assert dpg == 0
        dcs.append(sorted(name_of_actor[a] for a in acts) if acts else (["d"] if f == b.f["direct"] else None))
    assert dcs == gold["dcs"]
    assert len(rep["dcs"]) == gold["M"]
    # one element per DC, the elements the control table gives
    assert [el for (_, el, _, _) in rep["dcs"]] == [1, 2, 3]
    for a in ("a1", "a2", "a3"):
        assert rep["dc_of_actor"][b.a[a]] == 0
    assert rep["dc_of_actor"][b.a["a4"]] == 1
    # zero delays on an acyclic graph: every FIFO holds one firing's tokens at most
    assert rep["beta"] == [b.g.fifos[f][2] for f in range(len(b.g.fifos))]


# ---------------------------------------------------------------- Sec. IV rule illustrations
def test_rule1_linked_port_control():
    assert _dpg().codes() == set()
    b = _dpg(el_y=(2, 1))
    assert (an.RULE1, b.p["px1"], b.p["py1"]) in an.analyze(b.g)["violations"]
    # x and y controlled by different control output ports
    assert an.RULE1 in _dpg(two_q=True).codes()


def test_rule2_balanced_delay():
    for dx, dy, bad in ((0, 1, True), (1, 1, False), (2, 0, True)):
        b = B()
        b.act("src", SOURCE); b.act("q", CONFIG, n_elements=1); b.act("x", SWITCH)
        b.act("a", PASSTHROUGH); b.act("y", SELECT); b.act("snk", SINK)
        b.link("src", "x"); b.ctl("q", "x", delay=dx); b.ctl("q", "y", delay=dy)
        b.link("x", "a", ks=DRP, ps="px"); b.link("a", "y", kd=DRP, pd="py"); b.link("y", "snk")
        b.T("q", "px", 1); b.T("q", "py", 1)
        v = an.analyze(b.g)["violations"]
        assert ((an.RULE2, b.a["x"], b.a["y"]) in v) == bad


def test_rule3_connecting_subchain():
    # (c) of the figure: a2 lies on subchains of (x, y) and of (z, y)
    b = B()
    b.act("src", SOURCE); b.act("src2", SOURCE); b.act("q", CONFIG, n_elements=1)
    b.act("x", SWITCH); b.act("z", SWITCH); b.act("a1", PASSTHROUGH); b.act("a2", PASSTHROUGH)
    b.act("y", SELECT); b.act("snk", SINK)
    b.link("src", "x"); b.link("src2", "z")
    b.ctl("q", "x"); b.ctl("q", "z"); b.ctl("q", "y")
    b.link("x", "a1", ks=DRP, ps="px"); b.link("a1", "a2"); b.link("z", "a2", ks=DRP, ps="pz")
    b.link("a2", "y", kd=DRP, pd="py"); b.link("y", "snk")
    for p in ("px", "pz", "py"):
        b.T("q", p, 1)
    v = an.analyze(b.g)["violations"]
    assert (an.RULE3_SHARED, b.a["a2"], -1) in v
    # (1): a dynamic actor inside a connecting subchain
    b = B()
    b.act("src", SOURCE); b.act("q", CONFIG, n_elements=2); b.act("x", SWITCH)
    b.act("a1", PASSTHROUGH); b.act("w", SWITCH); b.act("y", SELECT); b.act("snk", SINK)
    b.act("snk2", SINK)
    b.link("src", "x"); b.ctl("q", "x"); b.ctl("q", "y"); b.ctl("q", "w")
    b.link("x", "a1", ks=DRP, ps="px"); b.link("a1", "w"); b.link("w", "y", kd=DRP, pd="py")
    b.link("w", "snk2", ks=DRP, ps="pw"); b.link("y", "snk")
    b.T("q", "px", 1); b.T("q", "py", 1); b.T("q", "pw", 2)
    assert (an.RULE3_KIND, b.a["w"], -1) in an.analyze(b.g)["violations"]


def test_rule4_single_sided_dynamism():
    b = B()
    b.act("src", SOURCE); b.act("q", CONFIG, n_elements=1); b.act("x", SELECT); b.act("snk", SINK)
    b.link("src", "x", kd=DRP, pd="pi"); b.ctl("q", "x"); b.link("x", "snk", ks=DRP, ps="po")
    b.T("q", "pi", 1); b.T("q", "po", 1)
    assert (an.RULE4, b.a["x"], -1) in an.analyze(b.g)["violations"]


def test_rule5_encapsulation():
    def build(b_on_chain):
        b = B()
        b.act("src", SOURCE); b.act("q", CONFIG, n_elements=1); b.act("x", SWITCH)
        b.act("a1", PASSTHROUGH); b.act("a2", PASSTHROUGH); b.act("y", SELECT); b.act("snk", SINK)
        b.act("b", PASSTHROUGH if b_on_chain else SOURCE)
        b.link("src", "x"); b.ctl("q", "x"); b.ctl("q", "y")
        b.link("x", "a1", ks=DRP, ps="px"); b.link("a1", "a2"); b.link("a2", "y", kd=DRP, pd="py")
        if b_on_chain:
            b.link("a1", "b"); b.link("b", "a2")
        else:
            b.link("b", "a2")          # b feeds a2 through its SRP, off every x-y chain
        b.link("y", "snk")
        b.T("q", "px", 1); b.T("q", "py", 1)
        return b
    b = build(False)
    assert (an.RULE5, b.a["b"], -1) in an.analyze(b.g)["violations"]
    assert an.RULE5 not in build(True).codes()


# ---------------------------------------------------------------- DPG validity, pairing
def test_dpg_validity_and_pairing():
    # (a): a DC attached to x only
    b = B()
    b.act("src", SOURCE); b.act("q", CONFIG, n_elements=2); b.act("x", SWITCH)
    b.act("a1", PASSTHROUGH); b.act("a2", PASSTHROUGH); b.act("y", SELECT); b.act("snk", SINK)
    b.act("snk2", SINK)
    b.link("src", "x"); b.ctl("q", "x"); b.ctl("q", "y")
    b.link("x", "a1", ks=DRP, ps="px1"); b.link("a1", "y", kd=DRP, pd="py1")
    b.link("x", "a2", ks=DRP, ps="px2"); b.link("a2", "snk2")
    b.link("y", "snk")
    b.T("q", "px1", 1); b.T("q", "py1", 1); b.T("q", "px2", 2)
    assert an.DPG_A in b.codes()
    # (c): an SRP of x feeding a DC actor
    b = _dpg()
    b.link("x", "a1")
    assert an.DPG_C in b.codes()
    # a lone dynamic actor is in no DPG
    b = B()
    b.act("src", SOURCE); b.act("q", CONFIG, n_elements=1); b.act("x", SWITCH); b.act("snk", SINK)
    b.link("src", "x"); b.ctl("q", "x"); b.link("x", "snk", ks=DRP, ps="px"); b.T("q", "px", 1)
    assert (an.UNPAIRED, b.a["x"], -1) in an.analyze(b.g)["violations"]
    # x linked to two different y
    b = _dpg()
    b.act("y2", SELECT); b.act("a3", PASSTHROUGH); b.act("snk3", SINK)
    b.ctl("q", "y2")
    b.link("x", "a3", ks=DRP, ps="px3"); b.link("a3", "y2", kd=DRP, pd="py3"); b.link("y2", "snk3")
    b.T("q", "px3", 1); b.T("q", "py3", 1)
    assert (an.PAIRING, b.a["x"], -1) in an.analyze(b.g)["violations"]


# ---------------------------------------------------------------- analysis vs execution
def _run(b, tokens, n_frames, r=2):
    b.g.finalize(3)
    b.g.push(b.a["src"], [np.full(r, f + 1.0) for f in range(n_frames)])
    for q in [k for k in ("q", "q2") if k in b.a]:
        b.g.push(b.a[q], [(0, r, 0, t) for t in tokens])
    b.g.run()


def test_valid_dpg_never_deadlocks():
    """The analysis finds no violation, and every control sequence of length
    <= 4 runs to completion in the executor."""
    assert an.analyze(_dpg().g)["violations"] == []
    for n in range(1, 5):
        for toks in itertools.product([0, 1], repeat=n):
            _run(_dpg(), list(toks), n)


def test_mismatched_elements_deadlock():
    """Sec. V: linked DRPs set to atr on one side and itr on the other
    deadlock.  The analysis flags the graph (rule 1); in the executor the
    first token activates a1 for x and a2 for y, and y waits for a2 forever."""
    b = _dpg(el_y=(2, 1))
    assert an.RULE1 in b.codes()
    with pytest.raises(PruneError) as e:
        _run(b, [0], 1)
    assert e.value.code == moc.E_DEADLOCK
    b = _dpg(two_q=True)
    assert an.RULE1 in b.codes()


# ---------------------------------------------------------------- liveness and buffer bounds
def _random_dc_graph(rng, n_mid, n_edges, r):
    b = B()
    b.act("src", SOURCE); b.act("q", CONFIG, n_elements=1); b.act("x", SWITCH)
    mids = [f"a{i}" for i in range(n_mid)]
    for m in mids:
        b.act(m, PASSTHROUGH)
    b.act("y", SELECT); b.act("snk", SINK)
    b.link("src", "x"); b.ctl("q", "x"); b.ctl("q", "y")
    # every middle actor sits on an x-y chain (encapsulation), one element
    for i, m in enumerate(mids):
        b.link("x", m, ks=DRP, r=r, ps=f"px{i}", delay=int(rng.integers(0, 2 * r + 1)))
        b.link(m, "y", kd=DRP, r=r, pd=f"py{i}", delay=int(rng.integers(0, 2 * r + 1)))
        b.T("q", f"px{i}", 1); b.T("q", f"py{i}", 1)
    for i in range(1, n_mid):                       # a spanning chain keeps one DC
        b.link(mids[rng.integers(0, i)], mids[i], r=r, delay=int(rng.integers(0, 2 * r + 1)))
    for _ in range(n_edges):
        u, w = rng.integers(0, n_mid, size=2)
        b.link(mids[u], mids[w], r=r, delay=int(rng.integers(0, 2 * r + 1)))
    b.link("y", "snk")
    return b


def _has_tokenless_cycle(nodes, edges):
    """Brute force: some directed cycle whose FIFOs all hold fewer tokens
    than one firing consumes."""
    adj = {v: [w for (u, w, ok) in edges if u == v and ok] for v in nodes}
    for start in nodes:
        stack = [(start, [start])]
        while stack:
            v, path = stack.pop()
            for w in adj[v]:
                if w == start:
                    return True
                if w not in path:
                    stack.append((w, path + [w]))
    return False


@pytest.mark.parametrize("seed", range(40))
def test_dc_liveness_and_bounds(seed):
    rng = np.random.default_rng(seed)
    r = int(rng.integers(1, 4))
    b = _random_dc_graph(rng, int(rng.integers(1, 6)), int(rng.integers(0, 5)), r)
    rep = an.analyze(b.g)
    assert not ({v[0] for v in rep["violations"]} - {an.DEADLOCK_DC})
    assert len(rep["dcs"]) == 1
    members = set(rep["dcs"][0][2]) | {b.a["x"], b.a["y"]}
    # the DC's FIFOs: data FIFOs among its actors and x, y (none joins x to y here)
    H = [f for f, (s, d, rate, Q) in enumerate(b.g.fifos)
         if b.g.ports[d].kind != CPORT and b.g.ports[s].actor in members
         and b.g.ports[d].actor in members]
    edges = [(b.g.ports[b.g.fifos[f][0]].actor, b.g.ports[b.g.fifos[f][1]].actor,
              b.g.fifos[f][3] < b.g.fifos[f][2]) for f in H]
    dead = _has_tokenless_cycle(sorted(members), edges)
    assert ((an.DEADLOCK_DC, 0, 0) in rep["violations"]) == dead
    for f in H:
        rate, Q = b.g.fifos[f][2], b.g.fifos[f][3]
        if dead:
            assert rep["beta"][f] == -1
        elif Q < rate:
            assert rep["beta"][f] == Q + rate      # the producer fires first
        else:
            assert rep["beta"][f] in (Q, Q + rate)


def test_linked_iff_same_dc():
    """With one dynamic pair, px and py are linked exactly when they attach
    to the same DC (connectivity of U - {x, y} against the component
    decomposition of Sec. V)."""
    rng = np.random.default_rng(7)
    for trial in range(30):
        b = B()
        b.act("src", SOURCE); b.act("q", CONFIG, n_elements=8); b.act("x", SWITCH)
        n = int(rng.integers(2, 6))
        mids = [f"a{i}" for i in range(n)]
        for m in mids:
            b.act(m, PASSTHROUGH)
        b.act("y", SELECT); b.act("snk", SINK)
        b.link("src", "x"); b.ctl("q", "x"); b.ctl("q", "y"); b.link("y", "snk")
        for _ in range(int(rng.integers(0, 4))):
            u, w = rng.integers(0, n, size=2)
            if u != w:
                b.link(mids[u], mids[w])
        for k in range(int(rng.integers(1, 4))):
            b.link("x", mids[int(rng.integers(0, n))], ks=DRP, ps=f"px{k}")
            b.link(mids[int(rng.integers(0, n))], "y", kd=DRP, pd=f"py{k}")
        rep = an.analyze(b.g)
        dc_of = rep["dc_of_actor"]
        linked = set(rep["linked"])
        px = [p for k, p in b.p.items() if k.startswith("px")]
        py = [p for k, p in b.p.items() if k.startswith("py")]
        for p in px:
            for p2 in py:
                u = b.g.ports[b.g.fifos[b.g.ports[p].fifos[0]][1]].actor
                w = b.g.ports[b.g.fifos[b.g.ports[p2].fifos[0]][0]].actor
                assert ((min(p, p2), max(p, p2)) in linked) == (dc_of[u] == dc_of[w] != -1)


# ---------------------------------------------------------------- the paper's graphs
def test_unfused_dpd_graph():
    """Fig. 8 before merging: one DPG (conf, poly, add), one DC per FIR
    branch, element b+1 for branch b, no violation."""
    K, L = 4, 3
    taps = np.ones((1, K, L), np.complex128)
    g, ids = graphs.build_unfused(taps, [L], K, 8, 3)
    rep = an.analyze(g)
    assert rep["violations"] == []
    assert [(q, x, y) for (q, x, y, _) in rep["dpgs"]] == [(ids["cfg"], ids["poly"], ids["add"])]
    assert [(acts, el) for (_, el, acts, _) in rep["dcs"]] == [((ids["firs"][b],), b + 1) for b in range(K)]


def test_merged_and_routed_graphs():
    taps = np.ones((1, 3, 4), np.complex128)
    g, ids = graphs.build_plain(taps, [4], 3, 8, 3)
    rep = an.analyze(g)
    assert rep["violations"] == [] and rep["dpgs"] == []
    taps2 = np.ones((2, 1, 3, 4), np.complex128)
    g, ids = graphs.build_routed(taps2, [4], 3, 8, 3, 2)
    rep = an.analyze(g)
    assert rep["violations"] == []
    assert len(rep["dpgs"]) == 2 and len(rep["dcs"]) == 4
    assert [len(acts) for (_, _, acts, _) in rep["dcs"]] == [1, 1, 1, 1]
