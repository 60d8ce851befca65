"""Compile-time analysis through the C ABI (host-only graphs, no GPU):
identical reports from libprune_hip.so and the oracle on the same seeded
structures, the paper's example graphs, and the finalize gate."""
import pytest

import graphgen as gg
from oracle import analysis as an
from oracle import moc
from paper_1802_06625_amd import _lib as L
from paper_1802_06625_amd.graph import Graph


def oracle_graph(S):
    g = moc.Graph()
    for a, k in enumerate(S.actors):
        if k == gg.CONFIG:
            g.actor(moc.CONFIG, mode="route", n_elements=S.n_elements[a])
        else:
            g.actor(k)
    for (a, d, k) in S.ports:
        g.port(a, d, k, 1)
    for (s, d, r, q) in S.fifos:
        g.connect(s, d, r, q)
    for (c, p, e) in S.table:
        g.control(c, p, e)
    return g


def native_graph(S):
    g = Graph(-1)
    for a, k in enumerate(S.actors):
        if k == gg.CONFIG:
            assert g.config(L.CONFIG_ROUTE, 1, S.n_elements[a]) == a
        else:
            assert g.actor(k) == a
    for i, (a, d, k) in enumerate(S.ports):
        assert g.port(a, d, k, 1) == i
    for i, (s, d, r, q) in enumerate(S.fifos):
        assert g.connect(s, d, r, q) == i
    for (c, p, e) in S.table:
        g.control(c, p, e)
    return g


def both(S):
    return an.analyze(oracle_graph(S)), native_graph(S).analyze()


@pytest.mark.parametrize("seed", range(150))
def test_parity_random_structures(seed):
    ref, got = both(gg.random_structure(seed))
    assert got == ref


@pytest.mark.parametrize("seed", range(150))
def test_parity_dpg_structures(seed):
    ref, got = both(gg.dpg_structure(seed))
    assert got == ref


def test_random_structures_cover_every_code():
    """The seeds above exercise every violation code, clean graphs and
    deadlocking ones."""
    seen, clean, deadlocks = set(), 0, 0
    for seed in range(150):
        for S in (gg.random_structure(seed), gg.dpg_structure(seed)):
            v = an.analyze(oracle_graph(S))["violations"]
            seen |= {c for c, _, _ in v}
            clean += not v
            deadlocks += any(c == an.DEADLOCK_DC for c, _, _ in v)
    assert {an.RULE1, an.RULE2, an.RULE3_KIND, an.RULE3_SHARED, an.RULE4, an.RULE5, an.DPG_A,
            an.DPG_B_DC, an.DPG_B_COUNT, an.DPG_C, an.DEADLOCK_DC, an.PAIRING,
            an.UNPAIRED} <= seen
    assert clean >= 30 and deadlocks >= 5


def _sec5_structure():
    S = gg.Structure()
    q = S.actor(gg.CONFIG, 3)
    src, x = S.actor(gg.SOURCE), S.actor(gg.SWITCH)
    a = [S.actor(gg.PASSTHROUGH) for _ in range(4)]
    y, snk = S.actor(gg.SELECT), S.actor(gg.SINK)
    qp = S.port(q, gg.OUT, gg.SRP)
    S.connect(S.port(src, gg.OUT, gg.SRP), S.port(x, gg.IN, gg.SRP), 4)
    S.connect(qp, S.port(x, gg.IN, gg.CPORT))
    S.connect(qp, S.port(y, gg.IN, gg.CPORT))
    px = [S.port(x, gg.OUT, gg.DRP) for _ in range(4)]
    py = [S.port(y, gg.IN, gg.DRP) for _ in range(3)]
    S.connect(px[0], S.port(a[0], gg.IN, gg.SRP), 4)
    S.connect(px[1], S.port(a[1], gg.IN, gg.SRP), 4)
    S.connect(S.port(a[0], gg.OUT, gg.SRP), S.port(a[2], gg.IN, gg.SRP), 4)
    S.connect(S.port(a[1], gg.OUT, gg.SRP), S.port(a[2], gg.IN, gg.SRP), 4)
    S.connect(S.port(a[2], gg.OUT, gg.SRP), py[0], 4)
    S.connect(px[2], S.port(a[3], gg.IN, gg.SRP), 4)
    S.connect(S.port(a[3], gg.OUT, gg.SRP), py[1], 4)
    direct = S.connect(px[3], py[2], 4)
    S.connect(S.port(y, gg.OUT, gg.SRP), S.port(snk, gg.IN, gg.SRP), 4)
    for p, e in zip(px + py, (1, 1, 2, 3, 1, 2, 3)):
        S.control(qp, p, e)
    return S, dict(px=px, py=py, a=a, x=x, y=y, q=q, qp=qp, direct=direct)


def test_sec5_example_native():
    """Sec. V example through the C ABI: four linked DRP pairs, three DCs
    {a1, a2, a3}, {a4} and the dummy of the direct px4-py3 FIFO."""
    S, ids = _sec5_structure()
    rep = native_graph(S).analyze()
    px, py, a = ids["px"], ids["py"], ids["a"]
    assert rep["linked"] == sorted([(px[0], py[0]), (px[1], py[0]), (px[2], py[1]), (px[3], py[2])])
    assert rep["violations"] == []
    assert rep["dpgs"] == [(ids["q"], ids["x"], ids["y"], ids["qp"])]
    assert [(el, acts) for (_, el, acts, _) in rep["dcs"]] == [(1, tuple(a[:3])), (2, (a[3],)), (3, ())]
    assert rep["dcs"][2][3] == ids["direct"]          # the direct FIFO px4 -> py3


def _dpd_structure(K):
    """The unfused DPD graph of Fig. 8 (poly as a switch, FIR_b as copy
    actors, add as a select)."""
    S = gg.Structure()
    q = S.actor(gg.CONFIG, K)
    src, poly = S.actor(gg.SOURCE), S.actor(gg.SWITCH)
    firs = [S.actor(gg.PASSTHROUGH) for _ in range(K)]
    add, snk = S.actor(gg.SELECT), S.actor(gg.SINK)
    qp = S.port(q, gg.OUT, gg.SRP)
    S.connect(S.port(src, gg.OUT, gg.SRP), S.port(poly, gg.IN, gg.SRP), 8)
    S.connect(qp, S.port(poly, gg.IN, gg.CPORT))
    S.connect(qp, S.port(add, gg.IN, gg.CPORT))
    for b in range(K):
        po = S.port(poly, gg.OUT, gg.DRP)
        ai = S.port(add, gg.IN, gg.DRP)
        S.connect(po, S.port(firs[b], gg.IN, gg.SRP), 17)
        S.connect(S.port(firs[b], gg.OUT, gg.SRP), ai, 8)
        S.control(qp, po, b + 1)
        S.control(qp, ai, b + 1)
    S.connect(S.port(add, gg.OUT, gg.SRP), S.port(snk, gg.IN, gg.SRP), 8)
    return S, firs


def test_dpd_graph_native():
    S, firs = _dpd_structure(10)
    ref, got = both(S)
    assert got == ref
    assert got["violations"] == []
    assert [acts for (_, _, acts, _) in got["dcs"]] == [(f,) for f in firs]
    assert [el for (_, el, _, _) in got["dcs"]] == list(range(1, 11))


def _routed_native(el_sel=(1, 2)):
    """The routed stream graph of the multi-stream workload, host-only."""
    g = Graph(-1)
    atr, H = 64, 7
    src = g.actor(L.SOURCE); cfg = g.config(L.CONFIG_ROUTE, 1, 2)
    sw = g.actor(L.SWITCH); fb = g.filterbank(1, [8], windowed=True, fixed_mask=1)
    ps = g.actor(L.PASSTHROUGH); sel = g.actor(L.SELECT); snk = g.actor(L.SINK)
    p_src = g.port(src, L.OUT, L.SRP, atr); p_ctl = g.port(cfg, L.OUT, L.SRP, 1)
    p_swc = g.port(sw, L.IN, L.CPORT, 1); p_swi = g.port(sw, L.IN, L.SRP, atr)
    p_sw0 = g.port(sw, L.OUT, L.DRP, atr + H, halo=H); p_sw1 = g.port(sw, L.OUT, L.DRP, atr)
    p_fbi = g.port(fb, L.IN, L.SRP, atr + H, halo=H); p_fbo = g.port(fb, L.OUT, L.SRP, atr)
    p_psi = g.port(ps, L.IN, L.SRP, atr); p_pso = g.port(ps, L.OUT, L.SRP, atr)
    p_slc = g.port(sel, L.IN, L.CPORT, 1); p_sl0 = g.port(sel, L.IN, L.DRP, atr)
    p_sl1 = g.port(sel, L.IN, L.DRP, atr); p_slo = g.port(sel, L.OUT, L.SRP, atr)
    p_snk = g.port(snk, L.IN, L.SRP, atr)
    g.connect(p_src, p_swi, atr); g.connect(p_ctl, p_swc, 1); g.connect(p_ctl, p_slc, 1)
    g.connect(p_sw0, p_fbi, atr + H); g.connect(p_sw1, p_psi, atr)
    g.connect(p_fbo, p_sl0, atr); g.connect(p_pso, p_sl1, atr); g.connect(p_slo, p_snk, atr)
    g.control(p_ctl, p_sw0, 1); g.control(p_ctl, p_sw1, 2)
    g.control(p_ctl, p_sl0, el_sel[0]); g.control(p_ctl, p_sl1, el_sel[1])
    return g, dict(fb=fb, ps=ps)


def test_finalize_gate():
    g, ids = _routed_native()
    rep = g.analyze()
    assert rep["violations"] == []
    assert [acts for (_, _, acts, _) in rep["dcs"]] == [(ids["fb"],), (ids["ps"],)]
    g.finalize(3, check_rules=True)
    g, _ = _routed_native(el_sel=(2, 1))
    assert any(c == an.RULE1 for c, _, _ in g.analyze()["violations"])
    with pytest.raises(L.PruneError) as e:
        g.finalize(3, check_rules=True)
    assert e.value.code == L.E_RULE
    g, _ = _routed_native(el_sel=(2, 1))
    g.finalize(3)                       # local checks only: the graph is accepted


def test_analysis_table_errors():
    g = Graph(-1)
    import ctypes as C
    n = C.c_size_t()
    assert L.lib().prune_graph_analysis_table(g.h, L.AN_BETA, None, 0, C.byref(n)) == L.E_STATE
    g.analyze()
    assert L.lib().prune_graph_analysis_table(g.h, 99, None, 0, C.byref(n)) == L.E_ARG
    assert L.lib().prune_graph_set_checks(g.h, 6) == L.E_ARG
