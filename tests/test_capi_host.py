"""Host-side checks of libprune_hip (no GPU needed): the library loads and
exports every entry point of include/prune.h, its integer rules equal the
oracle's, and host-only graphs validate like the oracle's graphs."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1802_06625_amd import _lib as L
from paper_1802_06625_amd.graph import Graph
from oracle import moc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "prune.h")).read()
    return sorted(set(re.findall(r"\b(prune_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    names = _declared()
    assert len(names) >= 35
    for n in names:
        assert hasattr(lib, n), n
    assert {s[0] for s in L.SIGNATURES} == set(names)


@pytest.mark.parametrize("r,Q,C", [(4, 1, 3), (4, 0, 3), (4, 8, 3), (4, 16, 3), (3, 2, 2), (5, 3, 3),
                                   (4, 12, 2), (6, 6, 2), (7, 3, 1), (16384, 0, 4096), (1, 0, 1),
                                   (65536, 0, 2048), (4, 5, 2), (10, 13, 4)])
def test_rules_match_oracle(r, Q, C):
    cap = C.c_uint64() if False else None
    cap = __import__("ctypes").c_uint64()
    st = L.lib().prune_rule_capacity(r, Q, C, __import__("ctypes").byref(cap))
    try:
        expect = moc.FifoState(0, r, Q, C, np.float64, False).capacity
    except moc.PruneError as e:
        assert st == L.E_DELAY and e.code == moc.E_DELAY
        return
    assert st == L.OK and cap.value == expect
    n = 50
    ws = (__import__("ctypes").c_uint64 * n)()
    rs = (__import__("ctypes").c_uint64 * n)()
    assert L.lib().prune_rule_slots(r, Q, C, n, ws, rs) == L.OK
    assert list(ws) == [moc.fifo_write_slot(r, Q, C, j) for j in range(n)]
    assert list(rs) == [moc.fifo_read_slot(r, Q, C, i) for i in range(n)]


def test_config_token_matches_oracle():
    import ctypes
    rng = np.random.default_rng(0)
    for _ in range(900):
        mode = int(rng.integers(0, 3))
        Kmax = int(rng.integers(1, 11))
        K = int(rng.integers(0, 1 << Kmax)) if mode == L.CONFIG_MASK else int(rng.integers(0, Kmax + 1))
        side = L.SideInfo(K, int(rng.integers(1, 70000)), int(rng.integers(0, 3)), int(rng.integers(0, 5)))
        tok = L.CtrlToken()
        assert L.lib().prune_rule_config_token(mode, Kmax, ctypes.byref(side), ctypes.byref(tok)) == 0
        mask, rate = moc.Graph.config_token(dict(mode=("prefix", "route", "mask")[mode], Kmax=Kmax),
                                            (side.K, side.n, side.bank, side.route))
        assert (tok.mask, tok.rate) == (mask, rate)


# ---- host-only graph validation -------------------------------------------
def _plain(g, atr=64, Kmax=4, bank_L=(8,), tweak=None):
    src = g.actor(L.SOURCE)
    cfg = g.config(L.CONFIG_PREFIX, Kmax, Kmax * len(bank_L))
    fb = g.filterbank(Kmax, bank_L)
    snk = g.actor(L.SINK)
    ps = g.port(src, L.OUT, L.SRP, atr)
    pc = g.port(cfg, L.OUT, L.SRP, 1)
    pcp = g.port(fb, L.IN, L.CPORT, 1)
    pin = g.port(fb, L.IN, L.SRP, atr if tweak != "rate" else atr + 1)
    pout = g.port(fb, L.OUT, L.SRP, atr)
    pk = g.port(snk, L.IN, L.SRP, atr)
    g.connect(ps, pin, atr)
    g.connect(pc, pcp, 1)
    if tweak != "unconnected":
        g.connect(pout, pk, atr)
    for d in range(Kmax * len(bank_L)):
        if tweak == "uncontrolled" and d == 1:
            continue
        g.control(pc, g.branch(fb, d), d + 1)
    return g


def test_host_only_plain_graph_validates_and_sizes():
    g = _plain(Graph(-1))
    g.finalize(3)
    assert g.required_bytes(0) == 8 * moc.fifo_capacity(64, 0, 3)
    assert g.required_bytes(1) == 8 * moc.fifo_capacity(1, 0, 3)


@pytest.mark.parametrize("tweak,code", [("rate", L.E_RATE_MISMATCH), ("unconnected", L.E_CONNECT),
                                        ("uncontrolled", L.E_PORT_KIND)])
def test_host_only_validation_errors(tweak, code):
    g = _plain(Graph(-1), tweak=tweak)
    with pytest.raises(L.PruneError) as e:
        g.finalize(3)
    assert e.value.code == code


def test_host_only_rule4_and_static_drp():
    g = Graph(-1)
    cfg = g.config(L.CONFIG_ROUTE, 1, 2)
    src = g.actor(L.SOURCE)
    x = g.actor(L.SELECT)
    snk = g.actor(L.SINK)
    pc = g.port(cfg, L.OUT, L.SRP, 1)
    ps = g.port(src, L.OUT, L.SRP, 4)
    p1 = g.port(x, L.IN, L.CPORT, 1)
    p2 = g.port(x, L.IN, L.DRP, 4)
    p3 = g.port(x, L.OUT, L.DRP, 4)
    pk = g.port(snk, L.IN, L.SRP, 4)
    g.connect(pc, p1, 1); g.connect(ps, p2, 4); g.connect(p3, pk, 4)
    g.control(pc, p2, 1); g.control(pc, p3, 1)
    with pytest.raises(L.PruneError) as e:
        g.finalize(3)
    assert e.value.code in (L.E_RULE4, L.E_ARG)
    g = Graph(-1)
    src = g.actor(L.SOURCE); mid = g.actor(L.PASSTHROUGH); snk = g.actor(L.SINK)
    a = g.port(src, L.OUT, L.SRP, 4); b = g.port(mid, L.IN, L.DRP, 4)
    c = g.port(mid, L.OUT, L.SRP, 4); d = g.port(snk, L.IN, L.SRP, 4)
    g.connect(a, b, 4); g.connect(c, d, 4)
    with pytest.raises(L.PruneError) as e:
        g.finalize(3)
    assert e.value.code == L.E_PORT_KIND


def test_host_only_delay_rules():
    for Q, C_, ok in [(1, 3, True), (13, 3, False), (8, 3, True), (1, 1, False)]:
        g = Graph(-1)
        src = g.actor(L.SOURCE); mid = g.actor(L.PASSTHROUGH); snk = g.actor(L.SINK)
        a = g.port(src, L.OUT, L.SRP, 4); b = g.port(mid, L.IN, L.SRP, 4)
        c = g.port(mid, L.OUT, L.SRP, 4); d = g.port(snk, L.IN, L.SRP, 4)
        g.connect(a, b, 4, Q); g.connect(c, d, 4)
        if ok:
            g.finalize(C_)
            assert g.required_bytes(0) == 8 * moc.fifo_capacity(4, Q, C_)
        else:
            with pytest.raises(L.PruneError) as e:
                g.finalize(C_)
            assert e.value.code == L.E_DELAY


def test_edit_after_finalize_is_state_error():
    g = _plain(Graph(-1))
    g.finalize(2)
    with pytest.raises(L.PruneError) as e:
        g.actor(L.SINK)
    assert e.value.code == L.E_STATE


def test_unsupported_shapes():
    g = Graph(-1)
    with pytest.raises(L.PruneError) as e:
        g.filterbank(11, (8,))
    assert e.value.code == L.E_UNSUPPORTED
    with pytest.raises(L.PruneError) as e:
        g.filterbank(4, (65,))
    assert e.value.code == L.E_UNSUPPORTED


def test_actor_count_limit():
    g = Graph(-1)
    lib, h = L.lib(), g.h
    out = C.c_uint32()
    for _ in range(65536):
        assert lib.prune_actor_create(h, L.PASSTHROUGH, None, 0, C.byref(out)) == L.OK
    with pytest.raises(L.PruneError) as e:
        g.finalize(2)
    assert e.value.code == L.E_UNSUPPORTED


def test_variant_selection_arguments():
    """Forward and backward kernel selection: valid indices are accepted,
    others rejected with E_ARG, and the names are stable."""
    lib = L.lib()
    n = lib.prune_fb_variant_count()
    assert n == 8
    names = [lib.prune_fb_variant_name(v).decode() for v in range(1, n + 1)]
    assert all(x.startswith("valu") for x in names[:5]) and all(x.startswith("mfma") for x in names[5:])
    assert lib.prune_set_fb_variant(n + 1) == L.E_ARG
    assert lib.prune_set_fb_variant(-1) == L.E_ARG
    assert lib.prune_set_fb_variant(0) == L.OK
    assert [lib.prune_bwd_variant_name(v).decode() for v in (0, 1, 2, 3)] == \
        ["auto", "valu_horner", "mfma_toeplitz", "mfma_gemm"]
    assert lib.prune_set_bwd_variant(4) == L.E_ARG
    assert lib.prune_set_bwd_variant(-1) == L.E_ARG
    for v in (3, 2, 1, 0):
        assert lib.prune_set_bwd_variant(v) == L.OK
    v = C.c_int()
    assert lib.prune_autotune_bwd(0, 7, 1024, C.byref(v)) == L.E_ARG
    assert lib.prune_autotune_bwd(65, 7, 1024, C.byref(v)) == L.E_ARG


def test_backward_needs_one_gradient_output():
    """prune_fb_backward checks its pointers before any device work: both
    gradient outputs null is an argument error (no GPU needed)."""
    from paper_1802_06625_amd import ops
    d = ops.make_desc(1, 1024, 4, (8,), 1, 1024)
    p = C.c_void_p(16)   # never dereferenced: the call returns before any device work
    assert L.lib().prune_fb_backward(C.byref(d), p, p, p, p, None, None, p, 1 << 20, None) == L.E_ARG


def test_pixel_actor_parameters():
    """Motion Detection actors: frame width a multiple of 4 (the kernels move
    words of four pixels), W*H a multiple of 8 (copies move 8-byte words),
    positive sizes, and a parameter block of the right size."""
    g = Graph(-1)
    for kind in (L.GAUSS5, L.THRES, L.MED5):
        assert g.actor(kind, L.PixelParams(40, 24, 20)) >= 0
        for (W, H), code in [((42, 24), L.E_UNSUPPORTED), ((4, 1), L.E_ARG), ((0, 8), L.E_ARG),
                             ((8, 0), L.E_ARG)]:
            with pytest.raises(L.PruneError) as e:
                g.actor(kind, L.PixelParams(W, H, 20))
            assert e.value.code == code, (kind, W, H)
        out = C.c_uint32()
        assert L.lib().prune_actor_create(g.h, kind, None, 0, C.byref(out)) == L.E_ARG


@pytest.mark.parametrize("Kmax,bank_L,tile", [(8, (16,), 512), (4, (8, 5), 512), (9, (16,), 1024),
                                              (8, (17,), 1024), (10, (64, 32), 1024)])
def test_backward_workspace_covers_the_form_tiles(Kmax, bank_L, tile):
    """prune_fb_workspace_bytes (host logic) sizes the adjoint's workspace for
    the smallest tile any backward form cuts frames into: 512 positions for
    shapes of at most 8 powers and 16 taps (the plain-product form's one-wave
    kernel), 1024 otherwise; the tile partial rows alone take items x
    entries x 8 bytes."""
    n_frames, mfl = 37, 5000
    d = ops_desc(Kmax, bank_L, n_frames, mfl)
    ws = C.c_size_t()
    assert L.lib().prune_fb_workspace_bytes(C.byref(d), C.byref(ws)) == L.OK
    E = len(bank_L) * Kmax * max(bank_L)
    items = n_frames * -(-mfl // tile)
    assert ws.value >= items * E * 8 + items * 8
    # and not sized for the smaller tile when the shape never uses it
    if tile == 1024:
        assert ws.value < n_frames * -(-mfl // 512) * E * 8


def ops_desc(Kmax, bank_L, n_frames, mfl):
    from paper_1802_06625_amd import ops
    return ops.make_desc(1, n_frames * mfl, Kmax, bank_L, n_frames, mfl)
