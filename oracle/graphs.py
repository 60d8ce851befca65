"""Oracle builders and runners for the graphs the workloads use.

* plain:   SOURCE -> FILTERBANK (dynamic: the merged DPG poly/FIR_b/add with
           its control port) -> SINK, and CONFIG -> FILTERBANK.cport.  Branch d
           of the bank is DC d, controlled by element d+1 of the control value.
* routed:  per stream, SOURCE -> SWITCH -> {FILTERBANK (static, windowed),
           PASSTHROUGH} -> SELECT -> SINK with one CONFIG broadcasting the
           same one-hot control token to SWITCH and SELECT (a DPG with two
           DCs; the switch holds the stream history, so both DCs are
           stateless, as the design rules require of DC actors).
* unfused: SOURCE -> POLY (x) -> FIR_b -> ADD (y) -> SINK, CONFIG -> POLY, ADD:
           the DPD graph of Fig. 8 before actor merging.
* motion:  SOURCE -> GAUSS5 -> THRES -> MED5 -> SINK on uint8 frames (Fig. 7);
           GAUSS5's output port feeds THRES twice, the second FIFO with a
           one-frame delay (the previous frame of the difference).

Parity: exercised by tests/test_oracle_moc.py (fused == unfused, token
conservation, schedule independence, frame-split invariance).
"""
from __future__ import annotations

import numpy as np

from . import moc
from .moc import (Graph, IN, OUT, SRP, DRP, CPORT, SOURCE, CONFIG, FILTERBANK,
                  SWITCH, SELECT, PASSTHROUGH, SINK, POLY, FIR, ADD, GAUSS5, THRES, MED5)


def _frames_of(wl, s):
    off = wl.frame_offsets(s)
    return [wl.x[s, off[f]:off[f + 1]] for f in range(wl.n_frames)]


def build_plain(taps, bank_L, Kmax, atr, C, param=False, cfg_mode="prefix"):
    g = Graph()
    D = len(bank_L) * Kmax
    src = g.actor(SOURCE)
    cfg = g.actor(CONFIG, mode=cfg_mode, Kmax=Kmax, n_elements=D)
    fb = g.actor(FILTERBANK, taps=np.asarray(taps), bank_L=list(bank_L), Kmax=Kmax)
    snk = g.actor(SINK)
    p_src = g.port(src, OUT, SRP, atr, param)
    p_ctl = g.port(cfg, OUT, SRP, 1)
    p_cp = g.port(fb, IN, CPORT, 1)
    p_in = g.port(fb, IN, SRP, atr, param)
    p_out = g.port(fb, OUT, SRP, atr, param)
    p_snk = g.port(snk, IN, SRP, atr, param)
    f_in = g.connect(p_src, p_in, atr)
    f_ctl = g.connect(p_ctl, p_cp, 1)
    f_out = g.connect(p_out, p_snk, atr)
    for d, drp in enumerate(g.actors[fb].branches):
        g.control(p_ctl, drp, d + 1)
    g.finalize(C)
    ids = dict(src=src, cfg=cfg, fb=fb, snk=snk, f_in=f_in, f_ctl=f_ctl, f_out=f_out)
    return g, ids


def run_plain(wl, C=3, s=0, atr=None, param=None, policy="round_robin", rng=None,
              cfg_mode="prefix"):
    """Run the plain graph over stream s of a workload; returns (y, logs, g, ids)."""
    n = wl.side[s, :, 1]
    if param is None:
        param = bool(np.any(n != n[0]))
    if atr is None:
        atr = int(wl.spec.n_max) if param else int(n[0])
    g, ids = build_plain(wl.taps[s], wl.bank_L, wl.Kmax, atr, C, param, cfg_mode)
    g.push(ids["src"], _frames_of(wl, s))
    g.push(ids["cfg"], wl.side[s])
    g.run(policy=policy, rng=rng)
    return g.sink_output(ids["snk"]), g.logs(), g, ids


def build_routed(taps_all, bank_L, Kmax, atr, C, n_streams, param=False):
    g = Graph()
    H = max(bank_L) - 1
    D = len(bank_L) * Kmax
    ids = []
    for s in range(n_streams):
        src = g.actor(SOURCE)
        cfg = g.actor(CONFIG, mode="route", Kmax=Kmax, n_elements=2)
        sw = g.actor(SWITCH)
        fb = g.actor(FILTERBANK, taps=np.asarray(taps_all[s]), bank_L=list(bank_L), Kmax=Kmax,
                     windowed=True, mask=(1 << D) - 1)
        ps = g.actor(PASSTHROUGH)
        sel = g.actor(SELECT)
        snk = g.actor(SINK)
        p_src = g.port(src, OUT, SRP, atr, param)
        p_ctl = g.port(cfg, OUT, SRP, 1)
        p_swc = g.port(sw, IN, CPORT, 1)
        p_swi = g.port(sw, IN, SRP, atr, param)
        p_sw0 = g.port(sw, OUT, DRP, atr + H, param, halo=H)
        p_sw1 = g.port(sw, OUT, DRP, atr, param)
        p_fbi = g.port(fb, IN, SRP, atr + H, param, halo=H)
        p_fbo = g.port(fb, OUT, SRP, atr, param)
        p_psi = g.port(ps, IN, SRP, atr, param)
        p_pso = g.port(ps, OUT, SRP, atr, param)
        p_slc = g.port(sel, IN, CPORT, 1)
        p_sl0 = g.port(sel, IN, DRP, atr, param)
        p_sl1 = g.port(sel, IN, DRP, atr, param)
        p_slo = g.port(sel, OUT, SRP, atr, param)
        p_snk = g.port(snk, IN, SRP, atr, param)
        f = {}
        f["in"] = g.connect(p_src, p_swi, atr)
        f["ctl_sw"] = g.connect(p_ctl, p_swc, 1)
        f["ctl_sel"] = g.connect(p_ctl, p_slc, 1)
        f["sw_fb"] = g.connect(p_sw0, p_fbi, atr + H)
        f["sw_ps"] = g.connect(p_sw1, p_psi, atr)
        f["fb_sel"] = g.connect(p_fbo, p_sl0, atr)
        f["ps_sel"] = g.connect(p_pso, p_sl1, atr)
        f["out"] = g.connect(p_slo, p_snk, atr)
        g.control(p_ctl, p_sw0, 1)
        g.control(p_ctl, p_sw1, 2)
        g.control(p_ctl, p_sl0, 1)
        g.control(p_ctl, p_sl1, 2)
        ids.append(dict(src=src, cfg=cfg, sw=sw, fb=fb, ps=ps, sel=sel, snk=snk, fifos=f))
    g.finalize(C)
    return g, ids


def run_routed(wl, C=3, policy="round_robin", rng=None):
    n = wl.side[0, :, 1]
    param = bool(np.any(wl.side[:, :, 1] != n[0]))
    atr = int(wl.spec.n_max) if param else int(n[0])
    g, ids = build_routed(wl.taps, wl.bank_L, wl.Kmax, atr, C, wl.n_streams, param)
    for s in range(wl.n_streams):
        g.push(ids[s]["src"], _frames_of(wl, s))
        g.push(ids[s]["cfg"], wl.side[s])
    g.run(policy=policy, rng=rng)
    ys = np.stack([g.sink_output(ids[s]["snk"]) for s in range(wl.n_streams)])
    return ys, g.logs(), g, ids


def build_unfused(taps, bank_L, Kmax, atr, C):
    """Fig. 8 DPD graph before merging: one bank only."""
    if len(bank_L) != 1:
        raise moc.PruneError(moc.E_UNSUPPORTED, "the unfused graph covers one bank")
    L = int(bank_L[0])
    g = Graph()
    src = g.actor(SOURCE)
    cfg = g.actor(CONFIG, mode="prefix", Kmax=Kmax, n_elements=Kmax)
    poly = g.actor(POLY, Kmax=Kmax, bank_L=[L])
    firs = [g.actor(FIR, taps=np.asarray(taps[0, b, :L])) for b in range(Kmax)]
    add = g.actor(ADD)
    snk = g.actor(SINK)
    p_src = g.port(src, OUT, SRP, atr)
    p_ctl = g.port(cfg, OUT, SRP, 1)
    p_pc = g.port(poly, IN, CPORT, 1)
    p_pi = g.port(poly, IN, SRP, atr)
    p_po = [g.port(poly, OUT, DRP, atr + L - 1, halo=L - 1) for _ in range(Kmax)]
    p_fi = [g.port(firs[b], IN, SRP, atr + L - 1, halo=L - 1) for b in range(Kmax)]
    p_fo = [g.port(firs[b], OUT, SRP, atr) for b in range(Kmax)]
    p_ac = g.port(add, IN, CPORT, 1)
    p_ai = [g.port(add, IN, DRP, atr) for _ in range(Kmax)]
    p_ao = g.port(add, OUT, SRP, atr)
    p_snk = g.port(snk, IN, SRP, atr)
    g.connect(p_src, p_pi, atr)
    g.connect(p_ctl, p_pc, 1)
    g.connect(p_ctl, p_ac, 1)
    for b in range(Kmax):
        g.connect(p_po[b], p_fi[b], atr + L - 1)
        g.connect(p_fo[b], p_ai[b], atr)
        g.control(p_ctl, p_po[b], b + 1)
        g.control(p_ctl, p_ai[b], b + 1)
    g.connect(p_ao, p_snk, atr)
    g.finalize(C)
    return g, dict(src=src, cfg=cfg, poly=poly, firs=firs, add=add, snk=snk)


def stream_frames(wl, s=0):
    """(t0, n, mask, route) per frame of stream s, using the configuration
    actor's mapping of side-information to a branch mask."""
    out = []
    off = wl.frame_offsets(s)
    route_mode = wl.spec.pass_prob > 0
    D = len(wl.bank_L) * wl.Kmax
    for f in range(wl.n_frames):
        K, n, bank, route = (int(v) for v in wl.side[s, f])
        if route_mode:
            mask = (1 << D) - 1
        else:
            mask, _ = Graph.config_token(dict(mode="prefix", Kmax=wl.Kmax), wl.side[s, f])
            route = 0
        out.append((int(off[f]), n, mask, route))
    return out


def build_motion(W, H, C, T=20):
    """Motion Detection graph (Sec. VII-A): a frame is W*H one-byte tokens."""
    npix = W * H
    g = Graph()
    src = g.actor(SOURCE)
    gau = g.actor(GAUSS5, W=W, H=H)
    thr = g.actor(THRES, W=W, H=H, T=T)
    med = g.actor(MED5, W=W, H=H)
    snk = g.actor(SINK)
    p_src = g.port(src, OUT, SRP, npix, u8=True)
    p_gi = g.port(gau, IN, SRP, npix, u8=True)
    p_go = g.port(gau, OUT, SRP, npix, u8=True)
    p_tc = g.port(thr, IN, SRP, npix, u8=True)
    p_tp = g.port(thr, IN, SRP, npix, u8=True)
    p_to = g.port(thr, OUT, SRP, npix, u8=True)
    p_mi = g.port(med, IN, SRP, npix, u8=True)
    p_mo = g.port(med, OUT, SRP, npix, u8=True)
    p_snk = g.port(snk, IN, SRP, npix, u8=True)
    g.connect(p_src, p_gi, npix)
    g.connect(p_go, p_tc, npix)
    g.connect(p_go, p_tp, npix, npix)     # one-frame delay: the previous frame
    g.connect(p_to, p_mi, npix)
    g.connect(p_mo, p_snk, npix)
    g.finalize(C)
    return g, dict(src=src, gauss=gau, thres=thr, med=med, snk=snk)


def run_motion(frames, C=3, T=20):
    """Run the Motion Detection graph over uint8 frames [F, H, W]; returns
    (motion maps [F, H, W], logs, g, ids)."""
    F, H, W = frames.shape
    g, ids = build_motion(W, H, C, T)
    g.push(ids["src"], [fr.ravel() for fr in frames])
    g.run()
    return g.sink_output(ids["snk"]).reshape(F, H, W), g.logs(), g, ids
