"""Small graphs whose finite runs stop, with the classification the end of the
run must get: a normal end (external input used up) or a deadlock (a cycle
of blocking reads and writes, or linked DRPs set differently by their control
tokens).

A case is a plain description (actor kinds by name, ports, FIFOs, control
table, pushed frames and side-information) that the tests build through the
oracle's graph API here and through the library's in the GPU tests.  The
frames are seeded random values; nothing here computes any actor's output.
"""
from __future__ import annotations

import numpy as np

IN, OUT = 0, 1
SRP, DRP, CPORT = 0, 1, 2


class Desc:
    def __init__(self, C):
        self.C = C
        self.actors = []       # (kind name, params)
        self.ports = []        # (actor, dir, kind, atr, u8)
        self.fifos = []        # (src port, dst port, rate, delay)
        self.table = []        # (control port, drp, element)
        self.frames = {}       # source actor -> list of frames (uint8 or complex64)
        self.side = {}         # config actor -> [F, 4] side-information
        self.expect = None     # "normal" or "deadlock"
        self.names = {}

    def actor(self, name, kind, **params):
        self.actors.append((kind, params))
        self.names[name] = len(self.actors) - 1
        return self.names[name]

    def port(self, a, d, k, atr, u8=False):
        self.ports.append((a, d, k, int(atr), bool(u8)))
        return len(self.ports) - 1

    def connect(self, s, d, rate, delay=0):
        self.fifos.append((s, d, int(rate), int(delay)))
        return len(self.fifos) - 1

    def control(self, c, p, e):
        self.table.append((c, p, int(e)))


def thres_med_cycle(delay_frames, n_frames, C=3, W=8, H=8, seed=0):
    """src -> THRES (current frame); THRES -> MED; MED -> THRES (previous
    frame, with a delay of delay_frames frames); MED -> sink."""
    d = Desc(C)
    npix = W * H
    src = d.actor("src", "SOURCE")
    thr = d.actor("thres", "THRES", W=W, H=H, T=20)
    med = d.actor("med", "MED5", W=W, H=H)
    snk = d.actor("snk", "SINK")
    p = lambda a, dr: d.port(a, dr, SRP, npix, u8=True)
    ps, ptc, ptp, pto = p(src, OUT), p(thr, IN), p(thr, IN), p(thr, OUT)
    pmi, pmo, pk = p(med, IN), p(med, OUT), p(snk, IN)
    d.connect(ps, ptc, npix)
    d.connect(pto, pmi, npix)
    d.connect(pmo, ptp, npix, delay_frames * npix)
    d.connect(pmo, pk, npix)
    rng = np.random.default_rng(seed)
    d.frames[src] = [rng.integers(0, 256, npix, dtype=np.uint8) for _ in range(n_frames)]
    d.expect = "normal" if delay_frames else "deadlock"
    return d


def gauss_delay_capacity(delay_frames, n_frames, C, W=8, H=8, seed=1):
    """src -> GAUSS5, whose output goes to THRES twice: directly, and through
    a FIFO with a delay of delay_frames frames.  When the delay fills that
    FIFO's Eq. 2 capacity (delay_frames == C), GAUSS5 waits for room THRES
    only makes after reading a frame GAUSS5 has not written: a cycle of a
    blocking write and a blocking read."""
    d = Desc(C)
    npix = W * H
    src = d.actor("src", "SOURCE")
    gau = d.actor("gauss", "GAUSS5", W=W, H=H)
    thr = d.actor("thres", "THRES", W=W, H=H, T=20)
    snk = d.actor("snk", "SINK")
    p = lambda a, dr: d.port(a, dr, SRP, npix, u8=True)
    ps, pgi, pgo = p(src, OUT), p(gau, IN), p(gau, OUT)
    ptc, ptp, pto, pk = p(thr, IN), p(thr, IN), p(thr, OUT), p(snk, IN)
    d.connect(ps, pgi, npix)
    d.connect(pgo, ptc, npix)
    d.connect(pgo, ptp, npix, delay_frames * npix)
    d.connect(pto, pk, npix)
    rng = np.random.default_rng(seed)
    d.frames[src] = [rng.integers(0, 256, npix, dtype=np.uint8) for _ in range(n_frames)]
    d.expect = "deadlock" if delay_frames >= C else "normal"
    return d


def switch_select(routes_x, routes_y, n_frames, C=3, r=2, Q_in=0, seed=2):
    """src -> x (switch) -> {a1, a2} -> y (select) -> sink.  With routes_y
    None one configuration actor broadcasts to x and y (a valid DPG);
    otherwise a second one feeds y its own routes (route k -> DC a(k+1))."""
    d = Desc(C)
    src = d.actor("src", "SOURCE")
    q1 = d.actor("q", "CONFIG", mode="route", n_elements=2)
    q2 = d.actor("q2", "CONFIG", mode="route", n_elements=2) if routes_y is not None else None
    x = d.actor("x", "SWITCH")
    a = [d.actor("a1", "PASSTHROUGH"), d.actor("a2", "PASSTHROUGH")]
    y = d.actor("y", "SELECT")
    snk = d.actor("snk", "SINK")
    ps = d.port(src, OUT, SRP, r)
    pq1 = d.port(q1, OUT, SRP, 1)
    pq2 = d.port(q2, OUT, SRP, 1) if q2 is not None else pq1
    xc, xi = d.port(x, IN, CPORT, 1), d.port(x, IN, SRP, r)
    xo = [d.port(x, OUT, DRP, r) for _ in range(2)]
    ai = [d.port(v, IN, SRP, r) for v in a]
    ao = [d.port(v, OUT, SRP, r) for v in a]
    yc = d.port(y, IN, CPORT, 1)
    yi = [d.port(y, IN, DRP, r) for _ in range(2)]
    yo = d.port(y, OUT, SRP, r)
    pk = d.port(snk, IN, SRP, r)
    d.connect(ps, xi, r, Q_in)
    d.connect(pq1, xc, 1)
    d.connect(pq2, yc, 1)
    for k in range(2):
        d.connect(xo[k], ai[k], r)
        d.connect(ao[k], yi[k], r)
        d.control(pq1, xo[k], k + 1)
        d.control(pq2, yi[k], k + 1)
    d.connect(yo, pk, r)
    rng = np.random.default_rng(seed)
    d.frames[src] = [(rng.standard_normal(r) + 1j * rng.standard_normal(r)).astype(np.complex64)
                     for _ in range(n_frames)]
    d.side[q1] = np.array([(0, r, 0, t) for t in routes_x], np.int64).reshape(-1, 4)
    if q2 is not None:
        d.side[q2] = np.array([(0, r, 0, t) for t in routes_y], np.int64).reshape(-1, 4)
    return d


def cases():
    """name -> description with its expected end."""
    out = {}
    out["thres_med_cycle_undelayed"] = thres_med_cycle(0, 2)
    out["thres_med_cycle_undelayed_input_pending"] = thres_med_cycle(0, 5)
    out["thres_med_cycle_delayed"] = thres_med_cycle(1, 4)
    out["gauss_delay_fills_capacity"] = gauss_delay_capacity(3, 4, C=3)
    out["gauss_delay_below_capacity"] = gauss_delay_capacity(3, 4, C=4)
    d = switch_select([0, 0, 1, 0], [1, 1, 1, 1], 4)
    d.expect = "deadlock"
    out["mismatched_control_streams"] = d
    d = switch_select([0], [1], 1)
    d.expect = "deadlock"
    out["mismatched_first_token"] = d
    d = switch_select([0, 1, 1, 0, 1], None, 5)
    d.expect = "normal"
    out["one_control_stream"] = d
    d = switch_select([1, 0, 0], None, 3, Q_in=2)
    d.expect = "normal"                      # a block of the delay is left on x's input
    out["delay_left_on_dynamic_input"] = d
    d = switch_select([0, 1], None, 7)
    d.expect = "normal"                      # control ran out; frames wait in a full FIFO
    out["more_frames_than_tokens"] = d
    d = switch_select([0, 1, 1, 0, 1], None, 2)
    d.expect = "normal"                      # frames ran out; x holds a token
    out["more_tokens_than_frames"] = d
    d = switch_select([0, 1, 0, 1, 0, 1, 0], [0, 1, 0, 1], 7)
    d.expect = "normal"                      # y's control ran out first
    out["matched_prefix_then_y_exhausted"] = d
    return out


# ---------------------------------------------------------------- oracle side
def build_oracle(d):
    from oracle import moc
    g = moc.Graph()
    for kind, params in d.actors:
        g.actor(getattr(moc, kind), **params)
    for (a, dr, k, atr, u8) in d.ports:
        g.port(a, dr, k, atr, u8=u8)
    for (s, t, r, q) in d.fifos:
        g.connect(s, t, r, q)
    for (c, p, e) in d.table:
        g.control(c, p, e)
    g.finalize(d.C)
    for a, fr in d.frames.items():
        g.push(a, fr)
    for a, side in d.side.items():
        g.push(a, side)
    return g


def run_oracle(d):
    """(status 'normal'|'deadlock', graph) after running to the stop."""
    from oracle import moc
    g = build_oracle(d)
    try:
        g.run()
        return "normal", g
    except moc.PruneError as e:
        if e.code != moc.E_DEADLOCK:
            raise
        return "deadlock", g
