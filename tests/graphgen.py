"""Seeded random graph structures for the analysis parity tests.

A structure is a plain description (actor kinds, ports, FIFOs, control-table
entries) that the tests build through each side's graph API.  This module
holds no part of the analysis."""
from __future__ import annotations

import numpy as np

SOURCE, CONFIG, SWITCH, SELECT, PASSTHROUGH, SINK = 0, 1, 3, 4, 5, 6
IN, OUT = 0, 1
SRP, DRP, CPORT = 0, 1, 2


class Structure:
    def __init__(self):
        self.actors = []          # kind
        self.n_elements = {}      # config actor -> control-value size
        self.ports = []           # (actor, dir, kind)
        self.fifos = []           # (src port, dst port, rate, delay)
        self.table = []           # (control port, drp, element)
        self._in_used = set()

    def actor(self, kind, n_elements=4):
        self.actors.append(kind)
        a = len(self.actors) - 1
        if kind == CONFIG:
            self.n_elements[a] = n_elements
        return a

    def port(self, a, d, k):
        self.ports.append((a, d, k))
        return len(self.ports) - 1

    def connect(self, s, d, rate=1, delay=0):
        assert d not in self._in_used
        self._in_used.add(d)
        self.fifos.append((s, d, int(rate), int(delay)))
        return len(self.fifos) - 1

    def control(self, c, p, e):
        self.table.append((c, p, int(e)))


def random_structure(seed):
    """Unconstrained graphs: every kind of violation shows up."""
    rng = np.random.default_rng(seed)
    S = Structure()
    cfg_ports = []
    for _ in range(int(rng.integers(1, 3))):
        q = S.actor(CONFIG, n_elements=4)
        for _ in range(int(rng.integers(1, 3))):
            cfg_ports.append(S.port(q, OUT, SRP))
    outs, ins, cports, drps = [], [], [], []
    for _ in range(int(rng.integers(1, 3))):
        outs.append(S.port(S.actor(SOURCE), OUT, SRP))
    for _ in range(int(rng.integers(0, 4))):
        x = S.actor(SWITCH)
        ins.append(S.port(x, IN, SRP))
        cports.append(S.port(x, IN, CPORT))
        for _ in range(int(rng.integers(1, 4))):
            p = S.port(x, OUT, DRP)
            outs.append(p); drps.append(p)
        if rng.random() < 0.1:
            p = S.port(x, IN, DRP)
            ins.append(p); drps.append(p)
    for _ in range(int(rng.integers(0, 4))):
        y = S.actor(SELECT)
        cports.append(S.port(y, IN, CPORT))
        for _ in range(int(rng.integers(1, 4))):
            p = S.port(y, IN, DRP)
            ins.append(p); drps.append(p)
        outs.append(S.port(y, OUT, SRP))
    for _ in range(int(rng.integers(0, 7))):
        a = S.actor(PASSTHROUGH)
        for _ in range(int(rng.integers(1, 3))):
            ins.append(S.port(a, IN, SRP))
        for _ in range(int(rng.integers(1, 3))):
            outs.append(S.port(a, OUT, SRP))
    for _ in range(int(rng.integers(1, 3))):
        ins.append(S.port(S.actor(SINK), IN, SRP))
    for d in ins:
        if rng.random() < 0.9:
            s = outs[int(rng.integers(0, len(outs)))]
            S.connect(s, d, rng.integers(1, 4), rng.integers(0, 5) if rng.random() < 0.4 else 0)
    for c in cports:
        if rng.random() < 0.95:
            S.connect(cfg_ports[int(rng.integers(0, len(cfg_ports)))], c, 1,
                      1 if rng.random() < 0.15 else 0)
    feeder = {}
    for (s, d, r, q) in S.fifos:
        if S.ports[d][2] == CPORT:
            feeder[S.ports[d][0]] = s
    for p in drps:
        a = S.ports[p][0]
        c = feeder.get(a, cfg_ports[0])
        if rng.random() < 0.1:
            c = cfg_ports[int(rng.integers(0, len(cfg_ports)))]
        if rng.random() < 0.9:
            S.control(c, p, rng.integers(0, 4) if rng.random() < 0.2 else rng.integers(1, 4))
    return S


def dpg_structure(seed):
    """One to three DPGs (switch x, select y) whose DCs are small random
    graphs of copy actors, some with cycles and delays, sometimes a direct
    x-y link, elements one per DC: mostly valid graphs."""
    rng = np.random.default_rng(seed)
    S = Structure()
    for _ in range(int(rng.integers(1, 4))):
        q = S.actor(CONFIG, n_elements=6)
        qp = S.port(q, OUT, SRP)
        src = S.port(S.actor(SOURCE), OUT, SRP)
        x = S.actor(SWITCH)
        xi = S.port(x, IN, SRP)
        xc = S.port(x, IN, CPORT)
        y = S.actor(SELECT)
        yc = S.port(y, IN, CPORT)
        yo = S.port(y, OUT, SRP)
        snk = S.port(S.actor(SINK), IN, SRP)
        r = int(rng.integers(1, 4))
        S.connect(src, xi, r)
        S.connect(yo, snk, r)
        S.connect(qp, xc, 1)
        S.connect(qp, yc, 1, 0 if rng.random() < 0.9 else 1)
        n_dc = int(rng.integers(1, 4))
        for k in range(n_dc):
            el = k + 1 if rng.random() < 0.93 else int(rng.integers(1, 4))
            m = int(rng.integers(1, 4))
            acts = [S.actor(PASSTHROUGH) for _ in range(m)]
            for i, a in enumerate(acts):
                px = S.port(x, OUT, DRP)
                S.connect(px, S.port(a, IN, SRP), r, rng.integers(0, 2 * r + 1) if rng.random() < 0.3 else 0)
                S.control(qp, px, el)
                py = S.port(y, IN, DRP)
                S.connect(S.port(a, OUT, SRP), py, r, rng.integers(0, 2 * r + 1) if rng.random() < 0.3 else 0)
                S.control(qp, py, el)
                if i:
                    prev = acts[int(rng.integers(0, i))]
                    S.connect(S.port(prev, OUT, SRP), S.port(a, IN, SRP), r,
                              rng.integers(0, 2 * r + 1) if rng.random() < 0.5 else 0)
            for _ in range(int(rng.integers(0, 3))):
                u, w = acts[int(rng.integers(0, m))], acts[int(rng.integers(0, m))]
                S.connect(S.port(u, OUT, SRP), S.port(w, IN, SRP), r, int(rng.integers(0, 2 * r + 1)))
        if rng.random() < 0.3:
            px = S.port(x, OUT, DRP)
            py = S.port(y, IN, DRP)
            S.connect(px, py, r, 0)
            S.control(qp, px, n_dc + 1)
            S.control(qp, py, n_dc + 1)
    return S
