"""Compile-time analysis of a PRUNE graph (oracle, test infrastructure only).

Follows Sec. IV (adjacency, chains, linked ports, design rules 1-5) and
Sec. V (dynamic processing graphs, their dynamic components, DPG validity,
consistency of each component as an SDF graph with its buffer bound
beta(f)).  Simple chains are found by exhaustive enumeration, which is the
definition written out; it is exponential and meant for the small graphs of
the tests.

Readings where the paper is silent or leaves a choice (each is listed with
its reason in the design notes):
* Adjacency and chains use data FIFOs only (FIFOs into control ports are
  left out): a chain through a configuration actor never connects two DRPs.
* A dynamic actor is an actor with at least one external DRP.  A filter bank
  whose branch DRPs are internal is a merged DPG and counts as a static
  processing actor here.
* Linked DRPs are DRPs of two distinct actors.
* DPGs: an actor x with output DRPs and an actor y with input DRPs form a
  DPG when a DRP of x and a DRP of y are linked; q is the parent of the
  control output port feeding x.  An actor linked to more than one partner,
  or a dynamic actor in no DPG, is reported.
* DPG validity adds (c) to the paper's (a) and (b): a FIFO with exactly one
  end in a DC attaches to a DRP of x or y.  Without it an SRP of x feeding a
  DC would produce while the DC is inactive, so the DC's schedule would not
  describe every execution.
* The periodic schedule P(Z_k) of a DC fires x, then the DC's actors in
  increasing id, then y, each once (symmetric rates make every repetition
  count one), always taking the first fireable actor in that order.  The
  buffer bound of a FIFO is its largest token count over the initial state
  and the state after each firing.  Actors outside every DC are scheduled
  the same way (in id order) for the FIFOs among them, control FIFOs
  included.  A schedule that cannot complete is a deadlock, and its FIFOs
  get no bound (-1).

Report (every list sorted, every id an int):
  linked      [(p, p2)] linked DRP pairs, p < p2
  dpgs        [(q, x, y, control port)] in increasing x, then y
  dcs         [(dpg, element, actors tuple, direct fifo or -1)]
  dc_of_actor [dc index or -1] per actor
  beta        [bound or -1] per FIFO
  violations  sorted unique [(code, a, b)] with the codes below

Parity unpinned parts: none; pinned by tests/test_oracle_analysis.py (the
Sec. V example and its three DCs, the rule illustrations of Sec. IV, the
deadlock of mismatched control elements against the executor, the liveness
of cycles against brute-force cycle enumeration, the paper's DPD graph).
"""
from __future__ import annotations

from .moc import IN, OUT, SRP, DRP, CPORT, CONFIG

# violation codes
RULE1, RULE2, RULE3_KIND, RULE3_SHARED, RULE4, RULE5 = 1, 2, 31, 32, 4, 5
DPG_A, DPG_B_DC, DPG_B_COUNT, DPG_C = 10, 11, 12, 13
PAIRING, UNPAIRED = 40, 41
DEADLOCK_DC, DEADLOCK_TOP = 20, 21


class _View:
    """Structure of a moc.Graph needed by the analysis."""

    def __init__(self, g):
        self.n_actors = len(g.actors)
        self.ports = g.ports
        self.fifos = g.fifos
        self.table = g.table
        self.kind = [a.kind for a in g.actors]
        self.ext_ports = [list(a.ports) for a in g.actors]
        # data FIFOs give adjacency; control FIFOs end in a control port
        self.is_ctrl = [g.ports[d].kind == CPORT for (s, d, r, q) in g.fifos]
        self.nbrs = [set() for _ in range(self.n_actors)]
        for f, (s, d, r, q) in enumerate(g.fifos):
            if self.is_ctrl[f]:
                continue
            u, v = g.ports[s].actor, g.ports[d].actor
            if u != v:
                self.nbrs[u].add(v)
                self.nbrs[v].add(u)

    def drps(self, a):
        return [p for p in self.ext_ports[a] if self.ports[p].kind == DRP]

    def dynamic(self, a):
        return bool(self.drps(a))

    def static_processing(self, a):
        return not self.dynamic(a) and self.kind[a] != CONFIG

    def controller(self, a):
        """Control output port feeding the control port of actor a, or -1."""
        for p in self.ext_ports[a]:
            port = self.ports[p]
            if port.dir == IN and port.kind == CPORT and port.fifos:
                return self.fifos[port.fifos[0]][0]
        return -1

    def cport_fifo(self, a):
        for p in self.ext_ports[a]:
            port = self.ports[p]
            if port.dir == IN and port.kind == CPORT and port.fifos:
                return port.fifos[0]
        return -1

    def other_end(self, f, p):
        s, d, _, _ = self.fifos[f]
        return self.ports[d].actor if s == p else self.ports[s].actor

    def simple_paths(self, u, v, banned):
        """Every simple path from u to v avoiding the actors in `banned`."""
        out = []
        if u in banned or v in banned:
            return out
        stack = [(u, [u])]
        while stack:
            a, path = stack.pop()
            if a == v:
                out.append(tuple(path))
                continue
            for b in sorted(self.nbrs[a]):
                if b not in banned and b not in path:
                    stack.append((b, path + [b]))
        return out

    def on_simple_path(self, b, x, y):
        """True if actor b lies on a simple chain connecting x and y."""
        if b in (x, y):
            return True
        return any(b in p for p in self.simple_paths(x, y, set()))


def _linked(V):
    """Linked DRP pairs with their connecting subchains (Sec. IV)."""
    drps = [p for a in range(V.n_actors) for p in V.drps(a)]
    pairs = {}
    for i, p in enumerate(drps):
        for p2 in drps[i + 1:]:
            x, y = V.ports[p].actor, V.ports[p2].actor
            if x == y:
                continue
            direct = any(f in V.ports[p2].fifos for f in V.ports[p].fifos)
            chains = set()
            for f in V.ports[p].fifos:
                if V.is_ctrl[f]:
                    continue
                u = V.other_end(f, p)
                for f2 in V.ports[p2].fifos:
                    if V.is_ctrl[f2] or f2 == f:
                        continue
                    w = V.other_end(f2, p2)
                    if u in (x, y) or w in (x, y):
                        continue
                    chains.update(V.simple_paths(u, w, {x, y}))
            if direct or chains:
                pairs[(min(p, p2), max(p, p2))] = sorted(chains)
    return pairs


def _schedule(V, order, fifos):
    """Fire every actor of `order` once, always the first fireable one in
    that order; returns {fifo: bound} or None on deadlock."""
    tok = {f: V.fifos[f][3] for f in fifos}
    bound = dict(tok)
    ins = {a: [f for f in fifos if V.ports[V.fifos[f][1]].actor == a] for a in order}
    outs = {a: [f for f in fifos if V.ports[V.fifos[f][0]].actor == a] for a in order}
    left = list(order)
    while left:
        for a in left:
            if all(tok[f] >= V.fifos[f][2] for f in ins[a]):
                break
        else:
            return None
        left.remove(a)
        for f in ins[a]:
            tok[f] -= V.fifos[f][2]
        for f in outs[a]:
            tok[f] += V.fifos[f][2]
        for f in fifos:
            bound[f] = max(bound[f], tok[f])
    return bound


def analyze(g):
    V = _View(g)
    viol = set()
    linked = _linked(V)

    # Rule 1: linked DRPs share the control output port and element.
    for (p, p2) in linked:
        c, c2 = V.controller(V.ports[p].actor), V.controller(V.ports[p2].actor)
        e, e2 = V.table.get((c, p), 0), V.table.get((c2, p2), 0)
        if not (c >= 0 and c == c2 and e == e2 and e > 0):
            viol.add((RULE1, p, p2))

    # Rule 2: one control output port reaches its dynamic actors with equal delay.
    by_port = {}
    for a in range(V.n_actors):
        if V.dynamic(a) and V.controller(a) >= 0:
            by_port.setdefault(V.controller(a), []).append(a)
    for c, acts in by_port.items():
        acts.sort()
        d0 = V.fifos[V.cport_fifo(acts[0])][3]
        for a in acts[1:]:
            if V.fifos[V.cport_fifo(a)][3] != d0:
                viol.add((RULE2, acts[0], a))

    # Rules 3 and 5 over the connecting subchains.
    assoc = {}
    for (p, p2), chains in linked.items():
        x, y = V.ports[p].actor, V.ports[p2].actor
        members = set()
        for S in chains:
            members.update(S)
        for a in members:
            if not V.static_processing(a):
                viol.add((RULE3_KIND, a, -1))
            assoc.setdefault(a, set()).add((min(x, y), max(x, y)))
        for a in members:
            for f, (s, d, r, q) in enumerate(V.fifos):
                if V.is_ctrl[f]:
                    continue
                ends = (V.ports[s].actor, V.ports[d].actor)
                if a not in ends:
                    continue
                b_port = d if V.ports[s].actor == a else s
                b = V.ports[b_port].actor
                if b == a or b in members or V.ports[b_port].kind != SRP:
                    continue
                if not V.on_simple_path(b, x, y):
                    viol.add((RULE5, b, -1))
    for a, prs in assoc.items():
        if len(prs) > 1:
            viol.add((RULE3_SHARED, a, -1))

    # Rule 4: single-sided dynamism.
    for a in range(V.n_actors):
        dirs = {V.ports[p].dir for p in V.drps(a)}
        if IN in dirs and OUT in dirs:
            viol.add((RULE4, a, -1))

    # DPGs: x with output DRPs linked to y with input DRPs.
    partners = {}
    for (p, p2) in linked:
        for (pa, pb) in ((p, p2), (p2, p)):
            if V.ports[pa].dir == OUT and V.ports[pb].dir == IN:
                partners.setdefault(V.ports[pa].actor, set()).add(V.ports[pb].actor)
    dpg_pairs = sorted((x, y) for x, ys in partners.items() for y in ys)
    seen_x, seen_y = {}, {}
    for x, y in dpg_pairs:
        seen_x[x] = seen_x.get(x, 0) + 1
        seen_y[y] = seen_y.get(y, 0) + 1
    for a, n in list(seen_x.items()) + list(seen_y.items()):
        if n > 1:
            viol.add((PAIRING, a, -1))
    in_dpg = {a for pr in dpg_pairs for a in pr}
    for a in range(V.n_actors):
        if V.dynamic(a) and a not in in_dpg:
            viol.add((UNPAIRED, a, -1))

    dpgs, dcs = [], []
    dc_of_actor = [-1] * V.n_actors
    beta = [-1] * len(V.fifos)
    dc_fifos = set()
    for di, (x, y) in enumerate(dpg_pairs):
        cx = V.controller(x)
        q = V.ports[cx].actor if cx >= 0 else -1
        dpgs.append((q, x, y, cx))
        removed = {x, y} | ({q} if q >= 0 else set())
        # components of the rest (Sec. V procedure, step 2)
        comp = {}
        for a in range(V.n_actors):
            if a in removed or a in comp:
                continue
            todo, members = [a], set()
            while todo:
                b = todo.pop()
                if b in members:
                    continue
                members.add(b)
                todo.extend(n for n in V.nbrs[b] if n not in removed)
            for b in members:
                comp[b] = min(members)
        # attachments of the DRPs of x and y; direct links become dummy DCs
        attach, direct = {}, []
        for p in V.drps(x) + V.drps(y):
            for f in V.ports[p].fifos:
                if V.is_ctrl[f]:
                    continue
                other = V.other_end(f, p)
                s, d = V.fifos[f][0], V.fifos[f][1]
                if {V.ports[s].actor, V.ports[d].actor} == {x, y}:
                    if V.ports[s].kind == DRP and V.ports[d].kind == DRP and f not in direct:
                        direct.append(f)
                    continue
                if other in comp:
                    attach.setdefault(comp[other], []).append(p)
        keys = sorted(attach)
        local = []
        for k in keys:
            local.append((tuple(sorted(a for a, c in comp.items() if c == k)), attach[k], -1))
        for f in sorted(direct):
            local.append(((), [V.fifos[f][0], V.fifos[f][1]], f))
        elements = []
        for ci, (acts, ports, f) in enumerate(local):
            idx = len(dcs)
            E = {V.table.get((V.controller(V.ports[p].actor), p), 0) for p in ports}
            el = E.pop() if len(E) == 1 else -1
            if el == -1:
                viol.add((DPG_B_DC, di, idx))
            if not (any(V.ports[p].actor == x for p in ports) and
                    any(V.ports[p].actor == y for p in ports)):
                viol.add((DPG_A, di, idx))
            elements.append(el)
            dcs.append((di, el, acts, f))
            for a in acts:
                dc_of_actor[a] = idx
            # validity (c) and the DC's FIFOs
            members = set(acts)
            H = [f] if f >= 0 else []
            for g_f, (s, d, r, qd) in enumerate(V.fifos):
                if V.is_ctrl[g_f] or g_f in H:
                    continue
                u, w = V.ports[s].actor, V.ports[d].actor
                if u not in members and w not in members:
                    continue
                inside = all(t in members or t in (x, y) for t in (u, w))
                if inside:
                    H.append(g_f)
                ok = (u in members and w in members) or \
                     (u == x and w in members and V.ports[s].kind == DRP) or \
                     (w == y and u in members and V.ports[d].kind == DRP)
                if not ok:
                    viol.add((DPG_C, di, g_f))
            order = [x] + sorted(members) + [y]
            bnd = _schedule(V, order, sorted(H))
            if bnd is None:
                viol.add((DEADLOCK_DC, di, idx))
            for h in H:
                dc_fifos.add(h)
                beta[h] = -1 if bnd is None else bnd[h]
        used = {V.table.get((V.controller(V.ports[p].actor), p), 0) for p in V.drps(x) + V.drps(y)}
        good = [e for e in elements if e != -1]
        if len(set(good)) != len(good) or len(used) != len(local):
            viol.add((DPG_B_COUNT, di, -1))

    # top level: actors outside every DC, FIFOs among them (control included)
    top = [a for a in range(V.n_actors) if dc_of_actor[a] == -1]
    tset = set(top)
    T = [f for f, (s, d, r, q) in enumerate(V.fifos)
         if f not in dc_fifos and V.ports[s].actor in tset and V.ports[d].actor in tset]
    bnd = _schedule(V, top, T)
    if bnd is None:
        viol.add((DEADLOCK_TOP, -1, -1))
    for f in T:
        beta[f] = -1 if bnd is None else bnd[f]

    return {"linked": sorted(linked), "dpgs": dpgs, "dcs": dcs,
            "dc_of_actor": dc_of_actor, "beta": beta, "violations": sorted(viol)}
