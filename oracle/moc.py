"""PRUNE model of computation, sequential float64 executor (oracle).

Follows Sec. III (graph G = (A, F), ports, FIFOs, actor types, Eq. 1,
delays), the design-rule checks that are local to one actor (Sec. IV, rule 4)
and the runtime of Sec. VI (actor functions init/control/fire, FIFO capacity
of Eq. 2 and the access pattern described with Fig. 6).

Readings where the paper is silent (each is listed with its reason in the
design notes):
* Rate parameter: a control token carries (mask, rate).  A port flagged
  ``param`` uses ``rate`` (plus its ``halo``) instead of its atr for the
  firing; Eq. 1 is unchanged otherwise and reduces to it when rate == atr.
  FIFOs between parameterised ports keep a block stride of atr (Eq. 2 and the
  slot rule are unchanged) and carry no delay.
* FIFO slot rule with delay Q and rate r (Fig. 6 text): aligned case
  (Q mod r == 0) is a ring of max(rC, Q) slots in blocks of r with Q/r blocks
  prefilled; unaligned case is a ring of rC slots with a Q-slot overflow
  area, write j at Q + (j mod C) r, read i at (i mod C) r, and every write that
  runs past slot rC-1 is followed by a copy of its overflow back to slot 0.
* Scheduling: round-robin over actors in creation order, each actor fires at
  most once per sweep; a dynamic actor peeks its control token, decodes it,
  checks availability of the decoded rates, and only then consumes it.
* Termination: the run ends when no actor can fire.  It is a normal end
  when every actor that cannot fire waits, through a chain of blocking reads,
  on a source or configuration actor whose external input is used up; it is
  a deadlock when some actor waits in a cycle or behind a FIFO that is never
  drained, or when a dynamic actor waits on data its linked partner's firing
  of the same control token did not send (linked DRPs set differently,
  Sec. V).

Parity: pinned by tests/test_oracle_moc.py (the Fig. 6 worked example, Eq. 2
in both cases, Eq. 1 and the control-table example, the Fig. 1 rates, token
conservation, FIFO order through delayed channels, schedule independence,
brute-force deadlock freedom on small valid graphs and the deadlock of
mismatched control streams).
"""
from __future__ import annotations

import numpy as np

from .filterbank import fb_frame, basis
from .motion import gauss5, thres, med5

# Status codes (names match the C library's; values are the library's too).
E_ARG, E_STATE, E_RATE_MISMATCH, E_PORT_KIND, E_RULE4, E_CONNECT = -1, -2, -3, -4, -5, -6
E_DELAY, E_TOKEN, E_DEADLOCK, E_CAPACITY, E_HIP, E_UNSUPPORTED = -7, -8, -9, -10, -11, -12

IN, OUT, INTERNAL = 0, 1, 2
SRP, DRP, CPORT = 0, 1, 2
(SOURCE, CONFIG, FILTERBANK, SWITCH, SELECT, PASSTHROUGH, SINK,
 POLY, FIR, ADD, GAUSS5, THRES, MED5) = range(13)
KIND_NAMES = ["SOURCE", "CONFIG", "FILTERBANK", "SWITCH", "SELECT", "PASSTHROUGH",
              "SINK", "POLY", "FIR", "ADD", "GAUSS5", "THRES", "MED5"]
PIXEL_KINDS = (GAUSS5, THRES, MED5)   # Motion Detection actors on uint8 frames


class PruneError(Exception):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


# --------------------------------------------------------------------------
# FIFO capacity (Eq. 2) and the slot rule (Fig. 6 access pattern)
# --------------------------------------------------------------------------

def fifo_capacity(r: int, Q: int, C: int) -> int:
    """Eq. 2 in tokens: r*C + Q when Q is not a multiple of r, else max(r*C, Q)."""
    if r <= 0 or C <= 0 or Q < 0:
        raise PruneError(E_ARG, "rate and C must be positive, delay non-negative")
    if Q % r:
        return r * C + Q
    return max(r * C, Q)


def _ring_blocks(r, Q, C):
    return fifo_capacity(r, Q, C) // r


def fifo_write_slot(r: int, Q: int, C: int, j: int) -> int:
    """First slot written by the j-th (0-based) write."""
    if Q % r == 0:
        return ((Q // r + j) % _ring_blocks(r, Q, C)) * r
    return Q + (j % C) * r


def fifo_read_slot(r: int, Q: int, C: int, i: int) -> int:
    """First slot read by the i-th (0-based) read."""
    if Q % r == 0:
        return (i % _ring_blocks(r, Q, C)) * r
    return (i % C) * r


class FifoState:
    """Physical buffer of Eq. 2 size plus counters.  Tokens are stored at the
    slots the rule gives, so reading back in order checks the rule itself."""

    def __init__(self, fid, rate, delay, C, token_dtype, block_counts):
        r, Q = rate, delay
        if Q % r and Q >= r * C:
            raise PruneError(E_DELAY, f"fifo {fid}: unaligned delay {Q} >= r*C = {r*C}")
        if Q % r and Q < r and Q + r > r * C:
            # Neither the first write (its ring slots still hold delay tokens)
            # nor the first read (fewer than r tokens) could ever start.
            raise PruneError(E_DELAY, f"fifo {fid}: delay {Q} and one block do not fit in r*C")
        self.id, self.r, self.Q, self.C = fid, r, Q, C
        self.capacity = fifo_capacity(r, Q, C)
        self.aligned = (Q % r == 0)
        self.buf = np.zeros(self.capacity, dtype=token_dtype)
        self.block_counts = block_counts
        self.counts = {}                  # slot -> count, for parameterised FIFOs
        self.writes = 0
        self.reads = 0
        self.tokens_written = 0
        self.tokens_read = 0
        self.max_occ = Q
        self.log_w = []                   # (writer firing#, j, slot, count)
        self.log_r = []                   # (reader firing#, i, slot, count)

    @property
    def occupancy(self):
        return self.Q + self.tokens_written - self.tokens_read

    def can_write(self) -> bool:
        r, Q, C = self.r, self.Q, self.C
        j, i = self.writes, self.reads
        if self.aligned:
            return (Q // r + j) - i < _ring_blocks(r, Q, C)
        return i * r >= Q + (j + 1) * r - r * C

    def can_read(self) -> bool:
        r, Q = self.r, self.Q
        i, w = self.reads, self.writes
        if self.aligned:
            return i < Q // r + w
        return Q + w * r >= (i + 1) * r

    def write(self, data, firing):
        r, Q, C = self.r, self.Q, self.C
        count = len(data)
        if not self.block_counts and count != r:
            raise PruneError(E_TOKEN, f"fifo {self.id}: write of {count} tokens, rate {r}")
        if count > r or count < 0:
            raise PruneError(E_TOKEN, f"fifo {self.id}: write of {count} > atr {r}")
        j = self.writes
        slot = fifo_write_slot(r, Q, C, j)
        self.buf[slot:slot + count] = data
        if not self.aligned and slot + r > r * C:
            end = slot + r
            self.buf[0:end - r * C] = self.buf[r * C:end]     # copy-back
        if self.block_counts:
            self.counts[slot] = count
        self.log_w.append((firing, j, slot, count))
        self.writes += 1
        self.tokens_written += count
        self.max_occ = max(self.max_occ, self.occupancy)
        if self.occupancy > self.capacity:
            raise PruneError(E_CAPACITY, f"fifo {self.id}: occupancy above Gamma")

    def peek_count(self):
        slot = fifo_read_slot(self.r, self.Q, self.C, self.reads)
        return self.counts.get(slot, self.r) if self.block_counts else self.r

    def peek(self):
        slot = fifo_read_slot(self.r, self.Q, self.C, self.reads)
        return self.buf[slot]

    def read(self, firing):
        r, Q, C = self.r, self.Q, self.C
        i = self.reads
        slot = fifo_read_slot(r, Q, C, i)
        count = self.counts.pop(slot, r) if self.block_counts else r
        data = self.buf[slot:slot + count].copy()
        self.log_r.append((firing, i, slot, count))
        self.reads += 1
        self.tokens_read += count
        return data


# --------------------------------------------------------------------------
# Graph description
# --------------------------------------------------------------------------

class Port:
    __slots__ = ("id", "actor", "dir", "kind", "atr", "param", "halo", "fifos", "u8")

    def __init__(self, pid, actor, dir, kind, atr, param, halo, u8=False):
        self.id, self.actor, self.dir, self.kind = pid, actor, dir, kind
        self.atr, self.param, self.halo = atr, param, halo
        self.u8 = u8             # one-byte tokens (pixels) instead of complex samples
        self.fifos = []


class Actor:
    def __init__(self, aid, kind, params):
        self.id, self.kind, self.params = aid, kind, params
        self.ports = []          # external port ids in creation order
        self.branches = []       # internal branch DRPs of a filter bank
        self.firings = 0
        self.state = {}


CTRL_DTYPE = np.dtype([("mask", np.uint32), ("rate", np.uint32)])


class Graph:
    """Build with actor()/port()/connect()/control(), then finalize(C)."""

    def __init__(self):
        self.actors = []
        self.ports = []
        self.fifos = []          # (src_pid, dst_pid, rate, delay)
        self.table = {}          # (control output pid, drp pid) -> element (1-based)
        self.finalized = False
        self.C = None

    # ---- construction ----------------------------------------------------
    def _check_open(self):
        if self.finalized:
            raise PruneError(E_STATE, "graph already finalized")

    def actor(self, kind, **params) -> int:
        self._check_open()
        if kind not in range(13):
            raise PruneError(E_ARG, f"unknown actor kind {kind}")
        a = Actor(len(self.actors), kind, dict(params))
        self.actors.append(a)
        if kind == FILTERBANK:
            taps = np.asarray(params["taps"])
            nb, Km = taps.shape[0], taps.shape[1]
            if params.get("Kmax", Km) != Km or len(params["bank_L"]) != nb:
                raise PruneError(E_ARG, "taps shape does not match Kmax / bank_L")
            a.params.setdefault("Kmax", Km)
            a.params.setdefault("windowed", False)
            for _ in range(nb * Km):
                pid = len(self.ports)
                self.ports.append(Port(pid, a.id, INTERNAL, DRP, 0, False, 0))
                a.branches.append(pid)
        return a.id

    def port(self, aid, dir, kind, atr, param=False, halo=0, u8=False) -> int:
        self._check_open()
        if not (0 <= aid < len(self.actors)) or dir not in (IN, OUT) or kind not in (SRP, DRP, CPORT):
            raise PruneError(E_ARG, "bad port arguments")
        if atr <= 0:
            raise PruneError(E_ARG, "atr must be positive")
        pid = len(self.ports)
        self.ports.append(Port(pid, aid, dir, kind, int(atr), bool(param), int(halo), bool(u8)))
        self.actors[aid].ports.append(pid)
        return pid

    def connect(self, src, dst, rate, delay=0) -> int:
        self._check_open()
        for p in (src, dst):
            if not (0 <= p < len(self.ports)):
                raise PruneError(E_ARG, "unknown port")
        ps, pd = self.ports[src], self.ports[dst]
        if ps.dir != OUT or pd.dir != IN:
            raise PruneError(E_CONNECT, "a FIFO runs from an output port to an input port")
        if pd.fifos:
            raise PruneError(E_CONNECT, "an input port has exactly one FIFO")
        if rate <= 0 or delay < 0:
            raise PruneError(E_ARG, "fiforate must be positive, delay non-negative")
        fid = len(self.fifos)
        self.fifos.append((src, dst, int(rate), int(delay)))
        ps.fifos.append(fid)
        pd.fifos.append(fid)
        return fid

    def control(self, ctl_port, drp, element):
        self._check_open()
        if not (0 <= ctl_port < len(self.ports)) or not (0 <= drp < len(self.ports)) or element < 0:
            raise PruneError(E_ARG, "bad control-table entry")
        self.table[(ctl_port, drp)] = int(element)

    # ---- helpers -----------------------------------------------------------
    def _ports(self, a, dir=None, kind=None):
        return [self.ports[p] for p in self.actors[a].ports
                if (dir is None or self.ports[p].dir == dir) and
                (kind is None or self.ports[p].kind == kind)]

    def cport(self, a):
        cps = self._ports(a, IN, CPORT)
        return cps[0] if cps else None

    def drps(self, a):
        act = self.actors[a]
        if act.kind == FILTERBANK:
            return [self.ports[p] for p in act.branches]
        return self._ports(a, kind=DRP)

    def controller(self, a):
        """Control output port feeding the cport of actor a."""
        cp = self.cport(a)
        f = self.fifos[cp.fifos[0]]
        return self.ports[f[0]]

    # ---- validation (Sec. III local rules, rule 4) + sizing (Eq. 2) -------
    def finalize(self, C: int):
        self._check_open()
        if C <= 0:
            raise PruneError(E_ARG, "C must be positive")
        for p in self.ports:
            if p.dir == IN and len(p.fifos) != 1:
                raise PruneError(E_CONNECT, f"input port {p.id} needs exactly one FIFO")
            if p.dir == OUT and not p.fifos:
                raise PruneError(E_CONNECT, f"output port {p.id} is not connected")
        for fid, (s, d, rate, Q) in enumerate(self.fifos):
            ps, pd = self.ports[s], self.ports[d]
            if ps.atr != rate or pd.atr != rate:
                raise PruneError(E_RATE_MISMATCH, f"fifo {fid}: atr differs from fiforate")
            if ps.param != pd.param or ps.halo != pd.halo:
                raise PruneError(E_RATE_MISMATCH, f"fifo {fid}: rate parameterisation differs")
            if ps.param and Q:
                raise PruneError(E_DELAY, f"fifo {fid}: delay on a parameterised FIFO")
            if ps.u8 != pd.u8:
                raise PruneError(E_RATE_MISMATCH, f"fifo {fid}: token types differ")
            if Q % rate and (Q >= rate * C or (Q < rate and Q + rate > rate * C)):
                raise PruneError(E_DELAY, f"fifo {fid}: unaligned delay does not fit r*C")
            if (pd.kind == CPORT) != (self.actors[ps.actor].kind == CONFIG):
                raise PruneError(E_PORT_KIND, f"fifo {fid}: control ports connect only to configuration actors")
        for a in self.actors:
            self._validate_actor(a)
        self.C = C
        self.finalized = True
        self._init_runtime()

    def _validate_actor(self, a):
        ins = self._ports(a.id, IN)
        outs = self._ports(a.id, OUT)
        cps = [p for p in ins if p.kind == CPORT]
        data_in = [p for p in ins if p.kind != CPORT]
        in_drp = [p for p in data_in if p.kind == DRP]
        out_drp = [p for p in outs if p.kind == DRP]
        for p in cps:
            if p.atr != 1:
                raise PruneError(E_PORT_KIND, f"control port {p.id} must have rate 1")
        dynamic_kinds = (SWITCH, SELECT, POLY, ADD)
        k = a.kind
        if k == CONFIG:
            if ins:
                raise PruneError(E_ARG, "configuration actors here take external side-information only")
            for p in outs:
                if p.kind != SRP or p.atr != 1:
                    raise PruneError(E_PORT_KIND, "control output ports are SRPs of rate 1")
                for f in p.fifos:
                    if self.ports[self.fifos[f][1]].kind != CPORT:
                        raise PruneError(E_PORT_KIND, "control output ports connect to control ports")
            if not outs:
                raise PruneError(E_ARG, "a configuration actor needs a control output port")
            return
        dynamic = k in dynamic_kinds or (k == FILTERBANK and cps)
        if not dynamic:
            if cps or in_drp or out_drp:
                raise PruneError(E_PORT_KIND, f"actor {a.id}: static actors have SRPs only")
        else:
            if len(cps) != 1:
                raise PruneError(E_PORT_KIND, f"actor {a.id}: a dynamic actor has exactly one control port")
            if k != FILTERBANK and not (in_drp or out_drp):
                raise PruneError(E_PORT_KIND, f"actor {a.id}: a dynamic actor needs a DRP")
            if in_drp and out_drp:
                raise PruneError(E_RULE4, f"actor {a.id}: dynamic inputs and outputs (rule 4)")
            ctl = self.controller(a.id)
            n_el = self.actors[ctl.actor].params.get("n_elements", 32)
            for p in self.drps(a.id):
                e = self.table.get((ctl.id, p.id), 0)
                if not (1 <= e <= n_el):
                    raise PruneError(E_PORT_KIND, f"DRP {p.id} is not controlled by the port feeding its actor")
        # Kind-specific shapes and rate relations.
        def need(cond, code, msg):
            if not cond:
                raise PruneError(code, f"actor {a.id} ({KIND_NAMES[k]}): {msg}")
        if k == SOURCE:
            need(not ins and len(outs) == 1, E_ARG, "one output port, no inputs")
        elif k == SINK:
            need(len(data_in) == 1 and not outs and not cps, E_ARG, "one input port")
        elif k in (PASSTHROUGH, FIR):
            need(len(data_in) == 1 and len(outs) == 1, E_ARG, "one input and one output")
            if k == PASSTHROUGH:
                need(data_in[0].atr == outs[0].atr and data_in[0].param == outs[0].param,
                     E_RATE_MISMATCH, "input and output rates differ")
            else:
                L = len(a.params["taps"])
                need(data_in[0].atr == outs[0].atr + L - 1, E_RATE_MISMATCH, "window = n + L - 1")
        elif k == FILTERBANK:
            need(len(data_in) == 1 and len(outs) == 1, E_ARG, "one data input and one output")
            H = max(a.params["bank_L"]) - 1
            pi, po = data_in[0], outs[0]
            need(pi.param == po.param, E_RATE_MISMATCH, "parameterisation differs")
            if a.params["windowed"]:
                need(pi.atr == po.atr + H and pi.halo == H and po.halo == 0, E_RATE_MISMATCH,
                     "windowed input = output + Lmax-1")
            else:
                need(pi.atr == po.atr and pi.halo == 0 and po.halo == 0, E_RATE_MISMATCH,
                     "input and output rates differ")
            if not cps:
                need("mask" in a.params, E_ARG, "a static filter bank needs a fixed mask")
        elif k in (SWITCH, POLY):
            need(len(data_in) == 1 and data_in[0].kind == SRP and outs and all(p.kind == DRP for p in outs),
                 E_ARG, "one SRP input, DRP outputs")
            for p in outs:
                need(p.atr == data_in[0].atr + p.halo and p.param == data_in[0].param,
                     E_RATE_MISMATCH, "output window = input + halo")
            if k == POLY:
                need(len(outs) == a.params["Kmax"], E_ARG, "one output per branch")
        elif k in PIXEL_KINDS:
            npix = a.params["W"] * a.params["H"]
            need(len(data_in) == (2 if k == THRES else 1) and len(outs) == 1, E_ARG,
                 "pixel actors: one input (two for THRES), one output")
            for p in data_in + outs:
                need(p.atr == npix and p.u8 and not p.param and not p.halo, E_RATE_MISMATCH,
                     "pixel ports carry one W*H frame of one-byte tokens")
        elif k in (SELECT, ADD):
            need(len(outs) == 1 and outs[0].kind == SRP and in_drp and len(in_drp) == len(data_in),
                 E_ARG, "DRP inputs, one SRP output")
            for p in in_drp:
                need(p.atr == outs[0].atr and p.param == outs[0].param and p.halo == 0,
                     E_RATE_MISMATCH, "input and output rates differ")

    # ---- runtime -------------------------------------------------------------
    def _init_runtime(self):
        self.fstate = []
        for fid, (s, d, rate, Q) in enumerate(self.fifos):
            ctrl = self.ports[d].kind == CPORT
            dt = CTRL_DTYPE if ctrl else (np.uint8 if self.ports[s].u8 else np.complex128)
            self.fstate.append(FifoState(fid, rate, Q, self.C, dt, self.ports[s].param))
        for a in self.actors:
            a.firings = 0
            a.log = []          # dynamic: (firing#, mask, rate, decoded bitmap over drps)
            if a.kind in (SOURCE, CONFIG):
                a.state["queue"] = []
            if a.kind == SINK:
                a.state["out"] = []
            if a.kind in (FILTERBANK, SWITCH, POLY):
                if a.kind == FILTERBANK:
                    H = max(a.params["bank_L"]) - 1
                elif a.kind == SWITCH:
                    H = max(p.halo for p in self._ports(a.id, OUT))
                else:
                    H = max(a.params["bank_L"]) - 1
                a.state["history"] = np.zeros(H, np.complex128)
            if a.kind == FILTERBANK:
                D = len(a.branches)
                a.state["branch_firings"] = np.zeros(D, np.int64)
                a.state["branch_tokens"] = np.zeros(D, np.int64)
            if a.kind == FIR:
                a.state["tokens"] = 0

    def push(self, aid, frames):
        """External input of a source (list of sample arrays) or of a
        configuration actor (array [F, 4] of side-information K, n, bank, route)."""
        a = self.actors[aid]
        if a.kind == SOURCE:
            u8 = self._ports(aid, OUT)[0].u8
            a.state["queue"].extend(np.asarray(f, np.uint8 if u8 else np.complex128).ravel()
                                    for f in frames)
        elif a.kind == CONFIG:
            a.state["queue"].extend(np.asarray(frames, np.int64).reshape(-1, 4))
        else:
            raise PruneError(E_ARG, "push goes to a source or configuration actor")

    # Configuration actor function: side-information -> control token.
    @staticmethod
    def config_token(params, side):
        K, n, bank, route = (int(v) for v in side)
        mode = params.get("mode", "prefix")
        if mode == "route":
            mask = 1 << route
        elif mode == "mask":
            # K carries any set of the bank's branches (bit b-1 = branch b)
            Kmax = params["Kmax"]
            if K >> Kmax:
                raise PruneError(E_TOKEN, "branch set beyond the bank size")
            mask = K << (bank * Kmax)
        else:
            Kmax = params["Kmax"]
            if K > Kmax:
                raise PruneError(E_TOKEN, "K above the bank size")
            mask = ((1 << K) - 1) << (bank * Kmax)
        return mask, n

    def _decode(self, a):
        """Eq. 1 with the rate parameter: returns (mask, rate, {drp pid: tokrate})."""
        cp = self.cport(a.id)
        tok = self.fstate[cp.fifos[0]].peek()
        mask, rate = int(tok["mask"]), int(tok["rate"])
        ctl = self.controller(a.id)
        n_el = self.actors[ctl.actor].params.get("n_elements", 32)
        if n_el < 32 and mask >> n_el:
            raise PruneError(E_TOKEN, "control value has more elements than the control port declares")
        rates = {}
        for p in self.drps(a.id):
            e = self.table[(ctl.id, p.id)]
            bit = (mask >> (e - 1)) & 1
            rates[p.id] = bit     # multiplied by the port's size below
        return mask, rate, rates

    def _count(self, p, rate, active=1):
        """Tokens moved through port p in this firing."""
        if not active:
            return 0
        if p.param:
            if rate < 1 or rate + p.halo > p.atr:
                raise PruneError(E_TOKEN, f"rate {rate} outside 1..atr for port {p.id}")
            return rate + p.halo
        return p.atr

    def try_fire(self, aid) -> bool:
        a = self.actors[aid]
        k = a.kind
        fs = self.fstate
        ins = [p for p in self._ports(aid, IN) if p.kind != CPORT]
        outs = self._ports(aid, OUT)

        def out_ready(ports_counts):
            for p, c in ports_counts:
                if c and not all(fs[f].can_write() for f in p.fifos):
                    return False
            return True

        def in_ready(ports_counts):
            for p, c in ports_counts:
                if c and not fs[p.fifos[0]].can_read():
                    return False
            return True

        if k == SOURCE:
            if not a.state["queue"]:
                return False
            p = outs[0]
            n = len(a.state["queue"][0])
            c = self._count(p, n) if p.param else p.atr
            if not p.param and n != p.atr:
                raise PruneError(E_TOKEN, "source frame length differs from its SRP rate")
            if not out_ready([(p, c)]):
                return False
            frame = a.state["queue"].pop(0)
            for f in p.fifos:
                fs[f].write(frame, a.firings)
            a.firings += 1
            return True

        if k == CONFIG:
            if not a.state["queue"]:
                return False
            if not out_ready([(p, 1) for p in outs]):
                return False
            side = a.state["queue"].pop(0)
            mask, rate = self.config_token(a.params, side)
            tok = np.array([(mask, rate)], dtype=CTRL_DTYPE)
            for p in outs:
                for f in p.fifos:
                    fs[f].write(tok, a.firings)
            a.firings += 1
            return True

        # Everything below may be dynamic.
        cp = self.cport(aid)
        dynamic = cp is not None
        if dynamic:
            if not fs[cp.fifos[0]].can_read():
                return False
            mask, rate, bits = self._decode(a)
        else:
            mask, bits = a.params.get("mask", 0), {}
            # rate of a static actor with parameterised ports follows its input block
            rate = None
            if ins and ins[0].param:
                f = fs[ins[0].fifos[0]]
                if not f.can_read():
                    return False
                rate = f.peek_count() - ins[0].halo

        def cnt(p):
            if p.kind == DRP:
                return self._count(p, rate, bits[p.id])
            return self._count(p, rate)

        ins_c = [(p, cnt(p)) for p in ins]
        outs_c = [(p, cnt(p)) for p in outs]
        if not in_ready(ins_c) or not out_ready(outs_c):
            return False
        # Parameterised input blocks must carry the count the firing expects.
        for p, c in ins_c:
            if c and p.param and fs[p.fifos[0]].peek_count() != c:
                raise PruneError(E_TOKEN, f"port {p.id}: block of {fs[p.fifos[0]].peek_count()} tokens, firing expects {c}")
        # Commit: consume control token, read inputs.
        firing = a.firings
        if dynamic:
            fs[cp.fifos[0]].read(firing)
            drps = self.drps(aid)
            bitmap = sum(int(bits[p.id]) << i for i, p in enumerate(drps))
            a.log.append((firing, mask, rate, bitmap))
        data = {p.id: fs[p.fifos[0]].read(firing) for p, c in ins_c if c}
        results = self._compute(a, ins_c, outs_c, data, mask, rate, bits)
        for p, c in outs_c:
            if c:
                out = results[p.id]
                for f in p.fifos:
                    fs[f].write(out, firing)
        a.firings += 1
        return True

    def _compute(self, a, ins_c, outs_c, data, mask, rate, bits):
        k = a.kind
        res = {}
        if k == SINK:
            a.state["out"].append(data[ins_c[0][0].id])
            return res
        if k in PIXEL_KINDS:
            shape = (a.params["H"], a.params["W"])
            frames = [data[p.id].reshape(shape) for p, c in ins_c]
            if k == GAUSS5:
                y = gauss5(frames[0])
            elif k == MED5:
                y = med5(frames[0])
            else:
                y = thres(frames[0], frames[1], a.params.get("T", 20))
            res[outs_c[0][0].id] = y.ravel()
            return res
        if k == PASSTHROUGH:
            res[outs_c[0][0].id] = data[ins_c[0][0].id]
            return res
        if k == FILTERBANK:
            pi, po = ins_c[0][0], outs_c[0][0]
            x = data[pi.id]
            H = max(a.params["bank_L"]) - 1
            if a.params["windowed"]:
                window = x
            else:
                window = np.concatenate([a.state["history"], x])
                a.state["history"] = window[len(window) - H:] if H else window[:0]
            n = len(window) - H
            # Branch d is active when its DRP decodes to its atr (Eq. 1); a
            # static bank uses its fixed mask.
            if bits:
                eff = sum(int(bits[b]) << d for d, b in enumerate(a.branches))
            else:
                eff = int(mask)
            y = fb_frame(window, H, a.params["taps"], a.params["bank_L"], a.params["Kmax"], eff)
            for d in range(len(a.branches)):
                if (eff >> d) & 1:
                    a.state["branch_firings"][d] += 1
                    a.state["branch_tokens"][d] += n
            res[po.id] = y
            return res
        if k in (SWITCH, POLY):
            pi = ins_c[0][0]
            x = data[pi.id]
            hist = a.state["history"]
            full = np.concatenate([hist, x])
            H = len(hist)
            a.state["history"] = full[len(full) - H:] if H else full[:0]
            for bi, (p, c) in enumerate(outs_c):
                if not c:
                    continue
                w = full[len(full) - c:]
                res[p.id] = basis(w, bi) if k == POLY else w
            return res
        if k == FIR:
            w = data[ins_c[0][0].id]
            h = np.asarray(a.params["taps"], np.complex128)
            L = len(h)
            n = len(w) - L + 1
            y = np.zeros(n, np.complex128)
            for l in range(L):
                y += h[l] * w[L - 1 - l: L - 1 - l + n]
            a.state["tokens"] += n
            res[outs_c[0][0].id] = y
            return res
        if k in (SELECT, ADD):
            po, c = outs_c[0]
            y = np.zeros(c, np.complex128)
            for p, ci in ins_c:
                if ci:
                    y = y + data[p.id]
            res[po.id] = y
            return res
        raise PruneError(E_UNSUPPORTED, f"no firing function for kind {k}")

    # ---- scheduler -------------------------------------------------------------
    def run(self, policy="round_robin", rng=None, max_firings=None):
        """Fire until nothing can fire.  policy 'random' fires one uniformly
        chosen fireable actor at a time (for schedule-independence checks)."""
        if not self.finalized:
            raise PruneError(E_STATE, "finalize first")
        total = 0
        while True:
            fired = False
            if policy == "round_robin":
                for a in self.actors:
                    if self.try_fire(a.id):
                        fired = True
                        total += 1
            else:
                order = rng.permutation(len(self.actors))
                for aid in order:
                    if self.try_fire(int(aid)):
                        fired = True
                        total += 1
                        break
            if not fired or (max_firings is not None and total >= max_firings):
                break
        if max_firings is None:
            self._check_termination()
        return total

    def _check_termination(self):
        stuck, linked = self.stop_classification()
        if stuck or linked:
            raise PruneError(E_DEADLOCK, f"no actor can fire; actors waiting in a cycle or behind "
                                         f"a FIFO that is never drained {stuck}, dynamic actors "
                                         f"waiting on a firing their linked partner has passed {linked}")

    # ---- end of a finite run: wait-for classification ------------------------
    def _waits(self, aid):
        """What an actor that cannot fire is missing, as (fifo, 'read'|'write')
        pairs: a blocking read stalls on an input FIFO holding less than a
        block, a blocking write on an output FIFO without room for one
        (Sec. III-A).  A dynamic actor without a control token waits on its
        control FIFO; with one, on the FIFOs of the ports its token sets
        active (Eq. 1).  Returns None for a source or configuration actor
        whose external input is used up, and [] for an actor that can fire."""
        a = self.actors[aid]
        fs = self.fstate
        if a.kind in (SOURCE, CONFIG) and not a.state["queue"]:
            return None
        bits = {}
        cp = self.cport(aid)
        if cp is not None:
            if not fs[cp.fifos[0]].can_read():
                return [(cp.fifos[0], "read")]
            bits = self._decode(a)[2]
        waits = []
        for p in self._ports(aid):
            if p.kind == CPORT or (p.kind == DRP and not bits[p.id]):
                continue
            if p.dir == IN:
                if not fs[p.fifos[0]].can_read():
                    waits.append((p.fifos[0], "read"))
            else:
                waits.extend((f, "write") for f in p.fifos if not fs[f].can_write())
        return waits

    def stop_classification(self):
        """Classify a state in which no actor can fire.

        Returns (stuck, linked): two lists of actor ids; both empty means a
        normal end of a finite run.
        * Starvation: a source or configuration actor with no external input
          left is exhausted.  An actor is starved when one of the FIFOs it
          waits on has, at its other end, an exhausted or starved actor (the
          writer for a read, the reader for a write): it stops because some
          external input ran out, and more of that input would move it.
          Every other actor that cannot fire is stuck: its waits only lead
          round a cycle (each waits on what the next has not read or
          written), which no external input can break.
        * Linked DRPs (Sec. V): a dynamic actor y that holds a control token
          and waits to read an active DRP input is followed upstream, through
          the read waits of the actors feeding it, to the dynamic actor x
          whose DRP output starts that chain.  In a valid DPG the k-th token
          of x and of y set the same DCs active, so y's k-th firing can lack
          data from x only while x has not fired its k-th firing; if x has
          (counting each actor's firings from its first non-delay control
          token), the two were set differently and y waits forever.
        """
        waits = {a.id: self._waits(a.id) for a in self.actors}
        writer = {fid: self.ports[s].actor for fid, (s, d, r, q) in enumerate(self.fifos)}
        reader = {fid: self.ports[d].actor for fid, (s, d, r, q) in enumerate(self.fifos)}
        starved = {aid for aid, w in waits.items() if w is None}
        grown = True
        while grown:
            grown = False
            for aid, w in waits.items():
                if aid in starved or not w:
                    continue
                if any((writer[f] if d == "read" else reader[f]) in starved for f, d in w):
                    starved.add(aid)
                    grown = True
        stuck = sorted(aid for aid in waits if aid not in starved)

        def token_index(aid):
            # firings counted from the first control token that is not a delay
            return self.actors[aid].firings - self.fifos[self.cport(aid).fifos[0]][3]

        linked = []
        for y in self.actors:
            cp = self.cport(y.id)
            w = waits[y.id]
            if cp is None or not w or not self.fstate[cp.fifos[0]].can_read():
                continue
            drp_in = {p.fifos[0] for p in self._ports(y.id, IN, DRP)}
            todo = [f for f, d in w if d == "read" and f in drp_in]
            seen = set()
            while todo:
                f = todo.pop()
                sp = self.ports[self.fifos[f][0]]
                if sp.kind == DRP:
                    x = sp.actor
                    if self.cport(x) is not None and token_index(x) > token_index(y.id):
                        linked.append(y.id)
                        break
                    continue
                if sp.actor in seen:
                    continue
                seen.add(sp.actor)
                cw = self.cport(sp.actor)
                cf = cw.fifos[0] if cw is not None else None
                todo.extend(g for g, d in (waits[sp.actor] or []) if d == "read" and g != cf)
        return stuck, linked

    # ---- results -------------------------------------------------------------
    def sink_output(self, aid):
        out = self.actors[aid].state["out"]
        if not out:
            u8 = self._ports(aid, IN)[0].u8
            return np.zeros(0, np.uint8 if u8 else np.complex128)
        return np.concatenate(out)

    def logs(self):
        """Canonical integer logs (compared bit-exactly with the device)."""
        fifos = {}
        for f in self.fstate:
            fifos[f.id] = dict(
                writes=[(fi, j, s, c) for (fi, j, s, c) in f.log_w],
                reads=[(fi, i, s, c) for (fi, i, s, c) in f.log_r],
                tokens_written=f.tokens_written, tokens_read=f.tokens_read,
                firings_w=f.writes, firings_r=f.reads, capacity=f.capacity,
                max_occ=f.max_occ)
        actors = {}
        for a in self.actors:
            entry = dict(kind=a.kind, firings=a.firings)
            if getattr(a, "log", None):
                entry["control"] = list(a.log)
            if a.kind == FILTERBANK:
                entry["branch_firings"] = a.state["branch_firings"].tolist()
                entry["branch_tokens"] = a.state["branch_tokens"].tolist()
            if a.kind == SINK:
                entry["tokens"] = int(sum(len(b) for b in a.state["out"]))
            actors[a.id] = entry
        return dict(fifos=fifos, actors=actors)
