"""Python face of the graph C ABI (same names, marshalling only) plus builders
for the filter-bank graphs: the plain graph SOURCE -> FILTERBANK -> SINK with
a CONFIG actor on the bank's control port, and the routed multi-stream graph
SOURCE -> SWITCH -> {FILTERBANK, PASSTHROUGH} -> SELECT -> SINK.

PyTorch tensors provide device memory (data_ptr) and streams only.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from ._lib import call


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


class Graph:
    def __init__(self, device: int = 0):
        h = C.c_void_p()
        call("prune_graph_create", device, C.byref(h))
        self.h = h
        self.device = device
        self._keep = []          # borrowed tensors must outlive the graph

    def __del__(self):
        if getattr(self, "h", None):
            try:
                L.lib().prune_graph_destroy(self.h)
            except Exception:
                pass
            self.h = None

    # ---- construction ------------------------------------------------------
    def actor(self, kind, params=None):
        out = C.c_uint32()
        if params is None:
            call("prune_actor_create", self.h, kind, None, 0, C.byref(out))
        else:
            call("prune_actor_create", self.h, kind, C.byref(params), C.sizeof(params), C.byref(out))
        return out.value

    def config(self, mode, Kmax, n_elements):
        return self.actor(L.CONFIG, L.ConfigParams(mode, Kmax, n_elements))

    def filterbank(self, Kmax, bank_L, windowed=False, fixed_mask=0):
        p = L.FbParams()
        p.n_banks = len(bank_L)
        p.Kmax = Kmax
        for i, v in enumerate(bank_L):
            p.L[i] = int(v)
        p.windowed = int(windowed)
        p.fixed_mask = int(fixed_mask)
        return self.actor(L.FILTERBANK, p)

    def port(self, actor, dir, kind, atr, token_bytes=8, flags=0, halo=0):
        out = C.c_uint32()
        call("prune_port_create", self.h, actor, dir, kind, int(atr), token_bytes, flags, int(halo),
             C.byref(out))
        return out.value

    def branch(self, fb, d):
        out = C.c_uint32()
        call("prune_filterbank_branch", self.h, fb, d, C.byref(out))
        return out.value

    def connect(self, src, dst, rate, delay=0):
        out = C.c_uint32()
        call("prune_fifo_connect", self.h, src, dst, int(rate), int(delay), C.byref(out))
        return out.value

    def control(self, ctl_port, drp, element):
        call("prune_control_table_set", self.h, ctl_port, drp, int(element))

    def finalize(self, C_, check_rules=False):
        """Validate and size the graph; with check_rules the library runs the
        compile-time analysis first and refuses a graph with violations."""
        call("prune_graph_set_checks", self.h, L.CHECK_RULES if check_rules else 0)
        call("prune_graph_finalize", self.h, int(C_))

    def _table(self, which):
        n = C.c_size_t()
        call("prune_graph_analysis_table", self.h, which, None, 0, C.byref(n))
        buf = (C.c_int64 * max(n.value, 1))()
        call("prune_graph_analysis_table", self.h, which, buf, n.value, C.byref(n))
        return [int(v) for v in buf[:n.value]]

    def analyze(self):
        """Compile-time analysis of Sec. IV-V (prune_graph_analyze): linked DRP
        pairs, DPGs (q, x, y, control port), DCs (dpg, element, actors,
        direct FIFO), the DC of each actor, the buffer bound of each FIFO and
        the sorted violations (code, a, b)."""
        cnt = L.AnalysisCounts()
        call("prune_graph_analyze", self.h, C.byref(cnt))
        lk = self._table(L.AN_LINKED)
        dp = self._table(L.AN_DPGS)
        dc = self._table(L.AN_DCS)
        acts = self._table(L.AN_DC_ACTORS)
        vi = self._table(L.AN_VIOLATIONS)
        dcs, k = [], 0
        for i in range(0, len(dc), 4):
            n = dc[i + 3]
            dcs.append((dc[i], dc[i + 1], tuple(acts[k:k + n]), dc[i + 2]))
            k += n
        return {"linked": [tuple(lk[i:i + 2]) for i in range(0, len(lk), 2)],
                "dpgs": [tuple(dp[i:i + 4]) for i in range(0, len(dp), 4)],
                "dcs": dcs,
                "dc_of_actor": self._table(L.AN_ACTOR_DC),
                "beta": self._table(L.AN_BETA),
                "violations": [tuple(vi[i:i + 3]) for i in range(0, len(vi), 3)]}

    # ---- storage and input ------------------------------------------------
    def required_bytes(self, fifo):
        out = C.c_size_t()
        call("prune_fifo_required_bytes", self.h, fifo, C.byref(out))
        return out.value

    def alloc_fifo(self, fifo, device="cuda"):
        """Allocate and bind a torch tensor as the FIFO's storage."""
        nbytes = self.required_bytes(fifo)
        t = torch.zeros(nbytes // 8, dtype=torch.complex64, device=device)
        self.bind_storage(fifo, t)
        return t

    def bind_storage(self, fifo, tensor):
        self._keep.append(tensor)
        call("prune_fifo_bind_storage", self.h, fifo, C.c_void_p(tensor.data_ptr()),
             tensor.numel() * tensor.element_size())

    def write_window(self, fifo, k):
        out = C.c_void_p()
        call("prune_fifo_write_window", self.h, fifo, k, C.byref(out))
        return out.value

    def set_taps(self, fb, taps, stream=None):
        taps = taps.contiguous()
        self._keep.append(taps)
        call("prune_filterbank_set_taps", self.h, fb, C.c_void_p(taps.data_ptr()), taps.numel(),
             _stream(stream))

    def reset_history(self, actor, stream=None):
        call("prune_actor_reset_history", self.h, actor, _stream(stream))

    def source_push(self, src, samples, counts):
        counts = np.ascontiguousarray(counts, dtype=np.uint32)
        ptr = None
        if samples is not None:
            self._keep.append(samples)
            ptr = C.c_void_p(samples.data_ptr())
        call("prune_source_push", self.h, src, ptr,
             counts.ctypes.data_as(C.POINTER(C.c_uint32)), len(counts))

    def config_push(self, cfg, side, stream=None):
        side = np.ascontiguousarray(side, dtype=np.uint32).reshape(-1, 4)
        call("prune_config_push", self.h, cfg, side.ctypes.data_as(C.POINTER(L.SideInfo)), len(side),
             _stream(stream))

    def stream_host(self, src, cfg, snk, host_in, side, host_out, batch, stream=None):
        """prune_graph_stream_host: frames from a (pinned) host tensor through
        the graph and back into a host tensor, copies overlapped with firing."""
        side = np.ascontiguousarray(side, dtype=np.uint32).reshape(-1, 4)
        call("prune_graph_stream_host", self.h, src, cfg, snk, C.c_void_p(host_in.data_ptr()),
             side.ctypes.data_as(C.POINTER(L.SideInfo)), C.c_void_p(host_out.data_ptr()), len(side),
             int(batch), _stream(stream))

    def sink_bind_output(self, snk, tensor):
        self._keep.append(tensor)
        call("prune_sink_bind_output", self.h, snk, C.c_void_p(tensor.data_ptr()), tensor.numel())

    # ---- execution -----------------------------------------------------------
    def fire(self, mode=L.PER_FIRING, max_firings=0, stream=None):
        out = C.c_uint64()
        call("prune_graph_fire", self.h, mode, max_firings, _stream(stream), C.byref(out))
        return out.value

    def sync(self, stream=None):
        call("prune_graph_sync", self.h, _stream(stream))

    def fifo_stats(self, fifo):
        s = L.FifoStats()
        call("prune_fifo_get_stats", self.h, fifo, C.byref(s))
        return {k: getattr(s, k) for k, _ in L.FifoStats._fields_}

    def branch_stats(self, fb, n):
        f = (C.c_uint64 * n)()
        t = (C.c_uint64 * n)()
        call("prune_filterbank_branch_stats", self.h, fb, f, t, n)
        return list(f), list(t)

    def actor_firings(self, actor):
        out = C.c_uint64()
        call("prune_actor_firings", self.h, actor, C.byref(out))
        return out.value

    def trace_enable(self, max_records):
        call("prune_trace_enable", self.h, max_records)

    def trace_fetch(self):
        used = C.c_size_t()
        call("prune_trace_fetch", self.h, None, 0, C.byref(used))
        n = used.value // C.sizeof(L.TraceRecord)
        buf = np.zeros((n, 8), dtype=np.uint32)
        if n:
            call("prune_trace_fetch", self.h, C.c_void_p(buf.ctypes.data), buf.nbytes, C.byref(used))
        return buf


def trace_logs(trace):
    """Group trace records into per-FIFO (writes, reads) lists sorted by index
    and per-actor control decodes sorted by firing number."""
    fifos, ctrl = {}, {}
    for (typ, a, b, c, d, e, f, _) in trace.tolist():
        if typ == 0:
            ent = fifos.setdefault(a, {"writes": [], "reads": []})
            ent["reads" if b else "writes"].append((c, d, e, f))
        else:
            ctrl.setdefault(a, []).append((c, d, e, f))
    for v in fifos.values():
        v["writes"].sort(key=lambda r: r[1])
        v["reads"].sort(key=lambda r: r[1])
    for v in ctrl.values():
        v.sort()
    return fifos, ctrl


# ---------------------------------------------------------------- builders
class PlainGraph:
    """SOURCE -> FILTERBANK (merged DPG with control port) -> SINK; CONFIG
    (prefix mode) feeds the control port; branch d <- element d+1."""

    def __init__(self, Kmax, bank_L, atr, C_, param=False, device=0, cfg_mode=L.CONFIG_PREFIX):
        g = self.g = Graph(device)
        D = len(bank_L) * Kmax
        fl = L.PORT_PARAM if param else 0
        self.src = g.actor(L.SOURCE)
        self.cfg = g.config(cfg_mode, Kmax, D)
        self.fb = g.filterbank(Kmax, bank_L)
        self.snk = g.actor(L.SINK)
        p_src = g.port(self.src, L.OUT, L.SRP, atr, flags=fl)
        p_ctl = g.port(self.cfg, L.OUT, L.SRP, 1)
        p_cp = g.port(self.fb, L.IN, L.CPORT, 1)
        p_in = g.port(self.fb, L.IN, L.SRP, atr, flags=fl)
        p_out = g.port(self.fb, L.OUT, L.SRP, atr, flags=fl)
        p_snk = g.port(self.snk, L.IN, L.SRP, atr, flags=fl)
        self.f_in = g.connect(p_src, p_in, atr)
        self.f_ctl = g.connect(p_ctl, p_cp, 1)
        self.f_out = g.connect(p_out, p_snk, atr)
        for d in range(D):
            g.control(p_ctl, g.branch(self.fb, d), d + 1)
        g.finalize(C_, check_rules=True)
        self.atr = atr
        self.fifo_in = g.alloc_fifo(self.f_in)
        self.fifo_out = g.alloc_fifo(self.f_out)


class UnfusedGraph:
    """The DPD graph before actor merging (Sec. VII-A, Fig. 8): SOURCE -> POLY
    (dynamic x; output b carries |x|^b x over the window of L-1 past samples
    and the frame) -> FIR_b (a static windowed filter bank with one branch,
    taps of branch b) -> SELECT (dynamic y, the add: sum of its active
    inputs) -> SINK; CONFIG (prefix mode) broadcasts one control value to
    POLY and SELECT, branch b <- element b+1.  One bank, Kmax <= PRUNE_MAX_IN."""

    def __init__(self, Kmax, L_, atr, C_, device=0):
        g = self.g = Graph(device)
        H = L_ - 1
        self.src = g.actor(L.SOURCE)
        self.cfg = g.config(L.CONFIG_PREFIX, Kmax, Kmax)
        self.poly = g.actor(L.POLY)
        self.firs = [g.filterbank(1, [L_], windowed=True, fixed_mask=1) for _ in range(Kmax)]
        self.add = g.actor(L.SELECT)
        self.snk = g.actor(L.SINK)
        p_src = g.port(self.src, L.OUT, L.SRP, atr)
        p_ctl = g.port(self.cfg, L.OUT, L.SRP, 1)
        p_pc = g.port(self.poly, L.IN, L.CPORT, 1)
        p_pi = g.port(self.poly, L.IN, L.SRP, atr)
        p_po = [g.port(self.poly, L.OUT, L.DRP, atr + H, halo=H) for _ in range(Kmax)]
        p_fi = [g.port(f, L.IN, L.SRP, atr + H, halo=H) for f in self.firs]
        p_fo = [g.port(f, L.OUT, L.SRP, atr) for f in self.firs]
        p_ac = g.port(self.add, L.IN, L.CPORT, 1)
        p_ai = [g.port(self.add, L.IN, L.DRP, atr) for _ in range(Kmax)]
        p_ao = g.port(self.add, L.OUT, L.SRP, atr)
        p_snk = g.port(self.snk, L.IN, L.SRP, atr)
        self.f_in = g.connect(p_src, p_pi, atr)
        g.connect(p_ctl, p_pc, 1)
        g.connect(p_ctl, p_ac, 1)
        self.f_win, self.f_br = [], []
        for b in range(Kmax):
            self.f_win.append(g.connect(p_po[b], p_fi[b], atr + H))
            self.f_br.append(g.connect(p_fo[b], p_ai[b], atr))
            g.control(p_ctl, p_po[b], b + 1)
            g.control(p_ctl, p_ai[b], b + 1)
        self.f_out = g.connect(p_ao, p_snk, atr)
        g.finalize(C_, check_rules=True)
        self.atr = atr
        self.fifo_in = g.alloc_fifo(self.f_in)
        self.fifo_out = g.alloc_fifo(self.f_out)
        self.storage = [g.alloc_fifo(f) for f in self.f_win + self.f_br]

    def set_taps(self, taps):
        """taps: [Kmax, L] complex (branch b's FIR)."""
        for b, f in enumerate(self.firs):
            self.g.set_taps(f, taps[b:b + 1].reshape(1, 1, -1).contiguous())


class MotionGraph:
    """Motion Detection (Sec. VII-A, Fig. 7): SOURCE -> GAUSS5 -> THRES -> MED5
    -> SINK on 8-bit W x H frames (a frame is W*H one-byte tokens).  The
    Gauss output feeds THRES twice; the second FIFO carries a one-frame
    delay, so THRES compares each frame with the previous one."""

    def __init__(self, W, H, C_, threshold=20, device=0):
        g = self.g = Graph(device)
        npix = W * H
        pp = L.PixelParams(W, H, threshold)
        self.src = g.actor(L.SOURCE)
        self.gauss = g.actor(L.GAUSS5, pp)
        self.thres = g.actor(L.THRES, pp)
        self.med = g.actor(L.MED5, pp)
        self.snk = g.actor(L.SINK)
        P = lambda a, d: g.port(a, d, L.SRP, npix, token_bytes=1)
        p_src, p_gi, p_go = P(self.src, L.OUT), P(self.gauss, L.IN), P(self.gauss, L.OUT)
        p_tc, p_tp, p_to = P(self.thres, L.IN), P(self.thres, L.IN), P(self.thres, L.OUT)
        p_mi, p_mo, p_snk = P(self.med, L.IN), P(self.med, L.OUT), P(self.snk, L.IN)
        self.f_in = g.connect(p_src, p_gi, npix)
        self.f_cur = g.connect(p_go, p_tc, npix)
        self.f_prev = g.connect(p_go, p_tp, npix, npix)
        self.f_map = g.connect(p_to, p_mi, npix)
        self.f_out = g.connect(p_mo, p_snk, npix)
        g.finalize(C_, check_rules=True)
        self.npix = npix
        self.storage = {}
        for f in (self.f_in, self.f_cur, self.f_prev, self.f_map, self.f_out):
            nbytes = g.required_bytes(f)
            t = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
            g.bind_storage(f, t)
            self.storage[f] = t
        self.fifo_in = self.storage[self.f_in]
        self.fifo_out = self.storage[self.f_out]


class RoutedGraph:
    """Per stream: SOURCE -> SWITCH -> {FILTERBANK (static, windowed),
    PASSTHROUGH} -> SELECT -> SINK, with one CONFIG (route mode)
    broadcasting its token to SWITCH and SELECT."""

    def __init__(self, n_streams, Kmax, bank_L, atr, C_, param=False, device=0):
        g = self.g = Graph(device)
        H = max(bank_L) - 1
        D = len(bank_L) * Kmax
        fl = L.PORT_PARAM if param else 0
        self.streams = []
        for s in range(n_streams):
            ids = {}
            ids["src"] = g.actor(L.SOURCE)
            ids["cfg"] = g.config(L.CONFIG_ROUTE, Kmax, 2)
            ids["sw"] = g.actor(L.SWITCH)
            ids["fb"] = g.filterbank(Kmax, bank_L, windowed=True, fixed_mask=(1 << D) - 1)
            ids["ps"] = g.actor(L.PASSTHROUGH)
            ids["sel"] = g.actor(L.SELECT)
            ids["snk"] = g.actor(L.SINK)
            p_src = g.port(ids["src"], L.OUT, L.SRP, atr, flags=fl)
            p_ctl = g.port(ids["cfg"], L.OUT, L.SRP, 1)
            p_swc = g.port(ids["sw"], L.IN, L.CPORT, 1)
            p_swi = g.port(ids["sw"], L.IN, L.SRP, atr, flags=fl)
            p_sw0 = g.port(ids["sw"], L.OUT, L.DRP, atr + H, flags=fl, halo=H)
            p_sw1 = g.port(ids["sw"], L.OUT, L.DRP, atr, flags=fl)
            p_fbi = g.port(ids["fb"], L.IN, L.SRP, atr + H, flags=fl, halo=H)
            p_fbo = g.port(ids["fb"], L.OUT, L.SRP, atr, flags=fl)
            p_psi = g.port(ids["ps"], L.IN, L.SRP, atr, flags=fl)
            p_pso = g.port(ids["ps"], L.OUT, L.SRP, atr, flags=fl)
            p_slc = g.port(ids["sel"], L.IN, L.CPORT, 1)
            p_sl0 = g.port(ids["sel"], L.IN, L.DRP, atr, flags=fl)
            p_sl1 = g.port(ids["sel"], L.IN, L.DRP, atr, flags=fl)
            p_slo = g.port(ids["sel"], L.OUT, L.SRP, atr, flags=fl)
            p_snk = g.port(ids["snk"], L.IN, L.SRP, atr, flags=fl)
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
            ids["fifos"] = f
            self.streams.append(ids)
        g.finalize(C_, check_rules=True)
        self.atr = atr
        self.storage = []
        for ids in self.streams:
            st = {k: g.alloc_fifo(v) for k, v in ids["fifos"].items() if not k.startswith("ctl")}
            self.storage.append(st)
