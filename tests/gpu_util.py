"""Helpers for the GPU parity tests: run the library's graphs on seeded
workloads and compare with the oracle."""
import numpy as np
import torch

from oracle import graphs as og
from paper_1802_06625_amd import _lib as L
from paper_1802_06625_amd.graph import PlainGraph, RoutedGraph, trace_logs

TOL = 2e-5


def rel_l2(a, b):
    a = np.asarray(a, np.complex128)
    b = np.asarray(b, np.complex128)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def announce(msg):
    print(msg, flush=True)


def run_plain_device(wl, C, mode, s=0, atr=None, param=None, inplace=False, trace=True,
                     batches=None, cfg_mode=L.CONFIG_PREFIX, src_rounds=False):
    n = wl.side[s, :, 1].astype(np.int64)
    if param is None:
        param = bool(np.any(n != n[0]))
    if atr is None:
        atr = int(wl.spec.n_max) if param else int(n[0])
    pg = PlainGraph(wl.Kmax, wl.bank_L, atr, C, param, cfg_mode=cfg_mode)
    g = pg.g
    g.set_taps(pg.fb, torch.from_numpy(wl.taps[s]).cuda())
    total = int(n.sum())
    out = torch.zeros(total, dtype=torch.complex64, device="cuda")
    g.sink_bind_output(pg.snk, out)
    if trace:
        g.trace_enable(64 * len(n) + 4096)
    x = torch.from_numpy(wl.x[s]).cuda()
    if inplace:
        assert len(n) <= C, "in-place frames need a FIFO that holds them all"
        off = np.concatenate([[0], np.cumsum(n)])
        for f in range(len(n)):
            ptr = g.write_window(pg.f_in, f)
            base = pg.fifo_in.data_ptr()
            k = (ptr - base) // 8
            pg.fifo_in[k:k + n[f]] = x[off[f]:off[f + 1]]
        torch.cuda.synchronize()
        g.source_push(pg.src, None, n)
    elif not src_rounds:
        g.source_push(pg.src, x, n)
    side = wl.side[s]
    if batches is None:
        g.config_push(pg.cfg, side)
        g.fire(mode)
    else:
        # push and fire in several rounds
        # push and fire in several rounds; a list of modes gives each round's
        # (src_rounds: source frames are pushed per round too, so that a
        # per-firing round ends at an iteration boundary)
        modes = list(mode) if isinstance(mode, (list, tuple)) else [mode] * batches
        edges = np.linspace(0, len(n), batches + 1).astype(int)
        off = np.concatenate([[0], np.cumsum(n)])
        for a, b, m in zip(edges[:-1], edges[1:], modes):
            if src_rounds:
                g.source_push(pg.src, x[off[a]:off[b]], n[a:b])
            g.config_push(pg.cfg, side[a:b])
            g.fire(m)
    g.sync()
    y = out.cpu().numpy()
    res = dict(y=y, pg=pg, g=g)
    if trace:
        res["fifos"], res["ctrl"] = trace_logs(g.trace_fetch())
    return res


def compare_logs(dev, logs_ref, actors_with_control):
    for fid, ref in logs_ref["fifos"].items():
        got = dev["fifos"].get(fid, {"writes": [], "reads": []})
        assert got["writes"] == [tuple(w) for w in ref["writes"]], f"fifo {fid}: writes differ"
        assert got["reads"] == [tuple(r) for r in ref["reads"]], f"fifo {fid}: reads differ"
    for aid in actors_with_control:
        assert dev["ctrl"].get(aid, []) == [tuple(c) for c in logs_ref["actors"][aid]["control"]], \
            f"actor {aid}: control decodes differ"


def compare_stats(g, logs_ref):
    for fid, ref in logs_ref["fifos"].items():
        st = g.fifo_stats(fid)
        assert st["writes"] == ref["firings_w"] and st["reads"] == ref["firings_r"], fid
        assert st["tokens_written"] == ref["tokens_written"], fid
        assert st["tokens_read"] == ref["tokens_read"], fid
        assert st["capacity"] == ref["capacity"], fid
        assert st["max_occ"] <= st["capacity"], fid


def run_routed_device(wl, C, mode, trace=True):
    n = wl.side[0, :, 1].astype(np.int64)
    atr = int(n[0])
    rg = RoutedGraph(wl.n_streams, wl.Kmax, wl.bank_L, atr, C)
    g = rg.g
    outs = []
    if trace:
        g.trace_enable(200 * wl.n_streams * wl.n_frames + 4096)
    for s, ids in enumerate(rg.streams):
        g.set_taps(ids["fb"], torch.from_numpy(wl.taps[s]).cuda())
        o = torch.zeros(int(wl.side[s, :, 1].sum()), dtype=torch.complex64, device="cuda")
        g.sink_bind_output(ids["snk"], o)
        outs.append(o)
        g.source_push(ids["src"], torch.from_numpy(wl.x[s]).cuda(), wl.side[s, :, 1])
        g.config_push(ids["cfg"], wl.side[s])
    g.fire(mode)
    g.sync()
    res = dict(y=np.stack([o.cpu().numpy() for o in outs]), rg=rg, g=g)
    if trace:
        res["fifos"], res["ctrl"] = trace_logs(g.trace_fetch())
    return res
