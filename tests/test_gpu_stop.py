"""GPU: the library's end-of-run status in per-firing mode against the
oracle's, on the graphs of stopcases (undelayed and delayed THRES/MED
cycles, a delay that fills its FIFO, linked DRPs set by mismatched control
streams, valid DPGs stopped by input running out).  Status, per-actor firing
counts, FIFO counters and the sink's tokens must match exactly."""
import numpy as np
import pytest
import torch

import stopcases
from gpu_util import announce
from paper_1802_06625_amd import _lib as L
from paper_1802_06625_amd.graph import Graph

pytestmark = pytest.mark.gpu

PIXEL = ("GAUSS5", "THRES", "MED5")


def run_library(d):
    g = Graph()
    for kind, params in d.actors:
        if kind in PIXEL:
            g.actor(getattr(L, kind), L.PixelParams(params["W"], params["H"], params.get("T", 0)))
        elif kind == "CONFIG":
            mode = L.CONFIG_ROUTE if params.get("mode") == "route" else L.CONFIG_PREFIX
            g.config(mode, 1, params["n_elements"])
        else:
            g.actor(getattr(L, kind))
    for (a, dr, k, atr, u8) in d.ports:
        g.port(a, dr, k, atr, token_bytes=1 if u8 else 8)
    for (s, t, r, q) in d.fifos:
        g.connect(s, t, r, q)
    for (c, p, e) in d.table:
        g.control(c, p, e)
    g.finalize(d.C)
    for f, (s, t, r, q) in enumerate(d.fifos):
        if d.ports[t][2] != stopcases.CPORT:
            g.bind_storage(f, torch.zeros(g.required_bytes(f), dtype=torch.uint8, device="cuda"))
    sinks = {}
    for a, (kind, _) in enumerate(d.actors):
        if kind == "SINK":
            u8 = next(p[4] for p in d.ports if p[0] == a)
            total = sum(sum(len(x) for x in fr) for fr in d.frames.values())
            out = torch.zeros(total, dtype=torch.uint8 if u8 else torch.complex64, device="cuda")
            g.sink_bind_output(a, out)
            sinks[a] = out
    for a, frames in d.frames.items():
        x = torch.from_numpy(np.concatenate(frames)).cuda()
        g.source_push(a, x, [len(f) for f in frames])
    for a, side in d.side.items():
        g.config_push(a, side)
    status = "normal"
    try:
        g.fire(L.PER_FIRING)
    except L.PruneError as e:
        assert e.code == L.E_DEADLOCK, str(e)
        status = "deadlock"
    g.sync()
    return status, g, sinks


@pytest.mark.parametrize("name", sorted(stopcases.cases()))
def test_stop_status_matches_oracle(name):
    announce(f"stop case {name}")
    d = stopcases.cases()[name]
    st_ref, ref = stopcases.run_oracle(d)
    assert st_ref == d.expect
    st, g, sinks = run_library(d)
    assert st == st_ref
    for a, A in enumerate(ref.actors):
        assert g.actor_firings(a) == A.firings, f"actor {a} firings"
    for f in ref.fstate:
        s = g.fifo_stats(f.id)
        assert (s["writes"], s["reads"]) == (f.writes, f.reads), f"fifo {f.id}"
        assert (s["tokens_written"], s["tokens_read"]) == (f.tokens_written, f.tokens_read), f"fifo {f.id}"
        assert s["capacity"] == f.capacity
    for a, out in sinks.items():
        y_ref = ref.sink_output(a)
        y = out.cpu().numpy()[:len(y_ref)]
        np.testing.assert_array_equal(y.astype(y_ref.dtype), y_ref)
        assert not np.any(out.cpu().numpy()[len(y_ref):])
