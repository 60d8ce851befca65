"""GPU test of the persistent autotuning cache: a first process tunes the
forward and adjoint on its own inputs and records the choices in the file
named by PRUNE_AUTOTUNE_CACHE; a second process with the same file takes the
choices from it, runs no tuning, and gives bit-identical outputs."""
import json
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest
import torch

from gpu_util import announce

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = textwrap.dedent("""
    import ctypes as C, json, sys
    import numpy as np, torch
    sys.path.insert(0, sys.argv[1])
    import synth
    from oracle.graphs import stream_frames
    from paper_1802_06625_amd import _lib as L, ops
    wl = synth.scaled("C5", cotangent=True)
    rows = [(s, t0, n, m, r) for s in range(wl.n_streams) for (t0, n, m, r) in stream_frames(wl, s)]
    fr = ops.frame_table(rows)
    x, t = torch.from_numpy(wl.x).cuda(), torch.from_numpy(wl.taps).cuda()
    gy = torch.from_numpy(wl.gy).cuda()
    mfl = int(wl.side[:, :, 1].max())
    y = ops.fb_forward(x, t, fr, wl.Kmax, wl.bank_L, mfl)
    gx, gt = ops.fb_backward(x, t, fr, gy, wl.Kmax, wl.bank_L, mfl)
    torch.cuda.synchronize()
    runs, hits = C.c_uint32(), C.c_uint32()
    L.call("prune_autotune_counts", C.byref(runs), C.byref(hits))
    np.save(sys.argv[2], np.concatenate([y.cpu().numpy().ravel(), gx.cpu().numpy().ravel(),
                                         gt.cpu().numpy().ravel()]))
    print(json.dumps({"runs": runs.value, "hits": hits.value,
                      "fwd": ops.tuned_variant(x, fr, wl.Kmax, wl.bank_L, mfl)}), flush=True)
""")


@pytest.fixture(autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _child(tmp_path, name, cache):
    env = dict(os.environ, PRUNE_AUTOTUNE_CACHE=str(cache))
    env.pop("PRUNE_AUTOTUNE", None)
    out = tmp_path / f"{name}.npy"
    res = subprocess.run([sys.executable, "-c", CHILD, ROOT, str(out)], env=env, capture_output=True,
                         text=True, timeout=240)
    assert res.returncode == 0, res.stderr[-2000:]
    line = [l for l in res.stdout.splitlines() if l.startswith("{")][-1]
    return json.loads(line), np.load(out)


def test_autotune_cache_reused_by_second_process(tmp_path):
    announce("autotune cache: tuning process, then a process reading the cache")
    cache = tmp_path / "tune.jsonl"
    first, a = _child(tmp_path, "first", cache)
    assert first["runs"] == 2 and first["hits"] == 0, first       # forward and adjoint tuned
    lines = [json.loads(l) for l in cache.read_text().splitlines()]
    assert len(lines) == 2 and all(set(l) == {"key", "choice", "ms"} for l in lines)
    assert {l["key"].split("|")[0] for l in lines} == {"fwd-direct", "bwd"}
    second, b = _child(tmp_path, "second", cache)
    assert second["runs"] == 0 and second["hits"] == 2, second    # no tuning launches
    assert second["fwd"] == first["fwd"]
    assert np.array_equal(a, b)
