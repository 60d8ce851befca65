"""Host code of the library built with AddressSanitizer and
UndefinedBehaviorSanitizer (g++, no GPU) and checked against the oracle:
* the per-firing stop classification (stop_rules.cpp) on the states the
  oracle's runs stop in: the stop cases, seeded switch/select graphs with
  matched and mismatched control streams, delays and FIFO depths;
* the compile-time analysis (design_analysis.cpp) on seeded structures;
* the FIFO and configuration rules the kernels use (prune_rules.h) under
  random traffic: order, Eq. 2 occupancy, counters, buffer bounds, and the
  invariant checks of PRUNE_DEBUG builds on that traffic and on planted
  mistakes."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import graphgen as gg
import stopcases
from oracle import analysis as an
from oracle import moc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1802_06625_amd", "csrc")
NATIVE = os.path.join(ROOT, "tests", "native")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="verify_asan_link_order=0:detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")


@pytest.fixture(scope="module")
def tools(tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    out = tmp_path_factory.mktemp("native")
    srcs = {"stop_check": [os.path.join(CSRC, "stop_rules.cpp")],
            "analysis_check": [os.path.join(CSRC, "design_analysis.cpp")],
            "rules_check": []}
    bins = {}
    for name, extra in srcs.items():
        exe = str(out / name)
        cmd = [gxx, "-std=c++17", "-O1", "-g"] + SAN + ["-I", os.path.join(ROOT, "include"), "-I", CSRC,
                                                         os.path.join(NATIVE, name + ".cpp")] + extra + ["-o", exe]
        subprocess.run(cmd, check=True, capture_output=True, text=True)
        bins[name] = exe
    return bins


def _run(exe, text):
    res = subprocess.run([exe], input=text, capture_output=True, text=True, env=ENV, timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr
    return res.stdout


# ---------------------------------------------------------------- FIFO rules
def test_fifo_and_config_rules(tools):
    out = _run(tools["rules_check"], "")
    assert out.startswith("ok "), out
    cases, accesses, planted = (int(v) for v in out.split()[1:4])
    assert cases > 300 and accesses > 100000 and planted > 5000


# ---------------------------------------------------------------- stop classification
def stop_view(g):
    """The library's view of a stopped oracle run (stop_rules.h layout)."""
    lines = [f"{g.C} {len(g.actors)} {len(g.ports)} {len(g.fifos)}"]
    for a in g.actors:
        cp = g.cport(a.id)
        cf = cp.fifos[0] if cp is not None else -1
        tok = int(cf >= 0 and g.fstate[cf].can_read())
        mask = int(g.fstate[cf].peek()["mask"]) if tok else 0
        ex = int(a.kind in (moc.SOURCE, moc.CONFIG) and not a.state["queue"])
        lines.append(f"{a.kind} {ex} {cf} {tok} {mask} {a.firings} {len(a.ports)} "
                     + " ".join(str(p) for p in a.ports))
    for p in g.ports:
        el = 0
        if p.kind == moc.DRP and p.dir != moc.INTERNAL and g.cport(p.actor) is not None:
            el = g.table.get((g.controller(p.actor).id, p.id), 0)
        d = p.dir if p.dir != moc.INTERNAL else 2
        lines.append(f"{p.actor} {d} {p.kind} {el} {len(p.fifos)} " + " ".join(str(f) for f in p.fifos))
    for f, (s, d, r, q) in zip(g.fstate, g.fifos):
        lines.append(f"{s} {d} {r} {q} {f.writes - f.reads}")
    return "\n".join(lines) + "\n"


def _parse_stops(out):
    rows = out.strip().splitlines()
    res = []
    for i in range(0, len(rows), 2):
        st = [int(v) for v in rows[i].split()[1:]]
        lk = [int(v) for v in rows[i + 1].split()[1:]]
        res.append((st, lk))
    return res


def _random_switch_select(rng):
    C = int(rng.integers(1, 4))
    r = int(rng.integers(1, 4))
    n = int(rng.integers(0, 7))
    nx = int(rng.integers(0, 7))
    routes_x = [int(v) for v in rng.integers(0, 2, size=nx)]
    if rng.random() < 0.5:
        routes_y = None
    else:
        routes_y = list(routes_x[:int(rng.integers(0, nx + 1))])
        for k in range(len(routes_y)):
            if rng.random() < 0.3:
                routes_y[k] ^= 1
        routes_y += [int(v) for v in rng.integers(0, 2, size=int(rng.integers(0, 3)))]
    Q = int(rng.integers(0, 2)) * r
    return stopcases.switch_select(routes_x, routes_y, n, C=C, r=r, Q_in=Q, seed=int(rng.integers(1 << 30)))


def test_stop_classification_matches_oracle(tools):
    graphs = [d for d in stopcases.cases().values()]
    rng = np.random.default_rng(77)
    graphs += [_random_switch_select(rng) for _ in range(300)]
    text, ref, kinds = "", [], set()
    for d in graphs:
        status, g = stopcases.run_oracle(d)
        stuck, linked = g.stop_classification()
        ref.append((stuck, linked))
        kinds.add((bool(stuck), bool(linked)))
        text += stop_view(g)
    got = _parse_stops(_run(tools["stop_check"], text))
    assert got == ref
    # normal ends, cycles of waits and linked-DRP deadlocks all occur
    assert {(False, False), (True, False), (False, True)} <= kinds


# ---------------------------------------------------------------- analysis
def _structure_text(S):
    lines = [f"{len(S.actors)} {len(S.ports)} {len(S.fifos)} {len(S.table)}",
             " ".join(str(k) for k in S.actors)]
    lines += [f"{a} {d} {k}" for (a, d, k) in S.ports]
    lines += [f"{s} {d} {r} {q}" for (s, d, r, q) in S.fifos]
    lines += [f"{c} {p} {e}" for (c, p, e) in S.table]
    return "\n".join(lines) + "\n"


def _oracle_graph(S):
    g = moc.Graph()
    for a, k in enumerate(S.actors):
        if k == gg.CONFIG:
            g.actor(moc.CONFIG, mode="route", n_elements=S.n_elements[a])
        else:
            g.actor(k)
    for (a, d, k) in S.ports:
        g.port(a, d, k, 1)
    for (s, d, r, q) in S.fifos:
        g.connect(s, d, r, q)
    for (c, p, e) in S.table:
        g.control(c, p, e)
    return g


def _parse_reports(out):
    rows = out.strip().splitlines()
    reps = []
    for i in range(0, len(rows), 6):
        f = [[int(v) for v in rows[i + k].split()[1:]] for k in range(6)]
        dcs, k = [], 0
        v = f[2]
        while k < len(v):
            dpg, el, direct, n = v[k:k + 4]
            dcs.append((dpg, el, tuple(v[k + 4:k + 4 + n]), direct))
            k += 4 + n
        reps.append({"linked": [tuple(f[0][j:j + 2]) for j in range(0, len(f[0]), 2)],
                     "dpgs": [tuple(f[1][j:j + 4]) for j in range(0, len(f[1]), 4)],
                     "dcs": dcs, "dc_of_actor": f[3], "beta": f[4],
                     "violations": [tuple(f[5][j:j + 3]) for j in range(0, len(f[5]), 3)]})
    return reps


def test_analysis_matches_oracle(tools):
    structs = [gg.random_structure(s) for s in range(150)] + [gg.dpg_structure(s) for s in range(150)]
    got = _parse_reports(_run(tools["analysis_check"], "".join(_structure_text(S) for S in structs)))
    assert len(got) == len(structs)
    for S, rep in zip(structs, got):
        assert rep == an.analyze(_oracle_graph(S))
