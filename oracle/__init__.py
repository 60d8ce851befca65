"""Oracle for the PRUNE filter-bank dataflow path (TEST INFRASTRUCTURE ONLY).

A plain, slow, sequential CPU implementation in float64 (numpy) of what the
HIP library computes: the model of computation (graph, ports, FIFOs with the
capacity of Eq. 2 and the delay access pattern of Fig. 6, control tokens
decoded per Eq. 1, blocking firing rules, a round-robin scheduler with
deadlock detection, per-firing logs), the compile-time analysis of Sec. IV-V
(design rules, DPGs and their dynamic components, per-component consistency
and buffer bounds), the Motion Detection actors (Gauss 5x5, frame-difference threshold,
5-pixel median), the memory-polynomial filter-bank actor
by its direct definition, its adjoint in closed form, finite differences and
the least-squares / Adam fit.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  It shares no code with the
HIP library and the HIP library never imports it.

Parity status of each function is stated in its docstring; every function
here is pinned by the ``-m "not gpu"`` tests against values the paper fixes,
closed forms, invariants or brute force (see ``tests/test_oracle_*.py``).
"""
from .moc import (PruneError, Graph, E_ARG, E_STATE, E_RATE_MISMATCH, E_PORT_KIND,
                  E_RULE4, E_CONNECT, E_DELAY, E_TOKEN, E_DEADLOCK, E_CAPACITY,
                  E_UNSUPPORTED, IN, OUT, SRP, DRP, CPORT, SOURCE, CONFIG,
                  FILTERBANK, SWITCH, SELECT, PASSTHROUGH, SINK, POLY, FIR, ADD,
                  fifo_capacity, fifo_write_slot, fifo_read_slot)
from .filterbank import (fb_frame, fb_stream, fb_stream_adjoint, basis)
from . import graphs, fit, analysis, motion

__all__ = [n for n in dir() if not n.startswith("_")]
