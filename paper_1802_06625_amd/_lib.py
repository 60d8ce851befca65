"""ctypes binding of libprune_hip.so (argument marshalling only).

Every function here forwards to the C ABI declared in include/prune.h; all
work runs in the library's HIP kernels.  Importing this module fails loudly
when the shared library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# PRUNE_DEBUG_LIBRARY=1 loads the PRUNE_DEBUG build, whose bookkeeping
# kernels check the FIFO invariants after every counter update
DEBUG_LIBRARY = os.environ.get("PRUNE_DEBUG_LIBRARY", "0") not in ("", "0")
LIB_PATH = os.path.join(HERE, "libprune_hip_debug.so" if DEBUG_LIBRARY else "libprune_hip.so")
BUILD_DEBUG = 1

# ---- enums (mirror include/prune.h) ---------------------------------------
OK = 0
E_ARG, E_STATE, E_RATE_MISMATCH, E_PORT_KIND, E_RULE4, E_CONNECT = -1, -2, -3, -4, -5, -6
E_DELAY, E_TOKEN, E_DEADLOCK, E_CAPACITY, E_HIP, E_UNSUPPORTED = -7, -8, -9, -10, -11, -12
E_RULE = -13
CHECK_RULES = 1
AN_LINKED, AN_DPGS, AN_DCS, AN_DC_ACTORS, AN_ACTOR_DC, AN_BETA, AN_VIOLATIONS = range(7)
IN, OUT = 0, 1
SRP, DRP, CPORT = 0, 1, 2
PORT_PARAM = 1
SOURCE, CONFIG, FILTERBANK, SWITCH, SELECT, PASSTHROUGH, SINK, POLY, GAUSS5, THRES, MED5 = range(11)
MAX_PORTS, MAX_IN, MAX_IO = 14, 10, 12
PER_FIRING, BATCHED, BATCHED_GRAPH = 0, 1, 2
CONFIG_PREFIX, CONFIG_ROUTE, CONFIG_MASK = 0, 1, 2
MAX_BANKS, MAX_BRANCHES, MAX_L = 4, 32, 64


class CtrlToken(C.Structure):
    _fields_ = [("mask", C.c_uint32), ("rate", C.c_uint32)]


class SideInfo(C.Structure):
    _fields_ = [("K", C.c_uint32), ("n", C.c_uint32), ("bank", C.c_uint32), ("route", C.c_uint32)]


class ConfigParams(C.Structure):
    _fields_ = [("mode", C.c_uint32), ("Kmax", C.c_uint32), ("n_elements", C.c_uint32)]


class PixelParams(C.Structure):
    _fields_ = [("W", C.c_uint32), ("H", C.c_uint32), ("threshold", C.c_uint32)]


class FbParams(C.Structure):
    _fields_ = [("n_banks", C.c_uint32), ("Kmax", C.c_uint32), ("L", C.c_uint32 * MAX_BANKS),
                ("windowed", C.c_uint32), ("fixed_mask", C.c_uint32)]


class AnalysisCounts(C.Structure):
    _fields_ = [("n_linked", C.c_uint32), ("n_dpgs", C.c_uint32), ("n_dcs", C.c_uint32),
                ("n_violations", C.c_uint32)]


class FifoStats(C.Structure):
    _fields_ = [("writes", C.c_uint64), ("reads", C.c_uint64), ("tokens_written", C.c_uint64),
                ("tokens_read", C.c_uint64), ("max_occ", C.c_uint64), ("capacity", C.c_uint64)]


class TraceRecord(C.Structure):
    _fields_ = [(n, C.c_uint32) for n in ("type", "a", "b", "c", "d", "e", "f", "pad")]


class ProbeResult(C.Structure):
    _fields_ = [("seconds", C.c_double), ("work", C.c_double), ("rate", C.c_double),
                ("clock_ghz", C.c_double), ("grid", C.c_uint32), ("block", C.c_uint32),
                ("n_cu", C.c_uint32), ("pad", C.c_uint32)]


PROBE_COPY, PROBE_FMA32, PROBE_MFMA32, PROBE_FMAC32, PROBE_FMA3V, PROBE_FMAMIX = 0, 1, 2, 3, 4, 5


class FbDesc(C.Structure):
    _fields_ = [("n_streams", C.c_uint32), ("n_frames", C.c_uint32), ("stream_len", C.c_uint64),
                ("n_banks", C.c_uint32), ("Kmax", C.c_uint32), ("L", C.c_uint32 * MAX_BANKS),
                ("max_frame_len", C.c_uint32), ("reserved", C.c_uint32)]


class FbFrame(C.Structure):
    _fields_ = [("stream", C.c_uint32), ("t0", C.c_uint32), ("n", C.c_uint32), ("mask", C.c_uint32),
                ("route", C.c_uint32), ("pad", C.c_uint32 * 3)]


_P = C.c_void_p
_ID = C.c_uint32
_ST = C.c_int32

# (name, restype, argtypes) of every entry point in include/prune.h
SIGNATURES = [
    ("prune_graph_create", _ST, [C.c_int, C.POINTER(_P)]),
    ("prune_graph_destroy", _ST, [_P]),
    ("prune_actor_create", _ST, [_P, C.c_int, _P, C.c_size_t, C.POINTER(_ID)]),
    ("prune_port_create", _ST, [_P, _ID, C.c_int, C.c_int, C.c_uint32, C.c_uint32, C.c_uint32,
                                C.c_uint32, C.POINTER(_ID)]),
    ("prune_filterbank_branch", _ST, [_P, _ID, C.c_uint32, C.POINTER(_ID)]),
    ("prune_fifo_connect", _ST, [_P, _ID, _ID, C.c_uint32, C.c_uint32, C.POINTER(_ID)]),
    ("prune_control_table_set", _ST, [_P, _ID, _ID, C.c_uint32]),
    ("prune_graph_finalize", _ST, [_P, C.c_uint32]),
    ("prune_graph_set_checks", _ST, [_P, C.c_uint32]),
    ("prune_graph_analyze", _ST, [_P, C.POINTER(AnalysisCounts)]),
    ("prune_graph_analysis_table", _ST, [_P, C.c_int, C.POINTER(C.c_int64), C.c_size_t,
                                         C.POINTER(C.c_size_t)]),
    ("prune_fifo_required_bytes", _ST, [_P, _ID, C.POINTER(C.c_size_t)]),
    ("prune_fifo_bind_storage", _ST, [_P, _ID, _P, C.c_size_t]),
    ("prune_fifo_write_window", _ST, [_P, _ID, C.c_uint32, C.POINTER(_P)]),
    ("prune_filterbank_set_taps", _ST, [_P, _ID, _P, C.c_size_t, _P]),
    ("prune_actor_reset_history", _ST, [_P, _ID, _P]),
    ("prune_source_push", _ST, [_P, _ID, _P, C.POINTER(C.c_uint32), C.c_uint32]),
    ("prune_config_push", _ST, [_P, _ID, C.POINTER(SideInfo), C.c_uint32, _P]),
    ("prune_sink_bind_output", _ST, [_P, _ID, _P, C.c_uint64]),
    ("prune_graph_fire", _ST, [_P, C.c_int, C.c_uint32, _P, C.POINTER(C.c_uint64)]),
    ("prune_graph_sync", _ST, [_P, _P]),
    ("prune_graph_stream_host", _ST, [_P, _ID, _ID, _ID, _P, C.POINTER(SideInfo), _P, C.c_uint32,
                                      C.c_uint32, _P]),
    ("prune_fifo_get_stats", _ST, [_P, _ID, C.POINTER(FifoStats)]),
    ("prune_filterbank_branch_stats", _ST, [_P, _ID, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                            C.c_uint32]),
    ("prune_actor_firings", _ST, [_P, _ID, C.POINTER(C.c_uint64)]),
    ("prune_trace_enable", _ST, [_P, C.c_size_t]),
    ("prune_trace_fetch", _ST, [_P, _P, C.c_size_t, C.POINTER(C.c_size_t)]),
    ("prune_fb_forward", _ST, [C.POINTER(FbDesc), _P, _P, _P, _P, _P]),
    ("prune_fb_forward_noalloc", _ST, [C.POINTER(FbDesc), _P, _P, _P, _P, _P]),
    ("prune_fb_workspace_bytes", _ST, [C.POINTER(FbDesc), C.POINTER(C.c_size_t)]),
    ("prune_fb_backward", _ST, [C.POINTER(FbDesc), _P, _P, _P, _P, _P, _P, _P, C.c_size_t, _P]),
    ("prune_set_fb_variant", _ST, [C.c_int]),
    ("prune_fb_variant_name", C.c_char_p, [C.c_int]),
    ("prune_fb_variant_count", C.c_int, []),
    ("prune_autotune_fb", _ST, [C.c_uint32, C.c_uint32, C.c_uint32, C.POINTER(C.c_int)]),
    ("prune_autotune_counts", _ST, [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]),
    ("prune_fb_tuned_variant", _ST, [C.POINTER(FbDesc), C.POINTER(C.c_int)]),
    ("prune_fb_check_frames", _ST, [C.c_void_p, C.c_void_p, C.POINTER(C.c_uint32), C.c_void_p]),
    ("prune_set_bwd_variant", _ST, [C.c_int]),
    ("prune_bwd_variant_name", C.c_char_p, [C.c_int]),
    ("prune_autotune_bwd", _ST, [C.c_uint32, C.c_uint32, C.c_uint32, C.POINTER(C.c_int)]),
    ("prune_timing_enable", _ST, [C.c_int]),
    ("prune_set_batch_pipeline", _ST, [C.c_int]),
    ("prune_last_fb_kernel_ms", _ST, [C.POINTER(C.c_float), C.POINTER(C.c_uint32)]),
    ("prune_rule_capacity", _ST, [C.c_uint32, C.c_uint32, C.c_uint32, C.POINTER(C.c_uint64)]),
    ("prune_rule_slots", _ST, [C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                               C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    ("prune_rule_config_token", _ST, [C.c_uint32, C.c_uint32, C.POINTER(SideInfo),
                                      C.POINTER(CtrlToken)]),
    ("prune_probe_ceiling", _ST, [C.c_int, C.c_uint32, C.c_uint64, C.c_uint32,
                                  C.POINTER(ProbeResult)]),
    ("prune_status_string", C.c_char_p, [_ST]),
    ("prune_build_flags", C.c_uint32, []),
    ("prune_last_error", C.c_char_p, []),
]


class PruneError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_lib = None


def lib():
    """Load libprune_hip.so, or its debug build with PRUNE_DEBUG_LIBRARY=1
    (both built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(the HIP library is required; there is no fallback)")
        # torch's HIP runtime first: the library then binds to the same one,
        # so torch's device memory and stream handles are valid in it
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status):
    if status != OK:
        L = lib()
        msg = (L.prune_last_error() or b"").decode()
        name = (L.prune_status_string(status) or b"").decode()
        raise PruneError(status, f"{name}: {msg}")
    return status


def call(name, *args):
    return check(getattr(lib(), name)(*args))
