"""MI355X-native PRUNE filter-bank dataflow path.

libprune_hip.so (HIP, gfx950) holds the graph executor, the control-token
decode and FIFO bookkeeping kernels and the filter-bank forward/adjoint
kernels; this package is its Python binding.
"""
from . import _lib
from ._lib import PruneError

__all__ = ["_lib", "PruneError", "graph", "ops"]
