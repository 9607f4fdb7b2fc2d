"""G-ES-MC global edge switching on AMD MI355X (gfx950).

The hot path -- Philox permutation keys, the radix permutation, the dependency
resolution and the rounds of decisions of each global switch -- runs in the HIP
kernels of ``libgesmc.so`` (C ABI in ``include/gesmc.h``); this package is its
thin ctypes binding.  PyTorch supplies device memory and streams only.
Three forms: ``Context.run`` (one graph), ``Context.run_batch`` (many graphs
in one call) and ``Server`` (a request loop with continuous batching).
"""
from ._binding import (E_AGAIN, E_CANCELED, E_DEVICE, E_INTERNAL, E_INVAL, E_NOMEM, E_NOT_SIMPLE, E_RANGE, EXPORTS,
                       LIB_PATH, OK, OPT_BUCKET_AVG, OPT_FAST_ROUNDS, OPT_FUSE_EMIT, OPT_GRAPH, OPT_LEVEL1_BITS, OPT_SMALL_GRAPHS, OPT_PACK_TUPLES, OPT_PERSIST, OPT_PROFILE,
                       OPT_PROFILE_ONLY, OPT_SORT_CAP, OPT_STRATEGY, STRATEGY_HBM_TABLE, STRATEGY_SORTED_TUPLES, Context, GesmcError,
                       Server, default_context, load_library, run)

__all__ = ["Context", "Server", "GesmcError", "default_context", "load_library", "run", "EXPORTS", "LIB_PATH", "OK",
           "E_INVAL", "E_NOT_SIMPLE", "E_RANGE", "E_NOMEM", "E_DEVICE", "E_AGAIN", "E_CANCELED", "E_INTERNAL",
           "OPT_BUCKET_AVG", "OPT_SORT_CAP", "OPT_FAST_ROUNDS", "OPT_PROFILE", "OPT_STRATEGY", "OPT_PERSIST",
           "OPT_PROFILE_ONLY", "OPT_LEVEL1_BITS", "OPT_FUSE_EMIT", "OPT_GRAPH", "OPT_SMALL_GRAPHS", "OPT_PACK_TUPLES", "STRATEGY_SORTED_TUPLES", "STRATEGY_HBM_TABLE"]
