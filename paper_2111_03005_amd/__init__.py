"""G-ES-MC global edge switching on AMD MI355X (gfx950).

The hot path -- Philox permutation keys, the radix permutation, the dependency
resolution and the rounds of decisions of each global switch -- runs in the HIP
kernels of ``libgesmc.so`` (C ABI in ``include/gesmc.h``); this package is its
thin ctypes binding.  PyTorch supplies device memory and streams only.
Forms: ``Context.run`` (one graph), ``Context.run_batch`` (many graphs in one
call), ``Server`` (a request loop with continuous batching),
``Context.run_noalloc`` (one graph, nothing allocated inside the call) and
``Context.run_es`` (ParES: the ES-MC chain in supersteps without source
dependencies).
"""
from . import _binding
from ._binding import (Context, GesmcError, Server, default_context, load_library, run, tune_cache_clear,
                       tune_cache_load, tune_cache_save, tune_cache_size)

_CONSTANTS = [k for k in dir(_binding) if k.isupper() and not k.startswith("_")]
globals().update({k: getattr(_binding, k) for k in _CONSTANTS})

__all__ = ["Context", "Server", "GesmcError", "default_context", "load_library", "run", "tune_cache_clear",
           "tune_cache_load", "tune_cache_save", "tune_cache_size"] + _CONSTANTS
