"""libnrlsh: norm-ranging LSH for maximum inner product search on MI355X.

The compute path lives in ``libnrlsh.so`` (HIP kernels for gfx950 behind the C
ABI of ``include/nrlsh.h``); this package is its thin ctypes binding.
"""
from ._lib import (Index, MultiPlan, NrlshError, header_symbols, lib, nrlsh_build, nrlsh_free,
                   nrlsh_get_query_stats, nrlsh_query_multi, nrlsh_tune_clear, nrlsh_tune_lookup,
                   nrlsh_last_error, nrlsh_profile_enable, nrlsh_profile_get,
                   nrlsh_profile_reset, nrlsh_query, nrlsh_query_noalloc)

__all__ = ["Index", "MultiPlan", "NrlshError", "header_symbols", "lib", "nrlsh_build", "nrlsh_free",
           "nrlsh_get_query_stats", "nrlsh_query_multi", "nrlsh_tune_clear", "nrlsh_tune_lookup",
           "nrlsh_last_error", "nrlsh_profile_enable", "nrlsh_profile_get",
           "nrlsh_profile_reset", "nrlsh_query", "nrlsh_query_noalloc"]
