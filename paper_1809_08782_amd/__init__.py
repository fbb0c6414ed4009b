"""libnrlsh: norm-ranging LSH for maximum inner product search on MI355X.

The compute path lives in ``libnrlsh.so`` (HIP kernels for gfx950 behind the C
ABI of ``include/nrlsh.h``); this package is its thin ctypes binding.
"""
from ._lib import (Index, NrlshError, header_symbols, lib, nrlsh_build, nrlsh_free,
                   nrlsh_get_query_stats,
                   nrlsh_last_error, nrlsh_profile_enable, nrlsh_profile_get,
                   nrlsh_profile_reset, nrlsh_query)

__all__ = ["Index", "NrlshError", "header_symbols", "lib", "nrlsh_build", "nrlsh_free",
           "nrlsh_get_query_stats",
           "nrlsh_last_error", "nrlsh_profile_enable", "nrlsh_profile_get",
           "nrlsh_profile_reset", "nrlsh_query"]
