"""DBL reachability index (arXiv 2101.09441) on one MI355X: labels, insertion, batched queries.

The work runs in libdbl.so (HIP for gfx950, C ABI in include/dbl.h); this package only binds it.
"""
from .binding import (CLASS_NAMES, DBL_ERR_DEVICE, DBL_ERR_INVALID_ARG, DBL_ERR_OUT_OF_MEMORY,
                      DBL_ERR_VERTEX_RANGE, DBL_OK, EXPORTS, LIB_PATH, DblError, Index,
                      QueryContext, cached_bytes, live_bytes, load_library, release_cache,
                      set_cache_limit, set_device_limit, to_device_ids)

__all__ = ["Index", "QueryContext", "DblError", "load_library", "to_device_ids", "CLASS_NAMES", "EXPORTS",
           "release_cache", "set_cache_limit", "cached_bytes", "live_bytes", "set_device_limit",
           "LIB_PATH", "DBL_OK", "DBL_ERR_INVALID_ARG", "DBL_ERR_VERTEX_RANGE",
           "DBL_ERR_OUT_OF_MEMORY", "DBL_ERR_DEVICE"]
