"""MI355X-native ranking of many-body occupation patterns (arXiv:2203.04158).

The computation lives in libmbrank.so (HIP for gfx950, C ABI in
include/mbrank.h); this package is its Python binding.
"""
from .binding import *  # noqa: F401,F403
from .binding import lib, declared_symbols, NOT_FOUND, MbrError  # noqa: F401
