"""Loader for oracle/liboracle.so (the plain-C part of the oracle).

Test infrastructure only: see the package docstring.  The library is compiled
with gcc from oracle.c by `build()`; loading compiles it only when no built
library is present.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build() -> str:
    """Compile oracle.c into liboracle.so (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-fopenmp", "-shared", "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    L = ctypes.CDLL(_LIB)
    u64, i64, i32, dbl, p = (ctypes.c_uint64, ctypes.c_int64, ctypes.c_int,
                             ctypes.c_double, ctypes.c_void_p)
    L.orc_binom.restype, L.orc_binom.argtypes = u64, [i32, i32]
    L.orc_cns_rank.restype, L.orc_cns_rank.argtypes = u64, [u64]
    L.orc_cns_rank_batch.restype, L.orc_cns_rank_batch.argtypes = None, [p, i64, p]
    L.orc_cns_unrank.restype, L.orc_cns_unrank.argtypes = u64, [u64, i32, i32]
    L.orc_sector_enumerate.restype = i64
    L.orc_sector_enumerate.argtypes = [i32, i32, p, p, p, i32, p, i64]
    L.orc_bisect_rank_batch.restype, L.orc_bisect_rank_batch.argtypes = None, [p, i64, p, i64, p]
    L.orc_partrank.restype, L.orc_partrank.argtypes = u64, [u64, i32, i32]
    L.orc_trie_paper_size.restype, L.orc_trie_paper_size.argtypes = i64, [p, i64, i32, p]
    L.orc_apply_terms_bra.restype = i64
    L.orc_apply_terms_bra.argtypes = [p, i64, i32, p, p, p, p, p, p, p, p, i64, i64]
    L.orc_terms_coo.restype = i64
    L.orc_terms_coo.argtypes = [p, i64, i32, p, p, p, p, p, p, p, p, i64]
    L.orc_hubbard_bisect_apply.restype = i64
    L.orc_hubbard_bisect_apply.argtypes = [p, i64, i32, i32, p, p, p, p, p, p, p, i64, i64, i32]
    L.orc_rank_batch_mt.restype = None
    L.orc_rank_batch_mt.argtypes = [p, i64, p, i64, p, i32, i32]
    _lib = L
    return L


def ptr(a):
    """Data pointer of a C-contiguous numpy array."""
    assert a.flags["C_CONTIGUOUS"]
    return ctypes.c_void_p(a.ctypes.data)
