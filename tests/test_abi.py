"""Host-side checks of the C-ABI library: it loads and exports every declared symbol."""
import ctypes
import os

import pytest

import paper_2203_04158_amd as mbr


def test_library_exports_every_declared_symbol():
    names = mbr.declared_symbols()
    assert len(names) >= 30
    L = ctypes.CDLL(mbr.binding.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_declared_symbols():
    assert set(mbr.declared_symbols()) <= set(mbr.binding._SIGS)


def test_status_strings_and_version():
    L = mbr.lib()
    assert L.mbr_status_str(0) == b"ok"
    assert L.mbr_status_str(-4) == b"state list not sorted"
    assert L.mbr_version() >= 10000


def test_argument_validation_without_gpu():
    # argument checks happen before any device work
    L = mbr.lib()
    h = ctypes.c_void_p()
    assert L.mbr_build_staggered_tables(0, 1, 8, 32, ctypes.byref(h), None) == -1
    assert L.mbr_build_staggered_tables(24, 12, 17, 32, ctypes.byref(h), None) == -1
    assert L.mbr_build_staggered_tables(40, 12, 8, 32, ctypes.byref(h), None) == -1
    assert L.mbr_sector_build(65, 64, 0, None, ctypes.byref(h), None) == -1
    assert L.mbr_rank_batch(None, None, 1, None, None) == -1
    assert b"null" in L.mbr_last_error()


def test_sector_from_list_argument_errors_without_gpu():
    # every one of these is refused before the list is touched
    L = mbr.lib()
    h = ctypes.c_void_p()
    assert L.mbr_sector_from_list(0, 32, None, 0, ctypes.byref(h), None) == -1      # M
    assert L.mbr_sector_from_list(40, 32, None, 0, ctypes.byref(h), None) == -1     # M > 32 in 32 bits
    assert L.mbr_sector_from_list(12, 16, None, 0, ctypes.byref(h), None) == -1     # width
    assert L.mbr_sector_from_list(12, 32, None, 5, ctypes.byref(h), None) == -1     # null list
    assert b"null state list" in L.mbr_last_error()
    assert L.mbr_sector_from_list(12, 32, ctypes.c_void_p(16), 0xFFFFFFFF, ctypes.byref(h), None) == -6
    assert L.mbr_sector_from_list(12, 32, None, 0, None, None) == -1                # null handle
    assert L.mbr_status_str(-5) == b"state list has duplicates"


def test_autotune_argument_errors_without_gpu():
    L = mbr.lib()
    h = ctypes.c_void_p()
    res = mbr.RankTuning()
    assert L.mbr_rank_autotune(None, 1, None, 0, None, 0, 1, ctypes.byref(res), ctypes.byref(h), None) == -1
    assert b"null sector" in L.mbr_last_error()
    assert L.mbr_rank_autotune(None, 1, None, 0, None, 0, 1, None, ctypes.byref(h), None) == -1
    assert L.mbr_learned_autotune(None, None, 0, 1, None, None, None) == -1
    assert b"not a learned ranker" in L.mbr_last_error()
    assert L.mbr_trie_bytes(None, None) == -1
    assert b"null ranker" in L.mbr_last_error()
