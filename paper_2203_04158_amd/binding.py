"""Thin ctypes binding of libmbrank.so (the C ABI declared in include/mbrank.h).

Only argument marshalling lives here: torch tensors supply device memory and
streams, every computation runs in the HIP library.  Importing this module
does not need a GPU; calling into the library does, and a missing library is
an error (there is no fallback path).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmbrank.so")
NOT_FOUND = 0xFFFFFFFF

RANKER_STAGGERED, RANKER_SPIN, RANKER_TRIE, RANKER_LEARNED, RANKER_BISECT, RANKER_CNS, RANKER_SAMPLED = (
    1, 2, 3, 4, 5, 6, 7)
RANKER_BITMAP_TRIE = 8
F64, F32 = 0, 1
RANK_HALVES, RANK_TRIE = 0, 1

_lib = None


class MbrError(RuntimeError):
    def __init__(self, fn: str, status: int, detail: str):
        super().__init__(f"{fn}: status {status} ({detail})")
        self.status = status


class PopcCons(C.Structure):
    _fields_ = [("mask", C.c_uint64), ("lo", C.c_int32), ("hi", C.c_int32)]


class RankerInfo(C.Structure):
    _fields_ = [("kind", C.c_int32), ("M", C.c_int32), ("k", C.c_int32),
                ("width_bits", C.c_int32), ("n_states", C.c_uint64), ("bytes", C.c_uint64),
                ("levels", C.c_int32), ("reserved", C.c_int32)]


class LearnedOpts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float),
                ("seed", C.c_uint64), ("max_window", C.c_uint64),
                ("samples_per_epoch", C.c_uint64), ("log2_leaves", C.c_int32)]


class LearnedInfo(C.Structure):
    _fields_ = [("n_leaves", C.c_uint64), ("max_window", C.c_uint64), ("mean_window", C.c_double),
                ("single_window_error", C.c_uint64), ("uses_window", C.c_int32)]


class RankTuning(C.Structure):
    _fields_ = [("kind", C.c_int32), ("k", C.c_int32), ("ms", C.c_double), ("from_cache", C.c_int32),
                ("tried", C.c_int32)]


class Term(C.Structure):
    _fields_ = [("v", C.c_double), ("m", C.c_uint64), ("l", C.c_uint64), ("r", C.c_uint64),
                ("x", C.c_uint64), ("s", C.c_uint64)]


class Coulomb(C.Structure):
    _fields_ = [("i", C.c_int32), ("j", C.c_int32), ("k", C.c_int32), ("l", C.c_int32),
                ("U", C.c_double)]


class Bond(C.Structure):
    _fields_ = [("i", C.c_int32), ("j", C.c_int32), ("t", C.c_double)]


class SpinSector(C.Structure):
    _fields_ = [("n_up", C.c_int32), ("n_dn", C.c_int32)]


class HubbardDesc(C.Structure):
    _fields_ = [("L", C.c_int32), ("n_bonds", C.c_int32), ("bonds", C.POINTER(Bond)),
                ("eps", C.POINTER(C.c_double)), ("U", C.POINTER(C.c_double)),
                ("n_sectors", C.c_int32), ("sectors", C.POINTER(SpinSector)),
                ("precision", C.c_int32), ("k", C.c_int32), ("rank_kind", C.c_int32)]


class HubbardCfg(C.Structure):
    _fields_ = [("k", C.c_int32), ("G", C.c_int32), ("block", C.c_int32), ("tiles", C.c_int32),
                ("lds_bytes", C.c_uint64), ("tuned_ms", C.c_double)]


class LanczosOpts(C.Structure):
    _fields_ = [("max_steps", C.c_int32), ("reorth", C.c_int32), ("batched", C.c_int32),
                ("use_graph", C.c_int32), ("breakdown_tol", C.c_double)]


_SIGS = {
    "mbr_status_str": (C.c_char_p, [C.c_int32]),
    "mbr_last_error": (C.c_char_p, []),
    "mbr_version": (C.c_int32, []),
    "mbr_sector_build": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(PopcCons),
                                     C.POINTER(C.c_void_p), C.c_void_p]),
    "mbr_sector_from_list": (C.c_int32, [C.c_int32, C.c_int32, C.c_void_p, C.c_uint64,
                                         C.POINTER(C.c_void_p), C.c_void_p]),
    "mbr_sector_size": (C.c_int32, [C.c_void_p, C.POINTER(C.c_uint64)]),
    "mbr_sector_states": (C.c_int32, [C.c_void_p, C.POINTER(C.c_void_p)]),
    "mbr_sector_destroy": (C.c_int32, [C.c_void_p]),
    "mbr_unrank_batch": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p]),
    "mbr_unrank_spin_batch": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p]),
    "mbr_build_staggered_tables": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                               C.POINTER(C.c_void_p), C.c_void_p]),
    "mbr_staggered_table_copy": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_uint64,
                                             C.POINTER(C.c_uint64), C.c_void_p]),
    "mbr_build_spin_ranker": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                          C.POINTER(C.c_void_p), C.c_void_p]),
    "mbr_build_trie": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.c_void_p]),
    "mbr_build_bitmap_trie": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.c_void_p]),
    "mbr_bitmap_trie_levels": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                           C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "mbr_learned_train": (C.c_int32, [C.c_void_p, C.POINTER(LearnedOpts), C.c_void_p,
                                      C.POINTER(C.c_void_p), C.c_void_p]),
    "mbr_learned_max_error": (C.c_int32, [C.c_void_p, C.POINTER(C.c_uint64),
                                          C.POINTER(C.c_int32)]),
    "mbr_learned_params": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "mbr_learned_autotune": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_int32,
                                         C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p]),
    "mbr_rank_autotune": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_uint64,
                                      C.c_int32, C.POINTER(RankTuning), C.POINTER(C.c_void_p), C.c_void_p]),
    "mbr_learned_stats": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "mbr_sector_build_mod": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                         C.c_int32, C.c_int32, C.POINTER(C.c_void_p), C.c_void_p]),
    "mbr_terms_from_hamiltonian": (C.c_int32, [C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                               C.c_int64, C.POINTER(C.c_int64)]),
    "mbr_operator_create": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                        C.POINTER(C.c_void_p), C.c_void_p]),
    "mbr_operator_apply": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mbr_operator_destroy": (C.c_int32, [C.c_void_p]),
    "mbr_operator_lanczos": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.POINTER(C.c_double),
                                         C.POINTER(C.c_int32), C.c_void_p, C.c_void_p, C.c_void_p]),
    "mbr_rank_batch64": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p]),
    "mbr_build_bisect_ranker": (C.c_int32, [C.c_void_p, C.POINTER(C.c_void_p)]),
    "mbr_build_sampled_ranker": (C.c_int32, [C.c_void_p, C.POINTER(C.c_void_p), C.c_void_p]),
    "mbr_build_cns_ranker": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_void_p),
                                         C.c_void_p]),
    "mbr_trie_bytes": (C.c_int32, [C.c_void_p, C.POINTER(C.c_uint64)]),
    "mbr_trie_level_entries": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_int32),
                                           C.POINTER(C.c_int32)]),
    "mbr_mlp_forward": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "mbr_mlp_gradients": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                      C.c_void_p, C.c_void_p, C.c_void_p]),
    "mbr_mlp_gradients_noalloc": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                              C.c_void_p, C.c_void_p, C.c_void_p]),
    "mbr_ranker_info_get": (C.c_int32, [C.c_void_p, C.POINTER(RankerInfo)]),
    "mbr_rank_batch": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p]),
    "mbr_ranker_destroy": (C.c_int32, [C.c_void_p]),
    "mbr_hubbard_create": (C.c_int32, [C.POINTER(HubbardDesc), C.POINTER(C.c_void_p), C.c_void_p]),
    "mbr_hubbard_dim": (C.c_int32, [C.c_void_p, C.POINTER(C.c_uint64), C.c_void_p]),
    "mbr_hubbard_apply": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mbr_hubbard_destroy": (C.c_int32, [C.c_void_p]),
    "mbr_hubbard_get_config": (C.c_int32, [C.c_void_p, C.POINTER(HubbardCfg)]),
    "mbr_hubbard_set_config": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p]),
    "mbr_hubbard_autotune": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p]),
    "mbr_lanczos_create": (C.c_int32, [C.c_void_p, C.POINTER(LanczosOpts), C.POINTER(C.c_void_p)]),
    "mbr_lanczos_start": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "mbr_lanczos_step": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p]),
    "mbr_lanczos_result": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mbr_lanczos_coeffs": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mbr_lanczos_destroy": (C.c_int32, [C.c_void_p]),
    "mbr_probe_gather": (C.c_int32, [C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64, C.c_int32, C.c_int32,
                                     C.c_void_p, C.c_void_p]),
    "mbr_tridiag_lowest": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                       C.c_void_p, C.c_void_p]),
}


def lib() -> C.CDLL:
    """Load libmbrank.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime with the same soname as the system one;
        # loading torch first makes libmbrank bind to that runtime, so the process
        # holds a single HIP runtime whose device memory and streams both sides share.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2203_04158_amd.build`")
        L = C.CDLL(LIB_PATH)
        missing = []
        for name, (res, args) in _SIGS.items():
            try:
                f = getattr(L, name)
            except AttributeError:
                missing.append(name)
                continue
            f.restype, f.argtypes = res, args
        if missing:
            # a library older than this binding: calling these raises
            for name in missing:
                setattr(L, name, _missing_symbol(name))
        _lib = L
    return _lib


def _missing_symbol(name: str):
    def call(*_a, **_k):
        raise RuntimeError(f"{LIB_PATH} does not export {name}: rebuild it with "
                           "`python -m paper_2203_04158_amd.build`")
    return call


def _check(fn: str, st: int) -> None:
    if st != 0:
        L = lib()
        detail = L.mbr_last_error().decode() or L.mbr_status_str(st).decode()
        raise MbrError(fn, st, detail)


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _dptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return C.c_void_p(t.data_ptr())


def _dvec(t, itemsize: int, n: int, what: str):
    """Device pointer of `t` after checking that it is a contiguous device
    tensor of `itemsize`-byte elements holding at least `n` of them (the C ABI
    takes raw pointers and cannot check sizes)."""
    if t is None or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{what}: expected a contiguous device tensor")
    if t.element_size() != itemsize:
        raise ValueError(f"{what}: expected {itemsize}-byte elements, got {t.element_size()}")
    if t.numel() < n:
        raise ValueError(f"{what}: {t.numel()} elements, need {n}")
    return C.c_void_p(t.data_ptr())


def _torch():
    import torch
    return torch


# --------------------------------------------------------------------------- sectors
class Sector:
    def __init__(self, handle, M: int, width_bits: int):
        self._h = handle
        self.M, self.width_bits = M, width_bits
        n = C.c_uint64()
        _check("mbr_sector_size", lib().mbr_sector_size(self._h, C.byref(n)))
        self.size = int(n.value)

    @property
    def handle(self):
        return self._h

    def states(self, stream=None):
        """The sorted state list as a new device tensor (int32/int64 storage)."""
        torch = _torch()
        idx = torch.arange(self.size, dtype=torch.int32, device="cuda")
        return unrank_batch(self, idx, stream=stream)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mbr_sector_destroy(self._h)
            self._h = None


def sector_build(M: int, constraints, width_bits: int = 32, stream=None) -> Sector:
    """constraints: iterable of (mask, lo, hi) popcount windows."""
    cons = list(constraints)
    arr = (PopcCons * max(1, len(cons)))(*[PopcCons(int(m), int(lo), int(hi)) for m, lo, hi in cons])
    h = C.c_void_p()
    _check("mbr_sector_build", lib().mbr_sector_build(M, width_bits, len(cons), arr, C.byref(h),
                                                      _stream(stream)))
    return Sector(h, M, width_bits)


def sector_from_list(M: int, states, width_bits: int = 32, stream=None) -> Sector:
    """A sector holding the caller's ascending device list `states` (int32 or
    int64 storage of uint32/uint64 patterns), copied and checked by the library."""
    n = states.numel()
    h = C.c_void_p()
    ptr = _dvec(states, width_bits // 8, n, "states") if n else None
    _check("mbr_sector_from_list", lib().mbr_sector_from_list(M, width_bits, ptr, n, C.byref(h),
                                                              _stream(stream)))
    return Sector(h, M, width_bits)


def sector_build_mod(M: int, constraints, weights, modulus: int, residue: int, width_bits: int = 32,
                     stream=None) -> Sector:
    """Popcount windows plus sum(weights of set bits) = residue (mod modulus)."""
    cons = list(constraints)
    arr = (PopcCons * max(1, len(cons)))(*[PopcCons(int(m), int(lo), int(hi)) for m, lo, hi in cons])
    w = (C.c_int32 * M)(*[int(v) for v in weights])
    h = C.c_void_p()
    _check("mbr_sector_build_mod", lib().mbr_sector_build_mod(M, width_bits, len(cons), arr, w, modulus,
                                                              residue, C.byref(h), _stream(stream)))
    return Sector(h, M, width_bits)


def unrank_batch(sector: Sector, idx, out=None, stream=None):
    torch = _torch()
    if out is None:
        dt = torch.int32 if sector.width_bits == 32 else torch.int64
        out = torch.empty(idx.numel(), dtype=dt, device="cuda")
    n = idx.numel()
    _check("mbr_unrank_batch", lib().mbr_unrank_batch(sector.handle, _dvec(idx, 4, n, "idx"), n,
                                                      _dvec(out, sector.width_bits // 8, n, "out"),
                                                      _stream(stream)))
    return out


# --------------------------------------------------------------------------- rankers
class Ranker:
    def __init__(self, handle, keep=()):
        self._h = handle
        self._keep = keep  # handles this ranker references

    @property
    def handle(self):
        return self._h

    def info(self) -> RankerInfo:
        i = RankerInfo()
        _check("mbr_ranker_info_get", lib().mbr_ranker_info_get(self._h, C.byref(i)))
        return i

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mbr_ranker_destroy(self._h)
            self._h = None


def build_staggered_tables(M: int, N: int, k: int, width_bits: int = 32, stream=None) -> Ranker:
    h = C.c_void_p()
    _check("mbr_build_staggered_tables",
           lib().mbr_build_staggered_tables(M, N, k, width_bits, C.byref(h), _stream(stream)))
    return Ranker(h)


def staggered_table(ranker: Ranker, stream=None) -> np.ndarray:
    n = C.c_uint64()
    L = lib()
    _check("mbr_staggered_table_copy",
           L.mbr_staggered_table_copy(ranker.handle, None, 0, C.byref(n), _stream(stream)))
    out = np.zeros(n.value, dtype=np.uint64)
    _check("mbr_staggered_table_copy",
           L.mbr_staggered_table_copy(ranker.handle, C.c_void_p(out.ctypes.data), out.size,
                                      C.byref(n), _stream(stream)))
    return out


def build_spin_ranker(L: int, n_up: int, n_dn: int, k: int, stream=None) -> Ranker:
    h = C.c_void_p()
    _check("mbr_build_spin_ranker",
           lib().mbr_build_spin_ranker(L, n_up, n_dn, k, C.byref(h), _stream(stream)))
    return Ranker(h)


def unrank_spin_batch(ranker: Ranker, idx, out=None, stream=None):
    """Patterns of the spin ranker's sector at int32 device indices `idx`."""
    torch = _torch()
    width = ranker.info().width_bits
    if out is None:
        out = torch.empty(idx.numel(), dtype=torch.int32 if width == 32 else torch.int64, device="cuda")
    n = idx.numel()
    _check("mbr_unrank_spin_batch", lib().mbr_unrank_spin_batch(ranker.handle, _dvec(idx, 4, n, "idx"), n,
                                                                _dvec(out, width // 8, n, "out"),
                                                                _stream(stream)))
    return out


def build_trie(sector: Sector, k: int, stream=None) -> Ranker:
    h = C.c_void_p()
    _check("mbr_build_trie", lib().mbr_build_trie(sector.handle, k, C.byref(h), _stream(stream)))
    return Ranker(h, keep=(sector,))


def build_bitmap_trie(sector: Sector, k: int, stream=None) -> Ranker:
    h = C.c_void_p()
    _check("mbr_build_bitmap_trie", lib().mbr_build_bitmap_trie(sector.handle, k, C.byref(h), _stream(stream)))
    return Ranker(h, keep=(sector,))


def trie_bytes(ranker: Ranker) -> int:
    """Device bytes of a packed or bitmap trie (f = bytes / (4 N_s))."""
    b = C.c_uint64()
    _check("mbr_trie_bytes", lib().mbr_trie_bytes(ranker.handle, C.byref(b)))
    return int(b.value)


def bitmap_trie_levels(ranker: Ranker):
    """(records per level, bytes per record, number of top levels staged in LDS)."""
    rec = np.zeros(64, dtype=np.uint64)
    rb = np.zeros(64, dtype=np.uint32)
    lv, ld = C.c_int32(), C.c_int32()
    _check("mbr_bitmap_trie_levels", lib().mbr_bitmap_trie_levels(
        ranker.handle, C.c_void_p(rec.ctypes.data), C.c_void_p(rb.ctypes.data), 64, C.byref(lv), C.byref(ld)))
    return [int(v) for v in rec[: lv.value]], [int(v) for v in rb[: lv.value]], int(ld.value)


def build_bisect_ranker(sector: Sector) -> Ranker:
    h = C.c_void_p()
    _check("mbr_build_bisect_ranker", lib().mbr_build_bisect_ranker(sector.handle, C.byref(h)))
    return Ranker(h, keep=(sector,))


def build_sampled_ranker(sector: Sector, stream=None) -> Ranker:
    h = C.c_void_p()
    _check("mbr_build_sampled_ranker", lib().mbr_build_sampled_ranker(sector.handle, C.byref(h),
                                                                      _stream(stream)))
    return Ranker(h, keep=(sector,))


def build_cns_ranker(M: int, N: int, width_bits: int = 32, stream=None) -> Ranker:
    h = C.c_void_p()
    _check("mbr_build_cns_ranker", lib().mbr_build_cns_ranker(M, N, width_bits, C.byref(h),
                                                              _stream(stream)))
    return Ranker(h)


def trie_level_entries(ranker: Ranker):
    """(entries per level, number of top levels staged in LDS) of a trie ranker."""
    out = np.zeros(64, dtype=np.uint64)
    lv, ld = C.c_int32(), C.c_int32()
    _check("mbr_trie_level_entries", lib().mbr_trie_level_entries(
        ranker.handle, C.c_void_p(out.ctypes.data), 64, C.byref(lv), C.byref(ld)))
    return [int(v) for v in out[: lv.value]], int(ld.value)


def learned_train(sector: Sector, fallback: Ranker, epochs: int = 4, batch: int = 4096,
                  lr: float = 1e-3, seed: int = 1, max_window: int = 1 << 16,
                  samples_per_epoch: int = 0, log2_leaves: int = 0, stream=None) -> Ranker:
    o = LearnedOpts(epochs, batch, lr, seed, max_window, samples_per_epoch, log2_leaves)
    h = C.c_void_p()
    _check("mbr_learned_train", lib().mbr_learned_train(sector.handle, C.byref(o), fallback.handle,
                                                        C.byref(h), _stream(stream)))
    return Ranker(h, keep=(sector, fallback))


def learned_max_error(ranker: Ranker):
    e = C.c_uint64()
    w = C.c_int32()
    _check("mbr_learned_max_error", lib().mbr_learned_max_error(ranker.handle, C.byref(e), C.byref(w)))
    return int(e.value), bool(w.value)


def learned_autotune(ranker: Ranker, queries, reps: int = 5, stream=None):
    """Time the learned ranker's window search and its fallback on `queries`
    (uint32 device tensor) and keep the faster; returns (ms_window, ms_fallback)."""
    tw, tf = C.c_double(), C.c_double()
    _check("mbr_learned_autotune", lib().mbr_learned_autotune(
        ranker.handle, _dptr(queries), queries.numel(), reps, C.byref(tw), C.byref(tf), _stream(stream)))
    return float(tw.value), float(tf.value)


def rank_autotune(sector: Sector, kind: int, queries, ks=None, reps: int = 5, stream=None):
    """Fastest chunk width of one ranker kind for `sector` on `queries` (device
    tensor of the sector's width); returns (ranker, tuning dict)."""
    res = RankTuning()
    h = C.c_void_p()
    karr = (C.c_int32 * len(ks))(*ks) if ks else None
    _check("mbr_rank_autotune", lib().mbr_rank_autotune(
        sector.handle, kind, karr, len(ks) if ks else 0, _dptr(queries), queries.numel(), reps,
        C.byref(res), C.byref(h), _stream(stream)))
    keep = (sector,) if kind in (RANKER_TRIE, RANKER_BITMAP_TRIE) else ()
    return Ranker(h, keep=keep), {"kind": int(res.kind), "k": int(res.k), "ms": float(res.ms),
                                  "from_cache": bool(res.from_cache), "tried": int(res.tried)}


def learned_stats(ranker: Ranker) -> dict:
    i = LearnedInfo()
    _check("mbr_learned_stats", lib().mbr_learned_stats(ranker.handle, C.byref(i)))
    return {"n_leaves": int(i.n_leaves), "max_window": int(i.max_window),
            "mean_window": float(i.mean_window), "single_window_error": int(i.single_window_error),
            "uses_window": bool(i.uses_window)}


def learned_params(ranker: Ranker, stream=None) -> np.ndarray:
    out = np.zeros(6337, dtype=np.float32)
    _check("mbr_learned_params", lib().mbr_learned_params(ranker.handle, C.c_void_p(out.ctypes.data),
                                                          _stream(stream)))
    return out


def mlp_forward(params, q, out=None, stream=None):
    torch = _torch()
    if out is None:
        out = torch.empty(q.numel(), dtype=torch.float32, device="cuda")
    n = q.numel()
    _check("mbr_mlp_forward", lib().mbr_mlp_forward(_dvec(params, 4, 6337, "params"), _dvec(q, 4, n, "q"), n,
                                                    _dvec(out, 4, n, "out"), _stream(stream)))
    return out


def mlp_gradients(params, q, target, stream=None):
    torch = _torch()
    grad = torch.empty(6337, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    n = q.numel()
    _check("mbr_mlp_gradients", lib().mbr_mlp_gradients(_dvec(params, 4, 6337, "params"), _dvec(q, 4, n, "q"),
                                                        _dvec(target, 4, n, "target"), n, _dptr(grad),
                                                        _dptr(loss), _stream(stream)))
    return grad, loss


def mlp_gradients_noalloc(params, q, target, grad, loss, stream=None):
    """mbr_mlp_gradients into caller-provided grad[6337] and loss[1] (fp32
    device tensors), with no allocation and no synchronisation in the library."""
    n = q.numel()
    _check("mbr_mlp_gradients_noalloc", lib().mbr_mlp_gradients_noalloc(
        _dvec(params, 4, 6337, "params"), _dvec(q, 4, n, "q"), _dvec(target, 4, n, "target"), n,
        _dvec(grad, 4, 6337, "grad"), _dvec(loss, 4, 1, "loss"), _stream(stream)))
    return grad, loss


def rank_batch(ranker: Ranker, q, out=None, stream=None):
    """Ranks of the patterns in q (int32/int64 storage of uint32/uint64 patterns)
    as an int32 tensor whose value -1 is MBR_NOT_FOUND."""
    torch = _torch()
    if out is None:
        out = torch.empty(q.numel(), dtype=torch.int32, device="cuda")
    n = q.numel()
    _check("mbr_rank_batch", lib().mbr_rank_batch(ranker.handle, _dvec(q, ranker.info().width_bits // 8, n, "q"),
                                                  n, _dvec(out, 4, n, "out"), _stream(stream)))
    return out


def rank_batch64(ranker: Ranker, q, out=None, stream=None):
    """64-bit ranks of the patterns in q as an int64 tensor whose value -1 is
    'not in the sector' (staggered rankers)."""
    torch = _torch()
    if out is None:
        out = torch.empty(q.numel(), dtype=torch.int64, device="cuda")
    n = q.numel()
    _check("mbr_rank_batch64", lib().mbr_rank_batch64(ranker.handle,
                                                      _dvec(q, ranker.info().width_bits // 8, n, "q"), n,
                                                      _dvec(out, 8, n, "out"), _stream(stream)))
    return out


# --------------------------------------------------------------------------- general operators
def terms_from_hamiltonian(M: int, t=None, coulomb=()):
    """Tuples of Eq. H: t is an M x M array (or None), coulomb an iterable of
    (i, j, k, l, U).  Returns a list of (v, m, l, r, x, s)."""
    tt = None
    if t is not None:
        tt = np.ascontiguousarray(np.asarray(t, dtype=np.float64).reshape(M, M))
    cl = list(coulomb)
    carr = (Coulomb * max(1, len(cl)))(*[Coulomb(int(i), int(j), int(k), int(l), float(u))
                                         for i, j, k, l, u in cl])
    n = C.c_int64()
    tp = C.c_void_p(tt.ctypes.data) if tt is not None else None
    L = lib()
    _check("mbr_terms_from_hamiltonian", L.mbr_terms_from_hamiltonian(M, tp, len(cl), carr, None, 0,
                                                                      C.byref(n)))
    out = (Term * max(1, n.value))()
    _check("mbr_terms_from_hamiltonian", L.mbr_terms_from_hamiltonian(M, tp, len(cl), carr, out,
                                                                      n.value, C.byref(n)))
    return [(o.v, o.m, o.l, o.r, o.x, o.s) for o in out[: n.value]]


class Operator:
    def __init__(self, handle, sector: Sector, ranker: Ranker, n_terms: int):
        self._h = handle
        self._keep = (sector, ranker)
        self.dim = sector.size
        self.n_terms = n_terms

    @property
    def handle(self):
        return self._h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mbr_operator_destroy(self._h)
            self._h = None


def operator_create(sector: Sector, ranker: Ranker, terms, stream=None) -> Operator:
    """terms: list of (v, m, l, r, x, s) tuples."""
    tl = list(terms)
    arr = (Term * max(1, len(tl)))(*[Term(float(v), int(m), int(l), int(r), int(x), int(s))
                                     for v, m, l, r, x, s in tl])
    h = C.c_void_p()
    _check("mbr_operator_create", lib().mbr_operator_create(sector.handle, ranker.handle, arr, len(tl),
                                                            C.byref(h), _stream(stream)))
    return Operator(h, sector, ranker, len(tl))


def operator_apply(op: Operator, x, y, stream=None):
    _check("mbr_operator_apply", lib().mbr_operator_apply(op.handle, _dvec(x, 8, op.dim, "x"),
                                                          _dvec(y, 8, op.dim, "y"), _stream(stream)))
    return y


def operator_lanczos(op: Operator, v0, nsteps: int, tol: float = 1e-12, stream=None):
    """(E0, steps taken, alpha[nsteps], beta[nsteps]) by fp64 Lanczos on the GPU."""
    e0 = C.c_double()
    nd = C.c_int32()
    al = np.zeros(nsteps)
    be = np.zeros(nsteps)
    _check("mbr_operator_lanczos", lib().mbr_operator_lanczos(op.handle, _dvec(v0, 8, op.dim, "v0"), nsteps,
                                                              tol, C.byref(e0),
                                                              C.byref(nd), C.c_void_p(al.ctypes.data),
                                                              C.c_void_p(be.ctypes.data), _stream(stream)))
    return float(e0.value), int(nd.value), al, be


# --------------------------------------------------------------------------- Hamiltonian
class Hubbard:
    def __init__(self, handle, precision: int, n_sectors: int):
        self._h = handle
        self.precision = precision
        self.n_sectors = n_sectors
        tot = C.c_uint64()
        offs = (C.c_uint64 * (n_sectors + 1))()
        _check("mbr_hubbard_dim", lib().mbr_hubbard_dim(self._h, C.byref(tot), offs))
        self.dim = int(tot.value)
        self.offsets = [int(v) for v in offs]

    @property
    def handle(self):
        return self._h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mbr_hubbard_destroy(self._h)
            self._h = None


def hubbard_create(L: int, bonds, sectors, U=None, eps=None, precision: int = F64, k: int = 0,
                   rank_kind: int = 0, stream=None) -> Hubbard:
    """bonds: [(i, j, t)]; sectors: [(n_up, n_dn)]; U, eps: per-site lists or None;
    rank_kind: RANK_HALVES (staggered halves) or RANK_TRIE (trie over full patterns)."""
    b = (Bond * max(1, len(bonds)))(*[Bond(int(i), int(j), float(t)) for i, j, t in bonds])
    s = (SpinSector * len(sectors))(*[SpinSector(int(u), int(d)) for u, d in sectors])
    Uv = (C.c_double * L)(*[float(u) for u in U]) if U is not None else None
    ev = (C.c_double * L)(*[float(e) for e in eps]) if eps is not None else None
    d = HubbardDesc(L=L, n_bonds=len(bonds), bonds=b, eps=ev, U=Uv, n_sectors=len(sectors),
                    sectors=s, precision=precision, k=k, rank_kind=rank_kind)
    h = C.c_void_p()
    _check("mbr_hubbard_create", lib().mbr_hubbard_create(C.byref(d), C.byref(h), _stream(stream)))
    return Hubbard(h, precision, len(sectors))


def hubbard_apply(h: Hubbard, x, y, stream=None):
    tsz = 8 if h.precision == F64 else 4
    _check("mbr_hubbard_apply", lib().mbr_hubbard_apply(h.handle, _dvec(x, tsz, h.dim, "x"),
                                                        _dvec(y, tsz, h.dim, "y"), _stream(stream)))
    return y


def hubbard_get_config(h: Hubbard) -> dict:
    c = HubbardCfg()
    _check("mbr_hubbard_get_config", lib().mbr_hubbard_get_config(h.handle, C.byref(c)))
    return {"k": c.k, "G": c.G, "block": c.block, "tiles": c.tiles, "lds_bytes": c.lds_bytes,
            "tuned_ms": c.tuned_ms}


def hubbard_set_config(h: Hubbard, k: int, G: int, block: int, stream=None):
    _check("mbr_hubbard_set_config", lib().mbr_hubbard_set_config(h.handle, k, G, block,
                                                                  _stream(stream)))


def hubbard_autotune(h: Hubbard, reps: int = 5, stream=None) -> dict:
    _check("mbr_hubbard_autotune", lib().mbr_hubbard_autotune(h.handle, reps, _stream(stream)))
    return hubbard_get_config(h)


# --------------------------------------------------------------------------- Lanczos
class Lanczos:
    def __init__(self, handle, h: Hubbard, max_steps: int):
        self._h = handle
        self.ham = h
        self.max_steps = max_steps

    @property
    def handle(self):
        return self._h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mbr_lanczos_destroy(self._h)
            self._h = None


def lanczos_create(h: Hubbard, max_steps: int, reorth: bool = False, batched: bool = True,
                   use_graph: bool = True, breakdown_tol: float = 0.0) -> Lanczos:
    o = LanczosOpts(max_steps, int(reorth), int(batched), int(use_graph), breakdown_tol)
    p = C.c_void_p()
    _check("mbr_lanczos_create", lib().mbr_lanczos_create(h.handle, C.byref(o), C.byref(p)))
    return Lanczos(p, h, max_steps)


def lanczos_start(lz: Lanczos, v0, stream=None):
    _check("mbr_lanczos_start", lib().mbr_lanczos_start(lz.handle, _dvec(v0, 8, lz.ham.dim, "v0"),
                                                        _stream(stream)))


def lanczos_step(lz: Lanczos, nsteps: int, stream=None):
    _check("mbr_lanczos_step", lib().mbr_lanczos_step(lz.handle, nsteps, _stream(stream)))


def lanczos_result(lz: Lanczos, stream=None):
    n = lz.ham.n_sectors
    e0 = np.zeros(n)
    steps = np.zeros(n, dtype=np.int32)
    _check("mbr_lanczos_result", lib().mbr_lanczos_result(lz.handle, C.c_void_p(e0.ctypes.data),
                                                          C.c_void_p(steps.ctypes.data),
                                                          _stream(stream)))
    return e0, steps


def lanczos_coeffs(lz: Lanczos, stream=None):
    n = lz.ham.n_sectors * lz.max_steps
    a = np.zeros(n)
    b = np.zeros(n)
    _check("mbr_lanczos_coeffs", lib().mbr_lanczos_coeffs(lz.handle, C.c_void_p(a.ctypes.data),
                                                          C.c_void_p(b.ctypes.data),
                                                          _stream(stream)))
    return a.reshape(lz.ham.n_sectors, -1), b.reshape(lz.ham.n_sectors, -1)


def tridiag_lowest(alpha, beta, lengths, ld: int, out=None, stream=None):
    torch = _torch()
    nb = lengths.numel()
    if out is None:
        out = torch.empty(nb, dtype=torch.float64, device="cuda")
    _check("mbr_tridiag_lowest", lib().mbr_tridiag_lowest(_dvec(alpha, 8, nb * ld, "alpha"),
                                                          _dvec(beta, 8, nb * ld, "beta"),
                                                          _dvec(lengths, 4, nb, "lengths"), ld, nb,
                                                          _dvec(out, 8, nb, "out"), _stream(stream)))
    return out


def probe_gather(table, idx, depth: int = 1, lds: bool = False, out=None, stream=None):
    """Gather probe: out[j] = the index reached after `depth` chained reads
    i <- table[i] mod len(table), starting from idx[j] mod len(table)."""
    torch = _torch()
    n = idx.numel()
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device="cuda")
    _check("mbr_probe_gather", lib().mbr_probe_gather(_dvec(table, 4, table.numel(), "table"), table.numel(),
                                                      _dvec(idx, 4, n, "idx"), n, depth, int(lds),
                                                      _dvec(out, 4, n, "out"), _stream(stream)))
    return out


def declared_symbols():
    """Names of every function declared in include/mbrank.h."""
    import re
    hdr = os.path.join(_HERE, "..", "include", "mbrank.h")
    text = open(hdr).read()
    return sorted(set(re.findall(r"^\s*(?:const char \*|mbr_status|int32_t)\s*(mbr_\w+)\(", text,
                                 re.M)))
