"""Python binding of libgenie (match-count search with c-PQ on MI355X).

Argument marshalling only: every step of the search runs in the library's
HIP kernels.  PyTorch supplies device memory and streams.  The functions
carry the names of the C-ABI calls in ``include/genie.h``.

The library must be built (``python -m paper_1603_08390_amd.build`` or
``__graft_entry__.build()``); importing works without it, but every call
raises ``GenieError`` when ``libgenie.so`` is missing -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgenie.so")

GENIE_OK = 0
GENIE_EINVAL = -22
GENIE_ENOMEM = -12
GENIE_EDEVICE = -5
GENIE_ERANGE = -34
GENIE_MAX_K = 1024
GENIE_MAX_ITEMS = 1024
GENIE_TILE_OBJECTS = 65535
STATUS_BAD_DIM = 1
STATUS_TOO_MANY_ITEMS = 2
STATUS_BAD_OFFSETS = 4
STATUS_RANGE_ON_SET = 8

EXPORTED = (
    "genie_build_index", "genie_build_index_tiled", "genie_free_index", "genie_index_info_get",
    "genie_search",
    "genie_search_workspace_size", "genie_search_async", "genie_match_count_async",
    "genie_lsh_signatures", "genie_last_error", "genie_kernel_timing_enable",
    "genie_kernel_timing_read", "genie_search_gated_async", "genie_gate_features_async",
    "genie_gate_forward_async", "genie_gate_workspace_size", "genie_gate_backward_async",
    "genie_gate_adam_async", "genie_lsh_items_async", "genie_index_set_scan_shape",
    "genie_index_set_scan_schedule", "genie_search_rows_async", "genie_parts_build",
    "genie_parts_free", "genie_parts_info_get", "genie_parts_workspace_size",
    "genie_parts_search_async", "genie_search_spq_async", "genie_rbh_signatures",
    "genie_build_index_sets", "genie_seq_build", "genie_seq_free", "genie_seq_info_get",
    "genie_seq_match_index", "genie_seq_decompose_async", "genie_seq_verify_async",
    "genie_seq_workspace_size", "genie_seq_search_async", "genie_search_noalloc_async",
    "genie_probe_lds_atomics", "genie_probe_hbm", "genie_index_set_hash_slots",
)
NOALLOC_WORKSPACE_BYTES = 64 << 20
GATE_FEATURES = 64
GATE_PARAMS = 24961


class GenieError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libgenie error {code}: {msg}")
        self.code = code


class _KernelTimes(ctypes.Structure):
    _fields_ = [("scan_launches", ctypes.c_uint64), ("scan_ms", ctypes.c_double),
                ("merge_launches", ctypes.c_uint64), ("merge_ms", ctypes.c_double),
                ("fallback_launches", ctypes.c_uint64), ("fallback_ms", ctypes.c_double)]


class _PartsInfo(ctypes.Structure):
    _fields_ = [("n_objects", ctypes.c_uint64), ("n_parts", ctypes.c_uint32),
                ("tiles_total", ctypes.c_uint32), ("part_objects", ctypes.c_uint64),
                ("host_bytes", ctypes.c_uint64), ("device_bytes", ctypes.c_uint64)]


class _SeqInfo(ctypes.Structure):
    _fields_ = [("n_sequences", ctypes.c_uint64), ("n_chars", ctypes.c_uint64),
                ("n_windows", ctypes.c_uint64), ("gram", ctypes.c_uint32),
                ("alphabet", ctypes.c_uint32), ("n_grams", ctypes.c_uint32),
                ("n_keys", ctypes.c_uint32), ("max_occurrences", ctypes.c_uint32),
                ("n_tiles", ctypes.c_uint32), ("device_bytes", ctypes.c_uint64)]


class _IndexInfo(ctypes.Structure):
    _fields_ = [("n_objects", ctypes.c_uint64), ("n_dims", ctypes.c_uint32),
                ("n_buckets", ctypes.c_uint32), ("n_tiles", ctypes.c_uint32),
                ("tile_objects", ctypes.c_uint32), ("n_postings", ctypes.c_uint64),
                ("device_bytes", ctypes.c_uint64), ("scan_threads", ctypes.c_uint32),
                ("scan_unroll", ctypes.c_uint32), ("scan_persistent", ctypes.c_uint32),
                ("map_compact", ctypes.c_uint32), ("map_bytes", ctypes.c_uint64)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libgenie.so; raises GenieError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise GenieError(GENIE_EDEVICE, f"{LIB_PATH} is not built; run "
                         "python -m paper_1603_08390_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, sz = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t
    lib.genie_build_index.argtypes = [vp, u64, u32, u32, ctypes.POINTER(vp)]
    lib.genie_build_index.restype = ctypes.c_int
    lib.genie_build_index_tiled.argtypes = [vp, u64, u32, u32, u32, ctypes.POINTER(vp)]
    lib.genie_build_index_tiled.restype = ctypes.c_int
    lib.genie_free_index.argtypes = [vp]
    lib.genie_free_index.restype = None
    lib.genie_index_info_get.argtypes = [vp, ctypes.POINTER(_IndexInfo)]
    lib.genie_index_info_get.restype = ctypes.c_int
    lib.genie_search.argtypes = [vp, vp, vp, u32, u32, vp, vp]
    lib.genie_search.restype = ctypes.c_int
    lib.genie_search_workspace_size.argtypes = [vp, u32, u32]
    lib.genie_search_workspace_size.restype = sz
    lib.genie_search_async.argtypes = [vp, vp, vp, u64, u32, u32, u32, vp, vp, vp, sz, vp]
    lib.genie_search_async.restype = ctypes.c_int
    lib.genie_match_count_async.argtypes = [vp, vp, vp, u64, u32, u32, vp, vp, sz, vp]
    lib.genie_match_count_async.restype = ctypes.c_int
    lib.genie_lsh_signatures.argtypes = [vp, u64, u32, vp, vp, ctypes.c_float, u32, vp, u32,
                                         vp, vp]
    lib.genie_lsh_signatures.restype = ctypes.c_int
    lib.genie_rbh_signatures.argtypes = [vp, u64, u32, vp, vp, vp, u32, u32, vp, vp]
    lib.genie_rbh_signatures.restype = ctypes.c_int
    lib.genie_kernel_timing_enable.argtypes = [ctypes.c_int]
    lib.genie_kernel_timing_enable.restype = ctypes.c_int
    lib.genie_kernel_timing_read.argtypes = [ctypes.POINTER(_KernelTimes), ctypes.c_int]
    lib.genie_kernel_timing_read.restype = ctypes.c_int
    f32 = ctypes.c_float
    lib.genie_search_gated_async.argtypes = [vp, vp, vp, u64, u32, u32, u32, vp, f32, vp, vp, vp,
                                             sz, vp]
    lib.genie_search_gated_async.restype = ctypes.c_int
    lib.genie_search_rows_async.argtypes = [vp, vp, vp, u64, u32, vp, u32, u32, vp, f32, vp, vp,
                                            vp, sz, vp]
    lib.genie_search_rows_async.restype = ctypes.c_int
    lib.genie_search_spq_async.argtypes = [vp, vp, vp, u64, u32, u32, u32, vp, vp, vp, sz, vp]
    lib.genie_search_spq_async.restype = ctypes.c_int
    lib.genie_search_noalloc_async.argtypes = [vp, vp, vp, u64, u32, u32, u32, vp, vp, vp]
    lib.genie_search_noalloc_async.restype = ctypes.c_int
    dp = ctypes.POINTER(ctypes.c_double)
    lib.genie_probe_lds_atomics.argtypes = [ctypes.c_int, u32, u32, vp, dp]
    lib.genie_probe_lds_atomics.restype = ctypes.c_int
    lib.genie_probe_hbm.argtypes = [vp, vp, u64, u32, vp, dp, dp]
    lib.genie_probe_hbm.restype = ctypes.c_int
    lib.genie_parts_build.argtypes = [vp, u64, u32, u32, u64, u32, ctypes.POINTER(vp)]
    lib.genie_parts_build.restype = ctypes.c_int
    lib.genie_parts_free.argtypes = [vp]
    lib.genie_parts_free.restype = None
    lib.genie_parts_info_get.argtypes = [vp, ctypes.POINTER(_PartsInfo)]
    lib.genie_parts_info_get.restype = ctypes.c_int
    lib.genie_parts_workspace_size.argtypes = [vp, u32, u32]
    lib.genie_parts_workspace_size.restype = sz
    lib.genie_parts_search_async.argtypes = [vp, vp, vp, u64, u32, u32, u32, vp, vp, vp, sz, vp]
    lib.genie_parts_search_async.restype = ctypes.c_int
    lib.genie_gate_features_async.argtypes = [vp, vp, vp, u64, u32, u32, vp, vp]
    lib.genie_gate_features_async.restype = ctypes.c_int
    lib.genie_gate_forward_async.argtypes = [vp, vp, vp, u32, vp, vp]
    lib.genie_gate_forward_async.restype = ctypes.c_int
    lib.genie_gate_workspace_size.argtypes = [u32]
    lib.genie_gate_workspace_size.restype = sz
    lib.genie_gate_backward_async.argtypes = [vp, vp, vp, vp, u32, f32, vp, vp, vp, sz, vp]
    lib.genie_gate_backward_async.restype = ctypes.c_int
    lib.genie_gate_adam_async.argtypes = [vp, vp, vp, vp, vp, u32, f32, f32, f32, f32, vp]
    lib.genie_gate_adam_async.restype = ctypes.c_int
    lib.genie_lsh_items_async.argtypes = [vp, u32, u32, vp, vp, vp]
    lib.genie_lsh_items_async.restype = ctypes.c_int
    lib.genie_index_set_scan_shape.argtypes = [vp, u32, u32]
    lib.genie_index_set_scan_shape.restype = ctypes.c_int
    lib.genie_index_set_scan_schedule.argtypes = [vp, u32]
    lib.genie_index_set_scan_schedule.restype = ctypes.c_int
    lib.genie_index_set_hash_slots.argtypes = [vp, u32]
    lib.genie_index_set_hash_slots.restype = ctypes.c_int
    lib.genie_build_index_sets.argtypes = [vp, vp, u64, u32, u32, ctypes.POINTER(vp)]
    lib.genie_build_index_sets.restype = ctypes.c_int
    lib.genie_seq_build.argtypes = [vp, vp, u64, u32, u32, ctypes.POINTER(vp)]
    lib.genie_seq_build.restype = ctypes.c_int
    lib.genie_seq_free.argtypes = [vp]
    lib.genie_seq_free.restype = None
    lib.genie_seq_info_get.argtypes = [vp, ctypes.POINTER(_SeqInfo)]
    lib.genie_seq_info_get.restype = ctypes.c_int
    lib.genie_seq_match_index.argtypes = [vp]
    lib.genie_seq_match_index.restype = vp
    lib.genie_seq_decompose_async.argtypes = [vp, vp, vp, u64, u32, vp, vp]
    lib.genie_seq_decompose_async.restype = ctypes.c_int
    lib.genie_seq_verify_async.argtypes = [vp, vp, vp, u64, u32, u32, vp, vp, u32, u32, vp, vp,
                                           vp, vp]
    lib.genie_seq_verify_async.restype = ctypes.c_int
    lib.genie_seq_workspace_size.argtypes = [vp, u32, u64, u32]
    lib.genie_seq_workspace_size.restype = sz
    lib.genie_seq_search_async.argtypes = [vp, vp, vp, u64, u32, u32, u32, u32, vp, vp, vp, vp,
                                           sz, vp]
    lib.genie_seq_search_async.restype = ctypes.c_int
    lib.genie_last_error.argtypes = []
    lib.genie_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc: int):
    if rc != GENIE_OK:
        raise GenieError(rc, load().genie_last_error().decode(errors="replace"))


def _np_ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _dev_ptr(t) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream or None


@dataclass
class IndexInfo:
    n_objects: int
    n_dims: int
    n_buckets: int
    n_tiles: int
    tile_objects: int
    n_postings: int
    device_bytes: int
    scan_shape: tuple      # (threads per workgroup, posting dwords per thread and step)
    scan_persistent: int   # 0: one workgroup per (query, tile) pair; 1: persistent; 2: auto
    map_compact: int = 0   # 1: Position Map in the compact form
    map_bytes: int = 0     # device bytes of the Position Map


class Index:
    """genie_build_index: the inverted index of Section 3.2 on the device."""

    def __init__(self, values: np.ndarray, n_buckets: int, tile_log2: int = 16):
        """tile_log2: tiles of 2^tile_log2 - 1 objects (15 or 16), see
        genie_build_index_tiled."""
        values = np.ascontiguousarray(values, dtype=np.uint32)
        if values.ndim != 2:
            raise ValueError("values must be [n_objects, n_dims]")
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.genie_build_index_tiled(_np_ptr(values), values.shape[0], values.shape[1],
                                           int(n_buckets), int(tile_log2), ctypes.byref(h)))
        self._h = h
        self.refresh_info()

    def refresh_info(self):
        info = _IndexInfo()
        _check(load().genie_index_info_get(self.handle, ctypes.byref(info)))
        self.info = IndexInfo(info.n_objects, info.n_dims, info.n_buckets, info.n_tiles,
                              info.tile_objects, info.n_postings, info.device_bytes,
                              (info.scan_threads, info.scan_unroll), info.scan_persistent,
                              info.map_compact, info.map_bytes)

    @property
    def handle(self):
        if self._h is None:
            raise GenieError(GENIE_EINVAL, "index is freed")
        return self._h

    def free(self):
        if getattr(self, "_h", None) is not None:
            load().genie_free_index(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class _BorrowedIndex(Index):
    """An index owned by another object (e.g. a sequence index's match index)."""

    def __init__(self, handle, owner):
        self._h = ctypes.c_void_p(handle)
        self._owner = owner
        self.refresh_info()

    def free(self):
        self._h = None


def genie_build_index_sets(obj_offsets: np.ndarray, keys: np.ndarray, n_keys: int,
                           tile_log2: int = 16) -> Index:
    """Index over keyword sets: object o holds keys[obj_offsets[o] ..
    obj_offsets[o+1]) (Sections 2.2 and 5); query items name one keyword each."""
    obj_offsets = np.ascontiguousarray(obj_offsets, dtype=np.uint64)
    keys = np.ascontiguousarray(keys, dtype=np.uint32)
    ix = Index.__new__(Index)
    h = ctypes.c_void_p()
    _check(load().genie_build_index_sets(_np_ptr(obj_offsets),
                                         _np_ptr(keys) if keys.size else None,
                                         obj_offsets.size - 1, int(n_keys), int(tile_log2),
                                         ctypes.byref(h)))
    ix._h = h
    ix.refresh_info()
    return ix


class SeqIndex:
    """genie_seq_build: sequences decomposed into ordered n-grams and indexed
    for match-count search, kept on the device for verification (Section 5.1)."""

    def __init__(self, chars: np.ndarray, offsets: np.ndarray, gram: int = 3,
                 tile_log2: int = 16):
        chars = np.ascontiguousarray(chars, dtype=np.uint8)
        offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
        h = ctypes.c_void_p()
        _check(load().genie_seq_build(_np_ptr(chars) if chars.size else None, _np_ptr(offsets),
                                      offsets.size - 1, int(gram), int(tile_log2),
                                      ctypes.byref(h)))
        self._h = h
        info = _SeqInfo()
        _check(load().genie_seq_info_get(self._h, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in _SeqInfo._fields_}
        self.match_index = _BorrowedIndex(load().genie_seq_match_index(self._h), self)

    @property
    def handle(self):
        if self._h is None:
            raise GenieError(GENIE_EINVAL, "sequence index is freed")
        return self._h

    def free(self):
        if getattr(self, "_h", None) is not None:
            self.match_index.free()
            load().genie_seq_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def workspace(self, n_queries: int, n_qchars: int, K: int, device="cuda"):
        import torch
        nbytes = load().genie_seq_workspace_size(self.handle, int(n_queries), int(n_qchars),
                                                 int(K))
        return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def genie_seq_build(chars: np.ndarray, offsets: np.ndarray, gram: int = 3,
                    tile_log2: int = 16) -> SeqIndex:
    return SeqIndex(chars, offsets, gram, tile_log2)


def genie_seq_free(sx: SeqIndex):
    sx.free()


def genie_seq_info_get(sx: SeqIndex) -> dict:
    return dict(sx.info)


def genie_seq_match_index(sx: SeqIndex) -> Index:
    return sx.match_index


def genie_seq_workspace_size(sx: SeqIndex, n_queries: int, n_qchars: int, K: int) -> int:
    return int(load().genie_seq_workspace_size(sx.handle, int(n_queries), int(n_qchars), int(K)))


def genie_seq_decompose_async(sx: SeqIndex, d_qchars, d_qoffsets, out_items=None, stream=None):
    """Items of the queries' ordered n-grams, one per query byte (Section 5.1.2)."""
    import torch
    nq = d_qoffsets.numel() - 1
    if out_items is None:
        out_items = torch.empty((max(d_qchars.numel(), 1), 3), dtype=torch.int32,
                                device=d_qoffsets.device)
    if nq > 0:
        _check(load().genie_seq_decompose_async(sx.handle, _dev_ptr(d_qchars),
                                                _dev_ptr(d_qoffsets), d_qchars.numel(), nq,
                                                _dev_ptr(out_items), _stream_handle(stream)))
    return out_items


def _seq_outputs(nq, k, dev, out_ids, out_dist, out_cert):
    import torch
    if out_ids is None:
        out_ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
    if out_dist is None:
        out_dist = torch.empty((nq, k), dtype=torch.int32, device=dev)
    if out_cert is None:
        out_cert = torch.empty((max(nq, 1),), dtype=torch.int32, device=dev)
    return out_ids, out_dist, out_cert


def genie_seq_verify_async(sx: SeqIndex, d_qchars, d_qoffsets, max_qlen: int, d_cand_ids,
                           d_cand_counts, k: int, out_ids=None, out_dist=None, out_cert=None,
                           stream=None):
    """Algorithm 2 over K candidates per query ([nq, K] in count order) and
    the certificate of Theorem 5.2; returns (ids, dist, cert)."""
    nq = d_qoffsets.numel() - 1
    K = d_cand_ids.shape[1]
    if (d_cand_ids.dim() != 2 or tuple(d_cand_counts.shape) != tuple(d_cand_ids.shape)
            or d_cand_ids.shape[0] < nq):
        raise ValueError("candidates must be [n_queries, K] ids and counts")
    out_ids, out_dist, out_cert = _seq_outputs(nq, k, d_qoffsets.device, out_ids, out_dist,
                                               out_cert)
    if nq > 0:
        _check(load().genie_seq_verify_async(sx.handle, _dev_ptr(d_qchars), _dev_ptr(d_qoffsets),
                                             d_qchars.numel(), nq, int(max_qlen),
                                             _dev_ptr(d_cand_ids), _dev_ptr(d_cand_counts),
                                             int(K), int(k), _dev_ptr(out_ids),
                                             _dev_ptr(out_dist), _dev_ptr(out_cert),
                                             _stream_handle(stream)))
    return out_ids, out_dist, out_cert


def genie_seq_search_async(sx: SeqIndex, d_qchars, d_qoffsets, max_qlen: int, K: int, k: int,
                           out_ids=None, out_dist=None, out_cert=None, workspace=None,
                           stream=None):
    """Decomposition, top-K match-count search and verification (Section 5.1);
    returns (ids, dist, cert, workspace)."""
    nq = d_qoffsets.numel() - 1
    dev = d_qoffsets.device
    out_ids, out_dist, out_cert = _seq_outputs(nq, k, dev, out_ids, out_dist, out_cert)
    if workspace is None:
        workspace = sx.workspace(max(nq, 0), d_qchars.numel(), K, dev)
    if nq > 0:
        _check(load().genie_seq_search_async(sx.handle, _dev_ptr(d_qchars), _dev_ptr(d_qoffsets),
                                             d_qchars.numel(), nq, int(max_qlen), int(K), int(k),
                                             _dev_ptr(out_ids), _dev_ptr(out_dist),
                                             _dev_ptr(out_cert), _dev_ptr(workspace),
                                             workspace.numel(), _stream_handle(stream)))
    return out_ids, out_dist, out_cert, workspace


class PartsIndex:
    """genie_parts_build: multiple loadings (Section 3.4).  The index is cut
    into parts of `part_objects` objects kept in pinned host memory and
    streamed through two device slots by every search."""

    def __init__(self, values: np.ndarray, n_buckets: int, part_objects: int,
                 tile_log2: int = 16):
        values = np.ascontiguousarray(values, dtype=np.uint32)
        if values.ndim != 2:
            raise ValueError("values must be [n_objects, n_dims]")
        h = ctypes.c_void_p()
        _check(load().genie_parts_build(_np_ptr(values), values.shape[0], values.shape[1],
                                        int(n_buckets), int(part_objects), int(tile_log2),
                                        ctypes.byref(h)))
        self._h = h
        info = _PartsInfo()
        _check(load().genie_parts_info_get(self._h, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in _PartsInfo._fields_}

    @property
    def handle(self):
        if self._h is None:
            raise GenieError(GENIE_EINVAL, "parts index is freed")
        return self._h

    def free(self):
        if getattr(self, "_h", None) is not None:
            load().genie_parts_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def workspace(self, n_queries: int, k: int, device="cuda"):
        import torch
        nbytes = load().genie_parts_workspace_size(self.handle, int(n_queries), int(k))
        return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def genie_parts_build(values: np.ndarray, n_buckets: int, part_objects: int,
                      tile_log2: int = 16) -> PartsIndex:
    return PartsIndex(values, n_buckets, part_objects, tile_log2)


def genie_parts_free(parts: PartsIndex):
    parts.free()


def genie_parts_info_get(parts: PartsIndex) -> dict:
    return dict(parts.info)


def genie_parts_workspace_size(parts: PartsIndex, n_queries: int, k: int) -> int:
    return int(load().genie_parts_workspace_size(parts.handle, int(n_queries), int(k)))


def genie_parts_search_async(parts: PartsIndex, d_q_offsets, d_items, k: int, max_items: int,
                             out_ids=None, out_counts=None, workspace=None, stream=None):
    """Top-k search over every part, identical to genie_search_async on one
    index of all the objects."""
    import torch
    nq = d_q_offsets.numel() - 1
    dev = d_q_offsets.device
    if out_ids is None:
        out_ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
    if out_counts is None:
        out_counts = torch.empty((nq, k), dtype=torch.int32, device=dev)
    if workspace is None:
        workspace = parts.workspace(nq, k, dev)
    if nq <= 0:
        return out_ids, out_counts, workspace
    _check(load().genie_parts_search_async(parts.handle, _dev_ptr(d_q_offsets), _dev_ptr(d_items),
                                           d_items.numel() // 3, nq, int(max_items), int(k),
                                           _dev_ptr(out_ids), _dev_ptr(out_counts),
                                           _dev_ptr(workspace), workspace.numel(),
                                           _stream_handle(stream)))
    return out_ids, out_counts, workspace


def genie_build_index(values: np.ndarray, n_buckets: int) -> Index:
    return Index(values, n_buckets)


def genie_build_index_tiled(values: np.ndarray, n_buckets: int, tile_log2: int) -> Index:
    return Index(values, n_buckets, tile_log2)


def genie_index_set_scan_shape(index: Index, threads: int, unroll: int):
    _check(load().genie_index_set_scan_shape(index.handle, int(threads), int(unroll)))
    index.refresh_info()


def genie_index_set_scan_schedule(index: Index, persistent: int):
    _check(load().genie_index_set_scan_schedule(index.handle, int(persistent)))
    index.refresh_info()


SCAN_SHAPES = ((512, 4), (512, 8), (1024, 4), (1024, 8))
SCAN_SCHEDULES = (0, 1)   # one workgroup per pair, persistent


def genie_index_set_hash_slots(index: Index, log2_slots: int):
    """Cap the c-PQ Hash Table at 2^log2_slots slots (0: default size)."""
    _check(load().genie_index_set_hash_slots(index.handle, int(log2_slots)))


def genie_search(index: Index, q_offsets: np.ndarray, items: np.ndarray, k: int
                 ) -> Tuple[np.ndarray, np.ndarray]:
    """Synchronous search with host arrays; returns (ids, counts) [nq, k] uint32."""
    q_offsets = np.ascontiguousarray(q_offsets, dtype=np.uint64)
    items = np.ascontiguousarray(items, dtype=np.uint32).reshape(-1, 3)
    nq = len(q_offsets) - 1
    ids = np.zeros((max(nq, 0), k), dtype=np.uint32)
    cts = np.zeros((max(nq, 0), k), dtype=np.uint32)
    if nq <= 0:
        return ids, cts
    items_p = _np_ptr(items) if items.size else None
    _check(load().genie_search(index.handle, _np_ptr(q_offsets), items_p, nq, int(k),
                               _np_ptr(ids), _np_ptr(cts)))
    return ids, cts


def genie_search_workspace_size(index: Index, n_queries: int, k: int) -> int:
    return int(load().genie_search_workspace_size(index.handle, int(n_queries), int(k)))


def alloc_workspace(index: Index, n_queries: int, k: int, device="cuda"):
    import torch
    nbytes = genie_search_workspace_size(index, n_queries, k)
    if nbytes == 0:
        raise GenieError(GENIE_EINVAL, "bad workspace request")
    # torch's caching allocator returns 256-byte aligned blocks
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def genie_search_async(index: Index, d_q_offsets, d_items, k: int, max_items: int,
                       out_ids=None, out_counts=None, workspace=None, stream=None):
    """Enqueue a search on a stream (device tensors); returns (ids, counts, workspace)."""
    import torch
    nq = d_q_offsets.numel() - 1
    dev = d_q_offsets.device
    if out_ids is None:
        out_ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
    if out_counts is None:
        out_counts = torch.empty((nq, k), dtype=torch.int32, device=dev)
    if workspace is None:
        workspace = alloc_workspace(index, nq, k, dev)
    if nq <= 0:
        return out_ids, out_counts, workspace
    _check(load().genie_search_async(index.handle, _dev_ptr(d_q_offsets), _dev_ptr(d_items),
                                     d_items.numel() // 3, nq, int(max_items), int(k), _dev_ptr(out_ids),
                                     _dev_ptr(out_counts), _dev_ptr(workspace),
                                     workspace.numel(), _stream_handle(stream)))
    return out_ids, out_counts, workspace


def genie_search_noalloc_async(index: Index, d_q_offsets, d_items, k: int, max_items: int,
                               out_ids, out_counts, stream=None):
    """genie_search_async with the workspace held by the library (the call
    allocates nothing; outputs are the caller's); returns (ids, counts).
    Calls that overlap on one GPU share that workspace and race."""
    nq = d_q_offsets.numel() - 1
    if nq > 0:
        _check(load().genie_search_noalloc_async(index.handle, _dev_ptr(d_q_offsets),
                                                 _dev_ptr(d_items), d_items.numel() // 3, nq,
                                                 int(max_items), int(k), _dev_ptr(out_ids),
                                                 _dev_ptr(out_counts), _stream_handle(stream)))
    return out_ids, out_counts


def genie_search_gated_async(index: Index, d_q_offsets, d_items, k: int, max_items: int,
                             d_gate, gate_delta: float, out_ids=None, out_counts=None,
                             workspace=None, stream=None):
    """Search with the AuditThreshold starting at the predicted k-th count
    (minus gate_delta); identical results to genie_search_async."""
    import torch
    nq = d_q_offsets.numel() - 1
    dev = d_q_offsets.device
    if out_ids is None:
        out_ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
    if out_counts is None:
        out_counts = torch.empty((nq, k), dtype=torch.int32, device=dev)
    if workspace is None:
        workspace = alloc_workspace(index, nq, k, dev)
    if nq <= 0:
        return out_ids, out_counts, workspace
    _check(load().genie_search_gated_async(index.handle, _dev_ptr(d_q_offsets), _dev_ptr(d_items),
                                           d_items.numel() // 3, nq, int(max_items), int(k),
                                           _dev_ptr(d_gate), float(gate_delta), _dev_ptr(out_ids),
                                           _dev_ptr(out_counts), _dev_ptr(workspace),
                                           workspace.numel(), _stream_handle(stream)))
    return out_ids, out_counts, workspace


def genie_search_spq_async(index: Index, d_q_offsets, d_items, k: int, max_items: int,
                           out_ids=None, out_counts=None, workspace=None, stream=None):
    """GEN-SPQ ablation: count every posting, then select from the exact
    counters (no Gate, no Hash Table); identical results to
    genie_search_async."""
    import torch
    nq = d_q_offsets.numel() - 1
    dev = d_q_offsets.device
    if out_ids is None:
        out_ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
    if out_counts is None:
        out_counts = torch.empty((nq, k), dtype=torch.int32, device=dev)
    if workspace is None:
        workspace = alloc_workspace(index, nq, k, dev)
    if nq <= 0:
        return out_ids, out_counts, workspace
    _check(load().genie_search_spq_async(index.handle, _dev_ptr(d_q_offsets), _dev_ptr(d_items),
                                         d_items.numel() // 3, nq, int(max_items), int(k),
                                         _dev_ptr(out_ids), _dev_ptr(out_counts),
                                         _dev_ptr(workspace), workspace.numel(),
                                         _stream_handle(stream)))
    return out_ids, out_counts, workspace


def genie_search_rows_async(index: Index, d_q_offsets, d_items, d_rows, k: int, max_items: int,
                            out_ids, out_counts, workspace, d_gate=None, gate_delta: float = 0.0,
                            stream=None):
    """Search (gated when d_gate is given) over the first d_rows[0] queries of
    a batch laid out for capacity = d_q_offsets.numel() - 1 queries; the row
    count is read on the device, so a HIP graph recorded once serves any
    batch size up to the capacity."""
    capacity = d_q_offsets.numel() - 1
    if d_rows.numel() != 1 or out_ids.shape[0] < capacity or out_counts.shape[0] < capacity:
        raise ValueError("buffers do not fit the capacity")
    _check(load().genie_search_rows_async(index.handle, _dev_ptr(d_q_offsets), _dev_ptr(d_items),
                                          d_items.numel() // 3, capacity, _dev_ptr(d_rows),
                                          int(max_items), int(k),
                                          _dev_ptr(d_gate) if d_gate is not None else None,
                                          float(gate_delta), _dev_ptr(out_ids),
                                          _dev_ptr(out_counts), _dev_ptr(workspace),
                                          workspace.numel(), _stream_handle(stream)))
    return out_ids, out_counts


def genie_gate_features_async(index: Index, d_q_offsets, d_items, k: int, out=None, stream=None):
    """Query features [nq, 64] float32 on the device."""
    import torch
    nq = d_q_offsets.numel() - 1
    if out is None:
        out = torch.empty((max(nq, 0), GATE_FEATURES), dtype=torch.float32,
                          device=d_q_offsets.device)
    if nq <= 0:
        return out
    _check(load().genie_gate_features_async(index.handle, _dev_ptr(d_q_offsets), _dev_ptr(d_items),
                                            d_items.numel() // 3, nq, int(k), _dev_ptr(out),
                                            _stream_handle(stream)))
    return out


def _weights(w):
    import torch
    if w.dtype == torch.int16 or w.dtype == torch.uint16:
        return _dev_ptr(w), None
    if w.dtype == torch.float32:
        return None, _dev_ptr(w)
    raise TypeError("weights must be bf16 bit patterns (int16) or float32")


def genie_gate_forward_async(weights, d_x, out=None, stream=None):
    import torch
    n = d_x.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=d_x.device)
    wb, wf = _weights(weights)
    _check(load().genie_gate_forward_async(wb, wf, _dev_ptr(d_x), n, _dev_ptr(out),
                                           _stream_handle(stream)))
    return out


def genie_gate_workspace_size(n: int) -> int:
    return int(load().genie_gate_workspace_size(int(n)))


def genie_gate_backward_async(weights, d_x, d_y, tau: float, grad=None, loss=None,
                              workspace=None, stream=None):
    import torch
    n = d_x.shape[0]
    dev = d_x.device
    if grad is None:
        grad = torch.empty(GATE_PARAMS, dtype=torch.float32, device=dev)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=dev)
    if workspace is None:
        workspace = torch.empty(genie_gate_workspace_size(n), dtype=torch.uint8, device=dev)
    wb, wf = _weights(weights)
    _check(load().genie_gate_backward_async(wb, wf, _dev_ptr(d_x), _dev_ptr(d_y), n, float(tau),
                                            _dev_ptr(grad), _dev_ptr(loss), _dev_ptr(workspace),
                                            workspace.numel(), _stream_handle(stream)))
    return grad, loss, workspace


def genie_gate_adam_async(master, w_bf16, grad, m, v, step: int, lr: float, beta1: float = 0.9,
                          beta2: float = 0.999, eps: float = 1e-8, stream=None):
    _check(load().genie_gate_adam_async(_dev_ptr(master),
                                        _dev_ptr(w_bf16) if w_bf16 is not None else None,
                                        _dev_ptr(grad), _dev_ptr(m), _dev_ptr(v), int(step),
                                        float(lr), float(beta1), float(beta2), float(eps),
                                        _stream_handle(stream)))


def genie_match_count_async(index: Index, d_q_offsets, d_items, max_items: int,
                            out=None, workspace=None, stream=None):
    """Full match-count vectors [nq, n] (uint32 stored in int32 tensors)."""
    import torch
    nq = d_q_offsets.numel() - 1
    dev = d_q_offsets.device
    if out is None:
        out = torch.empty((nq, index.info.n_objects), dtype=torch.int32, device=dev)
    if workspace is None:
        workspace = alloc_workspace(index, nq, 1, dev)
    if nq <= 0:
        return out, workspace
    _check(load().genie_match_count_async(index.handle, _dev_ptr(d_q_offsets),
                                          _dev_ptr(d_items), d_items.numel() // 3, nq, int(max_items), _dev_ptr(out),
                                          _dev_ptr(workspace), workspace.numel(),
                                          _stream_handle(stream)))
    return out, workspace


def genie_lsh_signatures(d_points, d_a, d_b, w: float, d_rehash, log2_buckets: int,
                         out=None, stream=None):
    """Signatures [n, m] (uint32 stored in int32) for float32 points on the device."""
    import torch
    n, dim = d_points.shape
    m = d_a.shape[0]
    if d_a.shape[1] != dim or d_b.numel() != m or d_rehash.numel() != 2 * m:
        raise ValueError("shape mismatch")
    if out is None:
        out = torch.empty((n, m), dtype=torch.int32, device=d_points.device)
    _check(load().genie_lsh_signatures(_dev_ptr(d_points), n, dim, _dev_ptr(d_a), _dev_ptr(d_b),
                                       float(w), m, _dev_ptr(d_rehash), int(log2_buckets),
                                       _dev_ptr(out), _stream_handle(stream)))
    return out


def genie_rbh_signatures(d_points, d_g, d_u, d_seeds, log2_buckets: int, out=None, stream=None):
    """RBH signatures [n, m] (uint32 stored in int32) for float32 points on
    the device (Laplacian kernel, MurmurHash3 re-hash)."""
    import torch
    n, dim = d_points.shape
    m = d_g.shape[0]
    if d_g.shape != (m, dim) or d_u.shape != (m, dim) or d_seeds.numel() != m:
        raise ValueError("shape mismatch")
    if out is None:
        out = torch.empty((n, m), dtype=torch.int32, device=d_points.device)
    _check(load().genie_rbh_signatures(_dev_ptr(d_points), n, dim, _dev_ptr(d_g), _dev_ptr(d_u),
                                       _dev_ptr(d_seeds), m, int(log2_buckets), _dev_ptr(out),
                                       _stream_handle(stream)))
    return out


def genie_probe_lds_atomics(mode: int, steps: int = 4096, n_blocks: int = 4096) -> float:
    """LDS atomic adds per second over the chip (mode 0: with return,
    conflict-free; 1: with return, random words; 2: without return, random)."""
    import torch
    sink = torch.empty(n_blocks * 1024, dtype=torch.int32, device="cuda")
    out = ctypes.c_double()
    _check(load().genie_probe_lds_atomics(int(mode), int(steps), int(n_blocks), _dev_ptr(sink),
                                          ctypes.byref(out)))
    return out.value


def genie_probe_hbm(nbytes: int = 2 << 30, reps: int = 5) -> Tuple[float, float]:
    """Streaming read and copy rates in GB/s over two device buffers of nbytes."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    rd, cp = ctypes.c_double(), ctypes.c_double()
    _check(load().genie_probe_hbm(_dev_ptr(src), _dev_ptr(dst), src.numel() * 4, int(reps),
                                  _dev_ptr(sink), ctypes.byref(rd), ctypes.byref(cp)))
    del src, dst
    return rd.value, cp.value


def genie_kernel_timing_enable(on: bool = True):
    _check(load().genie_kernel_timing_enable(1 if on else 0))


def genie_kernel_timing_read(reset: bool = True) -> dict:
    t = _KernelTimes()
    _check(load().genie_kernel_timing_read(ctypes.byref(t), 1 if reset else 0))
    return {"scan_launches": t.scan_launches, "scan_ms": t.scan_ms,
            "merge_launches": t.merge_launches, "merge_ms": t.merge_ms,
            "fallback_launches": t.fallback_launches, "fallback_ms": t.fallback_ms}


def genie_lsh_items_async(d_sig, out=None, stream=None):
    """Exact-match query items (i, sig[i], sig[i]) for signature rows; returns
    (q_offsets int64 [nq+1], items int32 [nq*m, 3]) on the device, written
    into `out` = (q_offsets, items) when given."""
    import torch
    nq, m = d_sig.shape
    if out is None:
        off = torch.empty(nq + 1, dtype=torch.int64, device=d_sig.device)
        items = torch.empty((max(nq * m, 1), 3), dtype=torch.int32, device=d_sig.device)
    else:
        off, items = out
        if off.numel() != nq + 1 or items.shape[0] < nq * m or items.shape[1] != 3:
            raise ValueError("output buffers do not fit the signatures")
    _check(load().genie_lsh_items_async(_dev_ptr(d_sig) if nq else None, nq, m, _dev_ptr(items),
                                        _dev_ptr(off), _stream_handle(stream)))
    return off, items


def workspace_stats(workspace) -> dict:
    """Status flags and counters left in a workspace by the last search."""
    head = workspace[:48].cpu().numpy()
    status = int(head[:4].view(np.uint32)[0])
    stats = head[8:40].view(np.uint64)
    return {"status": status, "postings_scanned": int(stats[0]),
            "ht_overflow_tiles": int(stats[1]), "ht_inserts": int(stats[2]),
            "gate_passes": int(stats[3]), "fallback_queries": int(head[40:44].view(np.uint32)[0])}


def queries_to_device(q_offsets: np.ndarray, items: np.ndarray, device="cuda"):
    """Copy a host query CSR to device tensors (uint64 offsets as int64)."""
    import torch
    off = torch.from_numpy(np.ascontiguousarray(q_offsets, dtype=np.uint64).view(np.int64))
    items = np.ascontiguousarray(items, dtype=np.uint32).reshape(-1, 3)
    if items.shape[0] == 0:
        items = np.zeros((1, 3), dtype=np.uint32)   # never read; keeps the pointer valid
    it = torch.from_numpy(items.view(np.int32))
    return off.to(device), it.to(device)


def as_uint32(t) -> np.ndarray:
    """A device int32 tensor holding uint32 values, as a host uint32 array."""
    return t.cpu().numpy().view(np.uint32)
