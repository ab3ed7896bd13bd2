"""ctypes binding of liblc.so (include/lc.h): argument marshalling only.

Every computation runs in the HIP library; this module converts arguments
(torch device tensors -> device pointers, numpy arrays -> host pointers,
torch streams -> hipStream_t) and turns status codes into exceptions.
The library must be built (``python -m paper_2205_11852_amd.build``); there is
no fallback path: a missing library raises ``LcLibraryMissing``.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblc.so")

LC_OK, LC_ERR_INVALID, LC_ERR_RANGE, LC_ERR_OVERFLOW, LC_ERR_HIP, LC_ERR_NOMEM = 0, -1, -2, -3, -4, -5
LC_LOS_Z, LC_LOS_MID, LC_LOS_RPPI = 0, 1, 2
LC_PERSISTENT, LC_PER_TASK, LC_GRAPH, LC_FORCE_EXACT = 0, 1, 2, 4
LC_QUEUE_XCD_RANGES, LC_QUEUE_XCD_DEALT, LC_QUEUE_SHARED = 0, 1, 2
LC_FP64, LC_FP32_MFMA, LC_FP32_MFMA_CHECKED, LC_ACC32 = 0, 1, 2, 8
LC_MAX_BINS, LC_MAX_NMU = 32768, 1024
LC_NOALLOC_PLAN_BYTES = 1 << 20

STATUS_NAMES = {0: "LC_OK", -1: "LC_ERR_INVALID", -2: "LC_ERR_RANGE", -3: "LC_ERR_OVERFLOW",
                -4: "LC_ERR_HIP", -5: "LC_ERR_NOMEM"}

# the exported symbols of include/lc.h
EXPORTS = ["lc_last_error", "lc_build_cells", "lc_free_cells", "lc_cells_get_info",
           "lc_pair_count_batch", "lc_pair_count_batch_noalloc", "lc_xi_multipoles", "lc_covariance", "lc_xi_split", "lc_sample_covariance", "lc_covcov",
           "lc_autotune", "lc_covariance_general", "lc_rebin_counts", "lc_map_vectors", "lc_map_matrix",
           "lc_map_multipoles", "lc_map_projected", "lc_map_rebin_blocks",
           "lc_release_caches"]


class LcLibraryMissing(RuntimeError):
    pass


class LcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class lc_binning(ctypes.Structure):
    _fields_ = [("periodic", ctypes.c_int32), ("box_units", ctypes.c_int32), ("los", ctypes.c_int32),
                ("n_r", ctypes.c_int32), ("r_edges", ctypes.POINTER(ctypes.c_int32)),
                ("n_mu", ctypes.c_int32), ("pi_max", ctypes.c_int32)]


class lc_task(ctypes.Structure):
    _fields_ = [("cat_a", ctypes.c_int32), ("cat_b", ctypes.c_int32)]


class lc_tuning(ctypes.Structure):
    _fields_ = [("cells_per_item", ctypes.c_int32), ("waves_per_block", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("flush_limit", ctypes.c_int32), ("queue_order", ctypes.c_int32),
                ("hist_bits", ctypes.c_int32), ("wrap_test", ctypes.c_int32)]


class lc_mesh_opts(ctypes.Structure):
    _fields_ = [("cell_units", ctypes.c_int32), ("sub", ctypes.c_int32),
                ("arrival_order", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class lc_cells_info(ctypes.Structure):
    _fields_ = [("n_cat", ctypes.c_int32), ("grid", ctypes.c_int32 * 3),
                ("cell_side", ctypes.c_double * 3), ("sub", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("n_total", ctypes.c_int64),
                ("bytes", ctypes.c_int64)]


class lc_autotune_result(ctypes.Structure):
    _fields_ = [("cell_units", ctypes.c_int32), ("sub", ctypes.c_int32), ("tune", lc_tuning),
                ("sample_ms", ctypes.c_double), ("n_tried", ctypes.c_int32), ("sample_tasks", ctypes.c_int32),
                ("cached", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        t = self.tune
        return {"cell_units": self.cell_units, "sub": self.sub,
                "tune": {"cells_per_item": t.cells_per_item, "waves_per_block": t.waves_per_block,
                         "blocks_per_cu": t.blocks_per_cu, "chunk": t.chunk, "queue_order": t.queue_order},
                "sample_ms": self.sample_ms, "n_tried": self.n_tried, "sample_tasks": self.sample_tasks,
                "cached": bool(self.cached)}


class lc_covcov_report(ctypes.Structure):
    _fields_ = [("chi2_2_lc", ctypes.c_double), ("chi2_2_smp", ctypes.c_double), ("cost_lc", ctypes.c_double),
                ("cost_smp", ctypes.c_double), ("ifom_lc", ctypes.c_double), ("ifom_smp", ctypes.c_double),
                ("gain", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class lc_cov_report(ctypes.Structure):
    _fields_ = [("chol_ok", ctypes.c_int32 * 2), ("n_neg_eig", ctypes.c_int32 * 2),
                ("min_eig", ctypes.c_double * 2), ("max_eig", ctypes.c_double * 2),
                ("rel_frob_vs_fp64", ctypes.c_double * 3)]

    def as_dict(self):
        return {"chol_ok": list(self.chol_ok), "n_neg_eig": list(self.n_neg_eig),
                "min_eig": list(self.min_eig), "max_eig": list(self.max_eig),
                "rel_frob_vs_fp64": list(self.rel_frob_vs_fp64)}


_lib = None


def lib():
    """Load liblc.so (raises LcLibraryMissing if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LcLibraryMissing("%s is not built; run python -m paper_2205_11852_amd.build" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, st = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32
    L.lc_last_error.restype = ctypes.c_char_p
    L.lc_last_error.argtypes = []
    L.lc_build_cells.restype = st
    L.lc_build_cells.argtypes = [vp, i64, vp, i32, ctypes.POINTER(lc_binning),
                                 ctypes.POINTER(lc_mesh_opts), vp, ctypes.POINTER(vp)]
    L.lc_free_cells.restype = None
    L.lc_free_cells.argtypes = [vp]
    L.lc_cells_get_info.restype = st
    L.lc_cells_get_info.argtypes = [vp, ctypes.POINTER(lc_cells_info)]
    L.lc_pair_count_batch.restype = st
    L.lc_pair_count_batch.argtypes = [vp, vp, i32, ctypes.POINTER(lc_binning), vp, i32,
                                      ctypes.POINTER(lc_tuning), vp, vp]
    L.lc_map_multipoles.restype = st
    L.lc_map_multipoles.argtypes = [i32, i32, i32, i32, i32, i32, vp, vp, vp]
    L.lc_map_projected.restype = st
    L.lc_map_projected.argtypes = [i32, i32, ctypes.c_double, vp, vp, vp]
    L.lc_map_rebin_blocks.restype = st
    L.lc_map_rebin_blocks.argtypes = [i32, i32, i32, vp, vp, vp]
    L.lc_pair_count_batch_noalloc.restype = st
    L.lc_pair_count_batch_noalloc.argtypes = [vp, vp, i32, ctypes.POINTER(lc_binning), vp, i32,
                                              ctypes.POINTER(lc_tuning), vp, vp]
    L.lc_xi_multipoles.restype = st
    L.lc_xi_multipoles.argtypes = [vp, vp, i32, vp, i32, vp, i32, i32, i32, vp, vp]
    L.lc_covariance.restype = st
    L.lc_covariance.argtypes = [vp, i32, i32, i32, i32, ctypes.c_double, i32, vp, vp, vp,
                                ctypes.POINTER(lc_cov_report), vp]
    L.lc_xi_split.restype = st
    L.lc_xi_split.argtypes = [vp, vp, i32, vp, i32, vp, i32, i32, i32, i32, vp, i64, vp]
    dbl = ctypes.c_double
    L.lc_covariance_general.restype = st
    L.lc_covariance_general.argtypes = [vp, i32, i32, i32, dbl, dbl, dbl, i32, vp, vp, vp,
                                        ctypes.POINTER(lc_cov_report), vp]
    L.lc_rebin_counts.restype = st
    L.lc_rebin_counts.argtypes = [vp, i32, i32, i32, i32, i32, vp, vp]
    L.lc_map_vectors.restype = st
    L.lc_map_vectors.argtypes = [vp, i64, i32, i64, vp, vp, i32, vp, i64, vp]
    L.lc_map_matrix.restype = st
    L.lc_map_matrix.argtypes = [vp, i32, vp, vp, i32, vp, vp]
    L.lc_sample_covariance.restype = st
    L.lc_sample_covariance.argtypes = [vp, i32, i32, i32, vp, vp]
    L.lc_covcov.restype = st
    L.lc_covcov.argtypes = [vp, vp, i32, i32, ctypes.c_double, vp, i32, vp, vp, ctypes.POINTER(lc_covcov_report),
                            vp]
    L.lc_autotune.restype = st
    L.lc_autotune.argtypes = [vp, i64, vp, i32, ctypes.POINTER(lc_binning), vp, i32, i32, vp,
                              ctypes.POINTER(lc_autotune_result)]
    L.lc_release_caches.restype = None
    L.lc_release_caches.argtypes = []
    _lib = L
    return L


def last_error() -> str:
    return lib().lc_last_error().decode()


def _check(status: int):
    if status != LC_OK:
        raise LcError(status, last_error())


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------

def _dptr(t) -> Optional[int]:
    """Device pointer of a torch tensor (or None / a raw int)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return int(t.data_ptr())


def _need(t, n_elems: int, name: str):
    """Refuse a torch tensor smaller than the n_elems 8-byte values (float64
    or uint64) the call reads or writes through it; raw pointers and None
    are passed through."""
    if t is None or isinstance(t, int):
        return
    if not t.is_contiguous() or t.numel() * t.element_size() < int(n_elems) * 8:
        raise ValueError("%s must be a contiguous tensor of at least %d 8-byte values (got %s, %s)"
                         % (name, int(n_elems), tuple(t.shape), t.dtype))


def _rows(n: int, ld: int, width: int) -> int:
    """Values spanned by n rows of `width` values at stride ld (0: width)."""
    return 0 if int(n) <= 0 else (int(n) - 1) * (int(ld) or int(width)) + int(width)


def _stream(stream) -> Optional[int]:
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return int(torch.cuda.current_stream().cuda_stream)
        except Exception:
            pass
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


class Binning:
    """Owns the host edge array that lc_binning points at."""

    def __init__(self, r_edges: Sequence[int], n_mu: int, periodic: bool, box_units: int = 0,
                 los: int = LC_LOS_Z, pi_max: int = 0):
        """los = LC_LOS_RPPI: r_edges bin r_p and n_mu counts the pi bins of
        [0, pi_max)."""
        self.edges = np.ascontiguousarray(np.asarray(r_edges, dtype=np.int32))
        self.n_r = len(self.edges) - 1
        self.n_mu = int(n_mu)
        self.pi_max = int(pi_max)
        self.c = lc_binning(int(bool(periodic)), int(box_units), int(los), int(self.n_r),
                            self.edges.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(n_mu),
                            int(pi_max))

    @property
    def P(self) -> int:
        return self.n_r * self.n_mu + 3 * self.n_r

    @classmethod
    def from_workload(cls, wl) -> "Binning":
        los = {"z": LC_LOS_Z, "mid": LC_LOS_MID, "rppi": LC_LOS_RPPI}[wl.los]
        return cls(wl.r_edges_units, wl.n_mu, wl.periodic, wl.box_units, los, wl.pi_max_units)


def tasks_array(tasks) -> np.ndarray:
    t = np.ascontiguousarray(np.asarray(tasks, dtype=np.int32).reshape(-1, 2))
    return t


# ---------------------------------------------------------------------------
# C-ABI calls
# ---------------------------------------------------------------------------

class Cells:
    """lc_cells handle; freed on close() / garbage collection."""

    def __init__(self, handle: int):
        self.handle = handle

    def info(self) -> dict:
        inf = lc_cells_info()
        _check(lib().lc_cells_get_info(self.handle, ctypes.byref(inf)))
        return {"n_cat": inf.n_cat, "grid": list(inf.grid), "cell_side": list(inf.cell_side),
                "sub": inf.sub, "n_total": inf.n_total, "bytes": inf.bytes}

    def close(self):
        if self.handle:
            lib().lc_free_cells(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lc_build_cells(xyz, cat_offsets, binning: Binning, cell_units: int = 0, sub: int = 0,
                   stream=None, arrival_order: bool = False) -> Cells:
    """xyz: int32 device tensor [3, n_total]; cat_offsets: int64 [n_cat+1];
    cell_units / sub / arrival_order: mesh options (0 = library defaults)."""
    off = np.ascontiguousarray(np.asarray(cat_offsets, dtype=np.int64))
    n_total = int(off[-1]) if len(off) else 0
    if xyz is not None and not isinstance(xyz, int):
        if tuple(xyz.shape) != (3, n_total) or str(xyz.dtype) != "torch.int32" or not xyz.is_contiguous():
            raise ValueError("xyz must be a contiguous int32 tensor of shape (3, %d)" % n_total)
    out = ctypes.c_void_p()
    opts = lc_mesh_opts(int(cell_units), int(sub), int(arrival_order))
    _check(lib().lc_build_cells(_dptr(xyz), n_total, off.ctypes.data, len(off) - 1,
                                ctypes.byref(binning.c), ctypes.byref(opts), _stream(stream),
                                ctypes.byref(out)))
    return Cells(out.value)


def _pair_count_args(cells, tasks, binning, counts, tune):
    t = tasks_array(tasks)
    if counts is not None and not isinstance(counts, int):
        if counts.numel() != len(t) * binning.n_r * binning.n_mu or counts.element_size() != 8:
            raise ValueError("counts must hold n_tasks * n_r * n_mu 64-bit integers")
    tn = None
    if tune:
        tn = lc_tuning(int(tune.get("cells_per_item", 0)), int(tune.get("waves_per_block", 0)),
                       int(tune.get("blocks_per_cu", 0)), int(tune.get("chunk", 0)),
                       int(tune.get("flush_limit", 0)), int(tune.get("queue_order", 0)),
                       int(tune.get("hist_bits", 0)), int(tune.get("wrap_test", 0)))
    return t, tn


def lc_pair_count_batch(cells: Cells, tasks, binning: Binning, counts, mode: int = LC_PERSISTENT,
                        tune: Optional[dict] = None, stats=None, stream=None):
    """counts: uint64-as-int64 device tensor [n_tasks, n_r, n_mu], added into."""
    t, tn = _pair_count_args(cells, tasks, binning, counts, tune)
    _check(lib().lc_pair_count_batch(cells.handle if cells else None, t.ctypes.data, len(t),
                                     ctypes.byref(binning.c), _dptr(counts), int(mode),
                                     ctypes.byref(tn) if tn is not None else None, _dptr(stats),
                                     _stream(stream)))


def lc_pair_count_batch_noalloc(cells: Cells, tasks, binning: Binning, counts, mode: int = LC_PERSISTENT,
                                tune: Optional[dict] = None, stats=None, stream=None):
    """As lc_pair_count_batch, through the entry point that allocates no
    device memory (its plan lives in the library's static device array)."""
    t, tn = _pair_count_args(cells, tasks, binning, counts, tune)
    _check(lib().lc_pair_count_batch_noalloc(cells.handle if cells else None, t.ctypes.data, len(t),
                                             ctypes.byref(binning.c), _dptr(counts), int(mode),
                                             ctypes.byref(tn) if tn is not None else None, _dptr(stats),
                                             _stream(stream)))


def lc_xi_multipoles(counts, tasks, cat_sizes, est, n_r: int, n_mu: int, xi, stream=None):
    t = tasks_array(tasks)
    sz = np.ascontiguousarray(np.asarray(cat_sizes, dtype=np.int64))
    e = np.ascontiguousarray(np.asarray(est, dtype=np.int32).reshape(-1, 5))
    _need(counts, len(t) * int(n_r) * int(n_mu), "counts")
    _need(xi, len(e) * 3 * (int(n_r) * int(n_mu) + 3 * int(n_r)), "xi")
    _check(lib().lc_xi_multipoles(_dptr(counts), t.ctypes.data, len(t), sz.ctypes.data, len(sz),
                                  e.ctypes.data, len(e), int(n_r), int(n_mu), _dptr(xi),
                                  _stream(stream)))


def lc_covariance(xi, n_mock: int, n_r: int, n_mu: int, m_a: int, M: float, precision: int,
                  A, B, C, report: bool = True, stream=None) -> Optional[dict]:
    P = int(n_r) * int(n_mu) + 3 * int(n_r)
    _need(xi, int(n_mock) * 3 * P, "xi")
    for name, t in (("A", A), ("B", B), ("C", C)):
        _need(t, P * P, name)
    rep = lc_cov_report() if report else None
    _check(lib().lc_covariance(_dptr(xi), int(n_mock), int(n_r), int(n_mu), int(m_a), float(M),
                               int(precision), _dptr(A), _dptr(B), _dptr(C),
                               ctypes.byref(rep) if rep is not None else None, _stream(stream)))
    return rep.as_dict() if rep is not None else None


def lc_xi_split(counts, tasks, cat_sizes, est, n_sub: int, n_r: int, n_mu: int, xi, stream=None,
                ld_xi: int = 0, offset: int = 0):
    """est: [n_mock][1 + 2 n_sub] task ids (DD, DR_1..DR_M, RR_1..RR_M);
    xi: float64 device tensor; row n written at element offset + n ld_xi
    (ld_xi = 0: rows of P back to back)."""
    t = tasks_array(tasks)
    sz = np.ascontiguousarray(np.asarray(cat_sizes, dtype=np.int64))
    e = np.ascontiguousarray(np.asarray(est, dtype=np.int32).reshape(-1, 1 + 2 * int(n_sub)))
    _need(counts, len(t) * int(n_r) * int(n_mu), "counts")
    _need(xi, int(offset) + _rows(len(e), ld_xi, int(n_r) * int(n_mu) + 3 * int(n_r)), "xi")
    _check(lib().lc_xi_split(_dptr(counts), t.ctypes.data, len(t), sz.ctypes.data, len(sz), e.ctypes.data,
                             int(n_sub), len(e), int(n_r), int(n_mu), _dptr(xi) + 8 * int(offset), int(ld_xi),
                             _stream(stream)))


def lc_covariance_general(xi, n_mock: int, P: int, n_split: int, m_a: float, m_b: float, M: float,
                          precision: int, A, B, C, report: bool = True, stream=None) -> Optional[dict]:
    _need(xi, int(n_mock) * 3 * int(P), "xi")
    for name, t in (("A", A), ("B", B), ("C", C)):
        _need(t, int(P) * int(P), name)
    rep = lc_cov_report() if report else None
    _check(lib().lc_covariance_general(_dptr(xi), int(n_mock), int(P), int(n_split), float(m_a), float(m_b),
                                       float(M), int(precision), _dptr(A), _dptr(B), _dptr(C),
                                       ctypes.byref(rep) if rep is not None else None, _stream(stream)))
    return rep.as_dict() if rep is not None else None


def lc_rebin_counts(counts, n_tasks: int, n_r: int, n_mu: int, w_r: int, w_mu: int, out, stream=None):
    _need(counts, int(n_tasks) * int(n_r) * int(n_mu), "counts")
    if int(w_r) >= 1 and int(w_mu) >= 1:
        _need(out, int(n_tasks) * (-(-int(n_r) // int(w_r))) * (int(n_mu) // int(w_mu)), "out")
    _check(lib().lc_rebin_counts(_dptr(counts), int(n_tasks), int(n_r), int(n_mu), int(w_r), int(w_mu),
                                 _dptr(out), _stream(stream)))


def _map_arrays(group, weight):
    g = np.ascontiguousarray(np.asarray(group, dtype=np.int32))
    w = np.ascontiguousarray(np.asarray(weight, dtype=np.float64))
    if g.shape != w.shape or g.ndim != 1:
        raise ValueError("group and weight must be 1-D arrays of the same length")
    return g, w


def lc_map_vectors(x, n_vec: int, P_in: int, group, weight, P_out: int, y, ld_x: int = 0, ld_y: int = 0,
                   stream=None):
    g, w = _map_arrays(group, weight)
    if len(g) != P_in:
        raise ValueError("group has %d entries, P_in = %d" % (len(g), P_in))
    _need(x, _rows(n_vec, ld_x, P_in), "x")
    _need(y, _rows(n_vec, ld_y, P_out), "y")
    _check(lib().lc_map_vectors(_dptr(x), int(n_vec), int(P_in), int(ld_x), g.ctypes.data, w.ctypes.data,
                                int(P_out), _dptr(y), int(ld_y), _stream(stream)))


def lc_map_matrix(X, P_in: int, group, weight, P_out: int, Y, stream=None):
    g, w = _map_arrays(group, weight)
    if len(g) != P_in:
        raise ValueError("group has %d entries, P_in = %d" % (len(g), P_in))
    _need(X, int(P_in) * int(P_in), "X")
    _need(Y, int(P_out) * int(P_out), "Y")
    _check(lib().lc_map_matrix(_dptr(X), int(P_in), g.ctypes.data, w.ctypes.data, int(P_out), _dptr(Y),
                               _stream(stream)))


def lc_sample_covariance(x, n_mock: int, P: int, precision: int, C, stream=None):
    _need(x, int(n_mock) * int(P), "x")
    _need(C, int(P) * int(P), "C")
    _check(lib().lc_sample_covariance(_dptr(x), int(n_mock), int(P), int(precision), _dptr(C),
                                      _stream(stream)))


def lc_covcov(A, B, P: int, m_a: int, M: float, Cref=None, n_mock: int = 0, sd_lc=None, sd_smp=None,
              report: bool = True, stream=None) -> Optional[dict]:
    for name, t in (("A", A), ("B", B), ("Cref", Cref), ("sd_lc", sd_lc), ("sd_smp", sd_smp)):
        _need(t, int(P) * int(P), name)
    rep = lc_covcov_report() if report else None
    _check(lib().lc_covcov(_dptr(A), _dptr(B), int(P), int(m_a), float(M), _dptr(Cref), int(n_mock),
                           _dptr(sd_lc), _dptr(sd_smp), ctypes.byref(rep) if rep is not None else None,
                           _stream(stream)))
    return rep.as_dict() if rep is not None else None


def lc_autotune(xyz, cat_offsets, binning: Binning, tasks, sample_tasks: int = 0, stream=None) -> dict:
    """Time candidate meshes and launch shapes; returns the chosen mesh
    options (cell_units, sub) and tuning dict (blocking)."""
    off = np.ascontiguousarray(np.asarray(cat_offsets, dtype=np.int64))
    t = tasks_array(tasks)
    res = lc_autotune_result()
    _check(lib().lc_autotune(_dptr(xyz), int(off[-1]) if len(off) else 0, off.ctypes.data, len(off) - 1,
                             ctypes.byref(binning.c), t.ctypes.data, len(t), int(sample_tasks),
                             _stream(stream), ctypes.byref(res)))
    return res.as_dict()


def lc_release_caches():
    lib().lc_release_caches()


INF = math.inf


def _map_out(P_in: int):
    return np.full(P_in, -1, dtype=np.int32), np.zeros(P_in, dtype=np.float64), ctypes.c_int32(0)


def lc_map_multipoles(n_r: int, n_mu: int, w: int, r_lo: int, r_hi: int, ell_mask: int):
    """(group, weight, P_out) of the multipole selection / re-binning map."""
    g, wt, P = _map_out(int(n_r) * int(n_mu) + 3 * int(n_r))
    _check(lib().lc_map_multipoles(int(n_r), int(n_mu), int(w), int(r_lo), int(r_hi), int(ell_mask),
                                   g.ctypes.data, wt.ctypes.data, ctypes.byref(P)))
    return g, wt, int(P.value)


def lc_map_projected(n_rp: int, n_pi: int, pi_max: float):
    """(group, weight, P_out) of the map to w_p(r_p)."""
    g, wt, P = _map_out(int(n_rp) * int(n_pi) + 3 * int(n_rp))
    _check(lib().lc_map_projected(int(n_rp), int(n_pi), float(pi_max), g.ctypes.data, wt.ctypes.data,
                                  ctypes.byref(P)))
    return g, wt, int(P.value)


def lc_map_rebin_blocks(n_blocks: int, n: int, w: int):
    """(group, weight, P_out) of the within-block averaging map."""
    g, wt, P = _map_out(int(n_blocks) * int(n))
    _check(lib().lc_map_rebin_blocks(int(n_blocks), int(n), int(w), g.ctypes.data, wt.ctypes.data,
                                     ctypes.byref(P)))
    return g, wt, int(P.value)
