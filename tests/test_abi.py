"""C-ABI checks that need no GPU: the library loads, exports every symbol
declared in include/lc.h, and rejects bad arguments with the documented
status before any HIP call."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_2205_11852_amd import lc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "lc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lc_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(lc.LIB_PATH):
        from paper_2205_11852_amd import build
        build.build()
    return lc.lib()


def test_exports_match_header(L):
    declared = _header_functions()
    assert set(declared) == set(lc.EXPORTS), declared
    for name in declared:
        assert hasattr(L, name), name


def test_no_fallback_when_library_missing(monkeypatch, tmp_path):
    monkeypatch.setattr(lc, "_lib", None)
    monkeypatch.setattr(lc, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(lc.LcLibraryMissing):
        lc.lib()


def _binning(**kw):
    d = dict(r_edges=[0, 10, 20, 30], n_mu=4, periodic=True, box_units=1000, los=lc.LC_LOS_Z)
    d.update(kw)
    return lc.Binning(**d)


def _build_status(L, b, n_total=4, offsets=(0, 4), out=True, xyz=0x1000):
    off = np.array(offsets, dtype=np.int64)
    h = ctypes.c_void_p()
    return L.lc_build_cells(xyz, n_total, off.ctypes.data, len(off) - 1, ctypes.byref(b.c), None, None,
                            ctypes.byref(h) if out else None)


@pytest.mark.parametrize("kw,code", [
    (dict(r_edges=[0, 20, 10]), lc.LC_ERR_INVALID),          # not increasing
    (dict(r_edges=[-1, 10]), lc.LC_ERR_INVALID),             # negative edge
    (dict(n_mu=0), lc.LC_ERR_INVALID),
    (dict(n_mu=lc.LC_MAX_NMU + 1), lc.LC_ERR_INVALID),
    (dict(r_edges=list(range(0, 34)), n_mu=1024), lc.LC_ERR_INVALID),         # too many bins (33 x 1024)
    (dict(r_edges=[0, 10, 500]), lc.LC_ERR_RANGE),           # r_max >= box/2
    (dict(box_units=999), lc.LC_ERR_INVALID),                # odd box
    (dict(box_units=(1 << 24) + 2), lc.LC_ERR_INVALID),
    (dict(los=lc.LC_LOS_MID), lc.LC_ERR_INVALID),            # midpoint needs open geometry
    (dict(los=7, periodic=False), lc.LC_ERR_INVALID),
    (dict(periodic=False, r_edges=[0, 1 << 25]), lc.LC_ERR_RANGE),
    (dict(los=lc.LC_LOS_RPPI), lc.LC_ERR_INVALID),                          # pi_max missing
    (dict(los=lc.LC_LOS_RPPI, pi_max=1 << 24, periodic=False), lc.LC_ERR_INVALID),
    (dict(los=lc.LC_LOS_RPPI, pi_max=500), lc.LC_ERR_RANGE),                # pi_max >= box/2
    (dict(los=3), lc.LC_ERR_INVALID),
])
def test_build_cells_rejects_bad_binning(L, kw, code):
    assert _build_status(L, _binning(**kw)) == code
    assert lc.last_error()


def test_build_cells_rejects_bad_options(L):
    b = _binning()
    off = np.array([0, 4], dtype=np.int64)
    h = ctypes.c_void_p()
    for opts in (lc.lc_mesh_opts(0, 3), lc.lc_mesh_opts(-5, 0), lc.lc_mesh_opts(0, 0, 2)):
        st = L.lc_build_cells(0x1000, 4, off.ctypes.data, 1, ctypes.byref(b.c), ctypes.byref(opts), None,
                              ctypes.byref(h))
        assert st == lc.LC_ERR_INVALID


def test_build_cells_rejects_bad_layout(L):
    b = _binning()
    assert _build_status(L, b, out=False) == lc.LC_ERR_INVALID
    assert _build_status(L, b, offsets=(1, 4)) == lc.LC_ERR_INVALID         # [0] != 0
    assert _build_status(L, b, offsets=(0, 3, 2, 4)) == lc.LC_ERR_INVALID   # decreasing
    assert _build_status(L, b, n_total=5) == lc.LC_ERR_INVALID              # last != n_total
    assert _build_status(L, b, xyz=0) == lc.LC_ERR_INVALID                  # NULL points
    assert "xyz" in lc.last_error()


@pytest.mark.parametrize("los", [lc.LC_LOS_MID, lc.LC_LOS_Z])
def test_build_cells_catalogue_limit(L, los):
    """A catalogue holds fewer than 2^28 points (checked on the host before
    any device work), whatever the line of sight."""
    b = _binning(periodic=False, los=los)
    n = 1 << 28
    assert _build_status(L, b, n_total=n + 5, offsets=(0, 5, n + 5)) == lc.LC_ERR_OVERFLOW
    assert "catalogue 1" in lc.last_error()


def test_pair_count_rejects_bad_arguments(L):
    b = _binning()
    t = np.array([[0, 0]], dtype=np.int32)
    st = L.lc_pair_count_batch(None, t.ctypes.data, 1, ctypes.byref(b.c), 0x1000, 0, None, None, None)
    assert st == lc.LC_ERR_INVALID and "cells" in lc.last_error()


def test_xi_rejects_inconsistent_tasks(L):
    tasks = np.array([[0, 0], [0, 1], [0, 2], [1, 1], [2, 2]], dtype=np.int32)
    sizes = np.array([10, 10, 10], dtype=np.int64)
    good = np.array([[0, 1, 2, 3, 4]], dtype=np.int32)
    bad_order = np.array([[1, 0, 2, 3, 4]], dtype=np.int32)
    bad_id = np.array([[0, 1, 2, 3, 9]], dtype=np.int32)
    for est in (bad_order, bad_id):
        st = L.lc_xi_multipoles(0x1000, tasks.ctypes.data, 5, sizes.ctypes.data, 3, est.ctypes.data, 1,
                                3, 4, 0x2000, None)
        assert st == lc.LC_ERR_INVALID
    tiny = np.array([1, 10, 10], dtype=np.int64)
    st = L.lc_xi_multipoles(0x1000, tasks.ctypes.data, 5, tiny.ctypes.data, 3, good.ctypes.data, 1, 3, 4,
                            0x2000, None)
    assert st == lc.LC_ERR_INVALID and ">= 2" in lc.last_error()


@pytest.mark.parametrize("args,code", [
    (dict(n_mock=1), lc.LC_ERR_INVALID),
    (dict(m_a=0), lc.LC_ERR_INVALID),
    (dict(M=0.0), lc.LC_ERR_INVALID),
    (dict(M=float("nan")), lc.LC_ERR_INVALID),
    (dict(precision=3), lc.LC_ERR_INVALID),
    (dict(precision=lc.LC_FP64 | lc.LC_ACC32), lc.LC_ERR_INVALID),    # float32 accumulation needs MFMA
    (dict(precision=16 | lc.LC_FP32_MFMA), lc.LC_ERR_INVALID),
    (dict(n_mu=0), lc.LC_ERR_INVALID),
    (dict(C=0), lc.LC_ERR_INVALID),
])
def test_covariance_rejects_bad_arguments(L, args, code):
    a = dict(xi=0x1000, n_mock=10, n_r=3, n_mu=4, m_a=1, M=50.0, precision=lc.LC_FP64, A=0, B=0, C=0x2000)
    a.update(args)
    st = L.lc_covariance(a["xi"], a["n_mock"], a["n_r"], a["n_mu"], a["m_a"], a["M"], a["precision"],
                         a["A"], a["B"], a["C"], None, None)
    assert st == code


def test_last_error_is_thread_local_string(L):
    assert isinstance(lc.last_error(), str)


def test_autotune_rejects_bad_arguments(L):
    b = _binning()
    off = np.array([0, 4], dtype=np.int64)
    t = np.array([[0, 0]], dtype=np.int32)
    res = lc.lc_autotune_result()
    assert L.lc_autotune(0x1000, 4, off.ctypes.data, 1, ctypes.byref(b.c), t.ctypes.data, 1, 8, None,
                         None) == lc.LC_ERR_INVALID
    assert L.lc_autotune(0x1000, 4, off.ctypes.data, 1, ctypes.byref(b.c), t.ctypes.data, 0, 8, None,
                         ctypes.byref(res)) == lc.LC_ERR_INVALID
    assert L.lc_autotune(0x1000, 4, off.ctypes.data, 1, ctypes.byref(b.c), None, 1, 8, None,
                         ctypes.byref(res)) == lc.LC_ERR_INVALID
    assert "tasks" in lc.last_error()


def test_xi_split_and_sample_covariance_reject_bad_arguments(L):
    tasks = np.array([[0, 0], [0, 1], [1, 1]], dtype=np.int32)
    sizes = np.array([10, 10], dtype=np.int64)
    good = np.array([[0, 1, 2]], dtype=np.int32)
    assert L.lc_xi_split(0x1000, tasks.ctypes.data, 3, sizes.ctypes.data, 2, good.ctypes.data, 0, 1, 3, 4,
                         0x2000, 0, None) == lc.LC_ERR_INVALID
    swapped = np.array([[0, 2, 1]], dtype=np.int32)
    assert L.lc_xi_split(0x1000, tasks.ctypes.data, 3, sizes.ctypes.data, 2, swapped.ctypes.data, 1, 1, 3, 4,
                         0x2000, 0, None) == lc.LC_ERR_INVALID
    assert "subset" in lc.last_error()
    # a row stride shorter than the vector (P = 3*4 + 3*3 = 21)
    assert L.lc_xi_split(0x1000, tasks.ctypes.data, 3, sizes.ctypes.data, 2, good.ctypes.data, 1, 1, 3, 4,
                         0x2000, 20, None) == lc.LC_ERR_INVALID
    assert "ld_xi" in lc.last_error()
    assert L.lc_sample_covariance(0x1000, 1, 10, lc.LC_FP64, 0x2000, None) == lc.LC_ERR_INVALID
    assert L.lc_sample_covariance(0x1000, 5, 10, 7, 0x2000, None) == lc.LC_ERR_INVALID
    assert L.lc_sample_covariance(None, 5, 10, lc.LC_FP64, 0x2000, None) == lc.LC_ERR_INVALID


def test_covcov_rejects_bad_arguments(L):
    rep = lc.lc_covcov_report()
    assert L.lc_covcov(None, 0x1000, 4, 1, 50.0, None, 10, None, None, ctypes.byref(rep), None) == lc.LC_ERR_INVALID
    assert L.lc_covcov(0x1000, 0x2000, 4, 0, 50.0, None, 10, None, None, ctypes.byref(rep), None) == lc.LC_ERR_INVALID
    assert L.lc_covcov(0x1000, 0x2000, 4, 1, -1.0, None, 10, None, None, ctypes.byref(rep), None) == lc.LC_ERR_INVALID
    assert L.lc_covcov(0x1000, 0x2000, 4, 1, 50.0, None, 1, 0x3000, None, ctypes.byref(rep), None) == lc.LC_ERR_INVALID


def test_covariance_general_rejects_bad_arguments(L):
    rep = lc.lc_cov_report()
    ok = dict(xi=0x1000, n=10, P=8, split=4, ma=1.0, mb=3.0, M=50.0, prec=lc.LC_FP64)

    def call(**kw):
        a = dict(ok, **kw)
        return L.lc_covariance_general(a["xi"], a["n"], a["P"], a["split"], a["ma"], a["mb"], a["M"], a["prec"],
                                       None, None, 0x2000, ctypes.byref(rep), None)

    assert call(xi=None) == lc.LC_ERR_INVALID
    assert call(n=1) == lc.LC_ERR_INVALID
    assert call(P=0) == lc.LC_ERR_INVALID
    assert call(split=9) == lc.LC_ERR_INVALID and "n_split" in lc.last_error()
    assert call(split=-1) == lc.LC_ERR_INVALID
    assert call(mb=1.0) == lc.LC_ERR_INVALID and "m_a" in lc.last_error()
    assert call(ma=0.0) == lc.LC_ERR_INVALID
    assert call(mb=float("inf")) == lc.LC_ERR_INVALID
    assert call(M=0.0) == lc.LC_ERR_INVALID
    assert call(prec=3) == lc.LC_ERR_INVALID
    assert call(prec=lc.LC_FP64 | lc.LC_ACC32) == lc.LC_ERR_INVALID


def test_rebin_counts_rejects_bad_arguments(L):
    assert L.lc_rebin_counts(0x1000, 3, 10, 6, 0, 1, 0x2000, None) == lc.LC_ERR_INVALID
    assert L.lc_rebin_counts(0x1000, 3, 10, 6, 11, 1, 0x2000, None) == lc.LC_ERR_INVALID
    assert L.lc_rebin_counts(0x1000, 3, 10, 6, 2, 4, 0x2000, None) == lc.LC_ERR_INVALID
    assert "divide" in lc.last_error()
    assert L.lc_rebin_counts(0x1000, 3, 10, 6, 2, 3, 0x1000, None) == lc.LC_ERR_INVALID
    assert "alias" in lc.last_error()
    assert L.lc_rebin_counts(None, 3, 10, 6, 2, 3, 0x2000, None) == lc.LC_ERR_INVALID
    assert L.lc_rebin_counts(None, 0, 10, 6, 2, 3, None, None) == lc.LC_OK   # nothing to do


def test_map_calls_reject_bad_arguments(L):
    g = np.array([0, 0, 1, -1], dtype=np.int32)
    w = np.array([0.5, 0.5, 1.0, 1.0])
    assert L.lc_map_vectors(0x1000, 0, 4, 0, g.ctypes.data, w.ctypes.data, 2, 0x2000, 0, None) == lc.LC_OK
    bad = np.array([0, 2, 1, -1], dtype=np.int32)
    assert L.lc_map_vectors(0x1000, 5, 4, 0, bad.ctypes.data, w.ctypes.data, 2, 0x2000, 0, None) == lc.LC_ERR_INVALID
    assert "group[1]" in lc.last_error()
    wn = np.array([0.5, np.nan, 1.0, 1.0])
    assert L.lc_map_vectors(0x1000, 5, 4, 0, g.ctypes.data, wn.ctypes.data, 2, 0x2000, 0, None) == lc.LC_ERR_INVALID
    # a NaN weight on a dropped element is never used
    wd = np.array([0.5, 0.5, 1.0, np.nan])
    assert L.lc_map_vectors(0x1000, 0, 4, 0, g.ctypes.data, wd.ctypes.data, 2, 0x2000, 0, None) == lc.LC_OK
    assert L.lc_map_vectors(0x1000, 5, 4, 3, g.ctypes.data, w.ctypes.data, 2, 0x2000, 0, None) == lc.LC_ERR_INVALID
    assert L.lc_map_vectors(0x1000, 5, 4, 0, g.ctypes.data, w.ctypes.data, 2, 0x1000, 0, None) == lc.LC_ERR_INVALID
    assert L.lc_map_vectors(0x1000, 5, 4, 0, None, w.ctypes.data, 2, 0x2000, 0, None) == lc.LC_ERR_INVALID
    assert L.lc_map_matrix(0x1000, 4, g.ctypes.data, w.ctypes.data, 0, 0x2000, None) == lc.LC_ERR_INVALID
    assert L.lc_map_matrix(0x1000, 4, bad.ctypes.data, w.ctypes.data, 2, 0x2000, None) == lc.LC_ERR_INVALID
    assert L.lc_map_matrix(None, 4, g.ctypes.data, w.ctypes.data, 2, 0x2000, None) == lc.LC_ERR_INVALID
    assert L.lc_map_matrix(0x1000, 4, g.ctypes.data, w.ctypes.data, 2, 0x1000, None) == lc.LC_ERR_INVALID


def test_map_builders_reject_bad_arguments(L):
    g = np.zeros(64, dtype=np.int32)
    w = np.zeros(64)
    P = ctypes.c_int32(0)
    assert L.lc_map_multipoles(4, 5, 1, 0, 4, 7, g.ctypes.data, w.ctypes.data, ctypes.byref(P)) == lc.LC_OK
    assert P.value == 12
    assert L.lc_map_multipoles(4, 5, 1, 3, 2, 7, g.ctypes.data, w.ctypes.data, ctypes.byref(P)) == lc.LC_ERR_INVALID
    assert L.lc_map_multipoles(4, 5, 0, 0, 4, 7, g.ctypes.data, w.ctypes.data, ctypes.byref(P)) == lc.LC_ERR_INVALID
    assert L.lc_map_multipoles(4, 5, 1, 0, 4, 8, g.ctypes.data, w.ctypes.data, ctypes.byref(P)) == lc.LC_ERR_INVALID
    assert L.lc_map_multipoles(4, 5, 1, 0, 4, 7, None, w.ctypes.data, ctypes.byref(P)) == lc.LC_ERR_INVALID
    assert L.lc_map_projected(4, 5, 0.0, g.ctypes.data, w.ctypes.data, ctypes.byref(P)) == lc.LC_ERR_INVALID
    assert L.lc_map_projected(4, 5, float("inf"), g.ctypes.data, w.ctypes.data, ctypes.byref(P)) == lc.LC_ERR_INVALID
    assert L.lc_map_rebin_blocks(3, 0, 2, g.ctypes.data, w.ctypes.data, ctypes.byref(P)) == lc.LC_ERR_INVALID
    assert L.lc_map_rebin_blocks(3, 4, 0, g.ctypes.data, w.ctypes.data, ctypes.byref(P)) == lc.LC_ERR_INVALID


def test_binding_refuses_short_buffers():
    """The Python binding checks tensor sizes before handing raw pointers to
    the library (which cannot): an [n_mock][P] array passed where the
    [n_mock][3][P] layout is read, or a short output matrix, is an error."""
    import torch
    n_r, n_mu, n_mock = 4, 5, 10
    P = n_r * n_mu + 3 * n_r
    xi = torch.zeros((n_mock, P), dtype=torch.float64)
    C = torch.zeros((P, P), dtype=torch.float64)
    with pytest.raises(ValueError, match="xi"):
        lc.lc_covariance(xi, n_mock, n_r, n_mu, 1, 50.0, lc.LC_FP64, None, None, C, report=False)
    with pytest.raises(ValueError, match="xi"):
        lc.lc_covariance_general(xi, n_mock, P, 0, 1.0, 2.0, 50.0, lc.LC_FP64, None, None, C, report=False)
    with pytest.raises(ValueError, match="C"):
        lc.lc_sample_covariance(xi, n_mock, P, lc.LC_FP64, C[:-1])
    counts = torch.zeros((3, n_r, n_mu), dtype=torch.int64)
    with pytest.raises(ValueError, match="out"):
        lc.lc_rebin_counts(counts, 3, n_r, n_mu, 2, 1, torch.zeros((3, 1, n_mu), dtype=torch.int64))
    with pytest.raises(ValueError, match="counts"):
        lc.lc_rebin_counts(counts, 4, n_r, n_mu, 1, 1, torch.zeros((4, n_r, n_mu), dtype=torch.int64))
    g = np.zeros(P, dtype=np.int32)
    w = np.ones(P)
    with pytest.raises(ValueError, match="y"):   # rows of 2 at a stride of 3 need 3 n - 1 values
        lc.lc_map_vectors(xi, n_mock, P, g, w, 2, torch.zeros((n_mock, 2), dtype=torch.float64), ld_y=3)
    with pytest.raises(ValueError, match="Y"):
        lc.lc_map_matrix(C, P, g, w, 2, torch.zeros(3, dtype=torch.float64))
    with pytest.raises(ValueError, match="sd_lc"):
        lc.lc_covcov(C, C, P, 1, 50.0, None, n_mock, C[:1], None, report=False)
