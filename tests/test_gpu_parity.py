"""GPU path vs the CPU oracle, through the C ABI.

Counts are compared bit for bit; xi and multipoles in float64 to 1e-12
relative to the magnitude of the terms summed; covariances from the float64
path to 1e-12 and from the float32-MFMA path to 1e-5 relative Frobenius.
"""
import dataclasses
import sys

import numpy as np
import pytest

import mockgen
from tests.fixtures import edge_pairs, two_point_catalogues

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return t


@pytest.fixture(scope="module")
def lcmod(torch):
    from paper_2205_11852_amd import lc
    lc.lib()  # raises if the library is not built
    return lc


@pytest.fixture(scope="module")
def c1(torch, lcmod, oracle_mod):
    from paper_2205_11852_amd.pipeline import Pipeline
    _say("[c1] generating")
    cats = mockgen.make_catalogues(mockgen.WORKLOADS["c1"])
    pl = Pipeline(cats)
    pl.build_cells()
    pl.count()
    torch.cuda.synchronize()
    gpu = pl.counts_host().copy()
    wl = cats.wl
    _say("[c1] oracle counts for %d tasks" % len(pl.tasks))
    ref = np.zeros_like(gpu)
    for t, (a, b) in enumerate(pl.tasks):
        ref[t] = oracle_mod.count_pairs(cats.cat(a), None if a == b else cats.cat(b), wl.r_edges_units,
                                        wl.n_mu, wl.box_units, wl.los)
    return dict(pl=pl, cats=cats, gpu=gpu, ref=ref)


def test_c1_counts_bit_exact(c1):
    assert np.array_equal(c1["gpu"], c1["ref"])
    st = c1["pl"].stats_host()
    assert st["binned"] == int(c1["ref"].sum())
    assert st["candidates"] >= st["binned"]


@pytest.mark.parametrize("mode_name", ["per_task", "graph", "graph_per_task", "force_exact"])
def test_c1_modes_identical(c1, lcmod, torch, mode_name):
    pl = c1["pl"]
    mode = {"per_task": lcmod.LC_PER_TASK, "graph": lcmod.LC_GRAPH,
            "graph_per_task": lcmod.LC_GRAPH | lcmod.LC_PER_TASK,
            "force_exact": lcmod.LC_FORCE_EXACT}[mode_name]
    reps = 3 if "graph" in mode_name else 1
    for r in range(reps):
        _say("[c1] mode", mode_name, "replay", r)
        pl.count(mode)
        torch.cuda.synchronize()
        assert np.array_equal(pl.counts_host(), c1["ref"]), (mode_name, r)
    if mode_name == "force_exact":
        # every queued pair took the integer rule: the binned ones plus the few
        # that phase A's float margin let through and the rule then dropped
        st = pl.stats_host()
        assert st["binned"] <= st["exact_fallback"] <= st["binned"] * (1 + 1e-4)


def test_graph_replay_after_mesh_rebuild(c1, lcmod, torch, oracle_mod):
    """A graph captured on a mesh is dropped when the mesh is freed: a new
    mesh of the same geometry (other points, possibly at the same host
    address) replays its own launch, whose counts match the oracle."""
    pl = c1["pl"]
    wl = c1["cats"].wl
    r = np.random.default_rng(11)
    off = pl.offsets
    for rep in range(3):
        # the catalogues shifted by a random vector (mod L): other sorted
        # points and cell starts, same geometry and plan
        sh = r.integers(0, wl.box_units, size=(3, 1))
        host = ((c1["cats"].xyz.astype(np.int64) + sh) % wl.box_units).astype(np.int32)
        xyz = torch.from_numpy(host).cuda()
        cells = lcmod.lc_build_cells(xyz, off, pl.binning, 0, 0)
        counts = torch.zeros_like(pl.counts)
        lcmod.lc_pair_count_batch(cells, pl.tasks, pl.binning, counts, lcmod.LC_GRAPH, None)
        torch.cuda.synchronize()
        got = counts.cpu().numpy().view(np.uint64)
        # translation mod L leaves every count unchanged
        assert np.array_equal(got, c1["ref"]), rep
        cells.close()
        del xyz


def test_c1_per_mock_baseline_identical(c1, torch):
    pl = c1["pl"]
    pl.count_per_mock()
    torch.cuda.synchronize()
    assert np.array_equal(pl.counts_host(), c1["ref"])


@pytest.mark.parametrize("tune", [dict(cells_per_item=1), dict(cells_per_item=7, waves_per_block=1),
                                  dict(waves_per_block=8, blocks_per_cu=1), dict(waves_per_block=2),
                                  dict(chunk=4), dict(chunk=12), dict(chunk=32), dict(chunk=64),
                                  dict(chunk=20, cells_per_item=3), dict(chunk=128), dict(chunk=256),
                                  dict(waves_per_block=16), dict(waves_per_block=16, chunk=64, cells_per_item=2),
                                  dict(queue_order=1), dict(queue_order=2), dict(queue_order=2, waves_per_block=16),
                                  dict(queue_order=1, cells_per_item=3, chunk=64)])
def test_c1_tunings_identical(c1, torch, tune):
    pl = c1["pl"]
    _say("[c1] tune", tune)
    pl.count(tune=tune)
    torch.cuda.synchronize()
    assert np.array_equal(pl.counts_host(), c1["ref"])


def test_bad_tuning_is_refused(c1, lcmod, torch):
    pl = c1["pl"]
    with pytest.raises(lcmod.LcError) as ei:
        pl.count(tune=dict(queue_order=3))
    assert ei.value.status == lcmod.LC_ERR_INVALID and "queue_order" in str(ei.value)
    for bits in (8, 24, 64):
        with pytest.raises(lcmod.LcError) as ei:
            pl.count(tune=dict(hist_bits=bits))
        assert ei.value.status == lcmod.LC_ERR_INVALID and "hist_bits" in str(ei.value)


def test_c1_autotuned_counts_identical(c1, torch):
    """The autotuner's choice counts the same pairs; a second call is cached."""
    pl = c1["pl"]
    res = pl.autotune(16)
    _say("[c1] autotune", res)
    assert res["n_tried"] > 3 and not res["cached"] and res["sample_ms"] > 0
    assert pl.autotune(16)["cached"]
    pl.build_cells()
    pl.count()
    torch.cuda.synchronize()
    assert np.array_equal(pl.counts_host(), c1["ref"])
    pl.tuned = None
    pl.build_cells()


@pytest.mark.parametrize("cell_mpc,sub", [(25.0, 1), (33.0, 2), (50.0, 4), (100.0, 1), (100.0, 2),
                                          (100.0, 4), (160.0, 4), (240.0, 4)])
def test_c1_cell_sizes_identical(c1, torch, cell_mpc, sub):
    pl = c1["pl"]
    _say("[c1] cell", cell_mpc, "sub", sub)
    pl.build_cells(int(cell_mpc * mockgen.UNITS_PER_MPC), sub)
    pl.count()
    torch.cuda.synchronize()
    assert np.array_equal(pl.counts_host(), c1["ref"]), (cell_mpc, sub)
    pl.build_cells()


@pytest.mark.parametrize("cell_mpc,sub", [(0.0, 0), (50.0, 2), (240.0, 4)])
def test_mesh_order_does_not_depend_on_arrival(c1, torch, cell_mpc, sub):
    """The mesh stores each sub-cell's points in (x, y, z) order, so a mesh built from the same catalogues with every catalogue's
    points shuffled (which changes the order in which points reach their
    sub-cells) leads to the same candidate tests, not only the same counts.
    Coarse cells put hundreds of points in one sub-cell."""
    from paper_2205_11852_amd.pipeline import Pipeline
    cats = c1["cats"]
    r = np.random.default_rng(11)
    xyz = cats.xyz.copy()
    for c in range(cats.n_cat):
        a, b = cats.offsets[c], cats.offsets[c + 1]
        xyz[:, a:b] = xyz[:, a + r.permutation(b - a)]
    shuffled = dataclasses.replace(cats, xyz=np.ascontiguousarray(xyz))
    seen = []
    for cs in (cats, shuffled, cats):
        pl = Pipeline(cs)
        pl.build_cells(int(cell_mpc * mockgen.UNITS_PER_MPC), sub)
        pl.count()
        torch.cuda.synchronize()
        assert np.array_equal(pl.counts_host(), c1["ref"]), (cell_mpc, sub)
        st = pl.stats_host()
        seen.append((st["candidates"], st["binned"]))
    _say("[order] cell", cell_mpc, "sub", sub, "candidates", seen)
    assert seen[0] == seen[1] == seen[2]


def test_edge_pairs_gpu(torch, lcmod):
    """Hand-derived bins of pairs exactly on r and mu edges (tests/golden)."""
    for scale in (1, 4096, 2 ** 18 // 5):
        for row in edge_pairs():
            a, b, edges, box = two_point_catalogues(row, scale=scale)
            xyz = np.concatenate([a, b], axis=1)
            los = lcmod.LC_LOS_MID if row["los"] == "mid" else lcmod.LC_LOS_Z
            bn = lcmod.Binning(edges, row["n_mu"], box > 0, box, los)
            t = torch.from_numpy(np.ascontiguousarray(xyz)).cuda()
            cells = lcmod.lc_build_cells(t, [0, 1, 2], bn)
            counts = torch.zeros((3, bn.n_r, bn.n_mu), dtype=torch.int64, device="cuda")
            for mode in (lcmod.LC_PERSISTENT, lcmod.LC_FORCE_EXACT):
                counts.zero_()
                lcmod.lc_pair_count_batch(cells, [[0, 1], [1, 0], [0, 0]], bn, counts, mode)
                got = counts.cpu().numpy()
                exp = np.zeros((bn.n_r, bn.n_mu), dtype=np.int64)
                if row["k"] >= 0:
                    exp[row["k"], row["m"]] = 1
                assert np.array_equal(got[0], exp), (row["note"], scale, mode)
                assert np.array_equal(got[1], exp), (row["note"], scale, mode, "swapped")
                assert got[2].sum() == 0
            cells.close()


def test_xi_multipoles_parity(c1, oracle_mod, torch):
    pl = c1["pl"]
    pl.count()
    pl.xi_multipoles()
    torch.cuda.synchronize()
    xi = pl.xi.cpu().numpy()
    counts = c1["ref"]
    sizes = pl.sizes
    wl = c1["cats"].wl
    W = oracle_mod.legendre_weights(wl.n_mu)
    nb = wl.n_r * wl.n_mu
    for m in range(pl.n_mock):
        e = pl.est[m]
        D, R1, R2 = pl.tasks[e[0]][0], pl.tasks[e[1]][1], pl.tasks[e[2]][1]
        V = oracle_mod.mock_vectors(*(counts[t] for t in e), sizes[D], sizes[R1], sizes[R2])
        g = xi[m]
        nan_g, nan_r = np.isnan(g), np.isnan(V)
        assert np.array_equal(nan_g, nan_r)
        ok = ~nan_r
        # xi(r, mu): same operations in the same order
        assert np.allclose(g[:, :nb][ok[:, :nb]], V[:, :nb][ok[:, :nb]], rtol=1e-12, atol=0)
        # multipoles: tolerance relative to the sum of |W xi| entering each one
        for q in range(3):
            x2 = V[q, :nb].reshape(wl.n_r, wl.n_mu)
            scale = np.abs(x2)[:, None, :] * np.abs(W)[None, :, :]
            scale = scale.sum(axis=2).T.ravel()
            d = np.abs(g[q, nb:] - V[q, nb:])
            fin = np.isfinite(V[q, nb:])
            assert np.all(d[fin] <= 1e-12 * scale[fin] + 1e-300)


@pytest.fixture(scope="module")
def c1_cov(c1, oracle_mod, torch):
    """Oracle data vectors (from the oracle's counts) and their LC matrices.
    The covariance tests feed the same vectors to the device, so the stage is
    compared on identical inputs."""
    pl = c1["pl"]
    counts = c1["ref"]
    V = np.stack([oracle_mod.mock_vectors(*(counts[t] for t in pl.est[m]), pl.sizes[pl.tasks[pl.est[m][0]][0]],
                                          pl.sizes[pl.tasks[pl.est[m][1]][1]], pl.sizes[pl.tasks[pl.est[m][2]][1]])
                  for m in range(pl.n_mock)])
    A, B, C, Ca, Cb = oracle_mod.lc_from_vectors(V, 1, 50.0)
    return dict(xi=V, A=A, B=B, C=C)


def _load_xi(pl, V, torch):
    pl.xi.copy_(torch.from_numpy(np.ascontiguousarray(V)).to(pl.xi.device))


def _rel_frob(x, y):
    m = np.isfinite(y)
    return np.linalg.norm((x - y)[m]) / np.linalg.norm(y[m])


def test_covariance_fp64_parity(c1, c1_cov, lcmod, torch):
    pl = c1["pl"]
    _load_xi(pl, c1_cov["xi"], torch)
    for M in (50.0, 1.0, 2.0, float("inf")):
        pl.covariance(lcmod.LC_FP64, report=False, M=M)
        torch.cuda.synchronize()
        A, B, C = (t.cpu().numpy() for t in (pl.A, pl.B, pl.C))
        exp_C = c1_cov["A"] if np.isinf(M) else c1_cov["A"] + c1_cov["B"] / M
        assert np.array_equal(np.isnan(C), np.isnan(exp_C))
        assert _rel_frob(A, c1_cov["A"]) < 1e-12
        assert _rel_frob(B, c1_cov["B"]) < 1e-12
        assert _rel_frob(C, exp_C) < 1e-12, M
        assert np.array_equal(C[np.isfinite(C)], C.T[np.isfinite(C)])


def test_covariance_fp32_mfma_parity(c1, c1_cov, lcmod, torch):
    pl = c1["pl"]
    _load_xi(pl, c1_cov["xi"], torch)
    rep = pl.covariance(lcmod.LC_FP32_MFMA_CHECKED, report=True)
    torch.cuda.synchronize()
    A, B, C = (t.cpu().numpy() for t in (pl.A, pl.B, pl.C))
    assert _rel_frob(C, c1_cov["C"]) < 1e-5
    assert _rel_frob(A, c1_cov["A"]) < 1e-5
    assert _rel_frob(B, c1_cov["B"]) < 1e-5
    for q in range(3):
        assert 0 <= rep["rel_frob_vs_fp64"][q] < 1e-5, rep


def _synthetic_vectors(n_mock, P, seed):
    """Float64 data vectors with a smooth correlation structure (input to the
    covariance stage only)."""
    r = np.random.default_rng(seed)
    L = r.normal(size=(P, P)) / np.sqrt(P) + np.eye(P)
    base = r.normal(size=(n_mock, P)) @ L.T
    V = np.stack([base + 0.3 * r.normal(size=(n_mock, P)) for _ in range(3)], axis=1)
    return V


@pytest.mark.parametrize("n_mock,n_r,n_mu", [(50, 4, 5), (300, 6, 10), (1000, 10, 20), (257, 3, 41)])
def test_covariance_synthetic_parity_and_check(lcmod, oracle_mod, torch, n_mock, n_r, n_mu):
    """Covariance stage on its own, at sizes that span several tiles with a
    ragged tail, plus the Cholesky / eigenvalue report against LAPACK."""
    P = n_r * n_mu + 3 * n_r
    V = _synthetic_vectors(n_mock, P, n_mock + P)
    xi = torch.from_numpy(V).cuda()
    A, B, C = (torch.empty((P, P), dtype=torch.float64, device="cuda") for _ in range(3))
    rA, rB, rC, _, _ = oracle_mod.lc_from_vectors(V, 1, 50.0)
    for prec, tol in ((lcmod.LC_FP64, 1e-12), (lcmod.LC_FP32_MFMA, 1e-5)):
        rep = lcmod.lc_covariance(xi, n_mock, n_r, n_mu, 1, 50.0, prec, A, B, C, report=True)
        torch.cuda.synchronize()
        gA, gB, gC = (t.cpu().numpy() for t in (A, B, C))
        assert _rel_frob(gC, rC) < tol and _rel_frob(gA, rA) < tol and _rel_frob(gB, rB) < tol, prec
        # the check runs on the matrix the device produced: compare with LAPACK on it
        nb0 = n_r * n_mu
        for blk, sl in enumerate((slice(0, nb0), slice(nb0, P))):
            ref = oracle_mod.check_matrix(gC[sl, sl])
            w = np.linalg.eigvalsh(gC[sl, sl])
            scale = np.abs(w).max()
            assert abs(rep["min_eig"][blk] - ref["min_eig"]) <= 1e-10 * scale, (blk, rep, ref)
            assert abs(rep["max_eig"][blk] - ref["max_eig"]) <= 1e-10 * scale, (blk, rep, ref)
            # counts and Cholesky agree unless an eigenvalue sits at rounding level
            if np.min(np.abs(w)) > 1e-8 * scale:
                assert rep["n_neg_eig"][blk] == ref["n_neg_eig"], (blk, rep, ref)
                assert rep["chol_ok"][blk] == ref["chol_ok"], (blk, rep, ref)


def test_covariance_nan_rows(lcmod, torch):
    """rr = 0 gives NaN xi; NaN propagates to its rows and the report flags it."""
    n_mock, n_r, n_mu = 20, 2, 3
    P = n_r * n_mu + 3 * n_r
    V = _synthetic_vectors(n_mock, P, 3)
    V[:, :, 1] = np.nan
    xi = torch.from_numpy(V).cuda()
    A, B, C = (torch.empty((P, P), dtype=torch.float64, device="cuda") for _ in range(3))
    rep = lcmod.lc_covariance(xi, n_mock, n_r, n_mu, 1, 50.0, lcmod.LC_FP64, A, B, C, report=True)
    g = C.cpu().numpy()
    assert np.all(np.isnan(g[1])) and np.all(np.isnan(g[:, 1]))
    assert np.all(np.isfinite(np.delete(np.delete(g, 1, 0), 1, 1)))
    assert rep["n_neg_eig"][0] == -1 and rep["chol_ok"][0] == 0


def test_wedge_midpoint_bit_exact(torch, oracle_mod, lcmod):
    """Open geometry with the midpoint line of sight (survey-like wedge)."""
    from paper_2205_11852_amd.pipeline import Pipeline
    wl = dataclasses.replace(mockgen.WORKLOADS["c4"], n_mock=3, n_mean=6000.0, n_parents=300,
                             n_subsets=2, subset_size=6000)
    cats = mockgen.make_catalogues(wl)
    pl = Pipeline(cats)
    for cell_mpc, sub in ((0, 0), (60.0, 1), (60.0, 4), (200.0, 2)):
        _say("[wedge] cell", cell_mpc, "sub", sub)
        pl.build_cells(int(cell_mpc * mockgen.UNITS_PER_MPC), sub)
        pl.count()
        torch.cuda.synchronize()
        gpu = pl.counts_host()
        for t, (a, b) in enumerate(pl.tasks):
            ref = oracle_mod.count_pairs(cats.cat(a), None if a == b else cats.cat(b), wl.r_edges_units,
                                         wl.n_mu, 0, "mid")
            assert np.array_equal(gpu[t], ref), (cell_mpc, t)


def test_wedge_midpoint_chunks_and_exact_mode(torch, oracle_mod, lcmod):
    """Midpoint line of sight: i chunks of 4 to 256 points (queued pairs
    keep their j offsets across chunks), the integer rule alone, per-task
    launches and graph replays all give the oracle's counts."""
    from paper_2205_11852_amd.pipeline import Pipeline
    wl = dataclasses.replace(mockgen.WORKLOADS["c4"], n_mock=2, n_mean=9000.0, n_parents=300,
                             n_subsets=2, subset_size=9000)
    cats = mockgen.make_catalogues(wl)
    pl = Pipeline(cats)
    pl.build_cells(int(150.0 * mockgen.UNITS_PER_MPC), 2)
    refs = [oracle_mod.count_pairs(cats.cat(a), None if a == b else cats.cat(b), wl.r_edges_units, wl.n_mu, 0,
                                   "mid") for a, b in pl.tasks]
    runs = [(lcmod.LC_PERSISTENT, dict(chunk=256)), (lcmod.LC_PERSISTENT, dict(chunk=132, waves_per_block=16)),
            (lcmod.LC_PERSISTENT, dict(chunk=4)), (lcmod.LC_PERSISTENT | lcmod.LC_FORCE_EXACT, None),
            (lcmod.LC_PER_TASK, dict(chunk=256)), (lcmod.LC_GRAPH, None), (lcmod.LC_GRAPH, None),
            (lcmod.LC_GRAPH | lcmod.LC_PER_TASK, None)]
    for mode, tune in runs:
        _say("[wedge] mode", mode, "tune", tune)
        pl.count(mode, tune)
        torch.cuda.synchronize()
        gpu = pl.counts_host()
        for t in range(len(pl.tasks)):
            assert np.array_equal(gpu[t], refs[t]), (mode, tune, t)
        st = pl.stats_host()
        if mode & lcmod.LC_FORCE_EXACT:
            # every pair phase A accepts takes the integer rule
            assert st["exact_fallback"] >= st["binned"] > 0


def test_midpoint_count_on_a_plane_parallel_mesh(torch, lcmod, oracle_mod):
    """A mesh built for the plane-parallel binning of the same geometry and
    reach also serves the midpoint binning (absolute coordinates come back
    from the cell origins): counts bit-exact against the oracle."""
    r = np.random.default_rng(5)
    xyz = r.integers(-3000000, 3000000, size=(3, 1500)).astype(np.int32)
    xyz[2] += 6000000
    off = np.array([0, 900, 1500], dtype=np.int64)
    edges = [0, 100000, 250000, 400000]
    bz = lcmod.Binning(edges, 7, False, 0, lcmod.LC_LOS_Z)
    bm = lcmod.Binning(edges, 7, False, 0, lcmod.LC_LOS_MID)
    cells = lcmod.lc_build_cells(torch.from_numpy(xyz).cuda(), off, bz, 0, 0)
    tasks = [(0, 0), (0, 1), (1, 1)]
    counts = torch.zeros((3, 3, 7), dtype=torch.int64, device="cuda")
    lcmod.lc_pair_count_batch(cells, tasks, bm, counts, lcmod.LC_PERSISTENT, None)
    torch.cuda.synchronize()
    got = counts.cpu().numpy()
    cats = [np.ascontiguousarray(xyz[:, 0:900]), np.ascontiguousarray(xyz[:, 900:1500])]
    for t, (a, b) in enumerate(tasks):
        ref = oracle_mod.count_pairs(cats[a], None if a == b else cats[b], edges, 7, 0, "mid")
        assert np.array_equal(got[t], ref), t
    cells.close()


def test_slab_open_geometry_bit_exact(torch, oracle_mod, lcmod):
    """The paper's slab shape (open 1500 x 1500 x 300 Mpc/h, z line of sight,
    200 x 100 bins: an 80 KB block histogram) at a density the oracle counts
    fully, on the default and the autotuned mesh."""
    from paper_2205_11852_amd.pipeline import Pipeline
    wl = dataclasses.replace(mockgen.WORKLOADS["slab"], n_mock=2, n_mean=6000.0, n_parents=7500)
    cats = mockgen.make_catalogues(wl)
    pl = Pipeline(cats)
    refs = {}
    for tuned in (False, True):
        if tuned:
            pl.autotune(8)
        pl.build_cells()
        _say("[slab] grid", pl.cells.info()["grid"], "tuned", tuned)
        pl.count()
        torch.cuda.synchronize()
        gpu = pl.counts_host()
        for t, (a, b) in enumerate(pl.tasks):
            if t not in refs:
                refs[t] = oracle_mod.count_pairs(cats.cat(a), None if a == b else cats.cat(b),
                                                 wl.r_edges_units, wl.n_mu, 0, "z")
            assert np.array_equal(gpu[t], refs[t]), (tuned, t)


def test_ragged_catalogues(torch, oracle_mod, lcmod):
    """Empty and one-point catalogues, coincident points, points on the box
    faces, everything in one cell, non-uniform edges with e_0 > 0; arrival
    and fixed mesh order."""
    L = 1 << 16
    r = np.random.default_rng(5)
    cats = [np.zeros((3, 0), np.int32), np.array([[5], [6], [7]], np.int32),
            np.repeat(np.array([[100], [200], [300]], np.int32), 5, axis=1),       # coincident
            np.array([[0, L - 1, 0, L - 1], [0, 0, L - 1, L - 1], [L - 1, 0, 0, L - 1]], np.int32),
            r.integers(1000, 1300, size=(3, 300)).astype(np.int32),                 # one cell
            r.integers(0, L, size=(3, 700)).astype(np.int32)]
    off = np.cumsum([0] + [c.shape[1] for c in cats])
    xyz = torch.from_numpy(np.ascontiguousarray(np.concatenate(cats, axis=1))).cuda()
    tasks = [(a, b) for a in range(len(cats)) for b in range(len(cats))]
    for edges in ([0, 100, 900, 2000, 3000, 6000], [40, 50, 64, 1000, 1001, 4321, 9000]):
        for n_mu in (1, 3, 10):
            bn = lcmod.Binning(edges, n_mu, True, L, lcmod.LC_LOS_Z)
            cells = lcmod.lc_build_cells(xyz, off, bn, sub=(1, 2, 4)[n_mu % 3], arrival_order=n_mu == 1)
            counts = torch.zeros((len(tasks), bn.n_r, n_mu), dtype=torch.int64, device="cuda")
            lcmod.lc_pair_count_batch(cells, tasks, bn, counts)
            got = counts.cpu().numpy().view(np.uint64)
            for t, (a, b) in enumerate(tasks):
                ref = oracle_mod.count_pairs(cats[a], None if a == b else cats[b], edges, n_mu, L, "z")
                assert np.array_equal(got[t], ref), (edges, n_mu, a, b)
            cells.close()


def test_maximum_bins_bit_exact(torch, lcmod, oracle_mod):
    """The largest histogram the library takes: 32 x 1024 = LC_MAX_BINS bins
    (128 KB of LDS, room for one 4-wave block per CU), plane-parallel and
    (r_p, pi), every task against the oracle; one bin more is refused."""
    cats = mockgen.make_catalogues(mockgen.WORKLOADS["c1"], 2)
    L = cats.wl.box_units
    xyz = torch.from_numpy(cats.xyz).cuda()
    tasks = [(0, 0), (0, 2), (1, 3), (2, 2)]
    edges = list(range(0, 33 * 3 * mockgen.UNITS_PER_MPC, 3 * mockgen.UNITS_PER_MPC))
    assert (len(edges) - 1) * 1024 == lcmod.LC_MAX_BINS
    for los, pi_max, name in ((lcmod.LC_LOS_Z, 0, "z"), (lcmod.LC_LOS_RPPI, 40 * mockgen.UNITS_PER_MPC, "rppi")):
        bn = lcmod.Binning(edges, 1024, True, L, los, pi_max)
        cells = lcmod.lc_build_cells(xyz, cats.offsets, bn)
        counts = torch.zeros((len(tasks), bn.n_r, 1024), dtype=torch.int64, device="cuda")
        lcmod.lc_pair_count_batch(cells, tasks, bn, counts)
        got = counts.cpu().numpy().view(np.uint64)
        for t, (a, b) in enumerate(tasks):
            ref = oracle_mod.count_pairs(cats.cat(a), None if a == b else cats.cat(b), edges, 1024, L, name,
                                         pi_max=pi_max)
            assert np.array_equal(got[t], ref), (name, t)
        cells.close()
    with pytest.raises(lcmod.LcError):
        lcmod.lc_build_cells(xyz, cats.offsets, lcmod.Binning(edges + [edges[-1] + 1], 1024, True, L))


@pytest.mark.parametrize("case", ["c1", "wedge", "max_bins"])
def test_overflow_guard_bit_exact(torch, lcmod, oracle_mod, case):
    """The overflow guard (a wave that has registered its share of the 2^32
    bound on a uint32 bin moves the live block histogram out with atomic
    exchanges while the block's other waves keep adding to it), forced by a
    small flush_limit, with 4- and 16-wave blocks and per-task launches:
    counts bit-exact against the oracle, and the guard taken many times
    (stats[1], apart from the block flushes in stats[3])."""
    from paper_2205_11852_amd.pipeline import Pipeline
    if case == "c1":
        cats = mockgen.make_catalogues(mockgen.WORKLOADS["c1"], 6)
        wl = cats.wl
        edges, n_mu, box, los = wl.r_edges_units, wl.n_mu, wl.box_units, "z"
        bn = None
    elif case == "wedge":
        wl = dataclasses.replace(mockgen.WORKLOADS["c4"], n_mock=2, n_mean=6000.0, n_parents=300,
                                 n_subsets=2, subset_size=6000)
        cats = mockgen.make_catalogues(wl)
        edges, n_mu, box, los = wl.r_edges_units, wl.n_mu, 0, "mid"
        bn = None
    else:
        cats = mockgen.make_catalogues(mockgen.WORKLOADS["c1"], 2)
        box = cats.wl.box_units
        edges = list(range(0, 33 * 3 * mockgen.UNITS_PER_MPC, 3 * mockgen.UNITS_PER_MPC))
        n_mu, los = 1024, "z"
        bn = lcmod.Binning(edges, n_mu, True, box, lcmod.LC_LOS_Z)
    pl = Pipeline(cats)
    if bn is not None:
        pl.binning = bn
        pl.counts = torch.zeros((len(pl.tasks), bn.n_r, n_mu), dtype=torch.int64, device="cuda")
    pl.build_cells()
    refs = [oracle_mod.count_pairs(cats.cat(a), None if a == b else cats.cat(b), edges, n_mu, box, los)
            for a, b in pl.tasks]
    runs = [(lcmod.LC_PERSISTENT, dict(flush_limit=3000)),
            (lcmod.LC_PERSISTENT, dict(flush_limit=1000, waves_per_block=16)),
            (lcmod.LC_PER_TASK, dict(flush_limit=1500))]
    if case != "max_bins":
        # a flush after every gathered j block (the 32768-bin histogram would
        # make this slow)
        runs.append((lcmod.LC_PERSISTENT, dict(flush_limit=1, waves_per_block=4, chunk=64)))
    for mode, tune in runs:
        _say("[guard]", case, "mode", mode, "tune", tune)
        pl.count(mode, tune)
        torch.cuda.synchronize()
        gpu = pl.counts_host()
        for t in range(len(pl.tasks)):
            assert np.array_equal(gpu[t], refs[t]), (case, mode, tune, t)
        st = pl.stats_host()
        _say("[guard]", case, st)
        assert st["guard_flushes"] > 100, st
        assert st["flushes"] > 0
    # the default limit never takes the guard on these workloads
    pl.count()
    torch.cuda.synchronize()
    assert pl.stats_host()["guard_flushes"] == 0


@pytest.mark.parametrize("case", ["c1", "wedge", "rppi"])
def test_sixteen_bit_bins_bit_exact(torch, lcmod, oracle_mod, case):
    """The packed 16-bit histogram (two bins per LDS word, each wrap from
    65535 to 0 corrected in the counts by the add that caused it), forced on
    small workloads, with bins started 16 below their wrap (wrap_test) so
    that wraps, carries from a low bin into its high neighbour and carries
    that wrap the high bin happen all the time: counts bit-exact against the
    oracle for 4-, 12- and 16-wave blocks, per-task launches and the
    integer-rule-only mode."""
    from paper_2205_11852_amd.pipeline import Pipeline
    if case == "c1":
        cats = mockgen.make_catalogues(mockgen.WORKLOADS["c1"], 6)
        wl = cats.wl
        edges, n_mu, box, los, pi_max = wl.r_edges_units, wl.n_mu, wl.box_units, "z", 0
        bn = None
    elif case == "wedge":
        wl = dataclasses.replace(mockgen.WORKLOADS["c4"], n_mock=2, n_mean=6000.0, n_parents=300,
                                 n_subsets=2, subset_size=6000)
        cats = mockgen.make_catalogues(wl)
        edges, n_mu, box, los, pi_max = wl.r_edges_units, wl.n_mu, 0, "mid", 0
        bn = None
    else:
        cats = mockgen.make_catalogues(mockgen.WORKLOADS["c1"], 3)
        box = cats.wl.box_units
        edges = list(range(0, 13 * 5 * mockgen.UNITS_PER_MPC, 5 * mockgen.UNITS_PER_MPC))
        n_mu, los, pi_max = 7, "rppi", 37 * mockgen.UNITS_PER_MPC
        bn = lcmod.Binning(edges, n_mu, True, box, lcmod.LC_LOS_RPPI, pi_max)
    pl = Pipeline(cats)
    if bn is not None:
        pl.binning = bn
        pl.counts = torch.zeros((len(pl.tasks), bn.n_r, n_mu), dtype=torch.int64, device="cuda")
    pl.build_cells()
    refs = [oracle_mod.count_pairs(cats.cat(a), None if a == b else cats.cat(b), edges, n_mu, box, los,
                                   pi_max=pi_max) for a, b in pl.tasks]
    runs = [(lcmod.LC_PERSISTENT, dict(hist_bits=16)),
            (lcmod.LC_PERSISTENT, dict(hist_bits=16, wrap_test=1)),
            (lcmod.LC_PERSISTENT, dict(hist_bits=16, wrap_test=1, waves_per_block=12)),
            (lcmod.LC_PERSISTENT, dict(hist_bits=16, wrap_test=1, waves_per_block=16, chunk=64)),
            (lcmod.LC_PERSISTENT | lcmod.LC_FORCE_EXACT, dict(hist_bits=16, wrap_test=1)),
            (lcmod.LC_PER_TASK, dict(hist_bits=16, wrap_test=1)),
            (lcmod.LC_PERSISTENT, dict(hist_bits=16, wrap_test=1, flush_limit=2000))]
    for mode, tune in runs:
        _say("[h16]", case, "mode", mode, "tune", tune)
        pl.count(mode, tune)
        torch.cuda.synchronize()
        gpu = pl.counts_host()
        for t in range(len(pl.tasks)):
            assert np.array_equal(gpu[t], refs[t]), (case, mode, tune, t)


def test_out_of_box_coordinate_is_an_error(torch, lcmod):
    L = 1000
    xyz = torch.tensor([[1, 2, L], [3, 4, 5], [6, 7, 8]], dtype=torch.int32, device="cuda")
    bn = lcmod.Binning([0, 10, 20], 2, True, L)
    with pytest.raises(lcmod.LcError) as ei:
        lcmod.lc_build_cells(xyz, [0, 3], bn)
    assert ei.value.status == lcmod.LC_ERR_RANGE
    big = torch.tensor([[1 << 24], [0], [0]], dtype=torch.int32, device="cuda")
    with pytest.raises(lcmod.LcError) as ei:
        lcmod.lc_build_cells(big, [0, 1], lcmod.Binning([0, 10], 1, False, 0, lcmod.LC_LOS_MID))
    assert ei.value.status == lcmod.LC_ERR_RANGE


def test_direct_split_estimate_and_sample_covariance(torch, oracle_mod, lcmod):
    """The direct estimate with M = 6 random sub-catalogues per mock (the
    sample covariance the linear construction replaces): counts bit-exact,
    the split estimate to 1e-12, its sample covariance to 1e-12 (float64) and
    1e-5 (float32 MFMA)."""
    from paper_2205_11852_amd.pipeline import Pipeline
    wl = dataclasses.replace(mockgen.WORKLOADS["c1"], n_mock=8, n_subsets=6, subset_size=3000)
    cats = mockgen.make_catalogues(wl)
    subsets = cats.random_catalogue_ids()
    assert len(subsets) == 6
    pl = Pipeline(cats)
    pl.build_cells()
    x, counts, tasks, est = pl.direct_estimates(range(cats.n_mock), subsets)
    torch.cuda.synchronize()
    got = counts.cpu().numpy().view(np.uint64)
    ref = np.zeros_like(got)
    for t, (a, b) in enumerate(tasks):
        ref[t] = oracle_mod.count_pairs(cats.cat(a), None if a == b else cats.cat(b), wl.r_edges_units,
                                        wl.n_mu, wl.box_units, wl.los)
    assert np.array_equal(got, ref)
    M = len(subsets)
    V = []
    for m in range(cats.n_mock):
        e = est[m]
        xs = oracle_mod.ls_split(ref[e[0]], [ref[t] for t in e[1:1 + M]], [ref[t] for t in e[1 + M:]],
                                 pl.sizes[m], [pl.sizes[s] for s in subsets])
        V.append(oracle_mod.data_vector(xs))
    V = np.array(V)
    g = x.cpu().numpy()
    assert np.array_equal(np.isnan(g), np.isnan(V))
    nb = wl.n_r * wl.n_mu
    ok = np.isfinite(V)
    assert np.allclose(g[:, :nb][ok[:, :nb]], V[:, :nb][ok[:, :nb]], rtol=1e-12, atol=0)
    W = oracle_mod.legendre_weights(wl.n_mu)
    for m in range(cats.n_mock):
        x2 = V[m, :nb].reshape(wl.n_r, wl.n_mu)
        scale = (np.abs(x2)[:, None, :] * np.abs(W)[None, :, :]).sum(axis=2).T.ravel()
        fin = np.isfinite(V[m, nb:])
        assert np.all(np.abs(g[m, nb:] - V[m, nb:])[fin] <= 1e-12 * scale[fin] + 1e-300)
    # sample covariance of the oracle's own vectors, on the device
    P = V.shape[1]
    xv = torch.from_numpy(np.ascontiguousarray(V)).cuda()
    C = torch.empty((P, P), dtype=torch.float64, device="cuda")
    refC = oracle_mod.sample_cov(V)
    for prec, tol in ((lcmod.LC_FP64, 1e-12), (lcmod.LC_FP32_MFMA, 1e-5)):
        lcmod.lc_sample_covariance(xv, V.shape[0], P, prec, C)
        torch.cuda.synchronize()
        assert _rel_frob(C.cpu().numpy(), refC) < tol, prec


def test_split_estimate_with_two_subsets_matches_xi_multipoles(c1, torch, lcmod):
    """lc_xi_split over (R1, R2) is the third estimate of lc_xi_multipoles."""
    pl = c1["pl"]
    pl.count()
    pl.xi_multipoles()
    x = torch.empty((pl.n_mock, pl.binning.P), dtype=torch.float64, device="cuda")
    lcmod.lc_xi_split(pl.counts, pl.tasks, pl.sizes, pl.est, 2, pl.binning.n_r, pl.binning.n_mu, x)
    torch.cuda.synchronize()
    a, b = x.cpu().numpy(), pl.xi[:, 2, :].cpu().numpy()
    assert np.array_equal(np.isnan(a), np.isnan(b))
    assert np.array_equal(a[np.isfinite(a)], b[np.isfinite(b)])


@pytest.mark.parametrize("P,M,use_ref,m_a", [(37, 50.0, False, 1), (2120, 50.0, False, 1), (2120, 10.0, True, 1),
                                             (120, float("inf"), False, 1), (37, 50.0, False, 2),
                                             (300, 7.0, True, 2), (64, 9.0, False, 3)])
def test_covcov_parity(torch, oracle_mod, lcmod, P, M, use_ref, m_a):
    """Covariance of the covariance estimates and the Table 3 summary on the
    device against the oracle (float64, 1e-12), for M_a = 1, 2 and 3 (the
    pair-count cost 1 + 6 M_a of Sect. 2.3 included)."""
    r = np.random.default_rng(P)
    G1, G2 = r.normal(size=(P, P)) / np.sqrt(P), r.normal(size=(P, P)) / np.sqrt(P)
    A = G1 @ G1.T + 0.1 * np.eye(P)      # positive definite, like the covariances
    B = 3.0 * (G2 @ G2.T)                # the random-catalogue part
    ref = (A + 2.0 * B) if use_ref else None
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dref = torch.from_numpy(ref).cuda() if use_ref else None
    sd_lc = torch.empty((P, P), dtype=torch.float64, device="cuda")
    sd_smp = torch.empty_like(sd_lc)
    n = 500
    rep = lcmod.lc_covcov(dA, dB, P, m_a, M, dref, n, sd_lc, sd_smp)
    exp = oracle_mod.covcov_summary(A, B, m_a, M, ref) if np.isfinite(M) else None
    if exp is not None:
        for k in ("chi2_2_lc", "chi2_2_smp", "ifom_lc", "ifom_smp", "gain"):
            assert abs(rep[k] - exp[k]) <= 1e-12 * abs(exp[k]), (k, rep[k], exp[k])
        assert rep["cost_lc"] == exp["cost_lc"] and rep["cost_smp"] == exp["cost_smp"]
    else:
        exp_lc = oracle_mod.chi2_2(oracle_mod.lc_cov_element_var(A, B, m_a, M, 2), A)
        assert abs(rep["chi2_2_lc"] - exp_lc) <= 1e-12 * exp_lc
    assert rep["cost_lc"] == oracle_mod.pair_cost_lc(m_a)
    v_lc = oracle_mod.lc_cov_element_var(A, B, m_a, M, n)
    v_smp = oracle_mod.sample_cov_element_var(A + (0.0 if np.isinf(M) else 1.0 / M) * B, n)
    assert np.allclose(sd_lc.cpu().numpy(), np.sqrt(v_lc), rtol=1e-12, atol=0)
    assert np.allclose(sd_smp.cpu().numpy(), np.sqrt(v_smp), rtol=1e-12, atol=0)


# ---------------------------------------------------------------------------
# co-added counts, 1D xi, linear maps and the general construction
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("w_r,w_mu", [(1, 1), (3, 2), (6, 5), (20, 10), (4, 10)])
def test_rebin_counts_parity(c1, oracle_mod, torch, lcmod, w_r, w_mu):
    """Co-added counts on the device, bit for bit against the oracle's
    co-adding of its own counts (ragged r groups, the 1D count, one bin)."""
    pl = c1["pl"]
    wl = c1["cats"].wl
    pl.count()
    out, b2 = pl.rebinned(w_r, w_mu)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint64)
    assert list(b2.edges) == oracle_mod.rebinned_edges(wl.r_edges_units, w_r)
    for t in range(len(pl.tasks)):
        assert np.array_equal(got[t], oracle_mod.rebin_counts(c1["ref"][t], w_r, w_mu)), t


def test_one_dimensional_xi_parity(c1, oracle_mod, torch, lcmod):
    """The 1D correlation function (counts co-added over mu, Sect. 4.3) and
    its vector: within 1e-12 of the oracle; xi_2 = xi_4 = 0 exactly."""
    pl = c1["pl"]
    wl = c1["cats"].wl
    pl.count()
    c, b1 = pl.rebinned(1, wl.n_mu)
    xi = pl.xi_of(c, b1)
    torch.cuda.synchronize()
    g = xi.cpu().numpy()
    n_r = wl.n_r
    for m in range(pl.n_mock):
        e = pl.est[m]
        D, R1, R2 = pl.tasks[e[0]][0], pl.tasks[e[1]][1], pl.tasks[e[2]][1]
        V = oracle_mod.mock_vectors(*(oracle_mod.rebin_counts(c1["ref"][t], 1, wl.n_mu) for t in e),
                                    pl.sizes[D], pl.sizes[R1], pl.sizes[R2])
        assert np.array_equal(np.isnan(g[m]), np.isnan(V))
        ok = np.isfinite(V)
        assert np.allclose(g[m][ok], V[ok], rtol=1e-12, atol=0)
        assert np.all(g[m][:, 2 * n_r:][ok[:, 2 * n_r:]] == 0.0)


def _random_map(r, P_in, P_out):
    g = r.integers(-1, P_out - 1, size=P_in).astype(np.int32)
    g[:P_out - 1] = np.arange(P_out - 1)  # every output but the last has a member
    g[P_out - 1] = -1                     # the last one has none (must be 0)
    w = r.normal(size=P_in)
    return g, w


def test_map_vectors_and_matrix_parity(torch, oracle_mod, lcmod):
    """Linear maps on the device against the oracle's dense T (float64,
    1e-12 of the summed magnitudes); strided rows; an empty output is 0."""
    r = np.random.default_rng(21)
    N, P_in, P_out = 37, 300, 61
    X = r.normal(size=(N, 3, P_in))
    g, w = _random_map(r, P_in, P_out)
    x = torch.from_numpy(X).cuda()
    y = torch.full((N, 3, P_out + 5), 7.0, dtype=torch.float64, device="cuda")
    lcmod.lc_map_vectors(x, 3 * N, P_in, g, w, P_out, y, ld_y=P_out + 5)
    torch.cuda.synchronize()
    gy = y.cpu().numpy()
    ref = oracle_mod.map_vectors(X, g, w, P_out)
    scale = oracle_mod.map_vectors(np.abs(X), g, np.abs(w), P_out)
    assert np.all(np.abs(gy[..., :P_out] - ref) <= 1e-12 * scale + 1e-300)
    assert np.all(gy[..., P_out:] == 7.0)            # the stride gap is untouched
    assert np.all(gy[..., P_out - 1] == 0.0)
    # the selection map of the paper's multipole vector picks elements exactly
    from paper_2205_11852_amd.pipeline import multipole_map
    gs, ws, Ps = multipole_map(20, 10, 1, 4, 20)
    xs = torch.from_numpy(r.normal(size=(5, 3, 20 * 10 + 60))).cuda()
    ys = torch.empty((5, 3, Ps), dtype=torch.float64, device="cuda")
    lcmod.lc_map_vectors(xs, 15, xs.shape[2], gs, ws, Ps, ys)
    torch.cuda.synchronize()
    assert np.array_equal(ys.cpu().numpy(), oracle_mod.map_vectors(xs.cpu().numpy(), gs, ws, Ps))
    # matrices
    S = r.normal(size=(P_in, P_in))
    S = S + S.T
    Y = torch.empty((P_out, P_out), dtype=torch.float64, device="cuda")
    lcmod.lc_map_matrix(torch.from_numpy(S).cuda(), P_in, g, w, P_out, Y)
    torch.cuda.synchronize()
    refY = oracle_mod.map_matrix(S, g, w, P_out)
    scY = oracle_mod.map_matrix(np.abs(S), g, np.abs(w), P_out)
    gY = Y.cpu().numpy()
    assert np.all(np.abs(gY - refY) <= 1e-12 * scY + 1e-300)
    assert np.all(gY[P_out - 1] == 0.0) and np.all(gY[:, P_out - 1] == 0.0)


@pytest.mark.parametrize("m_a,m_b,n_split", [(1.0, 3.0, 100), (2.0, 5.0, 0), (0.5, 4.0, 160), (1.0, 2.0, 37)])
def test_covariance_general_parity(torch, oracle_mod, lcmod, m_a, m_b, n_split):
    """Eq. CovAB on the device: float64 within 1e-12 and float32 MFMA within
    1e-5 of the oracle; the check of both blocks against LAPACK."""
    n_mock, P = 400, 160
    V = _synthetic_vectors(n_mock, P, int(10 * m_a + m_b))
    xi = torch.from_numpy(V).cuda()
    A, B, C = (torch.empty((P, P), dtype=torch.float64, device="cuda") for _ in range(3))
    for M in (50.0, float("inf")):
        rA, rB, rC, _, _ = oracle_mod.lc_from_vectors_general(V, m_a, m_b, M)
        for prec, tol in ((lcmod.LC_FP64, 1e-12), (lcmod.LC_FP32_MFMA_CHECKED, 1e-5)):
            rep = lcmod.lc_covariance_general(xi, n_mock, P, n_split, m_a, m_b, M, prec, A, B, C, report=True)
            torch.cuda.synchronize()
            gA, gB, gC = (t.cpu().numpy() for t in (A, B, C))
            assert _rel_frob(gA, rA) < tol and _rel_frob(gB, rB) < tol and _rel_frob(gC, rC) < tol, (M, prec)
        for blk, sl in enumerate((slice(0, n_split), slice(n_split, P))):
            if sl.stop - sl.start == 0:
                assert rep["chol_ok"][blk] == 1 and rep["n_neg_eig"][blk] == 0
                assert np.isnan(rep["min_eig"][blk]) and np.isnan(rep["max_eig"][blk])
                continue
            wv = np.linalg.eigvalsh(gC[sl, sl])
            scale = np.abs(wv).max()
            assert abs(rep["min_eig"][blk] - wv[0]) <= 1e-10 * scale
            assert abs(rep["max_eig"][blk] - wv[-1]) <= 1e-10 * scale
            assert rep["n_neg_eig"][blk] == int((wv < 0).sum())


@pytest.mark.parametrize("P,n_split", [(1, 0), (2, 1), (3, 0), (4, 1), (5, 3), (258, 2), (300, 43), (1100, 17)])
def test_check_block_sizes(torch, oracle_mod, lcmod, P, n_split):
    """The check's Householder and bisection on blocks of 1 to 1083 rows
    (both sides of the 256-row switch of the column kernel, and of the
    elements it holds in registers per lane: 512 and 1024), against
    LAPACK."""
    n_mock = 600
    V = _synthetic_vectors(n_mock, P, 1000 + P)
    xi = torch.from_numpy(V).cuda()
    A, B, C = (torch.empty((P, P), dtype=torch.float64, device="cuda") for _ in range(3))
    rep = lcmod.lc_covariance_general(xi, n_mock, P, n_split, 1.0, 2.0, 50.0, lcmod.LC_FP64, A, B, C, report=True)
    torch.cuda.synchronize()
    gC = C.cpu().numpy()
    for blk, sl in enumerate((slice(0, n_split), slice(n_split, P))):
        if sl.stop - sl.start == 0:
            assert rep["chol_ok"][blk] == 1 and rep["n_neg_eig"][blk] == 0
            continue
        ref = oracle_mod.check_matrix(gC[sl, sl])
        scale = max(abs(ref["min_eig"]), abs(ref["max_eig"]))
        assert abs(rep["min_eig"][blk] - ref["min_eig"]) <= 1e-10 * scale, (P, n_split, blk)
        assert abs(rep["max_eig"][blk] - ref["max_eig"]) <= 1e-10 * scale, (P, n_split, blk)
        assert rep["n_neg_eig"][blk] == ref["n_neg_eig"], (P, n_split, blk)
        assert rep["chol_ok"][blk] == ref["chol_ok"], (P, n_split, blk)


def test_covariance_general_at_paper_ratios_equals_lc_covariance(c1, c1_cov, torch, lcmod):
    """With M_b = 2 M_a and the (r, mu) block split, the general call is
    lc_covariance, bit for bit."""
    pl = c1["pl"]
    _load_xi(pl, c1_cov["xi"], torch)
    P, nb = pl.binning.P, pl.binning.n_r * pl.binning.n_mu
    pl.covariance(lcmod.LC_FP64, report=False)
    torch.cuda.synchronize()
    ref = [t.cpu().numpy().copy() for t in (pl.A, pl.B, pl.C)]
    A, B, C, _ = pl.covariance_general(pl.xi, P, nb, 1.0, 2.0, precision=lcmod.LC_FP64, report=False)
    torch.cuda.synchronize()
    for x, y in zip((A, B, C), ref):
        x = x.cpu().numpy()
        assert np.array_equal(np.isnan(x), np.isnan(y))
        assert np.array_equal(x[np.isfinite(x)], y[np.isfinite(y)])


def test_general_vectors_and_strided_split(c1, torch, lcmod, oracle_mod):
    """Estimates x, x' (M_a = 1) and y (M_b = 2) over the same pool
    sub-catalogues for every mock, written by lc_xi_split into the [n, 3, P]
    layout with a row stride, against the oracle's split estimator on the
    oracle's counts."""
    pl = c1["pl"]
    cats = c1["cats"]
    wl = cats.wl
    pool = cats.random_catalogue_ids()
    assert len(pool) >= 2
    sets = [[pool[0]], [pool[1]], [pool[0], pool[1]]]
    mocks = list(range(6))
    W = oracle_mod.legendre_weights(wl.n_mu)
    xi = pl.general_vectors(mocks, sets)
    torch.cuda.synchronize()
    g = xi.cpu().numpy()
    for m in mocks:
        dd = c1["ref"][pl.est[m][0]] if pl.tasks[pl.est[m][0]][0] == m else None
        assert dd is not None
        for e, S in enumerate(sets):
            DR = [oracle_mod.count_pairs(cats.cat(m), cats.cat(s), wl.r_edges_units, wl.n_mu, wl.box_units, wl.los)
                  for s in S]
            RR = [oracle_mod.count_pairs(cats.cat(s), None, wl.r_edges_units, wl.n_mu, wl.box_units, wl.los)
                  for s in S]
            V = oracle_mod.data_vector(oracle_mod.ls_split(dd, DR, RR, pl.sizes[m], [pl.sizes[s] for s in S]))
            assert np.array_equal(np.isnan(g[m, e]), np.isnan(V))
            ok = np.isfinite(V)
            nb = wl.n_r * wl.n_mu
            assert np.allclose(g[m, e, :nb][ok[:nb]], V[:nb][ok[:nb]], rtol=1e-12, atol=0)
            x2 = V[:nb].reshape(wl.n_r, wl.n_mu)
            scale = (np.abs(x2)[:, None, :] * np.abs(W)[None, :, :]).sum(axis=2).T.ravel()
            fin = np.isfinite(V[nb:])
            assert np.all(np.abs(g[m, e, nb:] - V[nb:])[fin] <= 1e-12 * scale[fin] + 1e-300)


def _random_config(r):
    """One random but valid binning, geometry, mesh and launch shape."""
    periodic = bool(r.integers(0, 2))
    los = ["z", "mid", "rppi"][int(r.integers(0, 3))]
    if los == "mid":
        periodic = False
    L = int(r.integers(20000, 200000)) * 2 if periodic else 0
    span = L if periodic else int(r.integers(20000, 400000))
    lo = 0 if periodic else int(r.integers(-(1 << 22), 1 << 22))
    reach = (L // 2 - 1) if periodic else span
    n_r = int(r.integers(1, 25))
    rmax = int(r.integers(max(n_r + 2, span // 40), max(n_r + 3, min(reach, span // 3))))
    if r.random() < 0.5:
        e0 = int(r.integers(0, rmax // 4 + 1)) if r.random() < 0.5 else 0
        de = max(1, (rmax - e0) // n_r)
        edges = [e0 + k * de for k in range(n_r + 1)]
    else:
        edges = sorted(set(int(v) for v in r.integers(0, rmax, size=n_r + 1)))
        if len(edges) < 2:
            edges = [0, rmax]
    n_mu = int(r.integers(1, 60))
    pi_max = int(r.integers(1, max(2, min(reach, span // 3)))) if los == "rppi" else 0
    cell = int(r.integers(0, 2)) * int(r.integers(max(1, edges[-1] // 4), max(2, edges[-1] + 1)))
    sub = [0, 1, 2, 4][int(r.integers(0, 4))]
    tune = dict(chunk=4 * int(r.integers(1, 65)),
                waves_per_block=[0, 1, 2, 4, 8, 16][int(r.integers(0, 6))],
                cells_per_item=int(r.integers(0, 5)),
                hist_bits=[0, 0, 16, 32][int(r.integers(0, 4))], wrap_test=int(r.integers(0, 2)))
    return dict(periodic=periodic, los=los, L=L, lo=lo, span=span, edges=edges, n_mu=n_mu, pi_max=pi_max,
                cell=cell, sub=sub, tune=tune)


@pytest.mark.parametrize("seed", range(60))
def test_random_configurations_bit_exact(torch, lcmod, oracle_mod, seed):
    """Seeded random binnings (uniform or not, e_0 >= 0, 1-59 mu bins),
    geometries (periodic boxes, open regions anywhere in |x| < 2^24),
    lines of sight (z, midpoint, (r_p, pi)), meshes (odd seeds in arrival
    order), launch shapes and histogram widths (16-bit bins, some started
    near their wrap), on clustered and uniform catalogues: every task
    bit-exact."""
    r = np.random.default_rng(1000 + seed)
    cfg = _random_config(r)
    _say("[random]", seed, {k: v for k, v in cfg.items() if k != "edges"}, "n_r", len(cfg["edges"]) - 1)
    cats = []
    for c in range(3):
        n = int(r.integers(0, 900)) if c else int(r.integers(200, 1500))
        if r.random() < 0.5:   # clustered around a few centres
            centres = r.integers(0, cfg["span"], size=(3, 6))
            pts = centres[:, r.integers(0, 6, size=n)] + r.normal(0, cfg["span"] / 30, size=(3, n)).astype(np.int64)
            pts = np.clip(pts, 0, cfg["span"] - 1)
        else:
            pts = r.integers(0, cfg["span"], size=(3, n))
        cats.append((pts + cfg["lo"]).astype(np.int32) if not cfg["periodic"] else (pts % cfg["L"]).astype(np.int32))
    off = np.cumsum([0] + [c.shape[1] for c in cats])
    xyz = torch.from_numpy(np.ascontiguousarray(np.concatenate(cats, axis=1))).cuda()
    los = {"z": lcmod.LC_LOS_Z, "mid": lcmod.LC_LOS_MID, "rppi": lcmod.LC_LOS_RPPI}[cfg["los"]]
    bn = lcmod.Binning(cfg["edges"], cfg["n_mu"], cfg["periodic"], cfg["L"], los, cfg["pi_max"])
    cells = lcmod.lc_build_cells(xyz, off, bn, cfg["cell"], cfg["sub"], arrival_order=seed % 2 == 1)
    tasks = [(a, b) for a in range(3) for b in range(3)]
    counts = torch.zeros((len(tasks), bn.n_r, bn.n_mu), dtype=torch.int64, device="cuda")
    lcmod.lc_pair_count_batch(cells, tasks, bn, counts, lcmod.LC_PERSISTENT, cfg["tune"])
    got = counts.cpu().numpy().view(np.uint64)
    for t, (a, b) in enumerate(tasks):
        ref = oracle_mod.count_pairs(cats[a], None if a == b else cats[b], cfg["edges"], cfg["n_mu"], cfg["L"],
                                     cfg["los"], pi_max=cfg["pi_max"])
        assert np.array_equal(got[t], ref), (seed, t)
    cells.close()
