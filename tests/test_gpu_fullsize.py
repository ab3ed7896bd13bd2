"""Parity at the benchmark's full size and in its launch configuration.

The 1000-mock, 1e5-galaxy periodic workload is counted exactly as bench.py
counts it (one persistent launch with the library defaults).  The oracle
checks sampled tasks one by one (brute force, bit for bit), the data vector
of one mock (float64, 1e-12), and properties that hold at any size: the
counts do not depend on the tiling, and per-task launches give the same
counts.  The covariance stage runs at the full data-vector sizes on seeded
synthetic vectors, and on the 5000 measured vectors of the
covariance-precision workload against the float64 oracle.  Smaller workloads of the other configurations' shapes
(100 mu bins with per-mock randoms) are compared task by task.
"""
import dataclasses
import sys

import numpy as np
import pytest

import mockgen

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel_frob(x, y):
    m = np.isfinite(y)
    return np.linalg.norm((x - y)[m]) / np.linalg.norm(y[m])


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return t


@pytest.fixture(scope="module")
def lcmod(torch):
    from paper_2205_11852_amd import lc
    lc.lib()
    return lc


@pytest.fixture(scope="module")
def c2(torch, lcmod):
    from paper_2205_11852_amd.pipeline import Pipeline
    _say("[c2] generating 1000 mocks")
    cats = mockgen.make_catalogues(mockgen.WORKLOADS["c2"])
    pl = Pipeline(cats)
    pl.build_cells()
    pl.count()
    pl.xi_multipoles()
    torch.cuda.synchronize()
    _say("[c2] counted %d tasks" % len(pl.tasks))
    return dict(pl=pl, cats=cats, counts=pl.counts_host().copy(), xi=pl.xi.cpu().numpy())


@pytest.fixture(scope="module")
def c2_mock0(c2, oracle_mod):
    """Oracle counts of every task of mock 0 (DD, DR1, DR2, RR1, RR2)."""
    pl, cats = c2["pl"], c2["cats"]
    wl = cats.wl
    out = {}
    for t in pl.est[0]:
        a, b = pl.tasks[t]
        _say("[c2] oracle task", int(t), (int(a), int(b)))
        out[int(t)] = oracle_mod.count_pairs(cats.cat(a), None if a == b else cats.cat(b), wl.r_edges_units,
                                             wl.n_mu, wl.box_units, wl.los)
    return out


def test_c2_sampled_tasks_bit_exact(c2, c2_mock0, oracle_mod):
    pl, cats = c2["pl"], c2["cats"]
    wl = cats.wl
    for t, ref in c2_mock0.items():
        assert np.array_equal(c2["counts"][t], ref), t
    # the last mock's auto pairs too (its catalogue sits at the far end of the point array)
    t = int(pl.est[-1][0])
    a, _ = pl.tasks[t]
    _say("[c2] oracle task", t)
    ref = oracle_mod.count_pairs(cats.cat(a), None, wl.r_edges_units, wl.n_mu, wl.box_units, wl.los)
    assert np.array_equal(c2["counts"][t], ref)


def test_c2_mock0_data_vector(c2, c2_mock0, oracle_mod):
    pl = c2["pl"]
    e = pl.est[0]
    D, R1, R2 = pl.tasks[e[0]][0], pl.tasks[e[1]][1], pl.tasks[e[2]][1]
    V = oracle_mod.mock_vectors(*(c2_mock0[int(t)] for t in e), pl.sizes[D], pl.sizes[R1], pl.sizes[R2])
    g = c2["xi"][0]
    assert np.array_equal(np.isnan(g), np.isnan(V))
    ok = np.isfinite(V)
    nb = pl.binning.n_r * pl.binning.n_mu
    assert np.allclose(g[:, :nb][ok[:, :nb]], V[:, :nb][ok[:, :nb]], rtol=1e-12, atol=0)
    W = oracle_mod.legendre_weights(pl.binning.n_mu)
    for q in range(3):
        x2 = V[q, :nb].reshape(pl.binning.n_r, pl.binning.n_mu)
        scale = (np.abs(x2)[:, None, :] * np.abs(W)[None, :, :]).sum(axis=2).T.ravel()
        d = np.abs(g[q, nb:] - V[q, nb:])
        fin = np.isfinite(V[q, nb:])
        assert np.all(d[fin] <= 1e-12 * scale[fin] + 1e-300)


def test_c2_counts_independent_of_tiling(c2, torch):
    """Every one of the 3050 tasks: another mesh, chunking and block shape
    give the same counts (the result cannot depend on the tiling)."""
    pl = c2["pl"]
    pl.build_cells(int(125.0 * mockgen.UNITS_PER_MPC), 4)
    pl.count(tune=dict(chunk=64, cells_per_item=3, waves_per_block=2))
    torch.cuda.synchronize()
    assert np.array_equal(pl.counts_host(), c2["counts"])
    pl.build_cells()


def test_c2_per_task_launches_identical(c2, torch):
    pl = c2["pl"]
    pl.count_per_mock()
    torch.cuda.synchronize()
    assert np.array_equal(pl.counts_host(), c2["counts"])


def test_c2_count_totals(c2):
    """No task holds more pairs than its catalogues can form."""
    pl = c2["pl"]
    tot = c2["counts"].reshape(len(pl.tasks), -1).sum(axis=1, dtype=np.float64)
    na = pl.sizes[pl.tasks[:, 0]].astype(np.float64)
    nb = pl.sizes[pl.tasks[:, 1]].astype(np.float64)
    cap = np.where(pl.tasks[:, 0] == pl.tasks[:, 1], na * (na - 1) / 2, na * nb)
    assert np.all(tot <= cap) and np.all(tot > 0)


@pytest.fixture(scope="module")
def slab(torch, lcmod):
    """Ten full-size paper-shaped slabs (156 158 points on average), counted
    in one persistent launch with the library defaults."""
    from paper_2205_11852_amd.pipeline import Pipeline
    wl = dataclasses.replace(mockgen.WORKLOADS["slab"], n_mock=10)
    _say("[slab] generating", wl.n_mock, "slabs")
    cats = mockgen.make_catalogues(wl)
    pl = Pipeline(cats)
    pl.build_cells()
    pl.count()
    torch.cuda.synchronize()
    _say("[slab] counted %d tasks" % len(pl.tasks))
    return dict(pl=pl, cats=cats, counts=pl.counts_host().copy())


def test_slab_full_size_sampled_tasks(slab, oracle_mod):
    """DD, DR1 and RR1 of one full-size slab, brute force, bit for bit."""
    pl, cats = slab["pl"], slab["cats"]
    wl = cats.wl
    m = 3
    for t in pl.est[m][[0, 1, 3]]:
        a, b = pl.tasks[t]
        _say("[slab] oracle task", int(t), (int(a), int(b)), cats.sizes()[a], cats.sizes()[b])
        ref = oracle_mod.count_pairs(cats.cat(a), None if a == b else cats.cat(b), wl.r_edges_units,
                                     wl.n_mu, 0, "z")
        assert np.array_equal(slab["counts"][t], ref), int(t)


def test_slab_counts_independent_of_tiling(slab, torch):
    pl = slab["pl"]
    pl.build_cells(int(75.0 * mockgen.UNITS_PER_MPC), 1)
    pl.count(tune=dict(chunk=128, waves_per_block=8))
    torch.cuda.synchronize()
    assert np.array_equal(pl.counts_host(), slab["counts"])
    pl.build_cells()


@pytest.fixture(scope="module")
def c5(torch, lcmod):
    """The covariance-precision workload at full size: 5000 mocks of
    Poisson(5e4) points, 40 x 50 bins, counted in one persistent launch with
    the library defaults; the data vectors (P = 2120) stay on the host."""
    from paper_2205_11852_amd.pipeline import Pipeline
    _say("[c5] generating 5000 mocks")
    cats = mockgen.make_catalogues(mockgen.WORKLOADS["c5"], progress=_say)
    pl = Pipeline(cats)
    pl.build_cells()
    pl.count()
    pl.xi_multipoles()
    torch.cuda.synchronize()
    _say("[c5] counted %d tasks" % len(pl.tasks))
    return dict(pl=pl, cats=cats, counts=pl.counts_host().copy(), xi=pl.xi.cpu().numpy())


def test_c5_sampled_tasks_and_data_vector(c5, oracle_mod):
    """Every task of mock 0 and the last mock's DD, brute force, bit for bit;
    mock 0's three estimates and their multipoles within 1e-12."""
    pl, cats = c5["pl"], c5["cats"]
    wl = cats.wl
    ref = {}
    for t in list(pl.est[0]) + [pl.est[-1][0]]:
        a, b = pl.tasks[t]
        _say("[c5] oracle task", int(t), (int(a), int(b)))
        ref[int(t)] = oracle_mod.count_pairs(cats.cat(a), None if a == b else cats.cat(b), wl.r_edges_units,
                                             wl.n_mu, wl.box_units, wl.los)
        assert np.array_equal(c5["counts"][t], ref[int(t)]), int(t)
    e = pl.est[0]
    D, R1, R2 = pl.tasks[e[0]][0], pl.tasks[e[1]][1], pl.tasks[e[2]][1]
    V = oracle_mod.mock_vectors(*(ref[int(t)] for t in e), pl.sizes[D], pl.sizes[R1], pl.sizes[R2])
    g = c5["xi"][0]
    assert np.array_equal(np.isnan(g), np.isnan(V))
    ok = np.isfinite(V)
    nb = pl.binning.n_r * pl.binning.n_mu
    assert np.allclose(g[:, :nb][ok[:, :nb]], V[:, :nb][ok[:, :nb]], rtol=1e-12, atol=0)


def test_c5_covariance_precision_against_oracle(c5, oracle_mod, lcmod, torch):
    """The 5000 measured data vectors (P = 2120): the float32-MFMA products
    give A, B and C^LC(50) within 1e-5 (relative Frobenius) of the float64
    oracle's, with float32 accumulation over blocks of 256 mocks and over all
    5000 (LC_ACC32), and the float64 path within 1e-12."""
    pl = c5["pl"]
    V = c5["xi"]
    rA, rB, rC, _, _ = oracle_mod.lc_from_vectors(V, 1, 50.0)
    for prec, tol in ((lcmod.LC_FP32_MFMA, 1e-5), (lcmod.LC_FP32_MFMA | lcmod.LC_ACC32, 1e-5),
                      (lcmod.LC_FP64, 1e-12)):
        _say("[c5] covariance, precision", prec)
        pl.covariance(prec, report=False, M=50.0)
        torch.cuda.synchronize()
        gA, gB, gC = (t.cpu().numpy() for t in (pl.A, pl.B, pl.C))
        errs = [_rel_frob(x, y) for x, y in ((gA, rA), (gB, rB), (gC, rC))]
        _say("[c5] rel. Frobenius A, B, C:", errs)
        assert max(errs) < tol, (prec, errs)


def _synthetic_vectors(n_mock, P, seed):
    r = np.random.default_rng(seed)
    L = r.normal(size=(P, P)) / np.sqrt(P) + np.eye(P)
    base = r.normal(size=(n_mock, P)) @ L.T
    return np.stack([base + 0.3 * r.normal(size=(n_mock, P)) for _ in range(3)], axis=1)


@pytest.mark.parametrize("n_mock", [1000, 5000])
def test_covariance_full_size(lcmod, oracle_mod, torch, n_mock):
    """The covariance stage at the full data-vector size (40 x 50 bins plus
    multipoles, P = 2120) for 1000 and 5000 mocks: float32-MFMA products
    within 1e-5 and float64 within 1e-12 of the oracle."""
    n_r, n_mu = 40, 50
    P = n_r * n_mu + 3 * n_r
    V = _synthetic_vectors(n_mock, P, 7 + n_mock)
    xi = torch.from_numpy(V).cuda()
    A, B, C = (torch.empty((P, P), dtype=torch.float64, device="cuda") for _ in range(3))
    rA, rB, rC, _, _ = oracle_mod.lc_from_vectors(V, 1, 50.0)
    for prec, tol in ((lcmod.LC_FP32_MFMA_CHECKED | lcmod.LC_ACC32, 1e-5), (lcmod.LC_FP32_MFMA_CHECKED, 1e-5),
                      (lcmod.LC_FP64, 1e-12)):
        _say("[cov] n_mock", n_mock, "precision", prec)
        rep = lcmod.lc_covariance(xi, n_mock, n_r, n_mu, 1, 50.0, prec, A, B, C, report=True)
        torch.cuda.synchronize()
        gA, gB, gC = (t.cpu().numpy() for t in (A, B, C))
        assert _rel_frob(gC, rC) < tol and _rel_frob(gA, rA) < tol and _rel_frob(gB, rB) < tol, prec
    nb0 = n_r * n_mu
    for blk, sl in enumerate((slice(0, nb0), slice(nb0, P))):
        w = np.linalg.eigvalsh(gC[sl, sl])
        scale = np.abs(w).max()
        assert abs(rep["min_eig"][blk] - w[0]) <= 1e-10 * scale
        assert abs(rep["max_eig"][blk] - w[-1]) <= 1e-10 * scale


def test_hundred_mu_bins_per_mock_randoms(torch, lcmod, oracle_mod):
    """The large-mock configuration's shape (2000 Mpc/h box, 100 mu bins,
    two random sub-catalogues per mock) at a size the oracle counts fully."""
    from paper_2205_11852_amd.pipeline import Pipeline
    wl = dataclasses.replace(mockgen.WORKLOADS["c3"], n_mock=2, n_mean=20000.0, n_parents=800)
    cats = mockgen.make_catalogues(wl)
    pl = Pipeline(cats)
    pl.build_cells()
    pl.count()
    torch.cuda.synchronize()
    gpu = pl.counts_host()
    _say("[c3-shape] grid", pl.cells.info()["grid"], "tasks", len(pl.tasks))
    for t, (a, b) in enumerate(pl.tasks):
        ref = oracle_mod.count_pairs(cats.cat(a), None if a == b else cats.cat(b), wl.r_edges_units, wl.n_mu,
                                     wl.box_units, wl.los)
        assert np.array_equal(gpu[t], ref), t
