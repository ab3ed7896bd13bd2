"""Parity at the full sizes of the large-mock and survey-wedge workloads.

Large mocks: 200 mocks of Poisson(1e6) clustered points in a 2000 Mpc/h
periodic box, each with two random sub-catalogues of its own size, 40 r bins
x 100 mu bins.  Survey wedge: 500 mocks of Poisson(3e5) points in the open
60 x 60 degree wedge with a shared pool of 20 x 3e5 randoms, midpoint line
of sight (integer rule in 128 bits).  Each is counted in one persistent
launch with the library defaults.

A full auto count of a 1e6-point mock is beyond the oracle (5e11 pair
tests), so the oracle checks sampled outputs: the cross counts of a
2048-point subset of a mock against the whole mock and against a random
sub-catalogue, counted in the same launch as every estimator task.  For the
wedge it also counts one whole DD task of a 3e5-point mock.
Properties that hold at any size cover the rest:
- the union identity DD(A u B) = DD(A) + DD(B) + DR(A, B) for a split of a
  whole mock into two halves (exact);
- the counts do not depend on the mesh or the launch shape (the autotuned
  configuration included), and per-task launches give the same counts;
- uniform random sub-catalogues in the periodic box: every bin's RR count
  against its expectation C(N, 2) p_k,m, p the bin's share of the box
  volume.  For uniform points in a periodic box two pair indicators that
  share a point are uncorrelated (given the shared point, the other two are
  independent and each lands in the bin with probability p), so the count's
  variance is exactly C(N, 2) p (1 - p).
"""
import sys

import numpy as np
import pytest

import mockgen

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

N_SAMPLE = 2048


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
    lc.lib()
    return lc


def _with_probes(cats, seed):
    """The workload's catalogues plus probe catalogues appended after them:
    a 2048-point subset of the first and of the last mock, and the two
    halves (even / odd positions) of the first mock.  Returns the extended
    catalogues, the probe tasks and their roles."""
    rng = np.random.default_rng(seed)
    last = cats.n_mock - 1
    d0, dl = cats.cat(0), cats.cat(last)
    probes = [d0[:, np.sort(rng.choice(d0.shape[1], N_SAMPLE, replace=False))],
              dl[:, np.sort(rng.choice(dl.shape[1], N_SAMPLE, replace=False))],
              d0[:, 0::2], d0[:, 1::2]]
    s0, sl, ha, hb = range(cats.n_cat, cats.n_cat + 4)
    r1_0 = int(cats.randoms[0, 0])
    r2_l = int(cats.randoms[last, 1])
    roles = {"S0xD0": (s0, 0), "S0xR1": (s0, r1_0), "SlxDl": (sl, last), "SlxR2": (sl, r2_l),
             "AA": (ha, ha), "BB": (hb, hb), "AB": (ha, hb)}
    xyz = np.concatenate([cats.xyz] + [np.ascontiguousarray(p, dtype=np.int32) for p in probes], axis=1)
    sizes = np.concatenate([cats.sizes(), [p.shape[1] for p in probes]]).astype(np.int64)
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    ext = mockgen.Catalogues(cats.wl, xyz, off, cats.n_mock, cats.randoms)
    return ext, list(roles.values()), list(roles.keys())


def _counted(name, torch, seed):
    from paper_2205_11852_amd.pipeline import Pipeline
    wl = mockgen.WORKLOADS[name]
    _say("[%s] generating %d mocks of Poisson(%g)" % (name, wl.n_mock, wl.n_mean))
    cats = mockgen.make_catalogues(wl, progress=_say)
    cats, probe_tasks, roles = _with_probes(cats, seed)
    pl = Pipeline(cats, extra_tasks=probe_tasks)
    n_est = len(pl.tasks) - len(probe_tasks)
    _say("[%s] %d points, %d catalogues, %d tasks; building the mesh" %
         (name, cats.xyz.shape[1], cats.n_cat, len(pl.tasks)))
    pl.build_cells()
    _say("[%s] mesh %s; counting" % (name, pl.cells.info()))
    pl.count()
    torch.cuda.synchronize()
    counts = pl.counts_host().copy()
    _say("[%s] counted: %s" % (name, pl.stats_host()))
    probe = {r: n_est + i for i, r in enumerate(roles)}
    return dict(pl=pl, cats=cats, counts=counts, probe=probe, n_est=n_est)


@pytest.fixture(scope="module")
def c3(torch, lcmod):
    return _counted("c3", torch, 31)


@pytest.fixture(scope="module")
def c4(torch, lcmod):
    return _counted("c4", torch, 41)


def _check_probes(run, oracle_mod):
    cats, wl = run["cats"], run["cats"].wl
    for role in ("S0xD0", "S0xR1", "SlxDl", "SlxR2"):
        t = run["probe"][role]
        a, b = run["pl"].tasks[t]
        _say("[%s] oracle %s: %d x %d points" % (wl.name, role, cats.sizes()[a], cats.sizes()[b]))
        ref = oracle_mod.count_pairs(cats.cat(a), cats.cat(b), wl.r_edges_units, wl.n_mu, wl.box_units, wl.los)
        assert np.array_equal(run["counts"][t], ref), role
        assert ref.sum() > 0


def _check_union(run):
    """DD of mock 0 from its estimator task equals the sum over its halves."""
    pl, c = run["pl"], run["counts"]
    p = run["probe"]
    dd0 = c[int(pl.est[0][0])]
    parts = c[p["AA"]] + c[p["BB"]] + c[p["AB"]]
    assert np.array_equal(dd0, parts)
    assert dd0.sum() > 0


def test_c3_sampled_cross_counts_bit_exact(c3, oracle_mod):
    _check_probes(c3, oracle_mod)


def test_c3_union_identity(c3):
    _check_union(c3)


def test_c3_uniform_randoms_match_shell_volumes(c3, oracle_mod):
    """RR of the first and last mock's random sub-catalogues (1e6 uniform
    points each, 4000 bins each) against the binomial expectation."""
    pl, c, wl = c3["pl"], c3["counts"], c3["cats"].wl
    frac = oracle_mod.shell_pair_fraction(wl.r_edges_units, wl.n_mu, wl.box_units)
    z = []
    for m in (0, c3["cats"].n_mock - 1):
        for t in pl.est[m][3:]:
            r = pl.tasks[int(t)][0]
            n = float(pl.sizes[r])
            e = n * (n - 1) / 2 * frac
            z.append((c[int(t)].astype(np.float64) - e) / np.sqrt(e * (1 - frac)))
    z = np.concatenate([v.ravel() for v in z])
    _say("[c3] RR z-scores: max |z| %.2f, mean z^2 %.4f over %d bins" % (np.abs(z).max(), np.mean(z * z), z.size))
    assert np.abs(z).max() < 6.0
    assert abs(np.mean(z * z) - 1.0) < 5.0 * np.sqrt(2.0 / z.size)
    assert abs(np.mean(z)) < 5.0 / np.sqrt(z.size)


def test_c3_counts_independent_of_tiling(c3, torch):
    """Every task, again with the autotuned configuration and with a mesh of
    r_max / 3 cells without sub-cells, 128-point chunks and 8-wave blocks."""
    pl = c3["pl"]
    tuned = pl.autotune()
    _say("[c3] autotuned:", tuned)
    pl.build_cells()
    pl.count()
    torch.cuda.synchronize()
    assert np.array_equal(pl.counts_host(), c3["counts"])
    pl.tuned = None
    pl.build_cells(int(200.0 / 3.0 * mockgen.UNITS_PER_MPC), 1)
    pl.count(tune=dict(chunk=128, waves_per_block=8))
    torch.cuda.synchronize()
    assert np.array_equal(pl.counts_host(), c3["counts"])
    pl.build_cells()


def test_c4_sampled_cross_counts_bit_exact(c4, oracle_mod):
    _check_probes(c4, oracle_mod)


def test_c4_union_identity(c4):
    _check_union(c4)


def test_c4_whole_auto_task_bit_exact(c4, oracle_mod):
    """One whole estimator task at full size: the DD count of the last mock
    (about 3e5 points, 4.5e10 pair tests in the oracle), every bin."""
    pl, cats, wl = c4["pl"], c4["cats"], c4["cats"].wl
    last = cats.n_mock - 1
    t = int(pl.est[last][0])
    a, b = pl.tasks[t]
    assert a == b == last
    _say("[c4] oracle DD of mock %d: %d points" % (last, cats.sizes()[a]))
    ref = oracle_mod.count_pairs(cats.cat(a), None, wl.r_edges_units, wl.n_mu, 0, "mid")
    _say("[c4] oracle done")
    assert np.array_equal(c4["counts"][t], ref)
    assert ref.sum() > 0


def test_c4_counts_independent_of_tiling(c4, torch):
    pl = c4["pl"]
    tuned = pl.autotune()
    _say("[c4] autotuned:", tuned)
    pl.build_cells()
    pl.count()
    torch.cuda.synchronize()
    assert np.array_equal(pl.counts_host(), c4["counts"])
    pl.tuned = None
    pl.build_cells(int(50.0 * mockgen.UNITS_PER_MPC), 1)
    pl.count(tune=dict(chunk=32, cells_per_item=2, waves_per_block=2))
    torch.cuda.synchronize()
    assert np.array_equal(pl.counts_host(), c4["counts"])
    pl.build_cells()


def test_c4_per_task_launches_identical(c4, torch):
    """One launch per estimator task, mock after mock (the probe tasks are
    not part of that loop and stay zero)."""
    pl = c4["pl"]
    pl.count_per_mock()
    torch.cuda.synchronize()
    n = c4["n_est"]
    got = pl.counts_host()
    assert np.array_equal(got[:n], c4["counts"][:n])
    assert not got[n:].any()
