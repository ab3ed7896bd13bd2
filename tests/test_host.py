"""Host-side logic (CPU only): the binding's task planner, and the library's
map builders (lc_map_multipoles, lc_map_projected, lc_map_rebin_blocks: host
calls of liblc that feed lc_map_vectors / lc_map_matrix), checked against
the oracle's definitions of the quantities they select or combine."""
import numpy as np
import pytest

from paper_2205_11852_amd import pipeline


def test_plan_tasks_counts_shared_rr_once():
    randoms = np.array([[10, 11], [12, 10], [11, 12]])
    tasks, est = pipeline.plan_tasks(3, randoms)
    assert est.shape == (3, 5)
    t = [tuple(x) for x in tasks]
    assert len(t) == len(set(t))                       # every task once
    for m in range(3):
        r1, r2 = randoms[m]
        assert [t[i] for i in est[m]] == [(m, m), (m, r1), (m, r2), (r1, r1), (r2, r2)]
    assert sum(1 for a, b in t if a == b and a >= 10) == 3   # RR of 10, 11, 12 once each


def test_plan_direct_tasks_layout():
    tasks, est = pipeline.plan_direct_tasks([0, 1], [5, 6, 7])
    t = [tuple(x) for x in tasks]
    assert t[:3] == [(5, 5), (6, 6), (7, 7)]
    for row, m in zip(est, (0, 1)):
        assert t[row[0]] == (m, m)
        assert [t[i] for i in row[1:4]] == [(m, 5), (m, 6), (m, 7)]
        assert [t[i] for i in row[4:]] == [(5, 5), (6, 6), (7, 7)]


def test_multipole_map_selects_the_paper_vector(oracle_mod):
    """200 x 100 bins, r = 20 .. 200 Mpc/h in 1 Mpc/h bins: the map picks
    xi_0, xi_2, xi_4 of r bins 20 .. 199 out of the data vector exactly
    (the 540-element vector of Sect. 5.3)."""
    r = np.random.default_rng(1)
    xi = r.normal(size=(200, 100))
    v = oracle_mod.data_vector(xi)
    g, w, P = pipeline.multipole_map(200, 100, 1, 20, 200)
    assert P == 540
    y = oracle_mod.map_vectors(v, g, w, P)
    mp = oracle_mod.multipoles(xi)
    assert np.array_equal(y, mp[:, 20:].ravel())


@pytest.mark.parametrize("w", [2, 7, 20])
def test_multipole_map_rebins_by_averaging(oracle_mod, w):
    n_r, n_mu, lo = 40, 5, 3
    xi = np.random.default_rng(w).normal(size=(n_r, n_mu))
    g, wt, P = pipeline.multipole_map(n_r, n_mu, w, lo, n_r)
    y = oracle_mod.map_vectors(oracle_mod.data_vector(xi), g, wt, P).reshape(3, -1)
    mp = oracle_mod.multipoles(xi)[:, lo:]
    n_out = (n_r - lo + w - 1) // w
    assert y.shape == (3, n_out)
    for j in range(n_out):
        assert np.allclose(y[:, j], mp[:, j * w:(j + 1) * w].mean(axis=1), rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("ells", [(2,), (0, 4), (4,), (0, 2)])
def test_multipole_map_selects_subsets(oracle_mod, ells):
    n_r, n_mu = 12, 7
    xi = np.random.default_rng(len(ells)).normal(size=(n_r, n_mu))
    g, wt, P = pipeline.multipole_map(n_r, n_mu, 1, 2, 11, ells)
    assert P == 9 * len(ells)
    y = oracle_mod.map_vectors(oracle_mod.data_vector(xi), g, wt, P).reshape(len(ells), 9)
    mp = oracle_mod.multipoles(xi)
    for j, ell in enumerate(ells):
        assert np.array_equal(y[j], mp[(0, 2, 4).index(ell), 2:11])
    with pytest.raises(ValueError):
        pipeline.multipole_map(n_r, n_mu, 1, 0, n_r, (4, 0))


def test_block_rebin_map_averages_within_blocks(oracle_mod):
    x = np.arange(3 * 180, dtype=float)
    g, w, P = pipeline.block_rebin_map(3, 180, 20)
    assert P == 27
    y = oracle_mod.map_vectors(x, g, w, P).reshape(3, 9)
    assert np.allclose(y, x.reshape(3, 9, 20).mean(axis=2), rtol=1e-15)
    g, w, P = pipeline.block_rebin_map(2, 7, 3)     # ragged: groups of 3, 3, 1
    y = oracle_mod.map_vectors(np.arange(14.0), g, w, P)
    assert np.allclose(y, [1.0, 4.0, 6.0, 8.0, 11.0, 13.0])


def test_projected_map_is_the_oracle_projection(oracle_mod):
    n_rp, n_pi = 6, 8
    xi = np.random.default_rng(4).normal(size=(n_rp, n_pi))
    g, w, P = pipeline.projected_map(n_rp, n_pi, 40.0)
    y = oracle_mod.map_vectors(oracle_mod.data_vector(xi), g, w, P)
    assert np.allclose(y, oracle_mod.projected(xi, 40.0), rtol=1e-14, atol=1e-14)


def test_map_builders_reject_bad_ranges():
    with pytest.raises(ValueError):
        pipeline.multipole_map(10, 5, 1, 8, 4)
    with pytest.raises(ValueError):
        pipeline.multipole_map(10, 5, 0)
    with pytest.raises(ValueError):
        pipeline.block_rebin_map(3, 0, 2)
