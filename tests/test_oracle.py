"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these retype the oracle's own formulas: they check hand-derived bins
(tests/golden/edge_pairs.txt), exact totals, invariances, closed forms that
follow from the estimator's definition, library routines (numpy covariance,
Legendre quadrature) and the paper's analytic covariance for uniform data.
"""
import math
import os

import numpy as np
import pytest

import mockgen
from tests.fixtures import edge_pairs, two_point_catalogues


# ---------------------------------------------------------------------------
# pair counts: hand-derived edge cases
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("scale", [1, 3, 4096, 2 ** 18 // 5])
def test_edge_pairs_fixture(oracle_mod, scale):
    for row in edge_pairs():
        a, b, edges, box = two_point_catalogues(row, scale=scale)
        n_mu = row["n_mu"]
        got = oracle_mod.count_pairs(a, b, edges, n_mu, box, row["los"])
        exp = np.zeros((len(edges) - 1, n_mu), dtype=np.uint64)
        if row["k"] >= 0:
            exp[row["k"], row["m"]] = 1
        assert np.array_equal(got, exp), (row["note"], scale)
        # the same two points as one catalogue: the single unordered pair
        both = np.concatenate([a, b], axis=1)
        got2 = oracle_mod.count_pairs(both, None, edges, n_mu, box, row["los"])
        assert np.array_equal(got2, exp), (row["note"], scale, "auto")


def test_edge_pairs_translation(oracle_mod):
    """z line of sight: bins do not change under translation (open and periodic)."""
    for row in edge_pairs():
        if row["los"] != "z":
            continue
        for shift in [(5, -7, 11), (123456, 654321, -222222)]:
            a, b, edges, box = two_point_catalogues(row, scale=7, shift=shift)
            got = oracle_mod.count_pairs(a, b, edges, row["n_mu"], box, "z")
            exp = np.zeros_like(got)
            if row["k"] >= 0:
                exp[row["k"], row["m"]] = 1
            assert np.array_equal(got, exp), (row["note"], shift)


# ---------------------------------------------------------------------------
# pair counts: totals, invariances, union identity
# ---------------------------------------------------------------------------

def _rand_pts(seed, n, lo, hi):
    r = np.random.default_rng(seed)
    return r.integers(lo, hi, size=(3, n)).astype(np.int32)


@pytest.mark.parametrize("los", ["z", "mid"])
def test_totals_open_geometry(oracle_mod, los):
    """With the last edge beyond the largest separation every pair is
    counted once: N(N-1)/2 auto pairs, N_a N_b cross pairs."""
    a = _rand_pts(1, 700, -3000, 3000)
    b = _rand_pts(2, 500, -3000, 3000)
    edges = [0, 1000, 4000, 12000]
    for n_mu in (1, 7, 50):
        dd = oracle_mod.count_pairs(a, None, edges, n_mu, 0, los)
        dr = oracle_mod.count_pairs(a, b, edges, n_mu, 0, los)
        assert int(dd.sum()) == 700 * 699 // 2
        assert int(dr.sum()) == 700 * 500


def test_totals_periodic_against_direct_distance_count(oracle_mod):
    """Sum over mu bins equals the number of pairs with e_0 <= r < e_n,
    counted here with a float64 distance (no pair lies within 1e-6 of an
    edge for these inputs, which the test asserts)."""
    L = 100000
    a = _rand_pts(3, 400, 0, L)
    edges = np.array([0, 3000, 9000, 20000, 30000])
    got = oracle_mod.count_pairs(a, None, edges, 9, L, "z").sum(axis=1)
    x = a.astype(np.float64)
    s = x[:, None, :] - x[:, :, None]
    s = (s + L / 2) % L - L / 2
    r = np.sqrt((s ** 2).sum(axis=0))
    iu = np.triu_indices(a.shape[1], 1)
    rr = r[iu]
    assert np.min(np.abs(rr[:, None] - edges[None, :])) > 1e-6
    exp = np.histogram(rr, bins=edges.astype(np.float64))[0]
    assert np.array_equal(got.astype(np.int64), exp)


def test_invariances_periodic(oracle_mod):
    L = 1 << 20
    a = _rand_pts(4, 600, 0, L)
    b = _rand_pts(5, 500, 0, L)
    edges = np.arange(0, 11) * 20000
    n_mu = 12
    base_dd = oracle_mod.count_pairs(a, None, edges, n_mu, L)
    base_dr = oracle_mod.count_pairs(a, b, edges, n_mu, L)
    # translation by an integer vector modulo L
    t = np.array([[123457], [L - 5], [777777]])
    at, bt = (a + t) % L, (b + t) % L
    assert np.array_equal(oracle_mod.count_pairs(at, None, edges, n_mu, L), base_dd)
    assert np.array_equal(oracle_mod.count_pairs(at, bt, edges, n_mu, L), base_dr)
    # swapping x and y (z line of sight unchanged)
    assert np.array_equal(oracle_mod.count_pairs(a[[1, 0, 2]], b[[1, 0, 2]], edges, n_mu, L), base_dr)
    # reflecting z -> -z (mod L)
    ar, br = a.copy(), b.copy()
    ar[2] = (L - ar[2]) % L
    br[2] = (L - br[2]) % L
    assert np.array_equal(oracle_mod.count_pairs(ar, br, edges, n_mu, L), base_dr)
    # point order
    p = np.random.default_rng(0).permutation(a.shape[1])
    assert np.array_equal(oracle_mod.count_pairs(a[:, p], None, edges, n_mu, L), base_dd)
    # cross counts are symmetric in the two catalogues
    assert np.array_equal(oracle_mod.count_pairs(b, a, edges, n_mu, L), base_dr)


@pytest.mark.parametrize("box,los", [(1 << 20, "z"), (0, "z"), (0, "mid")])
def test_union_identity(oracle_mod, box, los):
    """DD(A u B) = DD(A) + DD(B) + DR(A, B)."""
    lo, hi = (0, box) if box else (1 << 18, 1 << 19)
    a = _rand_pts(6, 500, lo, hi)
    b = _rand_pts(7, 400, lo, hi)
    edges = np.arange(0, 9) * 15000
    ab = np.concatenate([a, b], axis=1)
    lhs = oracle_mod.count_pairs(ab, None, edges, 10, box, los)
    rhs = (oracle_mod.count_pairs(a, None, edges, 10, box, los)
           + oracle_mod.count_pairs(b, None, edges, 10, box, los)
           + oracle_mod.count_pairs(a, b, edges, 10, box, los))
    assert np.array_equal(lhs, rhs)


def test_midpoint_rotation_invariance(oracle_mod):
    """Midpoint line of sight: a rotation by 90 degrees about any axis through
    the observer permutes and negates coordinates and keeps every bin."""
    a = _rand_pts(8, 300, -(1 << 20), 1 << 20)
    b = _rand_pts(9, 300, -(1 << 20), 1 << 20)
    edges = np.arange(0, 9) * 150000
    base = oracle_mod.count_pairs(a, b, edges, 10, 0, "mid")
    rot = lambda p: np.stack([-p[1], p[0], p[2]]).astype(np.int32)
    assert np.array_equal(oracle_mod.count_pairs(rot(a), rot(b), edges, 10, 0, "mid"), base)
    refl = lambda p: np.stack([p[0], p[1], -p[2]]).astype(np.int32)
    assert np.array_equal(oracle_mod.count_pairs(refl(a), refl(b), edges, 10, 0, "mid"), base)


def test_uniform_counts_match_shell_volume(oracle_mod):
    """Uniform points in a periodic box: E[RR_km] = N(N-1)/2 * G_p(k, m), with
    G_p = (4pi/3)(r_k+1^3 - r_k^3)/(L^3 n_mu) (mu uniform in [0, 1] for an
    isotropic separation).  Checked with a chi-square over the bins."""
    L = 1 << 22
    n = 3000
    pts = mockgen.uniform_box(np.random.default_rng(11), n, L)
    edges = np.linspace(0, L // 4, 9).astype(np.int64)
    n_mu = 5
    got = oracle_mod.count_pairs(pts, None, edges, n_mu, L).astype(np.float64)
    exp = n * (n - 1) / 2 * oracle_mod.shell_pair_fraction(edges, n_mu, L)
    chi2 = float(((got - exp) ** 2 / exp).sum())
    dof = got.size
    assert abs(chi2 - dof) < 6 * math.sqrt(2 * dof), chi2
    # the total within r_max has a relative scatter of about 1/sqrt(pairs)
    assert abs(got.sum() / exp.sum() - 1) < 0.02


# ---------------------------------------------------------------------------
# estimator
# ---------------------------------------------------------------------------

def test_ls_data_equals_random_closed_form(oracle_mod):
    """With the random catalogue equal to the data (R = D, N points):
    DR(D, D) = 2 DD away from r = 0 and RR = DD, so the estimator is
    (dd - 2 dr)/rr + 1 = 2 - 2 (N-1)/N = 2/N exactly.  The same holds for the
    split M = 2 estimate with R1 = R2 = D."""
    n = 400
    L = 1 << 20
    d = _rand_pts(12, n, 0, L)
    edges = np.arange(1, 12) * 30000           # e_0 > 0: no zero-separation pairs
    DD = oracle_mod.count_pairs(d, None, edges, 4, L)
    DR = oracle_mod.count_pairs(d, d, edges, 4, L)
    assert np.array_equal(DR, 2 * DD)
    xi1 = oracle_mod.ls_split(DD, [DR], [DD], n, [n])
    xi2 = oracle_mod.ls_split(DD, [DR, DR], [DD, DD], n, [n, n])
    ok = DD > 0
    assert np.allclose(xi1[ok], 2.0 / n, rtol=1e-12, atol=0)
    assert np.allclose(xi2[ok], 2.0 / n, rtol=1e-12, atol=0)
    assert np.all(np.isnan(xi1[~ok]))


def test_ls_doubled_random_closed_form(oracle_mod):
    """Random catalogue = every data point twice (N_r = 2N): DR = 2 DR(D,D),
    RR = 4 DD (+N coincident pairs at r = 0, excluded by e_0 > 0).  Then
    dd = 2DD/(N(N-1)), dr = 2DD/N^2, rr = 4DD/(N(2N-1)), and
    xi = (2N-1)/(2(N-1)) - (2N-1)/N + 1, independent of the counts.
    This fixes the DR and RR normalisations for N_r != N_d."""
    n = 300
    L = 1 << 20
    d = _rand_pts(13, n, 0, L)
    r = np.concatenate([d, d], axis=1)
    edges = np.arange(1, 10) * 40000
    DD = oracle_mod.count_pairs(d, None, edges, 3, L)
    DR = oracle_mod.count_pairs(d, r, edges, 3, L)
    RR = oracle_mod.count_pairs(r, None, edges, 3, L)
    assert np.array_equal(RR, 4 * DD)
    xi = oracle_mod.ls_split(DD, [DR], [RR], n, [2 * n])
    exp = (2 * n - 1) / (2 * (n - 1)) - (2 * n - 1) / n + 1
    ok = DD > 0
    assert np.allclose(xi[ok], exp, rtol=1e-12, atol=1e-15)


# ---------------------------------------------------------------------------
# multipoles
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n_mu", [1, 5, 10, 50, 100])
def test_legendre_weights_against_quadrature(oracle_mod, n_mu):
    """W[l, m] against Gauss-Legendre quadrature of (2l+1) P_l on each bin
    (numpy's Legendre module: an independent evaluation of P_l)."""
    from numpy.polynomial import legendre as npl
    W = oracle_mod.legendre_weights(n_mu)
    xg, wg = npl.leggauss(8)
    for li, ell in enumerate((0, 2, 4)):
        c = np.zeros(ell + 1)
        c[ell] = 1.0
        for m in range(n_mu):
            a, b = m / n_mu, (m + 1) / n_mu
            x = 0.5 * (b - a) * xg + 0.5 * (b + a)
            q = (2 * ell + 1) * 0.5 * (b - a) * np.sum(wg * npl.legval(x, c))
            assert abs(W[li, m] - q) < 1e-14
    # sums over mu: integral of P_0 over [0,1] is 1, of P_2 and P_4 is 0
    assert abs(W[0].sum() - 1) < 1e-14
    assert abs(W[1].sum()) < 1e-13 and abs(W[2].sum()) < 1e-13


def test_multipoles_of_legendre_shapes(oracle_mod):
    """A xi that is the bin average of c0 + c2 P_2 + c4 P_4 gives back
    (c0, c2, c4) as n_mu grows (orthogonality of P_l); constant xi gives
    exactly (c, 0, 0)."""
    from numpy.polynomial import legendre as npl
    n_mu = 2000
    e = np.arange(n_mu + 1) / n_mu
    coef = np.array([0.7, 0.0, -1.3, 0.0, 0.4])
    F = npl.legval(e, npl.legint(coef))
    xi = ((F[1:] - F[:-1]) * n_mu)[None, :].repeat(3, axis=0)
    mp = oracle_mod.multipoles(xi)
    assert np.allclose(mp[:, 0], [0.7, -1.3, 0.4], atol=2e-6)
    const = np.full((4, 10), 0.25)
    mc = oracle_mod.multipoles(const)
    assert np.allclose(mc[0], 0.25, atol=1e-15) and np.allclose(mc[1:], 0.0, atol=1e-15)


def test_data_vector_layout(oracle_mod):
    xi = np.arange(12.0).reshape(3, 4)
    v = oracle_mod.data_vector(xi)
    assert v.shape == (12 + 9,)
    assert np.array_equal(v[:12], xi.ravel())
    assert np.allclose(v[12:15], xi.mean(axis=1))        # xi_0 = bin average over mu


# ---------------------------------------------------------------------------
# covariance and linear construction
# ---------------------------------------------------------------------------

def test_sample_cov_matches_numpy(oracle_mod):
    V = np.random.default_rng(3).normal(size=(57, 9)) * np.arange(1, 10)
    assert np.allclose(oracle_mod.sample_cov(V), np.cov(V, rowvar=False), rtol=1e-13, atol=1e-15)


def _general_reconstruction(Ca, Cb, Ma, Mb):
    """A and B from two random-catalogue sizes M_a < M_b (Sect. 2.2, general
    form): A = (M_b C(M_b) - M_a C(M_a)) / (M_b - M_a),
    B = M_a M_b (C(M_a) - C(M_b)) / (M_b - M_a)."""
    A = (Mb * Cb - Ma * Ca) / (Mb - Ma)
    B = Ma * Mb * (Ca - Cb) / (Mb - Ma)
    return A, B


@pytest.mark.parametrize("m_a", [1, 2, 3])
def test_lc_equals_general_reconstruction(oracle_mod, m_a):
    """The component matrices of the linear construction (Sect. 2.3) are the
    general two-size reconstruction of Sect. 2.2 at M_b = 2 M_a."""
    r = np.random.default_rng(m_a)
    X = r.normal(size=(6, 6))
    Ca = X @ X.T
    Cb = 0.6 * Ca + 0.1 * np.eye(6)
    A, B, C = oracle_mod.linear_construction(Ca, Cb, m_a, 50.0)
    A2, B2 = _general_reconstruction(Ca, Cb, m_a, 2 * m_a)
    assert np.allclose(A, A2, rtol=1e-13) and np.allclose(B, B2, rtol=1e-13)


def test_lc_recovers_exact_model(oracle_mod):
    """If C(M) = A0 + B0/M exactly, C^a = C(M_a) and C^b = C(2 M_a) give back
    A0, B0 and C(M) for every M, including M -> infinity."""
    r = np.random.default_rng(5)
    X, Y = r.normal(size=(5, 5)), r.normal(size=(5, 5))
    A0, B0 = X @ X.T, Y @ Y.T
    for m_a in (1, 4):
        Ca, Cb = A0 + B0 / m_a, A0 + B0 / (2 * m_a)
        for M in (1.0, 2.0, 7.5, 50.0, np.inf):
            A, B, C = oracle_mod.linear_construction(Ca, Cb, m_a, M)
            assert np.allclose(A, A0, rtol=1e-12, atol=1e-12)
            assert np.allclose(B, B0, rtol=1e-12, atol=1e-12)
            exp = A0 if np.isinf(M) else A0 + B0 / M
            assert np.allclose(C, exp, rtol=1e-12, atol=1e-12)
        # the construction reproduces its inputs at M = M_a and M = 2 M_a
        assert np.allclose(oracle_mod.linear_construction(Ca, Cb, m_a, m_a)[2], Ca)
        assert np.allclose(oracle_mod.linear_construction(Ca, Cb, m_a, 2 * m_a)[2], Cb)


def test_check_matrix(oracle_mod):
    rep = oracle_mod.check_matrix(np.diag([3.0, 1.0, 2.0]))
    assert rep == {"chol_ok": 1, "n_neg_eig": 0, "min_eig": 1.0, "max_eig": 3.0}
    rep = oracle_mod.check_matrix(np.diag([3.0, -1.0, -2.0]))
    assert rep["chol_ok"] == 0 and rep["n_neg_eig"] == 2 and rep["min_eig"] == -2.0


# ---------------------------------------------------------------------------
# statistical pin: uniform data with independent randoms (Sect. 4.2, 5.1)
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def poisson_mock_vectors(oracle_mod):
    n_mock, n, L = 240, 800, 1 << 20
    xyz, off, ids = mockgen.independent_poisson_mocks(77, n_mock, n, L)
    edges = np.linspace(L // 40, L // 8, 9).astype(np.int64)
    n_mu = 1
    V = []
    for m in range(n_mock):
        cd, c1, c2 = (xyz[:, off[i]:off[i + 1]] for i in ids[m])
        DD, DR1, DR2, RR1, RR2 = oracle_mod.mock_counts(cd, c1, c2, edges, n_mu, L, "z")
        x1 = oracle_mod.ls_split(DD, [DR1], [RR1], n, [n]).ravel()
        x2 = oracle_mod.ls_split(DD, [DR2], [RR2], n, [n]).ravel()
        y = oracle_mod.ls_split(DD, [DR1, DR2], [RR1, RR2], n, [n, n]).ravel()
        V.append([x1, x2, y])
    G_p = oracle_mod.shell_pair_fraction(edges, n_mu, L).ravel()
    return np.array(V), n, G_p


def test_uniform_data_xi_unbiased(poisson_mock_vectors):
    V, n, G_p = poisson_mock_vectors
    mean = V[:, 2].mean(axis=0)
    sd = V[:, 2].std(axis=0, ddof=1) / math.sqrt(V.shape[0])
    assert np.all(np.abs(mean) < 4.5 * sd)


def test_lc_diagonal_matches_random_theory(oracle_mod, poisson_mock_vectors):
    """diag C^LC(M) for uniform data against the paper's analytic variance
    (2/(N_d(N_d-1)) + 4/(N_d N_r) + 2/(N_r(N_d-1)))/G_p with N_r = M N_d.
    At M = 1 and M = 2 the construction returns C^a and C^b; M = infinity is A.
    The tolerance is about 4 standard errors of the bin-averaged ratio."""
    V, n, G_p = poisson_mock_vectors
    A, B, C, Ca, Cb = oracle_mod.lc_from_vectors(V, 1, 50.0)
    for M, tol in ((1.0, 0.08), (2.0, 0.09), (50.0, 0.25), (np.inf, 0.3)):
        CM = A if np.isinf(M) else A + B / M
        if np.isinf(M):
            theory = 2.0 / (n * (n - 1.0)) / G_p
        else:
            theory = oracle_mod.random_theory_variance(n, M * n, G_p)
        ratio = np.diag(CM) / theory
        assert abs(ratio.mean() - 1.0) < tol, (M, ratio)


def test_lc_matches_direct_large_random_covariance(oracle_mod):
    """The linear construction predicts the covariance at any random-catalogue
    size M from the M = 1 and M = 2 estimates (Sect. 2.3): compare with the
    sample covariance of the split estimator computed directly with M = 6
    random sub-catalogues per mock, on the same uniform mocks.  Over seeds the
    mean diagonal ratio is 0.96 +- 0.03 (600 mocks of 600 points); using the
    M = 2 covariance instead would give about 5/3."""
    n_mock, n, L, M = 600, 600, 1 << 20, 6
    xyz, off, ids = mockgen.independent_poisson_mocks(101, n_mock, n, L, n_random=M)
    edges = np.linspace(L // 40, L // 8, 9).astype(np.int64)
    V, X = [], []
    for m in range(n_mock):
        c = [xyz[:, off[i]:off[i + 1]] for i in ids[m]]
        DD = oracle_mod.count_pairs(c[0], None, edges, 1, L, "z")
        DR = [oracle_mod.count_pairs(c[0], c[1 + r], edges, 1, L, "z") for r in range(M)]
        RR = [oracle_mod.count_pairs(c[1 + r], None, edges, 1, L, "z") for r in range(M)]
        x1 = oracle_mod.ls_split(DD, DR[:1], RR[:1], n, [n]).ravel()
        x2 = oracle_mod.ls_split(DD, DR[1:2], RR[1:2], n, [n]).ravel()
        y = oracle_mod.ls_split(DD, DR[:2], RR[:2], n, [n, n]).ravel()
        V.append([x1, x2, y])
        X.append(oracle_mod.ls_split(DD, DR, RR, n, [n] * M).ravel())
    A, B, C, Ca, Cb = oracle_mod.lc_from_vectors(np.array(V), 1, float(M))
    direct = np.diag(oracle_mod.sample_cov(np.array(X)))
    ratio = np.diag(C) / direct
    assert abs(ratio.mean() - 1.0) < 0.1, ratio
    assert np.all((ratio > 0.6) & (ratio < 1.5)), ratio
    # the M = 2 covariance is measurably larger than the M = 6 one
    assert np.diag(Cb).mean() / direct.mean() > 1.3


# ---------------------------------------------------------------------------
# covariance of the covariance estimates (Sect. 3) and Table 3 (Sect. 5.3)
# ---------------------------------------------------------------------------

def _exchangeable(P, seed):
    """Covariances S = Cov(x), T = Cov(x, x') of two exchangeable Gaussian
    estimate vectors (a valid joint covariance [[S, T], [T, S]])."""
    r = np.random.default_rng(seed)
    G = r.normal(size=(2 * P, 2 * P))
    J = G @ G.T + 0.5 * np.eye(2 * P)
    S = 0.5 * (J[:P, :P] + J[P:, P:])
    T = 0.5 * (J[:P, P:] + J[P:, :P])
    return S, 0.5 * (T + T.T)


@pytest.mark.parametrize("m_a,M", [(1, 50.0), (1, 2.0), (2, 7.0), (1, np.inf)])
def test_lc_element_var_equals_term_by_term_expansion(oracle_mod, m_a, M):
    """C^LC = a [c(x,x') + c(x',x)] + b [c(x,x) + c(x',x')] (Sect. 3.3) with
    a = (1 - M_a/M)/2, b = M_a/(2M); expand Var(C^LC_ij) over the 16 products
    with the Gaussian covariance of sample covariances, and compare with the
    compact form (which needs D = A + B/(2 M_a))."""
    P, N = 5, 40
    S, T = _exchangeable(P, 3 + m_a)
    A, B = T, m_a * (S - T)           # ensemble C^a = S, C^b = (S + T)/2
    inv_m = 0.0 if np.isinf(M) else 1.0 / M
    a, b = 0.5 * (1.0 - m_a * inv_m), 0.5 * m_a * inv_m

    def E(p, q):
        return S[p[1], q[1]] if p[0] == q[0] else T[p[1], q[1]]

    def covc(u, v, w, z):             # Cov[c(u, v), c(w, z)] for Gaussian u, v, w, z
        return (E(u, w) * E(v, z) + E(u, z) * E(v, w)) / (N - 1)

    var = oracle_mod.lc_cov_element_var(A, B, m_a, M, N)
    for i in range(P):
        for j in range(P):
            terms = [(a, (0, i), (1, j)), (a, (1, i), (0, j)), (b, (0, i), (0, j)), (b, (1, i), (1, j))]
            exact = sum(c1 * c2 * covc(u1, v1, u2, v2) for c1, u1, v1 in terms for c2, u2, v2 in terms)
            assert abs(var[i, j] - exact) <= 1e-12 * abs(exact)


def test_covariance_element_vars_monte_carlo(oracle_mod):
    """Gaussian x, x' with a known joint covariance, N = 12 realisations per
    trial: the spread over 20000 trials of the sample covariance and of the LC
    covariance built from c^a = (c(x) + c(x'))/2 and c^b = c((x + x')/2)
    matches the predicted element variances (Sect. 3.2, 3.3)."""
    P, N, trials, m_a, M = 3, 12, 20000, 1, 10.0
    S, T = _exchangeable(P, 11)
    J = np.block([[S, T], [T, S]])
    L = np.linalg.cholesky(J)
    r = np.random.default_rng(12)
    z = r.normal(size=(trials, N, 2 * P)) @ L.T
    x, xp = z[..., :P], z[..., P:]

    def scov(v):
        d = v - v.mean(axis=1, keepdims=True)
        return np.einsum("tni,tnj->tij", d, d) / (N - 1)

    ca = 0.5 * (scov(x) + scov(xp))
    cb = scov(0.5 * (x + xp))
    C = (2 * cb - ca) + 2 * m_a * (ca - cb) / M
    var_lc = C.var(axis=0, ddof=1)
    var_smp = scov(x).var(axis=0, ddof=1)
    A, B = T, m_a * (S - T)
    pred_lc = oracle_mod.lc_cov_element_var(A, B, m_a, M, N)
    pred_smp = oracle_mod.sample_cov_element_var(S, N)
    # the sample variance of 20000 draws is within about 3% of its mean
    assert np.all(np.abs(var_lc / pred_lc - 1.0) < 0.06), var_lc / pred_lc
    assert np.all(np.abs(var_smp / pred_smp - 1.0) < 0.06), var_smp / pred_smp


def _golden(name):
    rows = []
    for line in open(os.path.join(os.path.dirname(__file__), "golden", name)):
        if line.strip() and not line.startswith("#"):
            rows.append(line.split())
    return rows


def test_poisson_mock_std_ratio_matches_paper(oracle_mod):
    """Sect. 5.1: for random mocks at M = 50 the LC covariance's diagonal has
    2.7 times the standard deviation of the sample covariance's.  Their
    covariance is diagonal with C(M) ~ 1 + 3/M, i.e. A : B = 1 : 3."""
    g = {k: float(v) for k, v in _golden("poisson_std_ratio.txt")}
    M, m_a = g["M"], int(g["m_a"])
    A, B = np.eye(4), 3.0 * np.eye(4)
    ratio = np.sqrt(oracle_mod.lc_cov_element_var(A, B, m_a, M, 100)[0, 0]
                    / oracle_mod.sample_cov_element_var(A + B / M, 100)[0, 0])
    assert abs(ratio - g["ratio"]) < 0.05, ratio
    # the printed definition D = A + B/M_a would give about 4.0
    D_printed = A + B / m_a
    f = 1.0 / (2 * m_a) - 1.0 / M
    alt = np.sqrt((2 * D_printed[0, 0] ** 2 + f * f * 2 * B[0, 0] ** 2) / (2 * (A + B / M)[0, 0] ** 2))
    assert abs(alt - g["ratio"]) > 1.0


def _last_digit(txt):
    return 10.0 ** -(len(txt.split(".")[1]) if "." in txt else 0)


def test_table3_costs_and_figures_of_merit(oracle_mod):
    """Table 3: the pair-count cost per realisation (1 + 3M for the sample
    covariance, 7 for LC with M_a = 1), iFoM = cost x chi^2_2 and the ratio of
    the two iFoMs.  The printed iFoMs and ratios were formed from unrounded
    chi^2_2 and are themselves rounded (some LC values at M = 50 look
    truncated), so each is allowed one unit of its last printed digit plus
    the rounding of the printed chi^2_2."""
    for row in _golden("table3_covcov.txt"):
        M, dr, c_smp, c_lc, x_smp, x_lc, f_smp, f_lc, ratio = map(float, row)
        assert oracle_mod.pair_cost_sample(M) == c_smp
        assert oracle_mod.pair_cost_lc(1) == c_lc
        i_smp, i_lc = c_smp * x_smp, c_lc * x_lc
        assert abs(i_smp - f_smp) <= _last_digit(row[6]) + c_smp * 5e-4, row
        assert abs(i_lc - f_lc) <= _last_digit(row[7]) + c_lc * 5e-4, row
        assert abs(i_smp / i_lc - ratio) <= _last_digit(row[8]) + 0.01 * ratio, row


def _golden_value(txt):
    from fractions import Fraction
    if "/" in txt:
        num, den = txt.split("/")
        return float(Fraction(num) / Fraction(den))
    return float(Fraction(txt))


def _golden_matrix(txt, P):
    if txt == "-":
        return None
    if txt == "0":
        return np.zeros((P, P))
    if txt.startswith("I*"):
        return float(txt[2:]) * np.eye(P)
    return np.array([[float(v) for v in row.split(",")] for row in txt.split(";")])


def test_chi2_2_hand_derived_closed_forms(oracle_mod):
    """<chi^2_2> of both estimators, the pair-count costs and the iFoMs
    against values summed by hand (tests/golden/chi2_2_closed_forms.txt,
    with the derivations; Sect. 2.3, 3.2, 3.3, 5.3).  The cases separate the
    normalisation 1/P^2, the C_ii C_jj and C_ij^2 terms, D = A + B/(2 M_a),
    the factor f^2 and the reference diagonal."""
    for row in _golden("chi2_2_closed_forms.txt"):
        name, P, m_a, M = row[0], int(row[1]), int(row[2]), float(row[3])
        A, B = _golden_matrix(row[4], P), _golden_matrix(row[5], P)
        ref = _golden_matrix(row[6], P)
        x_smp, x_lc, c_smp, c_lc = (_golden_value(v) for v in row[7:11])
        s = oracle_mod.covcov_summary(A, B, m_a, M, ref)
        assert abs(s["chi2_2_smp"] - x_smp) <= 1e-12 * x_smp, (name, P, s["chi2_2_smp"], x_smp)
        assert abs(s["chi2_2_lc"] - x_lc) <= 1e-12 * x_lc, (name, P, s["chi2_2_lc"], x_lc)
        assert s["cost_smp"] == c_smp and s["cost_lc"] == c_lc, (name, s["cost_smp"], s["cost_lc"])
        assert abs(s["ifom_lc"] - c_lc * x_lc) <= 1e-12 * c_lc * x_lc
        assert abs(s["gain"] - (c_smp * x_smp) / (c_lc * x_lc)) <= 1e-12 * s["gain"]


def test_lc_pair_cost_counts_dd_once(oracle_mod):
    """Sect. 2.3: the split estimator at ratio M costs N_d^2/2 (1 + 3M); LC
    runs it twice at ratio M_a, 2 x N_d^2/2 (1 + 3 M_a), and counting DD once
    removes one N_d^2/2: 1 + 6 M_a.  The paper's M = 50, M_a = 1 gain
    151/7."""
    for m_a in (1, 2, 3, 5):
        assert oracle_mod.pair_cost_lc(m_a) == 2 * oracle_mod.pair_cost_sample(m_a) - 1
    assert oracle_mod.pair_cost_lc(1) == 7 and oracle_mod.pair_cost_lc(2) == 13
    assert abs(oracle_mod.pair_cost_sample(50) / oracle_mod.pair_cost_lc(1) - 21.6) < 0.05


def test_chi2_2_monte_carlo(oracle_mod):
    """<chi^2_2> by simulation, with no use of the variance formulas: Gaussian
    estimates x, x' with a known joint covariance, N = 2 realisations per
    trial, 200000 trials.  The spread of every element of the sample
    covariance and of the LC covariance (c^a = (c(x) + c(x'))/2, c^b from
    (x + x')/2, M_a = 1) over the trials, divided by Cref_ii Cref_jj and
    averaged over the P^2 elements, is the definition of Eq. chi2 at N = 2;
    covcov_summary must agree within the Monte Carlo error."""
    P, N, trials, m_a, M = 3, 2, 200000, 1, 10.0
    S, T = _exchangeable(P, 17)
    J = np.block([[S, T], [T, S]])
    L = np.linalg.cholesky(J)
    r = np.random.default_rng(18)
    z = r.normal(size=(trials, N, 2 * P)) @ L.T
    x, xp = z[..., :P], z[..., P:]

    def scov(v):
        d = v - v.mean(axis=1, keepdims=True)
        return np.einsum("tni,tnj->tij", d, d) / (N - 1)

    ca = 0.5 * (scov(x) + scov(xp))
    cb = scov(0.5 * (x + xp))
    C_lc = (2 * cb - ca) + 2 * m_a * (ca - cb) / M
    A, B = T, m_a * (S - T)            # ensemble C^a = S, C^b = (S + T)/2
    C_M = A + B / M                    # the covariance the LC estimates
    # the sample covariance of an estimate with that covariance
    Lm = np.linalg.cholesky(C_M)
    w = r.normal(size=(trials, N, P)) @ Lm.T
    C_smp = scov(w)
    d = np.diag(C_M)
    mc_lc = float((C_lc.var(axis=0, ddof=1) / np.outer(d, d)).mean())
    mc_smp = float((C_smp.var(axis=0, ddof=1) / np.outer(d, d)).mean())
    s = oracle_mod.covcov_summary(A, B, m_a, M)
    assert abs(s["chi2_2_lc"] / mc_lc - 1.0) < 0.03, (s["chi2_2_lc"], mc_lc)
    assert abs(s["chi2_2_smp"] / mc_smp - 1.0) < 0.03, (s["chi2_2_smp"], mc_smp)


def test_covcov_summary_consistency(oracle_mod):
    """covcov_summary: chi^2_2 of the sample covariance equals the LC one when
    M = 2 M_a (the two estimators coincide there, Sect. 3.3), and the gain is
    the ratio of the iFoMs."""
    S, T = _exchangeable(6, 21)
    A, B = T, S - T
    s2 = oracle_mod.covcov_summary(A, B, 1, 2.0)
    assert abs(s2["chi2_2_lc"] - s2["chi2_2_smp"]) <= 1e-12 * s2["chi2_2_smp"]
    s50 = oracle_mod.covcov_summary(A, B, 1, 50.0)
    assert abs(s50["gain"] - s50["ifom_smp"] / s50["ifom_lc"]) < 1e-12 * s50["gain"]
    assert s50["cost_smp"] == 151.0 and s50["cost_lc"] == 7.0


# ---------------------------------------------------------------------------
# co-added counts, linear maps, general M_a and M_b (Sect. 2.3, 4.3, 5.3)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("box,los", [(1 << 20, "z"), (0, "z"), (0, "mid")])
def test_rebin_counts_equals_counting_in_wide_bins(oracle_mod, box, los):
    """Co-added counts are the counts in the wider bins, counted directly by
    brute force with the co-added edges: for ragged r groups, mu groups that
    divide n_mu, and the 1D count over all mu (Sect. 4.3)."""
    lo = 0 if box else 1 << 21
    a = _rand_pts(31, 500, lo, lo + (1 << 20) if not box else box)
    b = _rand_pts(32, 400, lo, lo + (1 << 20) if not box else box)
    edges = np.array([0, 3000, 9000, 20000, 26000, 41000, 60000, 61000], dtype=np.int64)
    n_mu = 12
    for bb in (None, b):
        fine = oracle_mod.count_pairs(a, bb, edges, n_mu, box, los)
        for w_r, w_mu in ((1, 1), (3, 2), (2, 3), (7, 12), (4, 12), (5, 4)):
            got = oracle_mod.rebin_counts(fine, w_r, w_mu)
            e2 = oracle_mod.rebinned_edges(edges, w_r)
            ref = oracle_mod.count_pairs(a, bb, e2, n_mu // w_mu, box, los)
            assert np.array_equal(got, ref), (w_r, w_mu)
            assert got.sum() == fine.sum()


def test_rebinned_edges(oracle_mod):
    assert oracle_mod.rebinned_edges([0, 1, 2, 3, 4, 5, 6, 7], 3) == [0, 3, 6, 7]
    assert oracle_mod.rebinned_edges([0, 1, 2, 3, 4], 2) == [0, 2, 4]
    assert oracle_mod.rebinned_edges([5, 9], 1) == [5, 9]


def test_one_dimensional_xi_from_co_added_counts(oracle_mod):
    """The 1D correlation function is the estimator applied to counts
    co-added over mu (Sect. 4.3); its data vector has xi_0 = xi and
    xi_2 = xi_4 = 0 exactly (P_2 and P_4 integrate to zero over [0, 1])."""
    L = 1 << 20
    d, r1, r2 = _rand_pts(41, 600, 0, L), _rand_pts(42, 600, 0, L), _rand_pts(43, 600, 0, L)
    edges = np.linspace(0, L // 8, 7).astype(np.int64)
    c = oracle_mod.mock_counts(d, r1, r2, edges, 10, L, "z")
    c1 = [oracle_mod.rebin_counts(x, 1, 10) for x in c]
    V = oracle_mod.mock_vectors(*c1, 600, 600, 600)
    n_r = len(edges) - 1
    for q in range(3):
        xi1 = V[q, :n_r]
        assert np.array_equal(V[q, n_r:2 * n_r], xi1)
        assert np.all(V[q, 2 * n_r:] == 0.0)
    # and it is the estimator of counts made with one mu bin directly
    direct = oracle_mod.mock_counts(d, r1, r2, edges, 1, L, "z")
    assert all(np.array_equal(x, y) for x, y in zip(c1, direct))


def test_linear_map_small_example(oracle_mod):
    """Hand-computed: elements 0 and 1 averaged, 2 kept, 3 dropped."""
    g, w = [0, 0, 1, -1], [0.5, 0.5, 1.0, 1.0]
    x = np.array([1.0, 3.0, 5.0, 7.0])
    assert np.array_equal(oracle_mod.map_vectors(x, g, w, 2), [2.0, 5.0])
    C = np.arange(16.0).reshape(4, 4)
    # Y_00 = (C00 + C01 + C10 + C11)/4, Y_01 = (C02 + C12)/2, Y_11 = C22
    Y = oracle_mod.map_matrix(C, g, w, 2)
    assert np.allclose(Y, [[(0 + 1 + 4 + 5) / 4, (2 + 6) / 2], [(8 + 9) / 2, 10]], rtol=0, atol=1e-15)


def test_map_matrix_is_covariance_of_mapped_vectors(oracle_mod):
    """Cov(T x) = T Cov(x) T^T: re-binning the covariance (Sect. 5.3) equals
    the covariance of the re-binned vectors."""
    r = np.random.default_rng(12)
    P, P_out, N = 30, 11, 200
    V = r.normal(size=(N, P)) @ r.normal(size=(P, P))
    g = r.integers(-1, P_out, size=P)
    w = r.normal(size=P)
    lhs = oracle_mod.map_matrix(oracle_mod.sample_cov(V), g, w, P_out)
    rhs = oracle_mod.sample_cov(oracle_mod.map_vectors(V, g, w, P_out))
    assert np.allclose(lhs, rhs, rtol=1e-11, atol=1e-11 * np.abs(rhs).max())


@pytest.mark.parametrize("m_a,m_b", [(1.0, 2.0), (1.0, 3.0), (2.0, 5.0), (0.5, 4.0), (3.0, 6.0)])
def test_general_construction_recovers_exact_model(oracle_mod, m_a, m_b):
    """Eq. CovAB: if C(M) = A0 + B0/M exactly, the covariances at M_a and M_b
    give back A0 and B0, C(M) for any M, and the inputs at M = M_a, M_b."""
    r = np.random.default_rng(int(10 * m_a + m_b))
    X, Y = r.normal(size=(6, 6)), r.normal(size=(6, 6))
    A0, B0 = X @ X.T, Y @ Y.T
    Ca, Cb = A0 + B0 / m_a, A0 + B0 / m_b
    for M in (1.0, 7.5, 50.0, np.inf):
        A, B, C = oracle_mod.linear_construction_general(Ca, Cb, m_a, m_b, M)
        assert np.allclose(A, A0, rtol=1e-12, atol=1e-12)
        assert np.allclose(B, B0, rtol=1e-12, atol=1e-12)
        assert np.allclose(C, A0 if np.isinf(M) else A0 + B0 / M, rtol=1e-12, atol=1e-12)
    assert np.allclose(oracle_mod.linear_construction_general(Ca, Cb, m_a, m_b, m_a)[2], Ca)
    assert np.allclose(oracle_mod.linear_construction_general(Ca, Cb, m_a, m_b, m_b)[2], Cb)
    if m_b == 2 * m_a:
        ref = oracle_mod.linear_construction(Ca, Cb, int(m_a), 50.0)
        got = oracle_mod.linear_construction_general(Ca, Cb, m_a, m_b, 50.0)
        assert all(np.allclose(x, y, rtol=1e-13, atol=0) for x, y in zip(got, ref))


def test_general_construction_matches_random_theory(oracle_mod):
    """Uniform mocks with M_a = 1 (x from R1, x' from R2) and M_b = 3 (y split
    over R1, R2, R3): the diagonal of C(M) follows the analytic variance for
    uniform data at M = 1, 3 and 20, and at M = infinity its first term."""
    n_mock, n, L = 240, 700, 1 << 20
    xyz, off, ids = mockgen.independent_poisson_mocks(91, n_mock, n, L, n_random=3)
    edges = np.linspace(L // 40, L // 8, 9).astype(np.int64)
    V = []
    for m in range(n_mock):
        c = [xyz[:, off[i]:off[i + 1]] for i in ids[m]]
        DD = oracle_mod.count_pairs(c[0], None, edges, 1, L, "z")
        DR = [oracle_mod.count_pairs(c[0], c[1 + k], edges, 1, L, "z") for k in range(3)]
        RR = [oracle_mod.count_pairs(c[1 + k], None, edges, 1, L, "z") for k in range(3)]
        V.append([oracle_mod.ls_split(DD, DR[:1], RR[:1], n, [n]).ravel(),
                  oracle_mod.ls_split(DD, DR[1:2], RR[1:2], n, [n]).ravel(),
                  oracle_mod.ls_split(DD, DR, RR, n, [n] * 3).ravel()])
    V = np.array(V)
    G_p = oracle_mod.shell_pair_fraction(edges, 1, L).ravel()
    A, B, _, _, _ = oracle_mod.lc_from_vectors_general(V, 1.0, 3.0, 50.0)
    for M, tol in ((1.0, 0.08), (3.0, 0.1), (20.0, 0.2), (np.inf, 0.3)):
        CM = A if np.isinf(M) else A + B / M
        theory = (2.0 / (n * (n - 1.0)) / G_p if np.isinf(M)
                  else oracle_mod.random_theory_variance(n, M * n, G_p))
        ratio = np.diag(CM) / theory
        assert abs(ratio.mean() - 1.0) < tol, (M, ratio)


# ---------------------------------------------------------------------------
# (r_p, pi) binning and the projected correlation function (Sect. 2.3)
# ---------------------------------------------------------------------------

def _rppi_numpy(a, b, edges, n_pi, box, pi_max):
    """Every pair enumerated with numpy (a separate implementation of the
    definition): minimal image, r_p^2 = s_x^2 + s_y^2 against squared edges,
    pi bin = floor(n_pi |s_z| / pi_max) for |s_z| < pi_max."""
    a = a.astype(np.int64)
    bb = a if b is None else b.astype(np.int64)
    s = bb[:, None, :] - a[:, :, None]            # [3, n_a, n_b]
    if box:
        s = np.where(s >= box // 2, s - box, np.where(s < -(box // 2), s + box, s))
    rp2 = s[0] ** 2 + s[1] ** 2
    az = np.abs(s[2])
    keep = np.ones(rp2.shape, bool)
    if b is None:
        keep = np.triu(keep, 1)
    e2 = np.asarray(edges, np.int64) ** 2
    k = np.searchsorted(e2, rp2, side="right") - 1
    keep &= (k >= 0) & (k < len(edges) - 1) & (az < pi_max)
    m = (n_pi * az) // pi_max
    out = np.zeros((len(edges) - 1, n_pi), np.uint64)
    np.add.at(out, (k[keep], m[keep]), 1)
    return out


@pytest.mark.parametrize("box", [1 << 16, 0])
def test_rppi_counts_against_numpy_enumeration(oracle_mod, box):
    lo = 0 if box else 5000
    hi = box if box else 5000 + (1 << 16)
    a, b = _rand_pts(51, 300, lo, hi), _rand_pts(52, 250, lo, hi)
    for edges, n_pi, pi_max in (([0, 2000, 5000, 9000, 16000], 6, 12000), ([700, 800, 3001], 5, 32767),
                                ([0, 30000], 1, 1)):
        for bb in (None, b):
            got = oracle_mod.count_pairs(a, bb, edges, n_pi, box, "rppi", pi_max=pi_max)
            assert np.array_equal(got, _rppi_numpy(a, bb, edges, n_pi, box, pi_max)), (edges, n_pi, pi_max)


def test_rppi_edge_pairs(oracle_mod):
    """Hand-placed pairs: r_p exactly on an edge belongs to the upper bin;
    |s_z| = pi_max is dropped and pi_max - 1 kept; |s_z| on a pi edge opens
    that bin; a pair along the line of sight has r_p = 0; the periodic image
    across the box is used."""
    edges, n_pi, pi_max, L = [0, 30, 50, 80], 4, 40, 1000
    cases = [((0, 0, 0), (30, 0, 0), (1, 0)),       # r_p = 30 on an edge
             ((0, 0, 0), (18, 24, 0), (1, 0)),      # r_p = 30 (3-4-5)
             ((0, 0, 0), (29, 0, 0), (0, 0)),
             ((0, 0, 0), (0, 0, 40), None),         # |s_z| = pi_max
             ((0, 0, 0), (0, 0, 39), (0, 3)),
             ((0, 0, 0), (0, 0, 10), (0, 1)),       # |s_z| = pi_max / n_pi
             ((0, 0, 0), (0, 0, 9), (0, 0)),
             ((0, 0, 5), (0, 0, 995), (0, 1)),      # image: s_z = -10
             ((0, 0, 0), (80, 0, 0), None),         # r_p = e_n
             ((0, 0, 0), (50, 0, -20), (2, 2))]
    for pi, pj, km in cases:
        a = np.array(pi, np.int32).reshape(3, 1)
        b = np.array(pj, np.int32).reshape(3, 1)
        got = oracle_mod.count_pairs(a, b, edges, n_pi, L, "rppi", pi_max=pi_max)
        if km is None:
            assert got.sum() == 0, (pi, pj)
        else:
            assert got.sum() == 1 and got[km] == 1, (pi, pj, np.argwhere(got))


def test_rppi_union_identity(oracle_mod):
    L = 1 << 18
    a, b = _rand_pts(61, 400, 0, L), _rand_pts(62, 350, 0, L)
    edges = [0, 3000, 7000, 12000]
    ab = np.concatenate([a, b], axis=1)
    f = lambda x, y=None: oracle_mod.count_pairs(x, y, edges, 5, L, "rppi", pi_max=9000)
    assert np.array_equal(f(ab), f(a) + f(b) + f(a, b))


def test_rppi_uniform_counts_match_cylinder_volume(oracle_mod):
    """Uniform points in a periodic box: each (r_p, pi) bin holds the pair
    count times the volume of its cylindrical shell, 2 pi (e_k+1^2 - e_k^2)
    (pi_max / n_pi) / L^3, within Poisson noise."""
    L, n = 1 << 20, 3000
    a = _rand_pts(71, n, 0, L)
    edges = np.array([0, 20000, 40000, 60000, 80000])
    n_pi, pi_max = 4, 80000
    got = oracle_mod.count_pairs(a, None, edges, n_pi, L, "rppi", pi_max=pi_max).astype(np.float64)
    area = np.pi * np.diff(edges.astype(np.float64) ** 2)
    exp = (n * (n - 1) / 2) * (area[:, None] * 2 * (pi_max / n_pi)) / float(L) ** 3 * np.ones((1, n_pi))
    z = (got - exp) / np.sqrt(exp)
    assert np.all(np.abs(z) < 5), z
    assert abs(got.sum() / exp.sum() - 1) < 0.02


def test_projected_closed_forms(oracle_mod):
    """w_p of xi = c is 2 c pi_max; of xi_m = m (bin index) it is
    2 (pi_max / n) n (n - 1) / 2; it is linear."""
    n = 8
    xi = np.full((3, n), 0.25)
    assert np.allclose(oracle_mod.projected(xi, 40.0), 2 * 0.25 * 40.0)
    xi = np.tile(np.arange(n, dtype=float), (2, 1))
    assert np.allclose(oracle_mod.projected(xi, 40.0), 2 * (40.0 / n) * n * (n - 1) / 2)
    r = np.random.default_rng(3)
    x, y = r.normal(size=(5, n)), r.normal(size=(5, n))
    assert np.allclose(oracle_mod.projected(2 * x - y, 7.0),
                       2 * oracle_mod.projected(x, 7.0) - oracle_mod.projected(y, 7.0))
