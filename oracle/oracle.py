"""CPU oracle for the LC covariance hot path.  TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the CPU-baseline leg of the benchmark may
import this module; the product path never does, and it shares no code with
the GPU library (its pair counter is ``bf_count.c``, compiled by gcc).

Everything below is the plain definition from the paper, in float64:

* pair counts DD, DR_i, RR_i in (r, mu) bins: O(N^2) enumeration
  (``count_pairs``, C, exact integer bins; Sect. 2.1 and Sect. 4.3);
* normalised counts and the split Landy-Szalay estimator (Sect. 2.1):
  dd = DD / (N_d (N_d - 1) / 2), dr_i = DR_i / (N_d N_r,i),
  rr_i = RR_i / (N_r,i (N_r,i - 1) / 2),
  xi = (dd - (2/M) sum_i dr_i) / ((1/M) sum_i rr_i) + 1;
* Legendre multipoles l = 0, 2, 4 (Sect. 4.3), integrated exactly over each
  mu bin of |mu| in [0, 1];
* the sample covariance with the 1/(N-1) normalisation (Sect. 2.2, the
  "brute force" estimate) and the linear construction (Sect. 2.3):
  C^a = (Cov xi(D,R1) + Cov xi(D,R2)) / 2, C^b = Cov xi(D, R1 u R2),
  A = 2 C^b - C^a, B = 2 M_a (C^a - C^b), C^LC = A + B / M;
* the positive-definiteness check the paper recommends for C^LC (Sect. 3):
  Cholesky and the eigenvalue spectrum (numpy / LAPACK);
* the covariance of the covariance estimates for Gaussian data vectors
  (Sect. 3.2, 3.3): element variances of the sample and of the LC
  covariance, and their summaries chi^2_2, pair-count cost and inverse
  figure of merit (Sect. 5.3, Table 3);
* pair counts binned in (r_p, pi) along z (``count_pairs`` with los
  "rppi") and the projected correlation function w_p (Sect. 2.3);
* co-added (re-binned) pair counts, including the 1D count over all mu
  (Sect. 4.3); linear maps of data vectors and covariances (re-binning,
  selection; Sect. 2.3, 5.3); the construction from general M_a < M_b
  (Eq. CovAB).

Readings where the paper is silent (documented with the tests):
  mu is |mu| on [0, 1] with uniform bins, the last one closed at mu = 1;
  r bins are half-open [e_k, e_k+1); a pair at zero separation goes to mu
  bin 0; DR and RR are normalised by the actual sub-catalogue sizes; a bin
  with rr = 0 gives xi = NaN.  In the LC covariance of covariance, D is
  A + B/(2 M_a) (the printed A + B/M_a does not reproduce the term-by-term
  expansion), and the last term pairs B_il with B_jk.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bf_count.c")
_SO = os.path.join(_HERE, "_bf_count.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the brute-force counter with gcc (OpenMP)."""
    stale = not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC)
    if force or stale:
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99",
                               "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_SO)
        f = lib.oracle_count_pairs
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                      ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.c_int64,
                      ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                      ctypes.c_void_p, ctypes.c_int]
        _lib = lib
    return _lib


LOS = {"z": 0, "mid": 1, "rppi": 2}

_last_threads = 0


def threads_used() -> int:
    return _last_threads


def count_pairs(a: np.ndarray, b: Optional[np.ndarray], edges: Sequence[int], n_mu: int,
                box_units: int = 0, los: str = "z", threads: int = 0, pi_max: int = 0) -> np.ndarray:
    """Pair counts of catalogue ``a`` with itself (b is None: unordered i<j)
    or with catalogue ``b`` (all i in a, j in b).  a, b: int32 [3, n].
    los "rppi": bins in (r_p, pi) along z, edges bin r_p and n_mu uniform
    pi bins cover [0, pi_max).  Returns uint64 [n_r, n_mu]."""
    if los == "rppi" and not pi_max >= 1:
        raise ValueError("the (r_p, pi) binning needs pi_max >= 1")
    global _last_threads
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.int32)
    auto = b is None
    bb = a if auto else np.ascontiguousarray(b, dtype=np.int32)
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int64))
    n_r = len(e) - 1
    out = np.zeros((n_r, n_mu), dtype=np.uint64)
    _last_threads = lib.oracle_count_pairs(
        a.ctypes.data, a.shape[1], bb.ctypes.data, bb.shape[1], int(auto), int(box_units),
        LOS[los], int(pi_max), n_r, e.ctypes.data, int(n_mu), out.ctypes.data, int(threads))
    return out


# ---------------------------------------------------------------------------
# estimator (Sect. 2.1)
# ---------------------------------------------------------------------------

def norm_auto(n: int) -> float:
    return n * (n - 1) / 2.0


def norm_cross(n_a: int, n_b: int) -> float:
    return float(n_a) * float(n_b)


def ls_split(DD: np.ndarray, DRs: Sequence[np.ndarray], RRs: Sequence[np.ndarray],
             n_d: int, n_rs: Sequence[int]) -> np.ndarray:
    """Split Landy-Szalay estimate from raw counts, float64.

    M = len(DRs) random sub-catalogues; DR and RR of each are normalised
    by that sub-catalogue's own size.  rr = 0 gives NaN."""
    M = len(DRs)
    dd = DD.astype(np.float64) / norm_auto(n_d)
    dr = sum(DR.astype(np.float64) / norm_cross(n_d, nr) for DR, nr in zip(DRs, n_rs))
    rr = sum(RR.astype(np.float64) / norm_auto(nr) for RR, nr in zip(RRs, n_rs))
    num = dd - (2.0 / M) * dr
    den = (1.0 / M) * rr
    with np.errstate(divide="ignore", invalid="ignore"):
        xi = num / den + 1.0
    xi[den == 0] = np.nan
    return xi


# ---------------------------------------------------------------------------
# multipoles (Sect. 4.3)
# ---------------------------------------------------------------------------

def _legendre_antiderivative(ell: int, mu: np.ndarray) -> np.ndarray:
    """Integral of P_ell from 0 to mu, for ell = 0, 2, 4.
    P_0 = 1, P_2 = (3 mu^2 - 1)/2, P_4 = (35 mu^4 - 30 mu^2 + 3)/8."""
    if ell == 0:
        return mu
    if ell == 2:
        return (mu ** 3 - mu) / 2.0
    if ell == 4:
        return (7.0 * mu ** 5 - 10.0 * mu ** 3 + 3.0 * mu) / 8.0
    raise ValueError(ell)


def legendre_weights(n_mu: int, ells: Iterable[int] = (0, 2, 4)) -> np.ndarray:
    """W[l, m] = (2l+1) * integral of P_l over mu bin m of [0, 1].

    xi_l(r) = (2l+1)/2 * integral_{-1}^{1} xi(r, mu) P_l(mu) dmu; for a xi
    binned in |mu| (even in mu) and even l this is sum_m W[l, m] xi(r, m)."""
    edges = np.arange(n_mu + 1, dtype=np.float64) / n_mu
    rows = []
    for ell in ells:
        F = _legendre_antiderivative(ell, edges)
        rows.append((2 * ell + 1) * (F[1:] - F[:-1]))
    return np.array(rows)


def multipoles(xi: np.ndarray) -> np.ndarray:
    """xi [n_r, n_mu] -> [3, n_r] (l = 0, 2, 4)."""
    W = legendre_weights(xi.shape[1])
    return np.array([[float(np.sum(W[l] * xi[k])) for k in range(xi.shape[0])]
                     for l in range(3)])


def data_vector(xi: np.ndarray) -> np.ndarray:
    """[xi(r, mu) r-major | xi_0(r) | xi_2(r) | xi_4(r)], length n_r n_mu + 3 n_r."""
    return np.concatenate([xi.ravel(), multipoles(xi).ravel()])


def mock_vectors(DD, DR1, DR2, RR1, RR2, n_d, n_r1, n_r2) -> np.ndarray:
    """The three data vectors of one mock: xi(D,R1), xi(D,R2) with M = 1 and
    xi(D, R1 u R2) with the split estimator at M = 2 (Sect. 2.3)."""
    x1 = ls_split(DD, [DR1], [RR1], n_d, [n_r1])
    x2 = ls_split(DD, [DR2], [RR2], n_d, [n_r2])
    y = ls_split(DD, [DR1, DR2], [RR1, RR2], n_d, [n_r1, n_r2])
    return np.stack([data_vector(x1), data_vector(x2), data_vector(y)])


# ---------------------------------------------------------------------------
# covariance (Sect. 2.2, 2.3)
# ---------------------------------------------------------------------------

def sample_cov(V: np.ndarray) -> np.ndarray:
    """Sample covariance of the rows of V [N, P]: two passes, 1/(N-1)."""
    N = V.shape[0]
    mean = V.sum(axis=0) / N
    D = V - mean
    return (D.T @ D) / (N - 1)


def linear_construction(Ca: np.ndarray, Cb: np.ndarray, m_a: int, M: float):
    """A = 2 C^b - C^a, B = 2 M_a (C^a - C^b), C^LC = A + B / M (M = inf -> A)."""
    A = 2.0 * Cb - Ca
    B = 2.0 * m_a * (Ca - Cb)
    C = A.copy() if np.isinf(M) else A + B / M
    return A, B, C


def lc_from_vectors(V: np.ndarray, m_a: int, M: float):
    """V [N, 3, P]: the three estimates of every mock -> (A, B, C, Ca, Cb)."""
    Ca = 0.5 * (sample_cov(V[:, 0]) + sample_cov(V[:, 1]))
    Cb = sample_cov(V[:, 2])
    A, B, C = linear_construction(Ca, Cb, m_a, M)
    return A, B, C, Ca, Cb


def check_matrix(C: np.ndarray) -> Dict[str, float]:
    """Positive-definiteness report of a symmetric matrix: Cholesky success,
    number of negative eigenvalues, extreme eigenvalues (LAPACK)."""
    try:
        np.linalg.cholesky(C)
        ok = 1
    except np.linalg.LinAlgError:
        ok = 0
    w = np.linalg.eigvalsh(C)
    return {"chol_ok": ok, "n_neg_eig": int((w < 0).sum()),
            "min_eig": float(w[0]), "max_eig": float(w[-1])}


# ---------------------------------------------------------------------------
# covariance of the covariance estimates (Sect. 3) and its summaries (Sect. 5.3)
# ---------------------------------------------------------------------------

def sample_cov_element_var(C: np.ndarray, n_mock: int) -> np.ndarray:
    """Var of each element of the sample covariance for Gaussian estimates
    (Sect. 3.2, the covariance of the sample covariance with k = i, l = j):
    (C_ii C_jj + C_ij^2) / (N - 1)."""
    d = np.diag(C)
    return (np.outer(d, d) + C * C) / (n_mock - 1)


def lc_d_matrix(A: np.ndarray, B: np.ndarray, m_a: int) -> np.ndarray:
    """D = A + B / (2 M_a), the ensemble covariance at M = 2 M_a.  (The printed
    definition A + B / M_a is inconsistent with the formula it enters: expanding
    the LC covariance in the x, x' estimates term by term gives this D; the
    tests check the expansion.)"""
    return A + B / (2.0 * m_a)


def lc_cov_element_var(A: np.ndarray, B: np.ndarray, m_a: int, M: float, n_mock: int) -> np.ndarray:
    """Var of each element of C^LC(M) for Gaussian estimates (Sect. 3.3, the
    covariance of the LC covariance with k = i, l = j):
    (D_ii D_jj + D_ij^2 + (1/(2 M_a) - 1/M)^2 (B_ii B_jj + B_ij^2)) / (N - 1)."""
    D = lc_d_matrix(A, B, m_a)
    dd, bd = np.diag(D), np.diag(B)
    f = 1.0 / (2.0 * m_a) - (0.0 if np.isinf(M) else 1.0 / M)
    return (np.outer(dd, dd) + D * D + f * f * (np.outer(bd, bd) + B * B)) / (n_mock - 1)


def chi2_2(var_n2: np.ndarray, Cref: np.ndarray) -> float:
    """<chi^2_2> of Sect. 5.3: the element variances at N = 2, normalised by the
    reference diagonal, averaged over all P^2 elements."""
    d = np.diag(Cref)
    return float((var_n2 / np.outer(d, d)).sum() / Cref.shape[0] ** 2)


def pair_cost_sample(M: float) -> float:
    """Pair-count cost of one realisation of the sample covariance with the
    split estimator, in units of the pairs of one data catalogue (Sect. 2.2):
    DD (1) + DR with M N_d randoms (2M) + M split RR (M) = 1 + 3M."""
    return 1.0 + 3.0 * M


def pair_cost_lc(m_a: int) -> float:
    """Pair-count cost of one realisation for LC (Sect. 2.3), in units of the
    pairs of one data catalogue (N_d^2 / 2), with DD counted once: the two
    split estimates with ratio M_a each cost DD (1) + DR (2 M_a) + M_a split
    RR (M_a), and the shared DD is not counted again, so 1 + 6 M_a; 7 for
    M_a = 1."""
    return 1.0 + 6.0 * m_a


def covcov_summary(A: np.ndarray, B: np.ndarray, m_a: int, M: float, Cref: Optional[np.ndarray] = None):
    """<chi^2_2> of the LC and of the sample covariance at random ratio M (with
    A, B standing in for their ensemble values and C = A + B/M for the
    covariance), the pair-count costs, the inverse figures of merit
    (cost x chi^2_2) and their ratio, the gain of LC (Sect. 5.3, Table 3)."""
    C = A + B / M
    ref = C if Cref is None else Cref
    c_lc = chi2_2(lc_cov_element_var(A, B, m_a, M, 2), ref)
    c_smp = chi2_2(sample_cov_element_var(C, 2), ref)
    cost_lc, cost_smp = pair_cost_lc(m_a), pair_cost_sample(M)
    return {"chi2_2_lc": c_lc, "chi2_2_smp": c_smp, "cost_lc": cost_lc, "cost_smp": cost_smp,
            "ifom_lc": cost_lc * c_lc, "ifom_smp": cost_smp * c_smp,
            "gain": (cost_smp * c_smp) / (cost_lc * c_lc)}


# ---------------------------------------------------------------------------
# re-binning, the 1D correlation function and general M_a, M_b
# (Sect. 2.3 Eq. CovAB, Sect. 4.3, Sect. 5.3)
# ---------------------------------------------------------------------------

def rebin_counts(counts: np.ndarray, w_r: int, w_mu: int) -> np.ndarray:
    """Co-add pair counts [n_r, n_mu] over groups of w_r adjacent r bins (the
    last group keeps what is left) and w_mu adjacent mu bins (w_mu divides
    n_mu).  With w_mu = n_mu this is the 1D pair count of Sect. 4.3 (counts
    co-added over mu).  Plain loops, uint64."""
    n_r, n_mu = counts.shape
    assert n_mu % w_mu == 0
    n_r2 = (n_r + w_r - 1) // w_r
    out = np.zeros((n_r2, n_mu // w_mu), dtype=np.uint64)
    for k in range(n_r):
        for m in range(n_mu):
            out[k // w_r, m // w_mu] += np.uint64(counts[k, m])
    return out


def rebinned_edges(edges: Sequence[int], w_r: int) -> List[int]:
    """Edges of the co-added r bins: every w_r-th edge and the last one."""
    e = list(edges)
    n_r = len(e) - 1
    return [e[min(k * w_r, n_r)] for k in range((n_r + w_r - 1) // w_r + 1)]


def linear_map(group: np.ndarray, weight: np.ndarray, P_out: int) -> np.ndarray:
    """The dense matrix T [P_out, P_in] of a map that sends input element i
    with weight w_i to output element group_i (group_i = -1: dropped)."""
    T = np.zeros((P_out, len(group)))
    for i, (g, w) in enumerate(zip(group, weight)):
        if g >= 0:
            T[g, i] += w
    return T


def map_vectors(X: np.ndarray, group, weight, P_out: int) -> np.ndarray:
    """Rows of X [..., P_in] mapped by T: y = T x (re-binning or selecting the
    elements of a data vector; any linear function of xi, Sect. 2.3)."""
    return X @ linear_map(group, weight, P_out).T


def map_matrix(C: np.ndarray, group, weight, P_out: int) -> np.ndarray:
    """T C T^T: a covariance re-binned with the data vector (Sect. 5.3)."""
    T = linear_map(group, weight, P_out)
    return T @ C @ T.T


def projected(xi_rppi: np.ndarray, pi_max: float) -> np.ndarray:
    """The projected correlation function from xi binned in (r_p, pi) with
    n_pi uniform pi bins on [0, pi_max): w_p(r_p) = 2 * integral over
    [0, pi_max) of xi(r_p, pi) dpi, with xi constant within each pi bin,
    i.e. 2 (pi_max / n_pi) sum_m xi[k, m] (a linear function of xi,
    Sect. 2.3).  xi_rppi [n_rp, n_pi] -> [n_rp]; pi_max in the unit wanted
    for w_p."""
    n_pi = xi_rppi.shape[1]
    return 2.0 * (pi_max / n_pi) * xi_rppi.sum(axis=1)


def linear_construction_general(Ca: np.ndarray, Cb: np.ndarray, m_a: float, m_b: float, M: float):
    """Eq. CovAB: from covariances at random ratios M_a < M_b,
    A = (M_b C^b - M_a C^a) / (M_b - M_a), B = M_a M_b (C^a - C^b) / (M_b - M_a),
    and C = A + B / M (M = inf -> A)."""
    A = (m_b * Cb - m_a * Ca) / (m_b - m_a)
    B = (m_a * m_b) * (Ca - Cb) / (m_b - m_a)
    C = A.copy() if np.isinf(M) else A + B / M
    return A, B, C


def lc_from_vectors_general(V: np.ndarray, m_a: float, m_b: float, M: float):
    """V [N, 3, P]: two estimates at ratio M_a and one at M_b per mock ->
    (A, B, C, Ca, Cb) with C^a the mean of the two M_a covariances."""
    Ca = 0.5 * (sample_cov(V[:, 0]) + sample_cov(V[:, 1]))
    Cb = sample_cov(V[:, 2])
    A, B, C = linear_construction_general(Ca, Cb, m_a, m_b, M)
    return A, B, C, Ca, Cb


# ---------------------------------------------------------------------------
# end to end over catalogues
# ---------------------------------------------------------------------------

def mock_counts(cat_d: np.ndarray, cat_r1: np.ndarray, cat_r2: np.ndarray,
                edges, n_mu: int, box_units: int, los: str, threads: int = 0,
                rr_cache: Optional[dict] = None, r_ids: Tuple[int, int] = (-1, -1)):
    """DD, DR1, DR2, RR1, RR2 of one mock (RR optionally cached by id)."""
    DD = count_pairs(cat_d, None, edges, n_mu, box_units, los, threads)
    DR1 = count_pairs(cat_d, cat_r1, edges, n_mu, box_units, los, threads)
    DR2 = count_pairs(cat_d, cat_r2, edges, n_mu, box_units, los, threads)
    out = []
    for cat_r, rid in ((cat_r1, r_ids[0]), (cat_r2, r_ids[1])):
        if rr_cache is not None and rid >= 0 and rid in rr_cache:
            out.append(rr_cache[rid])
            continue
        RR = count_pairs(cat_r, None, edges, n_mu, box_units, los, threads)
        if rr_cache is not None and rid >= 0:
            rr_cache[rid] = RR
        out.append(RR)
    return DD, DR1, DR2, out[0], out[1]


def random_theory_variance(n_d: int, n_r: int, G_p: np.ndarray) -> np.ndarray:
    """Expected variance of xi for uniform ("random") data catalogues
    (Sect. 5.1, quoting Keihanen et al. 2019):
    (2/(N_d(N_d-1)) + 4/(N_d N_r) + 2/(N_r(N_d-1))) / G_p,
    with G_p the fraction of all pairs that fall in the bin."""
    return (2.0 / (n_d * (n_d - 1.0)) + 4.0 / (n_d * n_r) + 2.0 / (n_r * (n_d - 1.0))) / G_p


def shell_pair_fraction(edges_units: np.ndarray, n_mu: int, box_units: int) -> np.ndarray:
    """Fraction of uniformly distributed pairs in a periodic box that fall in
    each (r, mu) bin: (4 pi / 3)(r_k+1^3 - r_k^3) / (L^3 n_mu); exact in
    expectation for r_max < L/2 (minimal image)."""
    e = np.asarray(edges_units, dtype=np.float64)
    shell = (4.0 * np.pi / 3.0) * (e[1:] ** 3 - e[:-1] ** 3) / float(box_units) ** 3
    return np.repeat(shell[:, None] / n_mu, n_mu, axis=1)


def time_counts(fn, *args, **kw):
    t0 = time.perf_counter()
    out = fn(*args, **kw)
    return out, time.perf_counter() - t0
