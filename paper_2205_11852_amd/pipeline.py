"""Host orchestration of the LC path: task planning and the ordered C-ABI calls.

The paper's procedure (Sect. 2.3, 4.4): for every mock D with random
catalogues R1 and R2 count DD, DR1, DR2, RR1, RR2 (RR of a shared random
sub-catalogue is counted once), form xi(D,R1), xi(D,R2) and the split
xi(D, R1 u R2), then the covariances and the linear construction.  All
arithmetic happens in liblc.so; this module only builds the task table and
moves arguments.
"""
from __future__ import annotations

import time
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import lc


def plan_tasks(n_mock: int, randoms: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Task table (cat_a, cat_b) and, per mock, the task ids of DD, DR1, DR2,
    RR1, RR2.  RR of a sub-catalogue shared by several mocks appears once."""
    tasks: List[Tuple[int, int]] = []
    index: Dict[Tuple[int, int], int] = {}

    def tid(a: int, b: int) -> int:
        key = (int(a), int(b))
        if key not in index:
            index[key] = len(tasks)
            tasks.append(key)
        return index[key]

    est = np.zeros((n_mock, 5), dtype=np.int32)
    for m in range(n_mock):
        r1, r2 = int(randoms[m, 0]), int(randoms[m, 1])
        est[m] = (tid(m, m), tid(m, r1), tid(m, r2), tid(r1, r1), tid(r2, r2))
    return np.array(tasks, dtype=np.int32).reshape(-1, 2), est


def plan_direct_tasks(mocks: Sequence[int], subsets: Sequence[int]) -> Tuple[np.ndarray, np.ndarray]:
    """Task table and est rows for the direct estimate with every mock split
    over the same M random sub-catalogues: [DD, DR_1..DR_M, RR_1..RR_M] per
    mock; each RR_i is counted once for all mocks."""
    tasks: List[Tuple[int, int]] = [(int(s), int(s)) for s in subsets]
    rr = list(range(len(subsets)))
    est = []
    for m in mocks:
        row = [len(tasks)]
        tasks.append((int(m), int(m)))
        for s in subsets:
            row.append(len(tasks))
            tasks.append((int(m), int(s)))
        est.append(row + rr)
    return np.array(tasks, dtype=np.int32).reshape(-1, 2), np.array(est, dtype=np.int32)


def multipole_map(n_r: int, n_mu: int, w: int = 1, r_lo: int = 0, r_hi: Optional[int] = None,
                  ells: Sequence[int] = (0, 2, 4)) -> Tuple[np.ndarray, np.ndarray, int]:
    """Map (group, weight, P_out) for lc_map_vectors / lc_map_matrix from the
    data vector to the multipoles `ells` (increasing) over r bins
    [r_lo, r_hi), each output the mean of w adjacent r bins; built by the
    library (lc_map_multipoles).  w = 1 selects (the paper's 540-element
    vector); w > 1 re-bins (Table 3)."""
    r_hi = n_r if r_hi is None else int(r_hi)
    ells = list(ells)
    if ells != sorted(set(ells)) or any(e not in (0, 2, 4) for e in ells) or not ells:
        raise ValueError("ells must be an increasing subset of (0, 2, 4)")
    if not (0 <= r_lo < r_hi <= n_r) or w < 1:
        raise ValueError("bad r range [%d, %d) or width %d" % (r_lo, r_hi, w))
    mask = sum(1 << (0, 2, 4).index(e) for e in ells)
    return lc.lc_map_multipoles(n_r, n_mu, w, r_lo, r_hi, mask)


def projected_map(n_rp: int, n_pi: int, pi_max: float) -> Tuple[np.ndarray, np.ndarray, int]:
    """Map (group, weight, P_out) from the data vector of a (r_p, pi)
    binning to w_p(r_p), in the unit of pi_max; built by the library
    (lc_map_projected)."""
    return lc.lc_map_projected(n_rp, n_pi, pi_max)


def block_rebin_map(n_blocks: int, n: int, w: int) -> Tuple[np.ndarray, np.ndarray, int]:
    """Map (group, weight, P_out) that averages w adjacent elements within
    each of n_blocks consecutive blocks of n; built by the library
    (lc_map_rebin_blocks)."""
    if w < 1 or n < 1 or n_blocks < 1:
        raise ValueError("bad block map sizes")
    return lc.lc_map_rebin_blocks(n_blocks, n, w)


class Pipeline:
    """Device-resident catalogues of one workload and the calls of the path."""

    def __init__(self, cats, device: str = "cuda", M: float = 50.0, m_a: int = 1,
                 extra_tasks: Optional[Sequence[Tuple[int, int]]] = None):
        """extra_tasks: further (cat_a, cat_b) pairs counted in the same
        launches after the estimator's tasks (ids from len(plan) on)."""
        import torch
        self.torch = torch
        self.cats = cats
        self.wl = cats.wl
        self.device = device
        self.binning = lc.Binning.from_workload(self.wl)
        self.tasks, self.est = plan_tasks(cats.n_mock, cats.randoms)
        if extra_tasks is not None and len(extra_tasks):
            ex = np.asarray(extra_tasks, dtype=np.int32).reshape(-1, 2)
            self.tasks = np.concatenate([self.tasks, ex], axis=0)
        self.sizes = cats.sizes()
        self.offsets = cats.offsets
        self.M = float(M)
        self.m_a = int(m_a)
        self.xyz = torch.from_numpy(cats.xyz).to(device)
        self.n_mock = cats.n_mock
        nb = self.binning.n_r * self.binning.n_mu
        P = self.binning.P
        self.counts = torch.zeros((len(self.tasks), self.binning.n_r, self.binning.n_mu),
                                  dtype=torch.int64, device=device)
        self.stats = torch.zeros(4, dtype=torch.int64, device=device)
        self.xi = torch.empty((self.n_mock, 3, P), dtype=torch.float64, device=device)
        self.A = torch.empty((P, P), dtype=torch.float64, device=device)
        self.B = torch.empty((P, P), dtype=torch.float64, device=device)
        self.C = torch.empty((P, P), dtype=torch.float64, device=device)
        self.cells: Optional[lc.Cells] = None
        self._nb = nb
        self.tuned: Optional[dict] = None

    # -- steps ---------------------------------------------------------------
    def autotune(self, sample_tasks: int = 0) -> dict:
        """Pick the mesh and launch shape by timing (cached by the library);
        later build_cells() and count() calls without explicit options use it."""
        self.tuned = lc.lc_autotune(self.xyz, self.offsets, self.binning, self.tasks, sample_tasks)
        return self.tuned

    def build_cells(self, cell_units: int = 0, sub: int = 0, arrival_order: bool = False):
        if self.cells is not None:
            self.cells.close()
        if self.tuned is not None and cell_units == 0 and sub == 0:
            cell_units, sub = self.tuned["cell_units"], self.tuned["sub"]
        self.cells = lc.lc_build_cells(self.xyz, self.offsets, self.binning, cell_units, sub,
                                       arrival_order=arrival_order)
        return self.cells

    def count(self, mode: int = lc.LC_PERSISTENT, tune: Optional[dict] = None, zero: bool = True):
        if zero:
            self.counts.zero_()
            self.stats.zero_()
        if tune is None and self.tuned is not None:
            tune = self.tuned["tune"]
        lc.lc_pair_count_batch(self.cells, self.tasks, self.binning, self.counts, mode, tune,
                               self.stats)

    def count_per_mock(self, tune: Optional[dict] = None, sync: bool = True):
        """Baseline: one launch per task, mock after mock, synchronising after
        each mock (shared RR counted once, before the loop)."""
        torch = self.torch
        if tune is None and self.tuned is not None:
            tune = self.tuned["tune"]
        self.counts.zero_()
        self.stats.zero_()
        nbytes = self._nb * 8
        base = int(self.counts.data_ptr())
        sbase = int(self.stats.data_ptr())
        done = set()

        def one(t):
            lc.lc_pair_count_batch(self.cells, self.tasks[t:t + 1], self.binning, base + t * nbytes,
                                   lc.LC_PER_TASK, tune, sbase)

        for t in sorted(set(int(v) for v in self.est[:, 3:].ravel())):
            one(t)
            done.add(t)
        if sync:
            torch.cuda.synchronize()
        for m in range(self.n_mock):
            for t in self.est[m, :3]:
                if int(t) not in done:
                    one(int(t))
                    done.add(int(t))
            if sync:
                torch.cuda.synchronize()

    def xi_multipoles(self):
        b = self.binning
        lc.lc_xi_multipoles(self.counts, self.tasks, self.sizes, self.est, b.n_r, b.n_mu, self.xi)

    def covariance(self, precision: int = lc.LC_FP32_MFMA, report: bool = True, M: Optional[float] = None):
        b = self.binning
        return lc.lc_covariance(self.xi, self.n_mock, b.n_r, b.n_mu, self.m_a,
                                self.M if M is None else M, precision, self.A, self.B, self.C, report)

    def run(self, mode: int = lc.LC_PERSISTENT, precision: int = lc.LC_FP32_MFMA, report: bool = True,
            cell_units: int = 0, sub: int = 0, tune: Optional[dict] = None) -> dict:
        """The whole path on device-resident catalogues; returns the check report."""
        self.build_cells(cell_units, sub)
        self.count(mode, tune)
        self.xi_multipoles()
        return self.covariance(precision, report)

    def covcov(self, M: Optional[float] = None, n_mock: int = 0, sd: bool = False) -> dict:
        """Covariance-of-covariance summary (chi^2_2, cost, iFoM, gain) of the
        last lc_covariance call's A and B at ratio M; with sd, also the element
        standard deviations of both estimators at n_mock realisations."""
        P = self.binning.P
        sd_lc = sd_smp = None
        if sd:
            sd_lc = self.torch.empty((P, P), dtype=self.torch.float64, device=self.device)
            sd_smp = self.torch.empty_like(sd_lc)
        rep = lc.lc_covcov(self.A, self.B, P, self.m_a, self.M if M is None else M, None,
                           n_mock or self.n_mock, sd_lc, sd_smp)
        if sd:
            rep["sd_lc"], rep["sd_smp"] = sd_lc, sd_smp
        return rep

    def direct_estimates(self, mocks: Sequence[int], subsets: Sequence[int], tune: Optional[dict] = None):
        """The split estimate of each listed mock over all listed random
        sub-catalogues (M = len(subsets)): counts every needed task in one
        persistent launch on the current mesh, then lc_xi_split.  Returns
        (x [len(mocks), P] device tensor, counts, tasks, est)."""
        torch = self.torch
        tasks, est = plan_direct_tasks(mocks, subsets)
        b = self.binning
        counts = torch.zeros((len(tasks), b.n_r, b.n_mu), dtype=torch.int64, device=self.device)
        if tune is None and self.tuned is not None:
            tune = self.tuned["tune"]
        lc.lc_pair_count_batch(self.cells, tasks, b, counts, lc.LC_PERSISTENT, tune, None)
        x = torch.empty((len(mocks), b.P), dtype=torch.float64, device=self.device)
        lc.lc_xi_split(counts, tasks, self.sizes, est, len(subsets), b.n_r, b.n_mu, x)
        return x, counts, tasks, est

    def general_vectors(self, mocks: Sequence[int], sets: Sequence[Sequence[int]],
                        tune: Optional[dict] = None):
        """Three split estimates per listed mock (x, x' and y of the
        construction from general M_a < M_b, Eq. CovAB), estimate e over the
        random catalogues sets[e] (the same for every mock).  Counts every
        needed task in one launch, then one lc_xi_split per estimate into the
        [n, 3, P] layout.  Returns the device tensor."""
        torch = self.torch
        if len(sets) != 3:
            raise ValueError("need three subset lists: x, x' (ratio M_a) and y (ratio M_b)")
        union = sorted(set(int(c) for S in sets for c in S))
        tasks, est = plan_direct_tasks(mocks, union)
        b = self.binning
        counts = torch.zeros((len(tasks), b.n_r, b.n_mu), dtype=torch.int64, device=self.device)
        if tune is None and self.tuned is not None:
            tune = self.tuned["tune"]
        lc.lc_pair_count_batch(self.cells, tasks, b, counts, lc.LC_PERSISTENT, tune, None)
        xi = torch.empty((len(mocks), 3, b.P), dtype=torch.float64, device=self.device)
        n_u = len(union)
        for e, S in enumerate(sets):
            cols = np.array([union.index(int(c)) for c in S])
            est_e = np.concatenate([est[:, :1], est[:, 1 + cols], est[:, 1 + n_u + cols]], axis=1)
            lc.lc_xi_split(counts, tasks, self.sizes, est_e, len(S), b.n_r, b.n_mu, xi, ld_xi=3 * b.P,
                           offset=e * b.P)
        return xi

    def covariance_general(self, xi, P: int, n_split: int, m_a: float, m_b: float, M: Optional[float] = None,
                           precision: int = lc.LC_FP32_MFMA, report: bool = True):
        """lc_covariance_general on [n, 3, P] vectors; returns (A, B, C, report)."""
        torch = self.torch
        A, B, C = (torch.empty((P, P), dtype=torch.float64, device=self.device) for _ in range(3))
        rep = lc.lc_covariance_general(xi, xi.shape[0], P, n_split, m_a, m_b, self.M if M is None else M,
                                       precision, A, B, C, report)
        return A, B, C, rep

    def rebinned(self, w_r: int, w_mu: int):
        """Counts co-added over w_r r bins and w_mu mu bins (lc_rebin_counts)
        and the matching binning; w_mu = n_mu gives the 1D counts."""
        b = self.binning
        n_r2 = (b.n_r + w_r - 1) // w_r
        out = self.torch.empty((len(self.tasks), n_r2, b.n_mu // w_mu), dtype=self.torch.int64,
                               device=self.device)
        lc.lc_rebin_counts(self.counts, len(self.tasks), b.n_r, b.n_mu, w_r, w_mu, out)
        e = b.edges
        edges = [int(e[min(k * w_r, b.n_r)]) for k in range(n_r2 + 1)]
        return out, lc.Binning(edges, b.n_mu // w_mu, bool(b.c.periodic), int(b.c.box_units), int(b.c.los),
                               b.pi_max)

    def xi_of(self, counts, binning) -> "object":
        """lc_xi_multipoles of other counts of the same tasks (e.g. co-added)."""
        xi = self.torch.empty((self.n_mock, 3, binning.P), dtype=self.torch.float64, device=self.device)
        lc.lc_xi_multipoles(counts, self.tasks, self.sizes, self.est, binning.n_r, binning.n_mu, xi)
        return xi

    def map_vectors(self, xi, group, weight, P_out: int):
        """lc_map_vectors over every estimate row of an [n, 3, P] tensor."""
        n, q, P = xi.shape
        y = self.torch.empty((n, q, P_out), dtype=self.torch.float64, device=self.device)
        lc.lc_map_vectors(xi, n * q, P, group, weight, P_out, y)
        return y

    def map_matrix(self, X, group, weight, P_out: int):
        Y = self.torch.empty((P_out, P_out), dtype=self.torch.float64, device=self.device)
        lc.lc_map_matrix(X, X.shape[0], group, weight, P_out, Y)
        return Y

    # -- host copies ---------------------------------------------------------
    def counts_host(self) -> np.ndarray:
        return self.counts.cpu().numpy().view(np.uint64)

    def stats_host(self) -> Dict[str, int]:
        s = self.stats.cpu().numpy().view(np.uint64)
        return {"candidates": int(s[0]), "binned": int(self.counts_host().sum(dtype=np.uint64)),
                "exact_fallback": int(s[2]), "flushes": int(s[3]), "guard_flushes": int(s[1])}
