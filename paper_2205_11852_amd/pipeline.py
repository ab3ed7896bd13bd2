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


class Pipeline:
    """Device-resident catalogues of one workload and the calls of the path."""

    def __init__(self, cats, device: str = "cuda", M: float = 50.0, m_a: int = 1):
        import torch
        self.torch = torch
        self.cats = cats
        self.wl = cats.wl
        self.device = device
        self.binning = lc.Binning.from_workload(self.wl)
        self.tasks, self.est = plan_tasks(cats.n_mock, cats.randoms)
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

    def build_cells(self, cell_units: int = 0, sub: int = 0):
        if self.cells is not None:
            self.cells.close()
        if self.tuned is not None and cell_units == 0 and sub == 0:
            cell_units, sub = self.tuned["cell_units"], self.tuned["sub"]
        self.cells = lc.lc_build_cells(self.xyz, self.offsets, self.binning, cell_units, sub)
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

    # -- host copies ---------------------------------------------------------
    def counts_host(self) -> np.ndarray:
        return self.counts.cpu().numpy().view(np.uint64)

    def stats_host(self) -> Dict[str, int]:
        s = self.stats.cpu().numpy().view(np.uint64)
        return {"candidates": int(s[0]), "binned": int(self.counts_host().sum(dtype=np.uint64)),
                "exact_fallback": int(s[2]), "flushes": int(s[3])}
