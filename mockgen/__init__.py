"""Seeded synthetic catalogues for the LC covariance hot path.

This module only draws inputs: point positions, catalogue sizes and the
assignment of random sub-catalogues to mocks.  It contains none of the pair
counting, estimator or covariance arithmetic, so both the CPU oracle and the
GPU path can take their inputs from here without sharing any method code.

Coordinates are integers in units of 2^-12 Mpc/h (``UNITS_PER_MPC``).  The
paper's mocks are PINOCCHIO halo catalogues (Sect. 4) that are not available
here; Neyman-Scott cluster processes with a similar mean density stand in for
them, and uniform randoms play the role of the random catalogues (Sect. 4,
random catalogues drawn uniformly in the survey volume).

Every draw comes from ``rng_for(cfg_id, role, idx)``, a PCG64 generator
seeded with ``SeedSequence([220511852, cfg_id, role, idx])``; roles are
0 = cluster parents, 1 = data points, 2 = random points.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Tuple

import numpy as np

UNITS_PER_MPC = 4096
SEED_ROOT = 220511852
ROLE_PARENTS, ROLE_DATA, ROLE_RANDOM = 0, 1, 2


def rng_for(cfg_id: int, role: int, idx: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(
        np.random.SeedSequence([SEED_ROOT, int(cfg_id), int(role), int(idx)])))


def _quantise(pos_mpc: np.ndarray) -> np.ndarray:
    """float64 Mpc/h -> int32 units of 2^-12 Mpc/h (floor)."""
    return np.floor(pos_mpc * UNITS_PER_MPC).astype(np.int64)


# ---------------------------------------------------------------------------
# point processes
# ---------------------------------------------------------------------------

def uniform_box(rng: np.random.Generator, n: int, box_units: int) -> np.ndarray:
    """n uniform integer points in [0, box_units)^3, int32 [3, n]."""
    return rng.integers(0, box_units, size=(3, int(n)), dtype=np.int64).astype(np.int32)


def neyman_scott_box(rng_parents: np.random.Generator, rng_data: np.random.Generator,
                     n_mean: float, n_parents: int, sigma_mpc: float,
                     box_units: int) -> np.ndarray:
    """Neyman-Scott process in a periodic cube.

    N ~ Poisson(n_mean) children; each picks one of ``n_parents`` uniform
    parents and is offset by an isotropic Gaussian of width sigma; positions
    are wrapped into the box and quantised.  Returns int32 [3, N].
    """
    box_mpc = box_units / UNITS_PER_MPC
    parents = rng_parents.uniform(0.0, box_mpc, size=(3, n_parents))
    n = int(rng_data.poisson(n_mean))
    which = rng_data.integers(0, n_parents, size=n)
    pos = parents[:, which] + rng_data.normal(0.0, sigma_mpc, size=(3, n))
    q = _quantise(np.mod(pos, box_mpc)) % box_units
    return q.astype(np.int32)


# survey-like wedge: alpha, delta in [-30, 30] deg, chi in [1200, 2400] Mpc/h,
# number density falling linearly by a factor 3 from the near to the far edge.
WEDGE_HALF_ANGLE_DEG = 30.0
WEDGE_CHI = (1200.0, 2400.0)


def _wedge_chi(rng: np.random.Generator, n: int) -> np.ndarray:
    """Radial distances with pdf proportional to chi^2 n(chi), by rejection."""
    c0, c1 = WEDGE_CHI
    out = np.empty(0)
    # envelope: chi^2 n(chi) <= c1^2 * 1
    while out.size < n:
        m = max(2 * (n - out.size), 1024)
        chi = rng.uniform(c0, c1, size=m)
        dens = 1.0 - (2.0 / 3.0) * (chi - c0) / (c1 - c0)
        keep = rng.uniform(0.0, 1.0, size=m) < (chi * chi * dens) / (c1 * c1)
        out = np.concatenate([out, chi[keep]])
    return out[:n]


def _wedge_dirs(rng: np.random.Generator, n: int) -> np.ndarray:
    h = math.radians(WEDGE_HALF_ANGLE_DEG)
    alpha = rng.uniform(-h, h, size=n)
    sdec = rng.uniform(math.sin(-h), math.sin(h), size=n)
    cdec = np.sqrt(1.0 - sdec * sdec)
    return np.stack([cdec * np.cos(alpha), cdec * np.sin(alpha), sdec])


def _in_wedge(pos: np.ndarray) -> np.ndarray:
    h = math.radians(WEDGE_HALF_ANGLE_DEG)
    chi = np.sqrt((pos * pos).sum(axis=0))
    alpha = np.arctan2(pos[1], pos[0])
    sdec = pos[2] / np.maximum(chi, 1e-300)
    return ((chi >= WEDGE_CHI[0]) & (chi < WEDGE_CHI[1]) & (np.abs(alpha) <= h)
            & (np.abs(sdec) <= math.sin(h)) & (pos[0] > 0))


def wedge_uniform(rng: np.random.Generator, n: int) -> np.ndarray:
    """Points following the wedge selection (mask and n(chi)), int32 [3, n]."""
    pos = _wedge_dirs(rng, n) * _wedge_chi(rng, n)[None, :]
    return _quantise(pos).astype(np.int32)


def wedge_neyman_scott(rng_parents: np.random.Generator, rng_data: np.random.Generator,
                       n_mean: float, n_parents: int, sigma_mpc: float) -> np.ndarray:
    """Neyman-Scott clustering inside the wedge: parents follow the selection;
    a child that falls outside the mask is redrawn around the same parent."""
    parents = _wedge_dirs(rng_parents, n_parents) * _wedge_chi(rng_parents, n_parents)[None, :]
    n = int(rng_data.poisson(n_mean))
    which = rng_data.integers(0, n_parents, size=n)
    pos = parents[:, which] + rng_data.normal(0.0, sigma_mpc, size=(3, n))
    bad = ~_in_wedge(pos)
    while bad.any():
        k = int(bad.sum())
        pos[:, bad] = parents[:, which[bad]] + rng_data.normal(0.0, sigma_mpc, size=(3, k))
        bad = ~_in_wedge(pos)
    return _quantise(pos).astype(np.int32)


# paper-shaped slab (Sect. 4.1): a 1500 x 1500 x 300 Mpc/h slab cut from a
# 1500 Mpc/h box, thin along the line of sight (z), open (not periodic).
SLAB_SIDE_MPC = 1500.0
SLAB_DEPTH_MPC = 300.0
SLAB_COUNT_SCATTER = 0.03


def slab_neyman_scott(rng_parents: np.random.Generator, rng_data: np.random.Generator,
                      n_mean: float, n_parents: int, sigma_mpc: float) -> np.ndarray:
    """Neyman-Scott process in the periodic 1500 Mpc/h box, cut to the slab
    0 <= z < 300 Mpc/h.  ``n_mean`` is the mean count inside the slab and
    ``n_parents`` the number of parents in the whole box (about four children
    each: halo-like objects, weakly clustered at small separations).  The
    expected count of each slab is scaled by 1 + 0.03 g, g standard normal,
    standing in for the density modes larger than the slab that make the
    paper's slab counts vary by about 3% (Sect. 4.1).  Returns int32 [3, N]."""
    box_units = int(round(SLAB_SIDE_MPC * UNITS_PER_MPC))
    depth_units = int(round(SLAB_DEPTH_MPC * UNITS_PER_MPC))
    parents = rng_parents.uniform(0.0, SLAB_SIDE_MPC, size=(3, n_parents))
    scale = max(0.0, 1.0 + SLAB_COUNT_SCATTER * rng_parents.normal())
    n = int(rng_data.poisson(n_mean * scale * SLAB_SIDE_MPC / SLAB_DEPTH_MPC))
    which = rng_data.integers(0, n_parents, size=n)
    pos = parents[:, which] + rng_data.normal(0.0, sigma_mpc, size=(3, n))
    q = _quantise(np.mod(pos, SLAB_SIDE_MPC)) % box_units
    return q[:, q[2] < depth_units].astype(np.int32)


def slab_uniform(rng: np.random.Generator, n: int) -> np.ndarray:
    """n uniform integer points in the slab, int32 [3, n]."""
    side = int(round(SLAB_SIDE_MPC * UNITS_PER_MPC))
    depth = int(round(SLAB_DEPTH_MPC * UNITS_PER_MPC))
    hi = np.array([[side], [side], [depth]], dtype=np.int64)
    return rng.integers(0, hi, size=(3, int(n)), dtype=np.int64).astype(np.int32)


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic workload: mocks, random pool and binning."""
    name: str
    cfg_id: int
    n_mock: int
    n_mean: float
    n_parents: int
    sigma_mpc: float
    geometry: str                 # "periodic", "wedge" or "slab"
    box_mpc: float                # periodic side (ignored for the wedge)
    n_subsets: int                # shared random pool: number of sub-catalogues
    subset_size: int              # points per shared sub-catalogue (0: per-mock sizes)
    per_mock_randoms: bool        # True: every mock gets its own two sub-catalogues
    n_r: int
    r_max_mpc: float
    n_mu: int
    los: str                      # "z" (plane-parallel), "mid" (midpoint) or "rppi" ((r_p, pi) along z)
    pi_max_mpc: float = 0.0       # "rppi": line-of-sight extent; n_mu counts its pi bins

    @property
    def periodic(self) -> bool:
        return self.geometry == "periodic"

    @property
    def pi_max_units(self) -> int:
        return int(round(self.pi_max_mpc * UNITS_PER_MPC))

    @property
    def box_units(self) -> int:
        return int(round(self.box_mpc * UNITS_PER_MPC)) if self.periodic else 0

    @property
    def r_edges_units(self) -> np.ndarray:
        e = np.linspace(0.0, self.r_max_mpc, self.n_r + 1) * UNITS_PER_MPC
        ei = np.round(e).astype(np.int64)
        assert np.all(np.abs(ei - e) < 1e-6), "edges must be whole units"
        return ei

    def with_mocks(self, n_mock: int) -> "Workload":
        return dataclasses.replace(self, n_mock=int(n_mock))


WORKLOADS = {
    # 32 clustered mocks in a 500 Mpc/h box; one pool of 2 x 5000 randoms.
    "c1": Workload("c1", 1, 32, 5000.0, 250, 5.0, "periodic", 500.0, 2, 5000, False,
                   20, 100.0, 10, "z"),
    # 1000 mocks of 1e5 in a 1000 Mpc/h box; pool of 50 x 1e5 randoms.
    "c2": Workload("c2", 2, 1000, 1.0e5, 4000, 5.0, "periodic", 1000.0, 50, 100000, False,
                   40, 200.0, 50, "z"),
    # 200 mocks of 1e6 in a 2000 Mpc/h box; per-mock randoms, two of the mock's size.
    "c3": Workload("c3", 3, 200, 1.0e6, 40000, 5.0, "periodic", 2000.0, 0, 0, True,
                   40, 200.0, 100, "z"),
    # 500 mocks of 3e5 in a 60x60 deg wedge; pool of 20 x 3e5; midpoint line of sight.
    "c4": Workload("c4", 4, 500, 3.0e5, 12000, 5.0, "wedge", 0.0, 20, 300000, False,
                   40, 200.0, 50, "mid"),
    # 5000 mocks of 5e4 in a 1000 Mpc/h box; pool of 50 x 5e4.
    "c5": Workload("c5", 5, 5000, 5.0e4, 2000, 5.0, "periodic", 1000.0, 50, 50000, False,
                   40, 200.0, 50, "z"),
    # The paper's own shape (Sect. 4.1, 4.3): slabs of 156 158 weakly
    # clustered points on average (about +-3% from mock to mock), each with
    # two random sub-catalogues of its own size; 1 Mpc/h x 0.01 bins over
    # r < 200 Mpc/h.
    "slab": Workload("slab", 6, 100, 156158.0, 195000, 5.0, "slab", SLAB_SIDE_MPC, 0, 0, True,
                     200, 200.0, 100, "z"),
}


@dataclasses.dataclass
class Catalogues:
    """All catalogues of a workload packed for transfer.

    xyz      int32 [3, n_total], catalogues back to back
    offsets  int64 [n_cat + 1]
    n_mock   mocks are catalogues 0 .. n_mock-1
    randoms  (n_mock, 2) catalogue ids of R1 and R2 for every mock
    """
    wl: Workload
    xyz: np.ndarray
    offsets: np.ndarray
    n_mock: int
    randoms: np.ndarray

    @property
    def n_cat(self) -> int:
        return len(self.offsets) - 1

    def sizes(self) -> np.ndarray:
        return np.diff(self.offsets)

    def cat(self, c: int) -> np.ndarray:
        return self.xyz[:, self.offsets[c]:self.offsets[c + 1]]

    def random_catalogue_ids(self) -> List[int]:
        return sorted(set(int(v) for v in self.randoms.ravel()))


def mock_catalogue(wl: Workload, m: int) -> np.ndarray:
    rp = rng_for(wl.cfg_id, ROLE_PARENTS, m)
    rd = rng_for(wl.cfg_id, ROLE_DATA, m)
    if wl.periodic:
        return neyman_scott_box(rp, rd, wl.n_mean, wl.n_parents, wl.sigma_mpc, wl.box_units)
    if wl.geometry == "slab":
        return slab_neyman_scott(rp, rd, wl.n_mean, wl.n_parents, wl.sigma_mpc)
    return wedge_neyman_scott(rp, rd, wl.n_mean, wl.n_parents, wl.sigma_mpc)


def random_catalogue(wl: Workload, idx: int, n: int) -> np.ndarray:
    rr = rng_for(wl.cfg_id, ROLE_RANDOM, idx)
    if wl.periodic:
        return uniform_box(rr, n, wl.box_units)
    if wl.geometry == "slab":
        return slab_uniform(rr, n)
    return wedge_uniform(rr, n)


def subset_pair(wl: Workload, m: int) -> Tuple[int, int]:
    """Pool sub-catalogues (R1, R2) used by mock m: (2m mod K, 2m+1 mod K)."""
    k = wl.n_subsets
    return (2 * m) % k, (2 * m + 1) % k


def make_catalogues(wl: Workload, n_mock: Optional[int] = None,
                    progress: Optional[Callable[[str], None]] = None) -> Catalogues:
    """Draw every catalogue of a workload.

    Layout: mocks 0..n_mock-1, then the random sub-catalogues.  With a shared
    pool only the sub-catalogues some mock uses are drawn (pool index k is
    seeded by k, so a subset of mocks sees the same randoms as the full run).
    progress: called with a short message every 50 mocks (long workloads).
    """
    n_mock = wl.n_mock if n_mock is None else int(n_mock)
    cats = []
    for m in range(n_mock):
        cats.append(mock_catalogue(wl, m))
        if progress is not None and (m + 1) % 50 == 0:
            progress("%s: %d of %d mocks drawn" % (wl.name, m + 1, n_mock))
    randoms = np.zeros((n_mock, 2), dtype=np.int64)
    if wl.per_mock_randoms:
        for m in range(n_mock):
            n = cats[m].shape[1]
            for r in range(2):
                randoms[m, r] = len(cats)
                cats.append(random_catalogue(wl, 2 * m + r, n))
    else:
        used = sorted(set(k for m in range(n_mock) for k in subset_pair(wl, m)))
        pos = {}
        for k in used:
            pos[k] = len(cats)
            cats.append(random_catalogue(wl, k, wl.subset_size))
        for m in range(n_mock):
            a, b = subset_pair(wl, m)
            randoms[m] = (pos[a], pos[b])
    sizes = np.array([c.shape[1] for c in cats], dtype=np.int64)
    offsets = np.zeros(len(cats) + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    xyz = np.concatenate(cats, axis=1) if cats else np.zeros((3, 0), np.int32)
    return Catalogues(wl, np.ascontiguousarray(xyz, dtype=np.int32), offsets, n_mock, randoms)


def independent_poisson_mocks(cfg_id: int, n_mock: int, n_points: int, box_units: int,
                              n_random: int = 2) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Uniform ("random") mocks with their own random sub-catalogues of the
    same size (n_random of them: R1, R2, ...).

    Mirrors the paper's random-mock test (Sect. 4.2): data are themselves
    uniform with a fixed size, and every realisation has independent
    random catalogues.  Returns xyz int32 [3, n_total], offsets, and the
    (n_mock, 1 + n_random) catalogue ids (D, R1, R2, ...).
    """
    k = 1 + n_random
    cats, ids = [], np.zeros((n_mock, k), dtype=np.int64)
    for m in range(n_mock):
        for r in range(k):
            ids[m, r] = len(cats)
            cats.append(uniform_box(rng_for(cfg_id, ROLE_DATA if r == 0 else ROLE_RANDOM,
                                            k * m + r), n_points, box_units))
    sizes = np.array([c.shape[1] for c in cats], dtype=np.int64)
    offsets = np.zeros(len(cats) + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    return np.ascontiguousarray(np.concatenate(cats, axis=1)), offsets, ids
