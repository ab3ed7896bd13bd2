"""The seeded input generators (CPU): reproducibility, Poisson sizes,
coordinate ranges, the wedge selection and the slab shape."""
import dataclasses
import math

import numpy as np

import mockgen

U = mockgen.UNITS_PER_MPC


def _small(name, **kw):
    return dataclasses.replace(mockgen.WORKLOADS[name], **kw)


def test_catalogues_are_reproducible_and_seeded_by_config():
    wl = _small("c1", n_mock=3)
    a, b = mockgen.make_catalogues(wl), mockgen.make_catalogues(wl)
    assert np.array_equal(a.xyz, b.xyz) and np.array_equal(a.offsets, b.offsets)
    other = mockgen.make_catalogues(dataclasses.replace(wl, cfg_id=99))
    assert not np.array_equal(a.cat(0), other.cat(0))
    # a subset of the mocks sees the same catalogues as the full run
    full = mockgen.make_catalogues(_small("c1", n_mock=5))
    assert np.array_equal(full.cat(1), a.cat(1))


def test_neyman_scott_sizes_are_poisson():
    n_mean, draws = 400.0, 400
    sizes = [mockgen.neyman_scott_box(mockgen.rng_for(7, 0, i), mockgen.rng_for(7, 1, i), n_mean, 20, 5.0,
                                      1000 * U).shape[1] for i in range(draws)]
    m, v = np.mean(sizes), np.var(sizes, ddof=1)
    assert abs(m - n_mean) < 4 * math.sqrt(n_mean / draws)
    assert abs(v / n_mean - 1.0) < 0.25                      # Poisson: variance = mean


def test_periodic_coordinates_in_the_box():
    wl = _small("c1", n_mock=4)
    cats = mockgen.make_catalogues(wl)
    assert cats.xyz.min() >= 0 and cats.xyz.max() < wl.box_units
    r1, r2 = cats.randoms.T
    assert np.all(r1 != r2) and np.all(r1 >= cats.n_mock)          # two distinct random sub-catalogues


def test_wedge_mask_and_radial_density():
    """Points fill the 60 x 60 degree wedge between 1200 and 2400 Mpc/h, with a
    number density falling linearly by 3x from the near to the far edge."""
    pts = mockgen.wedge_uniform(mockgen.rng_for(4, 2, 0), 200000).astype(np.float64) / U
    chi = np.sqrt((pts ** 2).sum(axis=0))
    alpha = np.degrees(np.arctan2(pts[1], pts[0]))
    dec = np.degrees(np.arcsin(pts[2] / chi))
    assert chi.min() >= 1200 - 1e-3 and chi.max() < 2400 + 1e-3
    assert np.all(np.abs(alpha) <= 30 + 1e-3) and np.all(np.abs(dec) <= 30 + 1e-3)
    # n(chi) from counts in shells divided by shell volume (chi^2 dchi)
    h, e = np.histogram(chi, bins=12, range=(1200, 2400))
    c = 0.5 * (e[1:] + e[:-1])
    n = h / c ** 2
    ratio = n[0] / n[-1]
    assert 2.6 < ratio < 3.4, ratio
    slope = np.polyfit(c, n / n[0], 1)[0]
    assert slope < 0


def test_slab_shape_mean_and_scatter():
    """The paper's slabs: points inside 1500 x 1500 x 300 Mpc/h, about 156 158 on
    average with a few percent of scatter; randoms fill the same slab."""
    wl = mockgen.WORKLOADS["slab"]
    sizes = []
    for m in range(24):
        c = mockgen.mock_catalogue(wl, m)
        sizes.append(c.shape[1])
        if m < 2:
            assert c.min() >= 0 and c[:2].max() < 1500 * U and c[2].max() < 300 * U
    assert abs(np.mean(sizes) / wl.n_mean - 1.0) < 0.025
    assert 0.015 < np.std(sizes) / np.mean(sizes) < 0.06
    r = mockgen.random_catalogue(wl, 0, 50000)
    assert r.min() >= 0 and r[:2].max() < 1500 * U and r[2].max() < 300 * U
    # uniform in z across the slab's depth
    h = np.histogram(r[2], bins=6, range=(0, 300 * U))[0]
    assert np.all(np.abs(h / h.mean() - 1) < 0.05)


def test_independent_poisson_mocks_layout():
    xyz, off, ids = mockgen.independent_poisson_mocks(3, 4, 100, 1 << 16, n_random=3)
    assert ids.shape == (4, 4) and len(off) == 17
    assert np.all(np.diff(off) == 100)
    assert len(set(ids.ravel().tolist())) == 16
    assert xyz.min() >= 0 and xyz.max() < (1 << 16)
