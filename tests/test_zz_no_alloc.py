"""The allocation-free pair-count entry point against lc_pair_count_batch,
through the C ABI: two calls in a row (the second with a smaller input:
fewer and smaller catalogues, another binning), each bit-exact against the
allocating call on the same mesh, for the persistent and per-task launches;
plans beyond the static array and graph capture are refused."""
import dataclasses
import sys

import numpy as np
import pytest

import mockgen

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
    lc.lib()
    return lc


def _counts_both(lcmod, torch, pl, mode, tune=None):
    """Counts and stats of the allocating call, then of the allocation-free
    call, on the same mesh, tasks and binning."""
    out = []
    for fn in (lcmod.lc_pair_count_batch, lcmod.lc_pair_count_batch_noalloc):
        counts = torch.zeros_like(pl.counts)
        stats = torch.zeros(4, dtype=torch.int64, device="cuda")
        fn(pl.cells, pl.tasks, pl.binning, counts, mode, tune, stats)
        torch.cuda.synchronize()
        out.append((counts.cpu().numpy().view(np.uint64).copy(), stats.cpu().numpy().view(np.uint64).copy()))
    return out


@pytest.mark.parametrize("mode_name", ["persistent", "per_task"])
def test_noalloc_matches_allocating_call(torch, lcmod, mode_name):
    from paper_2205_11852_amd.pipeline import Pipeline
    mode = lcmod.LC_PERSISTENT if mode_name == "persistent" else lcmod.LC_PER_TASK
    big = mockgen.make_catalogues(mockgen.WORKLOADS["c1"], 8)
    wl_small = dataclasses.replace(mockgen.WORKLOADS["c1"], n_mean=2000.0, n_parents=100, subset_size=2000,
                                   n_r=12, r_max_mpc=60.0, n_mu=7)
    small = mockgen.make_catalogues(wl_small, 3)
    for step, cats in enumerate((big, small)):
        pl = Pipeline(cats)
        pl.build_cells()
        _say("[noalloc]", mode_name, "call", step, "tasks", len(pl.tasks), "bins", pl.binning.n_r, pl.binning.n_mu)
        (ref, sref), (got, sgot) = _counts_both(lcmod, torch, pl, mode)
        assert ref.sum() > 0
        assert np.array_equal(got, ref), (mode_name, step)
        assert sgot[0] == sref[0] and sgot[2] == sref[2], (sgot, sref)
        pl.cells.close()


def test_noalloc_repeated_calls_and_force_exact(torch, lcmod):
    """The array keeps the previous call's plan; every call rewrites it, its
    work-queue counters included: three calls in a row on one stream give
    the same counts, and the integer-rule-only mode agrees."""
    from paper_2205_11852_amd.pipeline import Pipeline
    cats = mockgen.make_catalogues(mockgen.WORKLOADS["c1"], 4)
    pl = Pipeline(cats)
    pl.build_cells()
    ref = None
    for rep in range(3):
        counts = torch.zeros_like(pl.counts)
        lcmod.lc_pair_count_batch_noalloc(pl.cells, pl.tasks, pl.binning, counts, lcmod.LC_PERSISTENT, None)
        torch.cuda.synchronize()
        got = counts.cpu().numpy().view(np.uint64).copy()
        if ref is None:
            (ref, _), _ = _counts_both(lcmod, torch, pl, lcmod.LC_PERSISTENT)
        assert np.array_equal(got, ref), rep
    (_, _), (ex, _) = _counts_both(lcmod, torch, pl, lcmod.LC_PERSISTENT | lcmod.LC_FORCE_EXACT)
    assert np.array_equal(ex, ref)
    pl.cells.close()


def test_noalloc_refuses_oversized_plan_and_graph(torch, lcmod):
    from paper_2205_11852_amd.pipeline import Pipeline
    cats = mockgen.make_catalogues(mockgen.WORKLOADS["c1"], 2)
    pl = Pipeline(cats)
    pl.build_cells()
    counts = torch.zeros_like(pl.counts)
    with pytest.raises(lcmod.LcError) as ei:
        lcmod.lc_pair_count_batch_noalloc(pl.cells, pl.tasks, pl.binning, counts, lcmod.LC_GRAPH, None)
    assert ei.value.status == lcmod.LC_ERR_INVALID
    # more tasks than the array's plan can hold: refused before any launch
    n = lcmod.LC_NOALLOC_PLAN_BYTES // 8 + 1
    many = np.zeros((n, 2), dtype=np.int32)
    big_counts = torch.zeros((n, pl.binning.n_r, pl.binning.n_mu), dtype=torch.int64, device="cuda")
    with pytest.raises(lcmod.LcError) as ei:
        lcmod.lc_pair_count_batch_noalloc(pl.cells, many, pl.binning, big_counts, lcmod.LC_PERSISTENT, None)
    assert ei.value.status == lcmod.LC_ERR_OVERFLOW
    assert not big_counts.any().item()
    # the array still serves a normal call afterwards
    (ref, _), (got, _) = _counts_both(lcmod, torch, pl, lcmod.LC_PERSISTENT)
    assert np.array_equal(got, ref)
    pl.cells.close()
