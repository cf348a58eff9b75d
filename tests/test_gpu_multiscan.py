"""Several independent reconstructions advanced together (ptyc_sweep_multi):
the same bytes as each context sweeping alone, and each context's batches
re-synced to the oracle."""
import numpy as np
import pytest

import oracle
import sim
from _parity import check_batches, engine_for, run_batches_resynced

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _scans():
    """Five small scans of three pattern sizes, uneven position counts."""
    out = []
    for k, (n, side, count) in enumerate([(64, 9, 81), (128, 12, 140), (64, 7, 40), (256, 6, 36), (128, 5, 25)]):
        step = max(1, int(round(0.094 * n)))
        cen = np.stack(np.meshgrid(np.arange(side), np.arange(side), indexing="ij"), -1).reshape(-1, 2)[:count] * step
        h, w, corners = sim.object_extent(cen, n, 32)
        r = {64: 20.0, 128: 40.0, 256: 70.0}[n]
        wl = sim.make_workload(n, None, r, 0.5 / r, corners, 1e7, 500 + k, h=h, w=w)
        out.append(wl)
    return out


@pytest.mark.parametrize("errors", [True, False])
def test_multi_equals_individual_sweeps(errors):
    """Same bytes as sweeping alone, with and without the per-sweep error
    reductions between the batch launches.  (This comparison caught a
    workgroup of the inverse stage reading a probe maximum that another
    workgroup of the same launch had already replaced, once launches
    started to stagger.)"""
    from paper_2308_10674_amd import sweep_multi
    scans = _scans()
    together = [engine_for(wl) for wl in scans]
    alone = [engine_for(wl) for wl in scans]
    empty = engine_for(scans[0], count=0)
    err_m = sweep_multi(together + [empty], 3, errors=errors)
    for e_alone, e_tog, k in zip(alone, together, range(len(scans))):
        err_a = e_alone.sweep(3, errors=True)
        np.testing.assert_array_equal(e_tog.get_object(), e_alone.get_object())
        np.testing.assert_array_equal(e_tog.get_probe(), e_alone.get_probe())
        if errors:
            np.testing.assert_allclose(err_m[k], err_a, rtol=1e-13)
        assert e_tog.sweeps_done == 3
    if errors:
        np.testing.assert_array_equal(err_m[-1], 0.0)
    # the next default schedules continue in step
    for e_alone, e_tog in zip(alone, together):
        oa, fa = e_alone.get_schedule()
        ot, ft = e_tog.get_schedule()
        np.testing.assert_array_equal(oa, ot)


def test_multi_each_scan_matches_oracle():
    """After a joint sweep, the next batch-by-batch sweep of every scan agrees
    with the FP64 oracle (the joint call leaves per-scan state consistent)."""
    from paper_2308_10674_amd import sweep_multi
    scans = _scans()[:3]
    engs = [engine_for(wl) for wl in scans]
    sweep_multi(engs, 1)
    for wl, eng in zip(scans, engs):
        order, off = eng.get_schedule()
        # start the oracle from the state the oracle itself reaches after the same first sweep
        o0, f0 = _first_schedule(wl)
        O1, P1, _, _ = oracle.sweep_coloured(wl.object0, wl.probe0, wl.positions, wl.intensities, o0, f0)
        rows, _ = run_batches_resynced(eng, wl, order, off, start=(O1, P1), label=f"multi n{wl.n}")
        check_batches(rows)


def _first_schedule(wl):
    e = engine_for(wl)
    return e.get_schedule()


def test_multi_small_and_mixed_sizes_together():
    """32 px contexts take the per-size launches and 64/128/256 px the
    mixed-size ones in the same call; every context still equals its own
    sweeps bit for bit, and its error agrees."""
    from paper_2308_10674_amd import sweep_multi
    scans = _scans()
    for k, (n, side) in enumerate([(32, 8), (32, 5)]):
        step = max(1, int(round(0.094 * n)))
        cen = np.stack(np.meshgrid(np.arange(side), np.arange(side), indexing="ij"), -1).reshape(-1, 2) * step
        h, w, corners = sim.object_extent(cen, n, 16)
        scans.append(sim.make_workload(n, None, 10.0, 0.05, corners, 1e6, 700 + k, h=h, w=w))
    together = [engine_for(wl) for wl in scans]
    err_m = sweep_multi(together, 2, errors=True)
    for k, (wl, e_tog) in enumerate(zip(scans, together)):
        e_alone = engine_for(wl)
        err_a = e_alone.sweep(2, errors=True)
        np.testing.assert_array_equal(e_tog.get_object(), e_alone.get_object(), err_msg=f"n{wl.n}")
        np.testing.assert_array_equal(e_tog.get_probe(), e_alone.get_probe(), err_msg=f"n{wl.n}")
        np.testing.assert_allclose(err_m[k], err_a, rtol=1e-13)


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5, 6])
def test_every_multi_variant_equals_individual_sweeps(variant):
    """The persistent launches (one kernel, a group of workgroups and its
    own barriers per scan; several inverse tiles and shares) and the
    stepped launches all give each scan the bytes of its own sweeps."""
    from paper_2308_10674_amd import sweep_multi
    scans = _scans()
    together = [engine_for(wl) for wl in scans]
    together[0].multi_variant = variant
    err_m = sweep_multi(together, 2, errors=True)
    for k, (wl, e_tog) in enumerate(zip(scans, together)):
        e_alone = engine_for(wl)
        err_a = e_alone.sweep(2, errors=True)
        np.testing.assert_array_equal(e_tog.get_object(), e_alone.get_object(), err_msg=f"scan {k}")
        np.testing.assert_array_equal(e_tog.get_probe(), e_alone.get_probe(), err_msg=f"scan {k}")
        np.testing.assert_allclose(err_m[k], err_a, rtol=1e-13)


def _spiral_scans():
    """Fermat spirals whose colour batches hold 1-9 positions (64, 128 and
    256 px), so the eight-slot inverse tile of the stepped launches runs
    with one and with two slot rounds."""
    out = []
    for k, (n, rfac, count) in enumerate([(64, 4.0, 300), (128, 12.0, 250), (256, 24.0, 300)]):
        t = np.arange(count, dtype=np.float64)
        rho = rfac * np.sqrt(t)
        th = t * np.pi * (3.0 - np.sqrt(5.0))
        cen = np.stack([np.rint(rho * np.sin(th)), np.rint(rho * np.cos(th))], 1)
        h, w, corners = sim.object_extent(cen, n, 32)
        r = {64: 20.0, 128: 40.0, 256: 70.0}[n]
        out.append(sim.make_workload(n, None, r, 0.5 / r, corners, 1e7, 520 + k, h=h, w=w))
    return out


@pytest.mark.parametrize("variant", [4, 5, 6])
def test_spiral_batches_equal_individual_sweeps(variant):
    """Stepped launches over spiral scans with batches of one to nine
    positions (the default and the eight-slot inverse tiles): each scan gets
    the bytes of its own sweeps."""
    from paper_2308_10674_amd import sweep_multi
    from paper_2308_10674_amd.engine import colour
    scans = _spiral_scans()
    sizes = set()
    for wl in scans:
        col, _ = colour(wl.positions, wl.n)
        sizes |= set(np.bincount(col).tolist())
    assert {1, 8, 9} <= sizes     # the eight-slot tile in one and in two slot rounds
    together = [engine_for(wl) for wl in scans]
    together[0].multi_variant = variant
    err_m = sweep_multi(together, 2, errors=True)
    for k, (wl, e_tog) in enumerate(zip(scans, together)):
        e_alone = engine_for(wl)
        err_a = e_alone.sweep(2, errors=True)
        np.testing.assert_array_equal(e_tog.get_object(), e_alone.get_object(), err_msg=f"scan {k}")
        np.testing.assert_array_equal(e_tog.get_probe(), e_alone.get_probe(), err_msg=f"scan {k}")
        np.testing.assert_allclose(err_m[k], err_a, rtol=1e-13)


def test_multi_graph_form_replays():
    """The persistent multi-scan launch captured as a graph, replayed by
    three calls in a row (the second and third reuse the graph): the same
    bytes as the cooperative launch."""
    from paper_2308_10674_amd import sweep_multi
    scans = _scans()
    g = [engine_for(wl) for wl in scans]
    b = [engine_for(wl) for wl in scans]
    g[0].form = "graph"
    for k in range(3):
        eg = sweep_multi(g, 1, errors=True)
        eb = sweep_multi(b, 1, errors=True)
        np.testing.assert_allclose(eg, eb, rtol=0)
    for e_g, e_b in zip(g, b):
        np.testing.assert_array_equal(e_g.get_object(), e_b.get_object())
        np.testing.assert_array_equal(e_g.get_probe(), e_b.get_probe())


def test_tune_multi_keeps_state():
    """The tuner times every variant and restores every scan's state and
    sweep counter: a joint sweep after tuning equals one without it."""
    from paper_2308_10674_amd import sweep_multi, tune_multi
    scans = _scans()
    t = [engine_for(wl) for wl in scans]
    r = [engine_for(wl) for wl in scans]
    sweep_multi(t, 1)
    sweep_multi(r, 1)
    v, ms = tune_multi(t, 1)
    assert 0 <= v < len(ms) and all(m > 0 for m in ms)
    assert all(e.sweeps_done == 1 for e in t)
    sweep_multi(t, 1)
    sweep_multi(r, 1)
    for e_t, e_r in zip(t, r):
        np.testing.assert_array_equal(e_t.get_object(), e_r.get_object())
        np.testing.assert_array_equal(e_t.get_probe(), e_r.get_probe())


def test_multi_rejects_bad_lists():
    from paper_2308_10674_amd import PtycError, sweep_multi
    scans = _scans()[:2]
    a = engine_for(scans[0])
    with pytest.raises(PtycError):
        sweep_multi([a, a], 1)
    with pytest.raises(PtycError):
        sweep_multi([], 1)
