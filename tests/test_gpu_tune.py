"""Tile variants of the per-batch kernels and the run-time tuner (through
the C ABI): every variant produces the same object and probe bytes, in the
batch and the graph form, and tuning leaves the reconstruction unchanged."""
import numpy as np
import pytest

import sim
from _parity import engine_for, progress

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _raster64(count=120):
    n, side = 64, 11
    step = max(1, int(round(0.094 * n)))
    cen = np.stack(np.meshgrid(np.arange(side), np.arange(side), indexing="ij"), -1).reshape(-1, 2)[:count] * step
    h, w, corners = sim.object_extent(cen, n, 32)
    return sim.make_workload(n, None, 20.0, 0.025, corners, 1e7, 900, h=h, w=w)


@pytest.mark.parametrize("which", ["n64", "n128", "n256"])
def test_variants_give_the_same_bytes(which):
    wl = {"n64": lambda: _raster64(), "n128": lambda: sim.make_config(1, n_positions=600),
          "n256": lambda: sim.make_config(2, n_positions=400)}[which]()
    ref = engine_for(wl)
    assert ref.tile == 0
    e_ref = ref.sweep(2, errors=True)
    O, P = ref.get_object(), ref.get_probe()
    assert ref.tile_count >= 2
    for form in ("batch", "graph"):
        for v in range(ref.tile_count):
            e = engine_for(wl, form=form)
            e.tile = v
            assert e.tile == v
            err = e.sweep(2, errors=True)
            np.testing.assert_array_equal(e.get_object(), O, err_msg=f"{form} variant {v}")
            np.testing.assert_array_equal(e.get_probe(), P, err_msg=f"{form} variant {v}")
            np.testing.assert_allclose(err, e_ref, rtol=1e-12)
            e.close()
    progress(f"tile variants {which}: {ref.tile_count} agree")


def test_graph_is_rebuilt_when_the_tile_changes():
    """A tile change between sweeps in the graph form rebuilds the graph; the
    bytes stay those of the batch form."""
    wl = sim.make_config(1, n_positions=600)
    g = engine_for(wl, form="graph")
    b = engine_for(wl)
    for v in (0, 2, 1, 0):
        g.tile = v
        g.sweep(1)
        b.sweep(1)
        np.testing.assert_array_equal(g.get_object(), b.get_object(), err_msg=f"variant {v}")
        np.testing.assert_array_equal(g.get_probe(), b.get_probe(), err_msg=f"variant {v}")


def test_tune_leaves_the_reconstruction_unchanged():
    wl = sim.make_config(1, n_positions=600)
    a = engine_for(wl)
    b = engine_for(wl)
    a.sweep(1)
    b.sweep(1)
    t, ms = a.tune(reps=2)
    print("tuned variant", t, "ms per sweep", ms)
    assert 0 <= t < a.tile_count and a.tile == t
    assert len(ms) == a.tile_count and all(m > 0 for m in ms)
    assert a.sweeps_done == b.sweeps_done
    np.testing.assert_array_equal(a.get_object(), b.get_object())
    np.testing.assert_array_equal(a.get_probe(), b.get_probe())
    oa, fa = a.get_schedule()
    ob, fb = b.get_schedule()
    np.testing.assert_array_equal(oa, ob)
    np.testing.assert_array_equal(fa, fb)
    a.sweep(2)
    b.sweep(2)
    np.testing.assert_array_equal(a.get_object(), b.get_object())
    np.testing.assert_array_equal(a.get_probe(), b.get_probe())


def test_tune_keeps_the_form_and_its_maxima():
    """Tuning a context in the persistent form times the batch form and
    hands back the persistent form with its own layout of the maxima."""
    wl = sim.make_config(1, n_positions=300)
    a = engine_for(wl, form="persistent")
    b = engine_for(wl, form="persistent")
    a.tune(reps=1)
    assert a.form == "persistent"
    a.sweep(2)
    b.sweep(2)
    np.testing.assert_array_equal(a.get_object(), b.get_object())
    np.testing.assert_array_equal(a.get_probe(), b.get_probe())


def test_tile_errors_and_trivial_cases():
    from paper_2308_10674_amd import PtycError
    wl = sim.make_config(0, n_positions=20)
    e = engine_for(wl)
    assert e.tile_count == 1
    with pytest.raises(PtycError):
        e.tile = 1
    with pytest.raises(PtycError):
        e.tile = -1
    with pytest.raises(PtycError):
        e.tune(reps=0)
    assert e.tune() == (0, [0.0])          # one variant: nothing to time
    empty = engine_for(sim.make_config(1, n_positions=10), count=0)
    t, ms = empty.tune()
    assert t == 0 and all(m == 0.0 for m in ms)
