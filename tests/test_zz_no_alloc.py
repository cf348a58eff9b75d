"""ptyc_sweep_noalloc (the sweep that allocates nothing, its work memory a
fixed device array) through the C ABI against ptyc_sweep: the same object
and probe bytes and the same running errors, on two calls in a row, the
second with a smaller input."""
import numpy as np
import pytest

import oracle
import sim
from _parity import engine_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_10674_amd import _lib
    _lib.lib()


def _subset_schedule(order, off, keep):
    """The batches of (order, off) restricted to the indices below ``keep``
    (still pairwise disjoint), empty batches dropped."""
    o2, f2 = [], [0]
    for b in range(len(off) - 1):
        part = [int(j) for j in order[off[b]:off[b + 1]] if j < keep]
        if part:
            o2 += part
            f2.append(len(o2))
    return np.array(o2, np.int64), np.array(f2, np.int64)


def _same(a, b):
    np.testing.assert_array_equal(a.get_object(), b.get_object())
    np.testing.assert_array_equal(a.get_probe(), b.get_probe())


@pytest.mark.parametrize("cfg,count,keep", [(1, 600, 150), (2, 400, 60)])
def test_noalloc_equals_sweep_on_two_calls(cfg, count, keep):
    wl = sim.make_config(cfg, n_positions=count)
    a = engine_for(wl)                       # ptyc_sweep
    b = engine_for(wl)                       # ptyc_sweep_noalloc
    order, off = a.get_schedule()
    # first call: two sweeps of the library's own schedule over all positions
    ea = a.sweep(2, errors=True)
    eb = b.sweep_noalloc(2, errors=True)
    _same(a, b)
    np.testing.assert_array_equal(ea, eb)
    assert a.sweeps_done == b.sweeps_done == 2
    # second call, smaller input: an explicit schedule over the first `keep` positions
    o2, f2 = _subset_schedule(order, off, keep)
    oracle.check_schedule(wl.positions, wl.n, o2, f2)
    ea = a.sweep(1, order=o2, batch_offsets=f2, errors=True)
    eb = b.sweep_noalloc(1, order=o2, batch_offsets=f2, errors=True)
    _same(a, b)
    np.testing.assert_array_equal(ea, eb)


def test_noalloc_strict_mode_and_other_size():
    """Sequential ePIE (every position its own batch) at 32 px."""
    wl = sim.make_config(0)
    a = engine_for(wl)
    b = engine_for(wl)
    for s in range(2):
        order = sim.sweep_order(wl.seed, s, wl.count)[: 100 - 40 * s]
        ea = a.sweep(1, order=order, errors=True)
        eb = b.sweep_noalloc(1, order=order, errors=True)
        _same(a, b)
        np.testing.assert_array_equal(ea, eb)


def test_noalloc_rejects_oversized_calls():
    from paper_2308_10674_amd import PtycError, _lib as L
    wl = sim.make_config(0)
    b = engine_for(wl)
    with pytest.raises(PtycError) as e:
        b.sweep_noalloc(L.PTYC_NOALLOC_BYTES // 8)
    assert e.value.status == L.PTYC_ERR_ARG
    assert b.sweeps_done == 0
    np.testing.assert_array_equal(b.get_object(), wl.object0.astype(np.complex64))
    b.sweep_noalloc(1)                       # still usable
    assert b.sweeps_done == 1
