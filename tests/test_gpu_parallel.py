"""The paper's subset-parallel scheme on the GPU: four round-robin subsets
iterated together (ptyc_sweep_multi) and synchronised by averaging object
and probe (ptyc_average), against the FP64 oracle's scheme."""
import numpy as np
import pytest

import oracle
import sim
from _parity import RTOL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _contexts(wl, subsets):
    from paper_2308_10674_amd import Engine
    engs = []
    for k, sub in enumerate(subsets):
        e = Engine(wl.n, wl.h, wl.w, wl.probe0, wl.object0, mode="coloured", seed=wl.seed + k)
        e.add_positions(wl.positions[sub], wl.intensities[sub])
        engs.append(e)
    return engs


def test_average_is_the_mean():
    from paper_2308_10674_amd import average, sweep_multi
    wl = sim.make_config(1, n_positions=200)
    subsets = oracle.round_robin(wl.count, 3)
    engs = _contexts(wl, subsets)
    sweep_multi(engs, 1)
    objs = [e.get_object().astype(np.complex128) for e in engs]
    probes = [e.get_probe().astype(np.complex128) for e in engs]
    average(engs)
    O = [e.get_object() for e in engs]
    P = [e.get_probe() for e in engs]
    for k in range(1, 3):
        np.testing.assert_array_equal(O[k], O[0])
        np.testing.assert_array_equal(P[k], P[0])
    np.testing.assert_allclose(O[0], sum(objs) / 3, rtol=3e-7, atol=1e-7)
    np.testing.assert_allclose(P[0], sum(probes) / 3, rtol=3e-7, atol=1e-7 * np.abs(P[0]).max())


def _floor(O, P, wl, subsets, scheds, mask):
    """FP32 rounding alone: the scheme run by the oracle in complex64 on
    globally phase-rotated copies (an exact symmetry)."""
    O64, P64, _ = oracle.subset_round(O, P, wl.positions, wl.intensities, subsets, scheds)
    fo = fp = 0.0
    for ang in (0.0, 0.7, 2.3):
        r = np.exp(1j * ang)
        O32, P32, _ = oracle.subset_round((O * r).astype(np.complex64), (P * r).astype(np.complex64), wl.positions,
                                          wl.intensities, subsets, scheds, dtype=np.complex64)
        fo = max(fo, oracle.rel_l2(O32 / np.complex64(r), O64, mask))
        fp = max(fp, oracle.rel_l2(P32 / np.complex64(r), P64))
    return fo, fp


def test_parallel_rounds_match_oracle():
    """Two rounds of one sweep per subset; each round re-synced to the
    oracle's state; the first round starts from the paper's initial values."""
    from paper_2308_10674_amd import average, sweep_multi
    wl = sim.make_config(1, n_positions=400)
    subsets = oracle.round_robin(wl.count, 4)
    engs = _contexts(wl, subsets)
    mask = oracle.union_mask(wl.positions, wl.n, wl.h, wl.w)
    O, P = wl.object0, wl.probe0
    for rnd in range(3):
        for e in engs:
            e.set_object(O.astype(np.complex64))
            e.set_probe(P.astype(np.complex64))
        scheds = [[e.get_schedule()] for e in engs]
        sweep_multi(engs, 1)
        average(engs)
        Og, Pg = engs[0].get_object(), engs[0].get_probe()
        On, Pn, _ = oracle.subset_round(O, P, wl.positions, wl.intensities, subsets, scheds)
        ro, rp = oracle.rel_l2(Og, On, mask), oracle.rel_l2(Pg, Pn)
        fo = fp = 0.0
        if max(ro, rp) > RTOL:
            fo, fp = _floor(O, P, wl, subsets, scheds, mask)
        print("round", rnd, "rel object", ro, "probe", rp, "fp32 floor", fo, fp, flush=True)
        assert ro <= max(RTOL, 10 * fo) and rp <= max(RTOL, 10 * fp)
        O, P = On, Pn


def test_average_rejects_mismatched_geometry():
    from paper_2308_10674_amd import Engine, PtycError, average
    a = sim.make_config(0)
    e1 = Engine(a.n, a.h, a.w, a.probe0, a.object0, mode="strict")
    e2 = Engine(a.n, a.h + 1, a.w, a.probe0, np.ones((a.h + 1, a.w), np.complex64), mode="strict")
    with pytest.raises(PtycError):
        average([e1, e2])
    with pytest.raises(PtycError):
        average([e1, e1])
