"""Shared helpers of the GPU parity tests: build an engine from a workload,
run the oracle on the same schedule, compare."""
from __future__ import annotations

import numpy as np

import oracle
import sim

RTOL = 1e-5   # relative L2 per re-synced sweep (FP32 GPU against the FP64 oracle)


def engine_for(wl, mode=None, max_batch=0, seed=None, count=None, alpha=None, beta=None):
    from paper_2308_10674_amd import Engine
    mode = mode or ("strict" if wl.mode == "strict" else "coloured")
    eng = Engine(wl.n, wl.h, wl.w, wl.probe0, wl.object0,
                 alpha=wl.alpha if alpha is None else alpha, beta=wl.beta if beta is None else beta,
                 mode=mode, max_batch=max_batch, seed=wl.seed if seed is None else seed)
    count = wl.count if count is None else count
    if count:
        eng.add_positions(wl.positions[:count], wl.intensities[:count])
    return eng


def oracle_sweep(O, P, wl, order, off, dtype=np.complex128, alpha=None, beta=None, count=None):
    count = wl.count if count is None else count
    a = wl.alpha if alpha is None else alpha
    b = wl.beta if beta is None else beta
    pos, inten = wl.positions[:count], wl.intensities[:count]
    if off is None:
        return oracle.sweep_strict(O, P, pos, inten, order, a, b, dtype)
    return oracle.sweep_coloured(O, P, pos, inten, order, off, a, b, dtype)


def fp32_floor(O, P, wl, order, off, mask, count=None, **kw):
    """Deviation of the oracle run in complex64 from the FP64 oracle on the
    same sweep: what any FP32 implementation inherits from the problem's
    conditioning."""
    O64, P64, _, _ = oracle_sweep(O, P, wl, order, off, count=count, **kw)
    O32, P32, _, _ = oracle_sweep(O.astype(np.complex64), P.astype(np.complex64), wl, order, off,
                                  dtype=np.complex64, count=count, **kw)
    return oracle.rel_l2(O32, O64, mask), oracle.rel_l2(P32, P64)


def gate(rel, floor):
    """The parity bar: 1e-5, unless even the FP32 oracle misses that on this
    sweep (ill-conditioned Fourier phases), then three times its deviation."""
    return max(RTOL, 3.0 * floor)


def run_resynced(eng, wl, n_sweeps, schedule, count=None, start=None, label=""):
    """For each sweep: take its (order, offsets) from ``schedule(s)``, reset
    the GPU to the oracle's state, run one sweep on both, compare.  Returns
    the rows (also printed) and the oracle's final (object, probe)."""
    count = wl.count if count is None else count
    mask = oracle.union_mask(wl.positions[:count], wl.n, wl.h, wl.w)
    O, P = (wl.object0, wl.probe0) if start is None else start
    rows = []
    for s in range(n_sweeps):
        order, off = schedule(s)
        if off is not None:
            oracle.check_schedule(wl.positions[:count], wl.n, order, off)
        eng.set_object(O.astype(np.complex64))
        eng.set_probe(P.astype(np.complex64))
        err = eng.sweep(1, order=order, batch_offsets=off, errors=True)[0]
        Og, Pg = eng.get_object(), eng.get_probe()
        On, Pn, num, den = oracle_sweep(O, P, wl, order, off, count=count)
        fo, fp = fp32_floor(O, P, wl, order, off, mask, count=count)
        rows.append(dict(sweep=s, rel_o=oracle.rel_l2(Og, On, mask), rel_p=oracle.rel_l2(Pg, Pn),
                         floor_o=fo, floor_p=fp, err_gpu=float(err), err_orc=num / den,
                         untouched_equal=bool(np.array_equal(Og[~mask], O.astype(np.complex64)[~mask]))))
        print(label, rows[-1], flush=True)
        O, P = On, Pn
    return rows, (O, P)


def check_rows(rows, final=None, err_rtol=1e-4):
    for r in rows:
        assert r["rel_o"] <= gate(r["rel_o"], r["floor_o"]), r
        assert r["rel_p"] <= gate(r["rel_p"], r["floor_p"]), r
        assert abs(r["err_gpu"] - r["err_orc"]) <= err_rtol * r["err_orc"] + 1e-12, r
        assert r["untouched_equal"], r


def library_schedule(eng):
    """Schedule source: the library's own next schedule, exported."""
    return lambda s: eng.get_schedule()


def strict_schedule(wl, count=None):
    count = wl.count if count is None else count
    return lambda s: (sim.sweep_order(wl.seed, s, count), None)
