"""Throughput benchmark: ePIE position updates per second on one MI355X.

A step is one sweep of the coloured-batch ePIE over every loaded position of
the 128 px workload: 60 x 60 raster (step 12 px, jitter +-2), 3600
positions, 1024 x 1024 object, Poisson data at 1e7 photons per pattern
(synthetic, seeded).  Inputs are resident in HBM before the timed region;
the library's own shuffled colour schedule runs each sweep.  By default the
256 px workload (20000-position Fermat spiral, 2048 x 2048 object, 1e8
photons) is timed as well and reported under "n256".

Roofline: the algorithmic HBM traffic of one position update is 20 N^2
bytes (read sqrt(I) 4 N^2, read the object window 8 N^2, write it 8 N^2);
the probe and the exchange buffers are not counted.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(n: int) -> int:
    return 20 * n * n


# algorithmic bytes per position update of each kernel: what it must move of
# the method's own state (the exchange buffers are not counted)
KERNEL_BYTES = {
    "k_rows_fwd": lambda n: 8 * n * n,    # read the object window
    "k_cols": lambda n: 4 * n * n,        # read sqrt(I)
    "k_rows_inv": lambda n: 16 * n * n,   # read and write the object window
    "k_sweep": lambda n: 20 * n * n,      # the whole update
}


KERNEL_SOURCES = ("kernels.hip", "kernels.h", "fft.h")


def kernel_source_hash():
    """sha256 prefix over the sources the kernels are compiled from."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2308_10674_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel, n):
    """HBM bytes per launch of ``kernel`` at pattern size ``n`` from the
    committed rocprofv3 counter summaries (lines 'traffic-json: {...}' in
    profiles/*.md), if they were taken on the current kernel source."""
    pdir = os.path.join(ROOT, "profiles")
    h = kernel_source_hash()
    try:
        names = sorted(os.listdir(pdir))
    except OSError:
        return None
    for name in names:
        if not name.endswith(".md"):
            continue
        with open(os.path.join(pdir, name)) as f:
            for line in f:
                if line.startswith("traffic-json:"):
                    rec = json.loads(line.split(":", 1)[1])
                    if rec.get("kernel") == kernel and rec.get("n") == n and rec.get("kernels_sha256") == h:
                        return rec
    return None


def run_gpu(cfg_id, steps, warmup, form, positions=None, tile=None):
    import torch

    import sim
    from paper_2308_10674_amd import Engine

    t0 = time.time()
    wl = sim.make_config(cfg_id, n_positions=positions)
    gen_s = time.time() - t0
    dev = torch.device("cuda:0")
    inten = torch.from_numpy(wl.intensities).to(dev)
    pos = torch.from_numpy(wl.positions).to(dev)
    eng = Engine(wl.n, wl.h, wl.w, wl.probe0, wl.object0, mode="coloured", seed=wl.seed, form=form)
    t1 = time.time()
    eng.add_positions(pos, inten)
    torch.cuda.synchronize()
    ingest_s = time.time() - t1
    del inten
    tile_ms = []
    if tile is None:
        tile, tile_ms = eng.tune(3)        # keep a clearly faster tile variant (state unchanged)
    else:
        eng.tile = tile
    order, off = eng.get_schedule()
    sizes = np.diff(off)
    eng.sweep(warmup)
    torch.cuda.synchronize()
    # exactly `steps` sweeps between the first and the last event; the
    # events between them split the run into (up to) five segments whose
    # per-sweep times give the median reported beside the total
    segs = [steps // 5 + (1 if k < steps % 5 else 0) for k in range(5)]
    segs = [k for k in segs if k > 0]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(segs) + 1)]
    ev[0].record()
    for k, n_s in enumerate(segs):
        eng.sweep(n_s)
        ev[k + 1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[-1])
    seg_ms = [ev[k].elapsed_time(ev[k + 1]) / segs[k] for k in range(len(segs))]
    err = eng.sweep(1, errors=True)[0]
    updates = wl.count * steps
    rate = updates / (ms / 1e3)
    achieved = algorithmic_bytes(wl.n) * rate / 1e9
    # per-kernel event timing over the same number of sweeps (a second pass,
    # so the events do not disturb the timed region above)
    eng.profile(True)
    eng.sweep(steps)
    kern = eng.profile_read()
    eng.profile(False)
    return dict(wl=wl, ms=ms, seg_ms=seg_ms, rate=rate, achieved_gbs=achieved, batches=int(len(sizes)),
                mean_batch=float(sizes.mean()), max_batch=int(sizes.max()), gen_s=gen_s,
                ingest_s=ingest_s, err=float(err), kernels=kern, tile=tile,
                tile_ms=[round(m, 4) for m in tile_ms])


def run_forms(wl, steps, strict_steps=1):
    """Updates/s of the other launch forms on the same workload: the sweep
    graph, the persistent kernel (one cooperative launch per sweep with
    software barriers between the stages; slower here than three launches
    per batch, kept for comparison), and strict ePIE (every position its own
    batch: one group of three launches per position)."""
    import torch

    from paper_2308_10674_amd import Engine

    out = {}
    inten = torch.from_numpy(wl.intensities).cuda()
    pos = torch.from_numpy(wl.positions).cuda()
    for name, form, mode, k in (("graph", "graph", "coloured", steps), ("persistent", "persistent", "coloured", steps),
                                ("per_position", "batch", "strict", strict_steps)):
        eng = Engine(wl.n, wl.h, wl.w, wl.probe0, wl.object0, mode=mode, seed=wl.seed, form=form)
        eng.add_positions(pos, inten)
        eng.sweep(1)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        eng.sweep(k)
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1])
        out[name] = {"value": round(wl.count * k / (ms / 1e3), 1), "ms_per_step": round(ms / k, 3), "steps": k,
                     "mode": mode}
        eng.close()
    out["unit"] = "position updates/s"
    return out


def run_config0(steps=20):
    """Sequential ePIE on the 32 px workload (10 x 10 raster, 128 x 128
    object), one sweep per step in the paper's order semantics: one group
    of three launches per position against the one-workgroup sequential
    kernel (the persistent form in strict mode)."""
    import torch

    import sim
    from paper_2308_10674_amd import Engine

    wl = sim.make_config(0)
    out = {"workload": "32x32 patterns, 10x10 raster (100 positions), 128x128 object, sequential (strict) ePIE",
           "unit": "position updates/s"}
    for name, form, k in (("per_position_launches", "batch", max(2, steps // 4)), ("sequential_kernel", "persistent", steps)):
        eng = Engine(wl.n, wl.h, wl.w, wl.probe0, wl.object0, mode="strict", seed=wl.seed, form=form)
        eng.add_positions(wl.positions, wl.intensities)
        eng.sweep(2)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        eng.sweep(k)
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1])
        out[name] = {"value": round(wl.count * k / (ms / 1e3), 1), "ms_per_step": round(ms / k, 4), "steps": k}
        eng.close()
    return out


def run_gradient(epochs=10, minibatch=512, lr=1e-2):
    """Gradient reconstruction throughput on the 128 px workload (3600
    positions, 1024 x 1024 object): Adam (fused) over shuffled minibatches of 512
    with the amplitude loss and its hand-written adjoint (AmplitudeLoss),
    timed over `epochs` epochs after one warm-up epoch.  Rate: position
    gradients per second (one position's loss term and its contribution to
    dL/dO and dL/dP).  Path roofline: 28 N^2 algorithmic bytes per position
    gradient (read sqrt(I) 4 N^2, read the window 8 N^2, read and write the
    window of dL/dO 16 N^2); Adam's own update of O and P is not counted."""
    import torch

    import sim
    from paper_2308_10674_amd import Engine, amplitude_loss

    wl = sim.make_config(3)
    eng = Engine(wl.n, wl.h, wl.w, wl.probe0, wl.object0, mode="coloured", seed=wl.seed)
    eng.add_positions(torch.from_numpy(wl.positions).cuda(), torch.from_numpy(wl.intensities).cuda())
    # the parameters are the real views (re, im) of O and P: PyTorch's Adam
    # treats a complex parameter as exactly that view, and its fused
    # implementation takes real tensors only
    Or = torch.view_as_real(torch.from_numpy(wl.object0.astype(np.complex64)).cuda()).requires_grad_(True)
    Pr = torch.view_as_real(torch.from_numpy(wl.probe0.astype(np.complex64)).cuda()).requires_grad_(True)
    O, P = torch.view_as_complex(Or), torch.view_as_complex(Pr)
    opt = torch.optim.Adam([Or, Pr], lr=lr, fused=True)
    rng = np.random.default_rng([wl.seed, 9])

    def epoch():
        perm = rng.permutation(wl.count)
        for b in range(0, wl.count, minibatch):
            opt.zero_grad(set_to_none=True)
            amplitude_loss(eng, torch.view_as_complex(Or), torch.view_as_complex(Pr), perm[b:b + minibatch]).backward()
            opt.step()

    epoch()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(epochs):
        epoch()
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1])
    rate = wl.count * epochs / (ms / 1e3)
    gbs = 28 * wl.n * wl.n * rate / 1e9
    err = eng.amp_loss(O.detach(), P.detach(), np.arange(wl.count)) / float(wl.intensities.sum(dtype=np.float64))
    eng.close()
    return {"workload": "128x128 patterns, 60x60 raster (3600 positions), 1024x1024 object; fused Adam lr 1e-2, "
                        f"minibatches of {minibatch}, {epochs} timed epochs",
            "value": round(rate, 1), "unit": "position gradients/s", "ms_per_epoch": round(ms / epochs, 3),
            "path": {"achieved": round(gbs, 2), "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 5),
                     "bytes_per_position_gradient": 28 * wl.n * wl.n},
            "error_after": round(float(err), 6)}


def run_live(wl, tile=None):
    """The live schedule of the 128 px workload: reveal 200 positions in scan
    order (patterns already in device memory, as a detector stream would
    leave them), run 2 sweeps, repeat until all 3600 are loaded, then sweep
    the full set until 50 sweeps have run; timed from the first reveal to
    the last sweep, ingest and schedule growth included."""
    import torch

    import sim
    from paper_2308_10674_amd import Engine

    inten = torch.from_numpy(wl.intensities).cuda()
    pos = torch.from_numpy(wl.positions).cuda()
    plan = sim.live_plan(wl.count, 200, 2, 50)
    eng = Engine(wl.n, wl.h, wl.w, wl.probe0, wl.object0, mode="coloured", seed=wl.seed)
    if tile is not None:
        eng.tile = tile
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loaded = 0
    updates = 0
    for n_loaded, k in plan:
        if n_loaded > loaded:
            eng.add_positions(pos[loaded:n_loaded], inten[loaded:n_loaded])
            loaded = n_loaded
        eng.sweep(k)
        updates += k * loaded
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    err = eng.sweep(1, errors=True)[0]     # the state reached (not timed)
    eng.close()
    return {"workload": "128 px raster, 3600 positions revealed 200 at a time with 2 sweeps each, "
                        "then full sweeps to 50 in all",
            "updates": updates, "seconds": round(dt, 4), "value": round(updates / dt, 1),
            "unit": "position updates/s", "error_after": float(err),
            "note": "wall time including add_positions of each increment; error_after from one more sweep"}


def _kernel_roofline(name, n, ms, launches, units):
    """Algorithmic bytes per launch of one kernel over its average duration."""
    per_launch_bytes = KERNEL_BYTES[name](n) * units / launches
    avg_s = ms / 1e3 / launches
    achieved = per_launch_bytes / avg_s / 1e9
    tr = load_traffic(name, n)
    return {
        "kernel": f"{name}<{n}>", "achieved": round(achieved, 2), "frac": round(achieved / HBM_PEAK_GBS, 5),
        "traffic": None if tr is None else int(tr["bytes_per_launch"]),
        "traffic_GBps": None if tr is None else round(tr["bytes_per_launch"] / avg_s / 1e9, 2),
        "algorithmic_bytes_per_launch": round(per_launch_bytes),
        "avg_launch_us": round(avg_s * 1e6, 3), "launches": launches,
    }


def roofline_of(r):
    """Roofline entry of the dominant kernel (largest summed event time), and
    the same figures for every stage of the path ("stages"): at 128 px the
    column and inverse stages take nearly the same time, so either can be
    the dominant one in a given run."""
    n = r["wl"].n
    name, (ms, launches, units) = max(r["kernels"].items(), key=lambda kv: kv[1][0])
    out = {"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    out.update(_kernel_roofline(name, n, ms, launches, units))
    out["timing"] = ("HIP events bound to each launch of the kernel (hipExtLaunchKernel) on its stream, "
                     "summed over one run of the timed number of sweeps")
    out["kernel_times_ms"] = {k: round(v[0], 3) for k, v in r["kernels"].items()}
    out["stages"] = [_kernel_roofline(k, n, *v) for k, v in r["kernels"].items()]
    return out


def copy_bandwidth(reps=5):
    """Measured stream-copy rate of this GPU (x -> -x over 512 MiB, read plus
    written bytes over the best of `reps` event-timed launches), reported
    beside the nominal HBM peak."""
    import torch

    x = torch.ones(128 << 20, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.neg(x, out=y)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.neg(x, out=y)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    gbs = 2 * x.numel() * 4 / (best / 1e3) / 1e9
    del x, y
    return round(gbs, 1)


def run_multi(steps, warmup, n_scans=16):
    """Sixteen independent scans of uneven size (pattern sizes 64/128/256,
    500-5000 positions, raster or spiral): per-scan sweeps one after the
    other against all scans advanced together by ptyc_sweep_multi."""
    import torch

    import sim
    from paper_2308_10674_amd import Engine, sweep_multi, tune_multi

    t0 = time.time()
    scans = sim.make_multiscan(n_scans)
    gen_s = time.time() - t0
    engs = []
    for wl in scans:
        e = Engine(wl.n, wl.h, wl.w, wl.probe0, wl.object0, mode="coloured", seed=wl.seed)
        e.add_positions(torch.from_numpy(wl.positions).cuda(), torch.from_numpy(wl.intensities).cuda())
        engs.append(e)
        wl.intensities = None
    total = sum(wl.count for wl in scans)
    bytes_per_sweep = sum(20 * wl.n * wl.n * wl.count for wl in scans)
    sweep_multi(engs, warmup)
    torch.cuda.synchronize()

    def timed(fn):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        fn()
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1])
        gbs = bytes_per_sweep * steps / (ms / 1e3) / 1e9
        return {"value": round(total * steps / (ms / 1e3), 1), "ms_per_step": round(ms / steps, 3),
                "achieved": round(gbs, 2), "frac": round(gbs / HBM_PEAK_GBS, 5)}

    out = {
        "workload": f"{n_scans} independent scans, pattern sizes {sorted(set(int(wl.n) for wl in scans))}, "
                    f"{total} positions in total ({min(wl.count for wl in scans)}-{max(wl.count for wl in scans)} per scan)",
        "steps": steps, "generation_s": round(gen_s, 1), "unit": "position updates/s",
        "sequential": timed(lambda: [e.sweep(steps) for e in engs]),
    }
    names = {2: "persistent_per_scan_barriers", 4: "stepped", 6: "stepped_small_batch_tile"}
    for v, name in names.items():
        engs[0].multi_variant = v
        out[name] = timed(lambda: sweep_multi(engs, steps))
    best, ms = tune_multi(engs, 1)
    out["tuned"] = {"variant": best, "variant_names": {str(k): n for k, n in names.items()},
                    "ms_per_variant_one_sweep": [round(m, 3) for m in ms]}
    out["together"] = timed(lambda: sweep_multi(engs, steps))
    out["together"]["variant"] = best
    for e in engs:
        e.close()
    return out


def run_adam_vs_epie(epochs, minibatch, lr, max_sweeps):
    """Gradient reconstruction against ePIE on the 128 px raster workload
    (3600 positions), both from the same start (flat object, Gaussian
    probe): Adam on the amplitude loss over shuffled minibatches (the last
    partial minibatch kept), and coloured ePIE sweeps.  Both are scored by
    the same full-data Fourier error, L(O, P) / sum I, evaluated by the loss
    kernel after every epoch or sweep; reported: Adam's final error and
    time, and the sweeps and time ePIE needs to reach that error."""
    import torch

    import sim
    from paper_2308_10674_amd import Engine, amplitude_loss

    wl = sim.make_config(3)
    eng = Engine(wl.n, wl.h, wl.w, wl.probe0, wl.object0, mode="coloured", seed=wl.seed)
    eng.add_positions(torch.from_numpy(wl.positions).cuda(), torch.from_numpy(wl.intensities).cuda())
    total_i = float(wl.intensities.sum(dtype=np.float64))
    full = np.arange(wl.count)

    def ferr(o, p):
        return eng.amp_loss(o, p, full) / total_i

    # Adam on the real views of O and P (as in run_gradient)
    Or = torch.view_as_real(torch.from_numpy(wl.object0.astype(np.complex64)).cuda()).requires_grad_(True)
    Pr = torch.view_as_real(torch.from_numpy(wl.probe0.astype(np.complex64)).cuda()).requires_grad_(True)
    O, P = torch.view_as_complex(Or), torch.view_as_complex(Pr)
    opt = torch.optim.Adam([Or, Pr], lr=lr, fused=True)
    rng = np.random.default_rng([wl.seed, 9])
    adam_curve = [ferr(O.detach(), P.detach())]
    adam_s = 0.0
    for _ in range(epochs):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        perm = rng.permutation(wl.count)
        for b in range(0, wl.count, minibatch):
            opt.zero_grad(set_to_none=True)
            amplitude_loss(eng, torch.view_as_complex(Or), torch.view_as_complex(Pr), perm[b:b + minibatch]).backward()
            opt.step()
        torch.cuda.synchronize()
        adam_s += time.perf_counter() - t0
        adam_curve.append(ferr(O.detach(), P.detach()))
    target = adam_curve[-1]
    epie_curve = [ferr(eng.get_object(device=True), eng.get_probe(device=True))]
    epie_s, match, match_s = 0.0, None, None
    for k in range(1, max_sweeps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        eng.sweep(1)
        torch.cuda.synchronize()
        epie_s += time.perf_counter() - t0
        epie_curve.append(ferr(eng.get_object(device=True), eng.get_probe(device=True)))
        if match is None and epie_curve[-1] <= target:
            match, match_s = k, epie_s
    pick = lambda c, step: [round(float(v), 6) for v in c[::step]] + ([round(float(c[-1]), 6)] if (len(c) - 1) % step else [])
    return {
        "workload": "128x128 patterns, 60x60 raster (3600 positions), 1024x1024 object, start: flat object, "
                    "Gaussian probe",
        "metric": "full-data Fourier error sum_j sum_k (|F(P S_j O)| - sqrt I)^2 / sum I",
        "adam": {"epochs": epochs, "minibatch": minibatch, "lr": lr, "optimizer": "torch.optim.Adam(fused=True) on the real views of O and P", "final_error": round(float(target), 6),
                 "seconds": round(adam_s, 3), "error_every_10_epochs": pick(adam_curve, 10)},
        "epie": {"sweeps_to_reach_adam_final": match,
                 "seconds_to_reach_adam_final": None if match_s is None else round(match_s, 4),
                 "sweeps": max_sweeps, "final_error": round(float(epie_curve[-1]), 6),
                 "error_every_5_sweeps": pick(epie_curve, 5)},
    }


def _oracle_batch(oracle, O, P, wl, idx):
    """One coloured batch through the oracle, handed only that batch's
    positions and patterns (re-indexed): the oracle prepares every pattern
    it is given on each call, so passing the whole workload per batch would
    time that preparation, not the update."""
    O, P, _, _ = oracle.sweep_coloured(O, P, wl.positions[idx], wl.intensities[idx],
                                       np.arange(len(idx)), [0, len(idx)], check=False)
    return O, P


def cpu_baseline(cfg_id, budget_s, wl256=None):
    """The FP64 oracle on the host: the same workload's coloured batches in
    schedule order, sweep after sweep, until ``budget_s`` seconds of work
    are done (and briefly the other pattern sizes, see cpu_other_configs)."""
    import oracle
    import sim
    from paper_2308_10674_amd import colour

    wl = sim.make_config(cfg_id)
    col, nc = colour(wl.positions, wl.n)
    base = np.argsort(col, kind="stable")
    off = np.concatenate([[0], np.cumsum(np.bincount(col))])
    O, P = wl.object0, wl.probe0
    done = 0
    t0 = time.perf_counter()
    b = 0
    while time.perf_counter() - t0 < budget_s:
        idx = base[off[b % nc]:off[b % nc + 1]]
        O, P = _oracle_batch(oracle, O, P, wl, idx)
        done += len(idx)
        b += 1
    dt = time.perf_counter() - t0
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = None
    return dict(value=done / dt, unit="position updates/s", cores=1, kind="oracle",
                sample=f"FP64 numpy oracle, {b} coloured batches ({b / nc:.2f} sweeps of the {nc}-batch "
                       f"schedule of {wl.count} positions), {done} position updates, {dt:.1f} s, single thread",
                host_cpus={"cpu_count": os.cpu_count(), "affinity": affinity},
                other_configs=cpu_other_configs(max(1.0, budget_s / 5), wl256))


def cpu_worker(data_dir, k, n_workers, budget_s):
    """One all-cores baseline worker (a child process): the oracle on the
    coloured batches of the 128 px workload, in schedule order from its
    own starting batch, for budget_s seconds; prints its update count."""
    import oracle

    pos = np.load(os.path.join(data_dir, "positions.npy"))
    inten = np.load(os.path.join(data_dir, "intensities.npy"), mmap_mode="r")
    O = np.load(os.path.join(data_dir, "object0.npy"))
    P = np.load(os.path.join(data_dir, "probe0.npy"))
    base = np.load(os.path.join(data_dir, "order.npy"))
    off = np.load(os.path.join(data_dir, "offsets.npy"))
    nc = len(off) - 1
    done, b = 0, (k * nc) // n_workers
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        idx = base[off[b % nc]:off[b % nc + 1]]
        O, P, _, _ = oracle.sweep_coloured(O, P, pos[idx], np.asarray(inten[idx]), np.arange(len(idx)),
                                           [0, len(idx)], check=False)
        done += len(idx)
        b += 1
    print(json.dumps({"updates": done, "seconds": time.perf_counter() - t0}), flush=True)


def cpu_baseline_all_cores(budget_s):
    """The same FP64 oracle on every host core at once: one single-threaded
    oracle process per core (started as child processes), each running the
    128 px workload's coloured batches from its own starting batch and the
    same starting state; the aggregate rate is the sum of their updates over
    the longest run.  A throughput of the unmodified oracle, not one
    coherent reconstruction (a sweep's batches depend on each other)."""
    import subprocess
    import tempfile

    import sim
    from paper_2308_10674_amd import colour

    try:
        n_workers = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n_workers = os.cpu_count() or 1
    wl = sim.make_config(1)
    col, nc = colour(wl.positions, wl.n)
    with tempfile.TemporaryDirectory(dir="/tmp") as d:
        np.save(os.path.join(d, "positions.npy"), wl.positions)
        np.save(os.path.join(d, "intensities.npy"), wl.intensities)
        np.save(os.path.join(d, "object0.npy"), wl.object0)
        np.save(os.path.join(d, "probe0.npy"), wl.probe0)
        np.save(os.path.join(d, "order.npy"), np.argsort(col, kind="stable"))
        np.save(os.path.join(d, "offsets.npy"), np.concatenate([[0], np.cumsum(np.bincount(col))]))
        del wl
        env = dict(os.environ)
        for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            env[v] = "1"
        procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", d, str(k),
                                   str(n_workers), str(budget_s)], stdout=subprocess.PIPE, env=env, text=True)
                 for k in range(n_workers)]
        res = []
        for p in procs:
            out, _ = p.communicate(timeout=budget_s * 10 + 120)
            if p.returncode != 0:
                raise RuntimeError(f"CPU baseline worker failed with status {p.returncode}")
            res.append(json.loads(out.strip().splitlines()[-1]))
    upd = sum(r["updates"] for r in res)
    sec = max(r["seconds"] for r in res)
    return {"value": upd / sec, "unit": "position updates/s", "cores": n_workers, "kind": "oracle",
            "sample": f"{n_workers} single-threaded FP64 numpy oracle processes on the 128 px workload's coloured "
                      f"batches, {upd} position updates in {sec:.1f} s"}


def cpu_other_configs(budget_s, wl256=None):
    """The same oracle on the other two pattern sizes, briefly: the 32 px
    raster swept strictly (sequential ePIE, whole sweeps) and, when the
    256 px spiral workload is at hand, the first coloured batches of its
    schedule, each for about ``budget_s`` seconds."""
    import oracle
    import sim
    from paper_2308_10674_amd import colour

    out = []
    wl = sim.make_config(0)
    O, P = wl.object0, wl.probe0
    done, s = 0, 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        order = sim.sweep_order(wl.seed, s, wl.count)
        O, P, _, _ = oracle.sweep_strict(O, P, wl.positions, wl.intensities, order)
        done += len(order)
        s += 1
    dt = time.perf_counter() - t0
    out.append({"workload": "32 px patterns, 10x10 raster, strict (sequential) ePIE", "value": done / dt,
                "unit": "position updates/s", "sample": f"{s} whole sweeps, {done} updates, {dt:.1f} s"})
    if wl256 is None:
        return out
    wl = wl256
    col, nc = colour(wl.positions, wl.n)
    base = np.argsort(col, kind="stable")
    off = np.concatenate([[0], np.cumsum(np.bincount(col))])
    O, P = wl.object0, wl.probe0
    done, b = 0, 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and b < nc:
        idx = base[off[b]:off[b + 1]]
        O, P = _oracle_batch(oracle, O, P, wl, idx)
        done += len(idx)
        b += 1
    dt = time.perf_counter() - t0
    out.append({"workload": "256 px patterns, 20000-position Fermat spiral, coloured batches",
                "value": done / dt, "unit": "position updates/s",
                "sample": f"coloured batches 0..{b - 1}, {done} updates, {dt:.1f} s"})
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--form", default="batch", choices=["batch", "persistent", "graph"],
                    help="batch: three launches per batch; persistent: one cooperative kernel per sweep; "
                         "graph: one HIP graph replay per sweep")
    ap.add_argument("--no-forms", action="store_true", help="skip timing the other launch forms")
    ap.add_argument("--tile", default=None,
                    help="tile variants of the per-batch kernels, 'A' or 'A,B' for the 128 px and the 256 px "
                         "workload (default: let ptyc_tune choose)")
    ap.add_argument("--no-256", action="store_true", help="skip the 256 px workload")
    ap.add_argument("--steps-256", type=int, default=3)
    ap.add_argument("--no-multi", action="store_true", help="skip the 16 independent scans advanced together")
    ap.add_argument("--steps-multi", type=int, default=3)
    ap.add_argument("--adam-vs-epie", action="store_true",
                    help="only compare gradient reconstruction (Adam) with ePIE at equal Fourier error")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-all-seconds", type=float, default=10.0,
                    help="budget of the all-cores oracle baseline (0 skips it)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 32 px sequential and the gradient workloads")
    ap.add_argument("--cpu-worker", nargs=4, metavar=("DIR", "K", "WORKERS", "SECONDS"), help=argparse.SUPPRESS)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 512 MiB device copy kernel (x -> -x), three times, to scale "
                         "the rocprofv3 FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.cpu_worker:
        cpu_worker(args.cpu_worker[0], int(args.cpu_worker[1]), int(args.cpu_worker[2]), float(args.cpu_worker[3]))
        return
    if args.calibrate_copy:
        import torch
        x = torch.ones(128 << 20, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.neg(x, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "neg copy", "bytes_read": x.numel() * 4, "bytes_written": y.numel() * 4}))
        return
    if args.adam_vs_epie:
        print(json.dumps({"adam_vs_epie": run_adam_vs_epie(100, 512, 1e-2, 100)}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library does not split the reconstruction of one scan "
              "across GPUs, so --gpus must be 1.", file=sys.stderr)
        sys.exit(2)

    tiles = [None, None]
    if args.tile is not None:
        parts = [int(x) for x in str(args.tile).split(",")]
        tiles = [parts[0], parts[-1]]
    r = run_gpu(1, args.steps, args.warmup, args.form, tile=tiles[0])
    wl = r["wl"]
    out = {
        "metric": "ePIE position updates/sec at 128^2 and 256^2 patterns; % HBM roofline",
        "value": round(r["rate"], 1),
        "unit": "position updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms"] / args.steps, 4),
        "median_ms_per_step": round(float(np.median(r["seg_ms"])), 4),
        "segment_ms_per_step": [round(x, 4) for x in r["seg_ms"]],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {
            "workload": "ePIE 128x128 patterns, 60x60 raster step 12 px (3600 positions), 1024x1024 object, "
                        "coloured batches of disjoint windows, one sweep per step",
            "n": wl.n, "object": [wl.h, wl.w], "positions": wl.count, "form": args.form,
            "batches_per_sweep": r["batches"], "mean_batch": round(r["mean_batch"], 2),
            "max_batch": r["max_batch"], "tile": r["tile"], "tile_ms_per_sweep": r["tile_ms"],
        },
        "roofline": dict(roofline_of(r), copy_GBps=copy_bandwidth()),
        "path": {
            "achieved": round(r["achieved_gbs"], 2), "unit": "GB/s", "frac": round(r["achieved_gbs"] / HBM_PEAK_GBS, 5),
            "bytes_per_update": algorithmic_bytes(wl.n),
            "note": "whole sweep: 20 N^2 algorithmic bytes per position update over the timed wall time",
        },
        "error_after": r["err"],
        "ingest": {
            "GB_per_s": round(wl.count * wl.n * wl.n * 4 / r["ingest_s"] / 1e9, 2),
            "note": "add_positions of device-resident float32 patterns (sqrt, schedule extension, "
                    "first-time buffer allocation included)",
        },
    }
    if not args.no_forms:
        out["forms"] = run_forms(wl, args.steps)
        out["live"] = run_live(wl, tiles[0])
    wl256 = None
    if not args.no_256:
        r2 = run_gpu(2, args.steps_256, 1, args.form, tile=tiles[1])
        wl256 = r2["wl"]
        out["n256"] = {
            "value": round(r2["rate"], 1), "unit": "position updates/s",
            "ms_per_step": round(r2["ms"] / args.steps_256, 3), "steps": args.steps_256,
            "workload": "ePIE 256x256 patterns, 20000-position Fermat spiral, 2048x2048 object",
            "achieved": round(r2["achieved_gbs"], 2), "frac": round(r2["achieved_gbs"] / HBM_PEAK_GBS, 5),
            "batches_per_sweep": r2["batches"], "mean_batch": round(r2["mean_batch"], 2),
            "tile": r2["tile"], "tile_ms_per_sweep": r2["tile_ms"],
            "roofline": roofline_of(r2),
        }
    if not args.no_multi:
        out["multi16"] = run_multi(args.steps_multi, 1)
    if not args.no_extra:
        out["config0"] = run_config0()
        out["gradient"] = run_gradient()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(1, args.cpu_seconds, wl256)
        if args.cpu_all_seconds > 0:
            out["cpu_baseline"]["all_cores"] = cpu_baseline_all_cores(args.cpu_all_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
