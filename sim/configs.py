"""Workload recipes (probe, object, scan, data) for the five benchmark shapes.

Every random quantity comes from numpy's PCG64 with its own stream
``default_rng([seed, id, ...])`` so that any one of them can be regenerated
alone.  Stream ids: 1 object amplitude, 2 object phase, 3 scan jitter,
4 Poisson noise (one sub-stream per position), 5 multi-scan parameters,
7 per-sweep position order.

The recipe follows the workloads of the paper's experiments (Materials and
Methods: 2^n-cropped far-field patterns, raster and spiral scans, object
sized from the scan bounding box padded by half the illumination) at the
sizes of the five benchmark configurations; the readings taken where the
configuration text is loose are listed in the design notes (probe defocus
for the larger apertures, object smoothing, photon scaling, jitter, scan
offsets, initial guesses).
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np
import scipy.fft
import scipy.ndimage


# --------------------------------------------------------------------------
# building blocks
# --------------------------------------------------------------------------

def make_probe(n: int, radius: float, kappa: float) -> np.ndarray:
    """Circular aperture with quadratic (defocus) phase, complex128 [n, n].

    P(r) = 1[|r - c| <= radius] * exp(i * kappa * |r - c|^2), c = (n/2, n/2),
    r the integer (row, col) pixel coordinate; the edge is inclusive.
    """
    rr, cc = np.mgrid[0:n, 0:n].astype(np.float64)
    d2 = (rr - n / 2) ** 2 + (cc - n / 2) ** 2
    amp = (d2 <= radius * radius).astype(np.float64)
    return amp * np.exp(1j * kappa * d2)


def make_object(h: int, w: int, seed: int, sigma: float = 2.0,
                amp_range=(0.8, 1.0), phase_range=(-math.pi / 4, math.pi / 4)
                ) -> np.ndarray:
    """Smoothed random complex transmission function, complex128 [h, w].

    Amplitude and phase are drawn i.i.d. uniform, each Gaussian-filtered
    (sigma px, periodic boundary, truncated at 4 sigma) and then min-max
    rescaled back onto the stated range (without the rescale the filter
    shrinks the amplitude spread to a few thousandths).
    """
    a = np.random.default_rng([seed, 1]).uniform(amp_range[0], amp_range[1], (h, w))
    p = np.random.default_rng([seed, 2]).uniform(phase_range[0], phase_range[1], (h, w))

    def smooth_rescale(x, lo, hi):
        y = scipy.ndimage.gaussian_filter(x, sigma, mode="wrap", truncate=4.0)
        y = (y - y.min()) / (y.max() - y.min())
        return lo + (hi - lo) * y

    a = smooth_rescale(a, *amp_range)
    p = smooth_rescale(p, *phase_range)
    return a * np.exp(1j * p)


def raster_positions(n_side: int, step: int, n: int, m: int, jitter: int,
                     seed: int) -> np.ndarray:
    """Raster scan, row-major scan order, int32 [n_side**2, 2] window corners.

    top-left = off + step * (i, k) + jitter with off = floor((m - (n_side-1)
    step - n) / 2) and an independent integer jitter, uniform on
    [-jitter, jitter] inclusive, per axis and position.
    """
    off = (m - (n_side - 1) * step - n) // 2
    i, k = np.meshgrid(np.arange(n_side), np.arange(n_side), indexing="ij")
    yx = np.stack([i.ravel(), k.ravel()], axis=1) * step + off
    if jitter:
        yx = yx + np.random.default_rng([seed, 3]).integers(
            -jitter, jitter, size=yx.shape, endpoint=True)
    return yx.astype(np.int32)


def fermat_positions(count: int, rho_step: float, n: int, m: int) -> np.ndarray:
    """Fermat spiral with golden-angle increment, int32 [count, 2] corners.

    rho = rho_step * sqrt(t), theta = t * pi * (3 - sqrt 5), t = 0..count-1,
    top-left = rint(m/2 + rho * (sin theta, cos theta) - n/2).
    """
    t = np.arange(count, dtype=np.float64)
    rho = rho_step * np.sqrt(t)
    th = t * math.pi * (3.0 - math.sqrt(5.0))
    y = np.rint(m / 2 + rho * np.sin(th) - n / 2)
    x = np.rint(m / 2 + rho * np.cos(th) - n / 2)
    return np.stack([y, x], axis=1).astype(np.int32)


def object_extent(pos_centre: np.ndarray, n: int, margin: int):
    """Object size covering every n x n illumination around the nominal
    scan, plus a margin, and the shift that turns centres into window corners.

    The object spans the bounding box of the scan centres padded by half the
    illumination on each side (Materials and Methods, "Determine
    parameters") plus ``margin`` pixels.  Returns (h, w, corners) where
    corners = centre - n//2 + (margin - min centre + n//2).
    """
    c = np.asarray(pos_centre, dtype=np.int64)
    lo = c.min(axis=0)
    hi = c.max(axis=0)
    h = int(hi[0] - lo[0]) + n + 2 * margin
    w = int(hi[1] - lo[1]) + n + 2 * margin
    corners = (c - lo + margin).astype(np.int32)
    return h, w, corners


def _windows(obj: np.ndarray, pos: np.ndarray, n: int) -> np.ndarray:
    r = np.arange(n)
    return obj[pos[:, 0, None, None] + r[None, :, None],
               pos[:, 1, None, None] + r[None, None, :]]


def simulate_intensities(probe: np.ndarray, obj: np.ndarray, pos: np.ndarray,
                         photons: float, noise: bool, seed: int,
                         dtype=np.float32, workers: int | None = None,
                         chunk: int = 16):
    """Far-field diffraction intensities for every scan position.

    I_j = Poisson(s * |FFT2(probe * O[window_j])|^2) with one global scale s
    chosen so that the mean total count per pattern equals ``photons``
    (by Parseval, sum_k |FFT2 psi|^2 = n^2 sum_r |psi|^2).  Without noise the
    exact expectation is returned.  Noise for position j comes from
    default_rng([seed, 4, j]).  Returns (I [count, n, n] dtype, s).
    """
    n = probe.shape[0]
    count = pos.shape[0]
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    starts = list(range(0, count, chunk))

    def run(fn):
        if workers > 1 and len(starts) > 1:
            with ThreadPoolExecutor(workers) as ex:
                return list(ex.map(fn, starts))
        return [fn(a) for a in starts]

    # pass 1: global photon scale from real-space energies (summed in a
    # fixed order, so the result does not depend on the thread count)
    p2 = np.abs(probe) ** 2

    def energy(a):
        w = _windows(obj, pos[a:a + chunk], n)
        return float(np.sum(p2[None] * (w.real ** 2 + w.imag ** 2)))

    e = math.fsum(run(energy))
    mean_energy = n * n * e / max(count, 1)
    s = photons / mean_energy if mean_energy > 0 else 1.0
    out = np.empty((count, n, n), dtype=dtype)

    def work(a):
        b = min(a + chunk, count)
        w = _windows(obj, pos[a:b], n)
        psi = probe[None] * w
        lam = s * np.abs(scipy.fft.fft2(psi, axes=(-2, -1), workers=1)) ** 2
        if noise:
            for j in range(a, b):
                out[j] = np.random.default_rng([seed, 4, j]).poisson(lam[j - a])
        else:
            out[a:b] = lam
        return b

    run(work)
    return out, s


def initial_probe(n: int, radius: float, mean_counts: float) -> np.ndarray:
    """Initial illumination guess: Gaussian amplitude (sigma = radius/2 px)
    centred at (n/2, n/2) with flat phase, scaled so that n^2 sum |P0|^2
    equals the mean total count per pattern (the paper starts every
    simulated reconstruction from a small Gaussian peak with zero phase)."""
    rr, cc = np.mgrid[0:n, 0:n].astype(np.float64)
    d2 = (rr - n / 2) ** 2 + (cc - n / 2) ** 2
    sig = radius / 2.0
    g = np.exp(-d2 / (2 * sig * sig))
    g *= math.sqrt(mean_counts / (n * n * np.sum(g * g)))
    return g.astype(np.complex128)


def sweep_order(seed: int, sweep: int, n_loaded: int) -> np.ndarray:
    """Random position order of one sweep: a permutation of the loaded
    indices drawn from default_rng([seed, 7, sweep])."""
    return np.random.default_rng([seed, 7, sweep]).permutation(n_loaded).astype(np.int64)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

CONFIGS = {
    0: dict(n=32, radius=10.0, kappa=0.05, m=128, scan=("raster", 10, 6, 1),
            photons=1e6, mode="strict", sweeps=10),
    1: dict(n=128, radius=40.0, kappa=0.5 / 40.0, m=1024, scan=("raster", 60, 12, 2),
            photons=1e7, mode="coloured", sweeps=50, live=(200, 2)),
    2: dict(n=256, radius=70.0, kappa=0.5 / 70.0, m=2048, scan=("fermat", 20000, 6.0),
            photons=1e8, mode="coloured", sweeps=20),
    3: dict(n=128, radius=40.0, kappa=0.5 / 40.0, m=1024, scan=("raster", 60, 12, 2),
            photons=1e7, mode="gradient", epochs=100, minibatch=512),
}


@dataclass
class Workload:
    """One reconstruction problem: truth, data and starting guesses."""
    config: int
    n: int
    h: int
    w: int
    radius: float
    kappa: float
    positions: np.ndarray          # int32 [count, 2] window corners (row, col)
    intensities: np.ndarray        # [count, n, n] (float32 unless asked)
    probe_true: np.ndarray         # complex128 [n, n], already scaled by sqrt(s)
    object_true: np.ndarray        # complex128 [h, w]
    probe0: np.ndarray             # complex128 [n, n]
    object0: np.ndarray            # complex128 [h, w]
    scale: float
    seed: int
    mode: str
    sweeps: int
    alpha: float = 1.0
    beta: float = 1.0
    extra: dict = field(default_factory=dict)

    @property
    def count(self) -> int:
        return int(self.positions.shape[0])


def make_workload(n, m, radius, kappa, positions, photons, seed, noise=True,
                  dtype=np.float32, h=None, w=None, config=-1, mode="coloured",
                  sweeps=1, workers=None) -> Workload:
    h = m if h is None else h
    w = m if w is None else w
    probe = make_probe(n, radius, kappa)
    obj = make_object(h, w, seed)
    inten, s = simulate_intensities(probe, obj, positions, photons, noise, seed,
                                    dtype=dtype, workers=workers)
    p0 = initial_probe(n, radius, photons)
    o0 = np.ones((h, w), dtype=np.complex128)
    return Workload(config=config, n=n, h=h, w=w, radius=radius, kappa=kappa,
                    positions=positions, intensities=inten,
                    probe_true=probe * math.sqrt(s), object_true=obj,
                    probe0=p0, object0=o0, scale=s, seed=seed, mode=mode,
                    sweeps=sweeps)


def make_config(k: int, noise: bool = True, dtype=np.float32,
                n_positions: int | None = None, seed: int | None = None,
                workers: int | None = None) -> Workload:
    """Build benchmark configuration k (0..3).  ``n_positions`` truncates
    the scan to its first positions in scan order (for quick tests)."""
    c = CONFIGS[k]
    seed = 1000 + k if seed is None else seed
    n, m = c["n"], c["m"]
    kind = c["scan"][0]
    if kind == "raster":
        _, side, step, jit = c["scan"]
        pos = raster_positions(side, step, n, m, jit, seed)
    else:
        _, cnt, rho = c["scan"]
        pos = fermat_positions(cnt if n_positions is None else n_positions, rho, n, m)
    if n_positions is not None:
        pos = pos[:n_positions]
    wl = make_workload(n, m, c["radius"], c["kappa"], pos, c["photons"], seed,
                       noise=noise, dtype=dtype, config=k, mode=c["mode"],
                       sweeps=c.get("sweeps", 1), workers=workers)
    wl.extra = {kk: vv for kk, vv in c.items() if kk in ("live", "epochs", "minibatch")}
    return wl


def live_plan(total: int, increment: int, sweeps_per_increment: int,
              total_sweeps: int):
    """Live acquisition schedule: reveal ``increment`` positions in scan order,
    run ``sweeps_per_increment`` sweeps, repeat until everything is loaded,
    then sweep the full set until ``total_sweeps`` sweeps have run.
    Returns a list of (n_loaded, sweeps) steps."""
    plan = []
    done = 0
    loaded = 0
    while loaded < total:
        loaded = min(total, loaded + increment)
        k = min(sweeps_per_increment, total_sweeps - done)
        plan.append((loaded, k))
        done += k
    if done < total_sweeps:
        plan.append((total, total_sweeps - done))
    return plan


def make_multiscan(n_scans: int = 16, seed: int = 1004, photons: float = 1e7,
                   margin: int = 32, sizes=(64, 128, 256),
                   count_range=(500, 5000), noise: bool = True,
                   max_count: int | None = None, workers=None):
    """Several independent scans of uneven size (pattern size, count, scan
    kind drawn per scan from default_rng([seed, 5])).  Raster scans use
    step 0.094 n; spiral scans rho = (6/256) n sqrt(t).  Each object covers
    its scan's windows plus ``margin`` px."""
    rng = np.random.default_rng([seed, 5])
    radius_of = {64: 20.0, 128: 40.0, 256: 70.0}
    out = []
    for i in range(n_scans):
        n = int(rng.choice(sizes))
        cnt = int(rng.integers(count_range[0], count_range[1], endpoint=True))
        if max_count is not None:
            cnt = min(cnt, max_count)
        kind = "raster" if rng.random() < 0.5 else "fermat"
        if kind == "raster":
            side = int(math.ceil(math.sqrt(cnt)))
            step = max(1, int(round(0.094 * n)))
            cen = np.stack(np.meshgrid(np.arange(side), np.arange(side),
                                       indexing="ij"), -1).reshape(-1, 2)[:cnt] * step
        else:
            t = np.arange(cnt, dtype=np.float64)
            rho = (6.0 / 256.0) * n * np.sqrt(t)
            th = t * math.pi * (3.0 - math.sqrt(5.0))
            cen = np.stack([np.rint(rho * np.sin(th)), np.rint(rho * np.cos(th))], 1)
        h, w, corners = object_extent(cen, n, margin)
        r = radius_of[n]
        wl = make_workload(n, None, r, 0.5 / r, corners, photons, seed * 100 + i,
                           noise=noise, h=h, w=w, config=4, mode="coloured",
                           workers=workers)
        wl.extra = {"scan": kind}
        out.append(wl)
    return out
