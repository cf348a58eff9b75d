"""FP64 ePIE, written from the method's definition.  Test infrastructure only.

Notation (the paper's ePIE, after Maiden & Rodenburg 2009, cited in the
paper's Introduction and "ePIE Implementation"):

  N         pattern / probe side; the object O is H x W
  r_j       integer (row, col) top-left corner of scan position j's window
  S_j O     the N x N window O[y_j:y_j+N, x_j:x_j+N]
  F         unnormalised 2D DFT, exp(-2 pi i k.r / N), DC at [0, 0]
  F^-1      its inverse including 1/N^2
  sgn z     z/|z| for z != 0 and 0 for z == 0

One position update, with pre-update P and S_j O on both right-hand sides
(simultaneous object and probe updates):

  psi    = P * S_j O                              exit wave
  Psi    = F psi
  Psi'   = sqrt(I_j) * sgn(Psi)                   modulus replacement
  psi'   = F^-1 Psi'
  Delta  = psi' - psi
  S_j O <- S_j O + alpha conj(P) Delta / max|P|^2
  P     <- P + beta conj(S_j O) Delta / max|S_j O|^2

The max in the object step runs over the whole probe array; the max in the
probe step runs over the position's own (pre-update) window.  alpha = beta = 1
in all of the paper's reconstructions.  A sweep visits every loaded position
once in a randomly shuffled order; the order is an explicit input here.

Coloured batches: a batch is a set of positions whose windows are pairwise
disjoint.  Every position of batch b is updated from the same probe P_b (its
object steps then touch disjoint pixels and commute); the probe increments
d_j = conj(S_j O) Delta_j / max|S_j O|^2 are averaged:
P_{b+1} = P_b + (beta / |B_b|) sum_j d_j.  A batch of one position is exactly
the sequential update above.

Running Fourier error of a sweep:
  E = sum_j sum_k (|Psi_j| - sqrt I_j)^2 / sum_j sum_k I_j
with Psi_j the transform computed while updating position j.
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------- transforms

def fft2(x):
    """Unnormalised forward 2D DFT over the last two axes (numpy pocketfft)."""
    return np.fft.fft2(x, axes=(-2, -1))


def ifft2(x):
    """Inverse 2D DFT over the last two axes, including the 1/N^2 factor."""
    return np.fft.ifft2(x, axes=(-2, -1))


def dft2_bruteforce(x):
    """The DFT written out: X[k, l] = sum_{r,c} x[r, c] exp(-2 pi i (k r / n0
    + l c / n1)).  O(n^4); only for pinning the transform convention."""
    x = np.asarray(x, dtype=np.complex128)
    n0, n1 = x.shape
    out = np.zeros((n0, n1), dtype=np.complex128)
    for k in range(n0):
        for l in range(n1):
            acc = 0j
            for r in range(n0):
                for c in range(n1):
                    acc += x[r, c] * np.exp(-2j * np.pi * (k * r / n0 + l * c / n1))
            out[k, l] = acc
    return out


# ---------------------------------------------------------------- one update

def sgn(z):
    """z/|z| where z != 0, else 0."""
    a = np.abs(z)
    out = np.zeros_like(z)
    nz = a > 0
    out[nz] = z[nz] / a[nz]
    return out


def modulus_replace(Psi, sqrt_i, mask=None):
    """Psi' = sqrt(I) * sgn(Psi): keep the phase, impose the measured modulus.
    Where ``mask`` is False there is no measurement and Psi' = Psi."""
    out = sqrt_i * sgn(Psi)
    if mask is not None:
        out = np.where(mask, out, Psi)
    return out


def _err(Psi, sqrt_i, mask):
    r = (np.abs(Psi) - sqrt_i) ** 2
    if mask is not None:
        r = np.where(mask, r, 0.0)
    return r


def position_update(probe, win, sqrt_i, alpha, mask=None):
    """One ePIE position update from pre-update values.

    Returns (new window, probe increment d, error term) where the caller
    applies P <- P + beta * d (sequential) or averages d over a batch.
    ``mask`` (bool, N x N) marks measured detector pixels.
    """
    psi = probe * win
    Psi = fft2(psi)
    err = float(np.sum(_err(Psi, sqrt_i, mask)))
    psi_new = ifft2(modulus_replace(Psi, sqrt_i, mask))
    delta = psi_new - psi
    pmax = np.max(np.abs(probe) ** 2)
    omax = np.max(np.abs(win) ** 2)
    new_win = win + alpha * np.conj(probe) * delta / pmax
    d = np.conj(win) * delta / omax
    return new_win, d, err


# ---------------------------------------------------------------- sweeps

def _prep(obj, probe, intensities, dtype):
    cdt = np.dtype(dtype)
    rdt = np.float64 if cdt == np.complex128 else np.float32
    sq = np.sqrt(np.asarray(intensities, dtype=np.float64)).astype(rdt)
    return np.array(obj, dtype=cdt), np.array(probe, dtype=cdt), sq


def sweep_strict(obj, probe, positions, intensities, order, alpha=1.0,
                 beta=1.0, dtype=np.complex128, mask=None):
    """One sequential ePIE sweep over ``order``.

    Returns (object, probe, error numerator, error denominator)."""
    O, P, sq = _prep(obj, probe, intensities, dtype)
    n = P.shape[0]
    num = 0.0
    den = 0.0
    for j in order:
        y, x = int(positions[j][0]), int(positions[j][1])
        win = O[y:y + n, x:x + n].copy()
        new_win, d, e = position_update(P, win, sq[j], alpha, mask)
        O[y:y + n, x:x + n] = new_win
        P = P + beta * d
        num += e
        den += float(np.sum(np.asarray(intensities[j], dtype=np.float64)))
    return O, P, num, den


def sweep_coloured(obj, probe, positions, intensities, order, batch_offsets,
                   alpha=1.0, beta=1.0, dtype=np.complex128, check=True, mask=None):
    """One coloured-batch sweep: batches order[off[b]:off[b+1]] in turn.

    Within a batch every position uses the batch's probe P_b; the windows
    are disjoint (checked), so the object steps commute; the probe moves by
    beta times the mean of the batch's increments.  The positions of a batch
    are processed together as one stack (the FFT applied to each member of
    the stack), which is the same computation as visiting them one by one.
    Returns (object, probe, error numerator, error denominator)."""
    O, P, sq = _prep(obj, probe, intensities, dtype)
    n = P.shape[0]
    order = np.asarray(order, dtype=np.int64)
    off = np.asarray(batch_offsets, dtype=np.int64)
    if check:
        check_schedule(positions, n, order, off)
    r = np.arange(n)
    num = 0.0
    den = 0.0
    pmax_dtype = np.float64 if O.dtype == np.complex128 else np.float32
    for b in range(len(off) - 1):
        idx = order[off[b]:off[b + 1]]
        if len(idx) == 0:
            continue
        pos = np.asarray(positions, dtype=np.int64)[idx]
        rows = pos[:, 0, None, None] + r[None, :, None]
        cols = pos[:, 1, None, None] + r[None, None, :]
        win = O[rows, cols]                              # [B, n, n]
        psi = P[None] * win
        Psi = fft2(psi)
        a = sq[idx]
        num += float(np.sum(_err(np.abs(Psi).astype(np.float64), a, mask)))
        den += float(np.sum(np.asarray(intensities[idx], dtype=np.float64)))
        delta = ifft2(modulus_replace(Psi, a, mask)) - psi
        pmax = np.max(np.abs(P) ** 2).astype(pmax_dtype)
        omax = np.max(np.abs(win) ** 2, axis=(1, 2)).astype(pmax_dtype)
        O[rows, cols] = win + alpha * np.conj(P)[None] * delta / pmax
        d = np.conj(win) * delta / omax[:, None, None]
        acc = np.zeros_like(P)
        for s in range(len(idx)):          # slot order, as listed
            acc = acc + d[s]
        P = P + (beta / len(idx)) * acc
    return O, P, num, den


# ---------------------------------------------------------------- schedules

def windows_overlap(a, b, n):
    """Two n x n windows with corners a, b share a pixel."""
    return abs(int(a[0]) - int(b[0])) < n and abs(int(a[1]) - int(b[1])) < n


def check_schedule(positions, n, order, batch_offsets, n_loaded=None,
                   require_partition=False):
    """Brute-force validation of a batch schedule: offsets are monotone and
    span ``order``; every index is loaded; no two windows in a batch share a
    pixel.  Raises ValueError on the first violation."""
    order = np.asarray(order, dtype=np.int64)
    off = np.asarray(batch_offsets, dtype=np.int64)
    n_loaded = len(positions) if n_loaded is None else n_loaded
    if len(off) < 1 or off[0] != 0 or off[-1] != len(order) or np.any(np.diff(off) < 0):
        raise ValueError("batch offsets do not span the order")
    if len(order) and (order.min() < 0 or order.max() >= n_loaded):
        raise ValueError("order index out of range")
    if require_partition and not np.array_equal(np.sort(order), np.arange(n_loaded)):
        raise ValueError("order is not a permutation of the loaded positions")
    for b in range(len(off) - 1):
        idx = order[off[b]:off[b + 1]]
        for u in range(len(idx)):
            for v in range(u + 1, len(idx)):
                if windows_overlap(positions[idx[u]], positions[idx[v]], n):
                    raise ValueError(f"batch {b}: windows {idx[u]} and {idx[v]} overlap")
    return True


def greedy_colouring(positions, n, max_batch=1024):
    """First-fit colouring in index order: position j joins the lowest
    colour that has room and holds no window overlapping j's.  Brute force,
    O(count^2); returns an int array of colours."""
    colours = np.full(len(positions), -1, dtype=np.int64)
    members: list[list[int]] = []
    for j in range(len(positions)):
        for c, mem in enumerate(members):
            if len(mem) < max_batch and not any(
                    windows_overlap(positions[j], positions[i], n) for i in mem):
                mem.append(j)
                colours[j] = c
                break
        else:
            members.append([j])
            colours[j] = len(members) - 1
    return colours


# ---------------------------------------------------------------- metrics

def union_mask(positions, n, h, w):
    """Pixels covered by at least one window."""
    m = np.zeros((h, w), dtype=bool)
    for y, x in np.asarray(positions):
        m[y:y + n, x:x + n] = True
    return m


def rel_l2(x, ref, mask=None):
    """||x - ref||_2 / ||ref||_2, optionally over a boolean mask."""
    x = np.asarray(x)
    ref = np.asarray(ref)
    if mask is not None:
        x = x[mask]
        ref = ref[mask]
    den = np.linalg.norm(ref.astype(np.complex128))
    return float(np.linalg.norm(x.astype(np.complex128) - ref.astype(np.complex128)) / den)


def reconstruct(obj, probe, positions, intensities, schedules, alpha=1.0,
                beta=1.0, dtype=np.complex128, mask=None):
    """Run a list of sweeps.  Each schedule entry is (order, batch_offsets)
    for a coloured sweep or (order, None) for a sequential one.
    Returns (object, probe, [E per sweep])."""
    O, P = obj, probe
    errs = []
    for order, off in schedules:
        if off is None:
            O, P, num, den = sweep_strict(O, P, positions, intensities, order,
                                          alpha, beta, dtype, mask=mask)
        else:
            O, P, num, den = sweep_coloured(O, P, positions, intensities, order,
                                            off, alpha, beta, dtype, mask=mask)
        errs.append(num / den if den > 0 else 0.0)
    return O, P, errs
