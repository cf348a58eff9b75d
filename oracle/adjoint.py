"""Amplitude loss and its gradient, FP64.  Test infrastructure only.

Gradient-based reconstruction (beside ePIE) minimises the amplitude loss over
a set of positions J:

  L(O, P) = sum_{j in J} sum_k (|F(P * S_j O)|_k - sqrt I_j,k)^2

Gradients follow PyTorch's convention for a real function of complex
variables, grad = dL/dRe + i dL/dIm:

  g_Psi = 2 (|Psi| - sqrt I) sgn(Psi)
  g_psi = F^H g_Psi = N^2 F^-1 g_Psi
  grad_O[window j] += conj(P) g_psi          (windows may overlap: summed)
  grad_P           += conj(S_j O) g_psi

The ePIE object step of one position equals -alpha / (2 N^2 max|P|^2) times
that position's grad_O (Psi = |Psi| sgn Psi, so F^-1 of |Psi| sgn Psi is psi).
"""
from __future__ import annotations

import numpy as np

from .epie import fft2, ifft2, sgn


def amplitude_loss(obj, probe, positions, intensities, idx=None, mask=None):
    n = probe.shape[0]
    idx = range(len(positions)) if idx is None else idx
    total = 0.0
    for j in idx:
        y, x = int(positions[j][0]), int(positions[j][1])
        Psi = fft2(probe * obj[y:y + n, x:x + n])
        a = np.sqrt(np.asarray(intensities[j], dtype=np.float64))
        r = (np.abs(Psi) - a) ** 2
        total += float(np.sum(r if mask is None else np.where(mask, r, 0.0)))
    return total


def amplitude_loss_grad(obj, probe, positions, intensities, idx=None, mask=None):
    """Returns (loss, grad_O, grad_P) in complex128."""
    obj = np.asarray(obj, dtype=np.complex128)
    probe = np.asarray(probe, dtype=np.complex128)
    n = probe.shape[0]
    idx = range(len(positions)) if idx is None else idx
    g_o = np.zeros_like(obj)
    g_p = np.zeros_like(probe)
    total = 0.0
    for j in idx:
        y, x = int(positions[j][0]), int(positions[j][1])
        win = obj[y:y + n, x:x + n]
        Psi = fft2(probe * win)
        a = np.sqrt(np.asarray(intensities[j], dtype=np.float64))
        r = np.abs(Psi) - a
        if mask is not None:
            r = np.where(mask, r, 0.0)   # no measurement: no loss, no gradient
        total += float(np.sum(r ** 2))
        g_psi = (n * n) * ifft2(2.0 * r * sgn(Psi))
        g_o[y:y + n, x:x + n] += np.conj(probe) * g_psi
        g_p += np.conj(win) * g_psi
    return total, g_o, g_p
