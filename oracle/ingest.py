"""Detector-frame preprocessing, written from its definition.  Test
infrastructure only.

The paper crops patterns to 2^n and rotates or flips them so that their
coordinate system and handedness match the position encoders ("ePIE
Implementation", "Preprocessing"); its Discussion lists masking invalid
pixels.  Here: keep the n x n crop at (crop_y, crop_x) of each raw frame;
apply the orientation (bit 0: transpose, then bit 1: flip rows, then bit 2:
flip columns); if the crop is DC-centred, move DC from (n/2, n/2) to (0, 0);
multiply counts by the gain scale.  Masked pixels (no measurement) are
stored as 0.
"""
from __future__ import annotations

import numpy as np


def orient_crop(crop, orient, centred):
    """The n x n crop (or a stack of them) in the stored layout."""
    x = np.asarray(crop)
    if orient & 1:
        x = np.swapaxes(x, -1, -2)
    if orient & 2:
        x = np.flip(x, axis=-2)
    if orient & 4:
        x = np.flip(x, axis=-1)
    if centred:
        x = np.fft.ifftshift(x, axes=(-2, -1))
    return np.ascontiguousarray(x)


def preprocess(frames, n, crop=(0, 0), orient=0, centred=False, scale=1.0, mask=None, dtype=np.float64):
    """Raw frames [count, fh, fw] -> (intensities [count, n, n] in dtype,
    stored mask [n, n] bool or None).  Masked pixels become 0."""
    y, x = crop
    c = np.asarray(frames)[..., y:y + n, x:x + n].astype(dtype)
    out = orient_crop(c, orient, centred) * dtype(scale)
    m = None
    if mask is not None:
        m = orient_crop(np.asarray(mask)[y:y + n, x:x + n] != 0, orient, centred)
        out = np.where(m, out, dtype(0))
    return out, m
