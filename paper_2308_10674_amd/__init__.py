"""Live ePIE ptychography on AMD Instinct MI355X (gfx950).

The reconstruction runs in libptyc.so (hand-written HIP kernels behind a
C ABI, include/ptyc.h); this package is its thin Python binding.
"""
from ._lib import PtycError, lib  # noqa: F401
from .engine import Engine, average, check_batches, colour, current_stream_handle, sweep_multi, tune_multi  # noqa: F401

try:  # the autograd wrapper needs torch
    from .autograd import AmplitudeLoss, amplitude_loss  # noqa: F401
except ImportError:  # pragma: no cover
    pass

__all__ = ["Engine", "PtycError", "colour", "check_batches", "lib", "current_stream_handle", "sweep_multi", "average",
           "tune_multi"]
