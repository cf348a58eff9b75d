"""Reference implementation used ONLY as test infrastructure.

A plain, slow, obviously correct FP64 CPU version of what the GPU path
computes: the ePIE per-position update (Maiden & Rodenburg 2009, the method
the paper uses in "Materials and Methods / ePIE Implementation"), the
sweep in a given (randomly shuffled) order, the coloured-batch variant,
the Fourier error, and the amplitude-loss gradient.  It uses numpy's
pocketfft for the Fourier transforms and shares no code with the HIP
library.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package; the library never calls it.
"""
from .epie import (  # noqa: F401
    dft2_bruteforce, fft2, ifft2, sgn, modulus_replace,
    position_update, sweep_strict, sweep_coloured,
    check_schedule, greedy_colouring, windows_overlap, rel_l2, union_mask,
    reconstruct,
)
from .adjoint import amplitude_loss, amplitude_loss_grad  # noqa: F401
from .parallel import round_robin, subset_round  # noqa: F401
from .ingest import orient_crop, preprocess  # noqa: F401
