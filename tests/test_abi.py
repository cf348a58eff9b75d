"""C-ABI contract checks that need no GPU: the library loads, exports every
declared entry point, rejects bad arguments before touching the device, and
its host-side schedule helpers agree with the oracle's brute force."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import sim
from paper_2308_10674_amd import _lib as L
from paper_2308_10674_amd import check_batches, colour

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ptyc.h")


def _lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libptyc.so not built")
    return L.lib()


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ptyc_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for must in ("ptyc_init", "ptyc_add_positions", "ptyc_sweep", "ptyc_get_object", "ptyc_get_probe"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = _lib()
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert set(declared_symbols()) == set(L.SIGNATURES)
    assert lib.ptyc_version() >= 100


def test_binding_constants_match_header():
    """Every numeric #define of the header that the binding names has the
    header's value, and every kernel kind has a name."""
    text = open(HEADER).read()
    defs = {k: int(v) for k, v in re.findall(r"#define\s+(PTYC_[A-Z0-9_]+)\s+\(?(-?\d+)\)?", text)}
    named = {k: getattr(L, k) for k in dir(L) if k.startswith("PTYC_") and isinstance(getattr(L, k), int)}
    assert named, "binding names no constants"
    for k, v in named.items():
        assert k in defs, k
        assert defs[k] == v, (k, defs[k], v)
    assert sorted(L.KERNEL_NAMES) == list(range(defs["PTYC_KERNEL_KINDS"]))


def _cfg(**kw):
    base = dict(n=32, h=64, w=64, alpha=1.0, beta=1.0, mode=0, max_batch=0, seed=1, flags=0, reserved=0)
    base.update(kw)
    return L.Config(**base)


@pytest.mark.parametrize("bad", [
    dict(n=48), dict(n=8), dict(n=512), dict(h=16), dict(w=31), dict(h=70000), dict(mode=3),
    dict(reserved=1), dict(max_batch=-1), dict(alpha=float("nan")), dict(beta=float("inf")), dict(flags=8),
])
def test_init_rejects_bad_config_before_device(bad):
    lib = _lib()
    ctx = C.c_void_p()
    cfg = _cfg(**bad)
    p = np.ones((cfg.n, cfg.n), np.complex64) if cfg.n > 0 and cfg.n <= 256 else np.ones((1,), np.complex64)
    o = np.ones((64, 64), np.complex64)
    rc = lib.ptyc_init(C.byref(ctx), C.byref(cfg), p.ctypes.data, o.ctypes.data, 0, None)
    assert rc == L.PTYC_ERR_ARG
    assert ctx.value is None
    assert lib.ptyc_init_error().decode()


def test_init_rejects_null_pointers_and_kind():
    lib = _lib()
    ctx = C.c_void_p()
    cfg = _cfg()
    p = np.ones((32, 32), np.complex64)
    o = np.ones((64, 64), np.complex64)
    assert lib.ptyc_init(None, C.byref(cfg), p.ctypes.data, o.ctypes.data, 0, None) == L.PTYC_ERR_ARG
    assert lib.ptyc_init(C.byref(ctx), None, p.ctypes.data, o.ctypes.data, 0, None) == L.PTYC_ERR_ARG
    assert lib.ptyc_init(C.byref(ctx), C.byref(cfg), None, o.ctypes.data, 0, None) == L.PTYC_ERR_ARG
    assert lib.ptyc_init(C.byref(ctx), C.byref(cfg), p.ctypes.data, None, 0, None) == L.PTYC_ERR_ARG
    assert lib.ptyc_init(C.byref(ctx), C.byref(cfg), p.ctypes.data, o.ctypes.data, 7, None) == L.PTYC_ERR_ARG


def test_null_context_is_harmless():
    lib = _lib()
    assert lib.ptyc_num_positions(None) == -1
    assert lib.ptyc_sweep_count(None) == -1
    assert lib.ptyc_last_error(None)
    lib.ptyc_destroy(None)
    assert lib.ptyc_sweep(None, 1, None, 0, None, 0, None) == L.PTYC_ERR_ARG
    assert lib.ptyc_add_positions(None, 0, None, None, 0) == L.PTYC_ERR_ARG
    assert lib.ptyc_synchronize(None) == L.PTYC_ERR_ARG


def test_init_without_device_reports_hip_error():
    """On a host without a GPU a valid config fails with PTYC_ERR_HIP, not a crash."""
    lib = _lib()
    try:
        import torch
        has_gpu = torch.cuda.device_count() > 0
    except Exception:
        has_gpu = False
    if has_gpu:
        pytest.skip("a GPU is present")
    ctx = C.c_void_p()
    cfg = _cfg()
    p = np.ones((32, 32), np.complex64)
    o = np.ones((64, 64), np.complex64)
    rc = lib.ptyc_init(C.byref(ctx), C.byref(cfg), p.ctypes.data, o.ctypes.data, 0, None)
    assert rc == L.PTYC_ERR_HIP
    assert "device" in lib.ptyc_init_error().decode().lower()


@pytest.mark.parametrize("case", ["raster128", "fermat256", "random32", "cap"])
def test_library_colouring_equals_oracle_greedy(case):
    _lib()
    if case == "raster128":
        pos, n, cap = sim.raster_positions(20, 12, 128, 500, 2, 5), 128, 0
    elif case == "fermat256":
        pos, n, cap = sim.fermat_positions(600, 6.0, 256, 2048), 256, 0
    elif case == "random32":
        pos, n, cap = np.random.default_rng(3).integers(0, 300, (400, 2)).astype(np.int32), 32, 0
    else:
        pos, n, cap = sim.raster_positions(12, 40, 32, 600, 0, 0), 32, 7
    got, nc = colour(pos, n, cap)
    want = oracle.greedy_colouring(pos, n, cap if cap else 1024)
    np.testing.assert_array_equal(got, want)
    assert nc == want.max() + 1


def test_colouring_statistics_of_the_128px_raster():
    """The 60 x 60 raster (step 12, 128 px windows): an 11 x 11 block of
    positions overlaps pairwise, so at least 121 colours are needed."""
    _lib()
    pos = sim.raster_positions(60, 12, 128, 1024, 2, 1001)
    col, nc = colour(pos, 128)
    assert nc >= 121
    sizes = np.bincount(col)
    order = np.argsort(col, kind="stable")
    off = np.concatenate([[0], np.cumsum(sizes)])
    assert check_batches(pos, 128, order, off) == L.PTYC_OK
    assert 25 < sizes.mean() < 36


def test_library_validator_matches_oracle():
    _lib()
    rng = np.random.default_rng(4)
    pos = rng.integers(0, 200, (60, 2)).astype(np.int32)
    n = 24
    for trial in range(40):
        order = rng.permutation(60)
        cuts = np.sort(rng.choice(np.arange(1, 60), size=rng.integers(5, 40), replace=False))
        off = np.concatenate([[0], cuts, [60]])
        try:
            oracle.check_schedule(pos, n, order, off)
            ok = True
        except ValueError:
            ok = False
        assert (check_batches(pos, n, order, off) == L.PTYC_OK) == ok
    assert check_batches(pos, n, [0, 1], [0, 1, 3]) == L.PTYC_ERR_ARG
    assert check_batches(pos, n, [0, 99], [0, 2]) == L.PTYC_ERR_ARG
    assert check_batches(pos, n, [0, 0], [0, 2]) == L.PTYC_ERR_ARG   # a position twice in one batch


def test_colour_rejects_bad_input():
    lib = _lib()
    pos = np.array([[0, 0], [-1, 3]], np.int32)
    out = np.zeros(2, np.int32)
    nc = C.c_int32()
    assert lib.ptyc_colour(2, pos.ctypes.data, 16, 0, out.ctypes.data_as(C.POINTER(C.c_int32)),
                           C.byref(nc)) == L.PTYC_ERR_BOUNDS
    assert lib.ptyc_colour(2, None, 16, 0, out.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(nc)) == L.PTYC_ERR_ARG
