"""Python face of libptyc: argument marshalling onto the C ABI, nothing else.

Every step of the reconstruction runs in the library's HIP kernels; torch is
used only for device tensors (inputs and outputs that live on the GPU) and
for the current HIP stream.  There is no CPU fallback: if libptyc.so is
missing or no GPU is present, the calls fail.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L

try:  # torch is optional for host-only use
    import torch
except Exception:  # pragma: no cover
    torch = None


def _check(rc: int, ctx=None):
    if rc != L.PTYC_OK:
        lib = L.lib()
        msg = lib.ptyc_last_error(ctx).decode() if ctx else lib.ptyc_init_error().decode()
        raise L.PtycError(rc, msg)


def _buffer(x, np_dtype, torch_dtype):
    """(pointer, mem_kind, keepalive) for a numpy array or torch tensor."""
    if torch is not None and isinstance(x, torch.Tensor):
        t = x.detach()
        if t.dtype != torch_dtype:
            t = t.to(torch_dtype)
        t = t.contiguous()
        kind = L.PTYC_MEM_DEVICE if t.is_cuda else L.PTYC_MEM_HOST
        return t.data_ptr(), kind, t
    a = np.ascontiguousarray(x, dtype=np_dtype)
    return a.ctypes.data, L.PTYC_MEM_HOST, a


def _i64(a):
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(C.POINTER(C.c_int64))


def current_stream_handle():
    """The raw hipStream_t of torch's current stream (None without a GPU)."""
    if torch is not None and torch.cuda.is_available():
        return torch.cuda.current_stream().cuda_stream
    return None


class Engine:
    """A live ePIE reconstruction (one libptyc context).

    Geometry is fixed at construction; positions and patterns are appended
    with add_positions while sweeps run.  mode "strict" is sequential ePIE,
    "coloured" batches positions with disjoint windows.
    """

    def __init__(self, n, h, w, probe0, object0, *, alpha=1.0, beta=1.0, mode="coloured",
                 max_batch=0, seed=0, sqrt_input=False, centred=False, stream=None, form="default"):
        lib = L.lib()
        cfg = L.Config(n=n, h=h, w=w, alpha=alpha, beta=beta,
                       mode=L.PTYC_MODE_STRICT if mode == "strict" else L.PTYC_MODE_COLOURED,
                       max_batch=max_batch, seed=seed,
                       flags=(L.PTYC_I_IS_SQRT if sqrt_input else 0) | (L.PTYC_I_CENTERED if centred else 0),
                       reserved=0)
        tdt = torch.complex64 if torch is not None else None
        pp, pk, pkeep = _buffer(probe0, np.complex64, tdt)
        op, ok, okeep = _buffer(object0, np.complex64, tdt)
        if pk != ok:
            raise ValueError("probe0 and object0 must both be host or both be device buffers")
        if stream is None:
            stream = current_stream_handle()
        self._ctx = C.c_void_p()
        self.n, self.h, self.w, self.mode = n, h, w, mode
        _check(lib.ptyc_init(C.byref(self._ctx), C.byref(cfg), pp, op, pk, stream))
        if form != "default":
            self.form = form

    # ------------------------------------------------------------------ data
    def add_positions(self, positions, intensities):
        """positions: [count, 2] int32 window corners (row, col);
        intensities: [count, n, n] float32 (host or device)."""
        lib = L.lib()
        tf = torch.float32 if torch is not None else None
        ti = torch.int32 if torch is not None else None
        pp, pk, pkeep = _buffer(positions, np.int32, ti)
        ip, ik, ikeep = _buffer(intensities, np.float32, tf)
        count = int(np.prod(pkeep.shape) // 2)
        if pk != ik:
            # positions are tiny: bring them to the intensities' side
            pos_np = np.ascontiguousarray(
                positions.cpu().numpy() if (torch is not None and isinstance(positions, torch.Tensor))
                else positions, dtype=np.int32)
            if ik == L.PTYC_MEM_DEVICE:
                pkeep = torch.from_numpy(pos_np).to(ikeep.device)
                pp = pkeep.data_ptr()
            else:
                pkeep = pos_np
                pp = pos_np.ctypes.data
        _check(lib.ptyc_add_positions(self._ctx, count, pp, ip, ik), self._ctx)
        return self

    def set_ingest(self, frame=None, crop=(0, 0), orient=0, scale=1.0, centred=False, sqrt_input=False):
        """Preprocessing of raw frames (see ptyc_set_ingest): frame size,
        top-left corner of the n x n crop, orientation 0..7 (bit 0
        transpose, bit 1 flip rows, bit 2 flip columns), gain scale, DC at
        the crop centre, amplitudes instead of counts."""
        fh, fw = (self.n, self.n) if frame is None else frame
        spec = L.Ingest(frame_h=fh, frame_w=fw, crop_y=crop[0], crop_x=crop[1], orient=orient, scale=scale,
                        flags=(L.PTYC_I_IS_SQRT if sqrt_input else 0) | (L.PTYC_I_CENTERED if centred else 0),
                        reserved=0)
        _check(L.lib().ptyc_set_ingest(self._ctx, C.byref(spec)), self._ctx)

    def set_mask(self, mask):
        """Detector mask in raw frame coordinates (nonzero = measured)."""
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        _check(L.lib().ptyc_set_mask(self._ctx, m.ctypes.data, L.PTYC_MEM_HOST), self._ctx)

    def get_patterns(self, first=0, count=None):
        """Stored amplitudes sqrt(I) after preprocessing, [count, n, n]."""
        count = self.num_positions - first if count is None else count
        out = np.empty((count, self.n, self.n), dtype=np.float32)
        _check(L.lib().ptyc_get_patterns(self._ctx, first, count, out.ctypes.data, L.PTYC_MEM_HOST), self._ctx)
        return out

    # ----------------------------------------------------------------- sweep
    def sweep(self, n_sweeps=1, order=None, batch_offsets=None, errors=False):
        """Run sweeps; returns the running Fourier error per sweep when
        ``errors`` (this synchronises), else None."""
        lib = L.lib()
        o, op = _i64(order)
        b, bp = _i64(batch_offsets)
        olen = 0 if o is None else len(o)
        nb = 0 if b is None else len(b) - 1
        err = np.zeros(n_sweeps, dtype=np.float64) if errors else None
        ep = err.ctypes.data_as(C.POINTER(C.c_double)) if errors else None
        _check(lib.ptyc_sweep(self._ctx, n_sweeps, op, olen, bp, nb, ep), self._ctx)
        return err

    def sweep_noalloc(self, n_sweeps=1, order=None, batch_offsets=None, errors=False):
        """sweep() through ptyc_sweep_noalloc: the same sweeps with the
        library's fixed work memory (no allocation in the call)."""
        lib = L.lib()
        o, op = _i64(order)
        b, bp = _i64(batch_offsets)
        olen = 0 if o is None else len(o)
        nb = 0 if b is None else len(b) - 1
        err = np.zeros(n_sweeps, dtype=np.float64) if errors else None
        ep = err.ctypes.data_as(C.POINTER(C.c_double)) if errors else None
        _check(lib.ptyc_sweep_noalloc(self._ctx, n_sweeps, op, olen, bp, nb, ep), self._ctx)
        return err

    def get_schedule(self):
        """(order, batch_offsets) of the next default sweep."""
        lib = L.lib()
        nb = C.c_int64()
        _check(lib.ptyc_get_schedule(self._ctx, None, None, C.byref(nb)), self._ctx)
        n = self.num_positions
        order = np.zeros(n, dtype=np.int64)
        off = np.zeros(nb.value + 1, dtype=np.int64)
        _check(lib.ptyc_get_schedule(self._ctx, order.ctypes.data_as(C.POINTER(C.c_int64)),
                                     off.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(nb)), self._ctx)
        return order, off

    # ---------------------------------------------------------------- state
    def _get(self, fn, shape, device):
        lib = L.lib()
        if device:
            out = torch.empty(shape, dtype=torch.complex64, device="cuda")
            _check(fn(self._ctx, out.data_ptr(), L.PTYC_MEM_DEVICE), self._ctx)
            return out
        out = np.empty(shape, dtype=np.complex64)
        _check(fn(self._ctx, out.ctypes.data, L.PTYC_MEM_HOST), self._ctx)
        return out

    def get_object(self, device=False):
        return self._get(L.lib().ptyc_get_object, (self.h, self.w), device)

    def get_probe(self, device=False):
        return self._get(L.lib().ptyc_get_probe, (self.n, self.n), device)

    def set_object(self, obj):
        p, k, keep = _buffer(obj, np.complex64, torch.complex64 if torch is not None else None)
        _check(L.lib().ptyc_set_object(self._ctx, p, k), self._ctx)

    def set_probe(self, probe):
        p, k, keep = _buffer(probe, np.complex64, torch.complex64 if torch is not None else None)
        _check(L.lib().ptyc_set_probe(self._ctx, p, k), self._ctx)

    # ------------------------------------------------------------ gradient
    def amp_loss(self, obj, probe, idx, grad=False, scale=1.0):
        """Amplitude loss sum_j || |F(P S_j O)| - sqrt(I_j) ||^2 over the
        positions ``idx`` for the device tensors ``obj`` and ``probe``
        (complex64).  With ``grad`` also returns scale * dL/dO and
        scale * dL/dP (PyTorch convention) as new device tensors."""
        o = obj.detach()
        p = probe.detach()
        if not (o.is_cuda and p.is_cuda) or o.dtype != torch.complex64 or p.dtype != torch.complex64:
            raise ValueError("obj and probe must be complex64 CUDA tensors")
        o = o.contiguous()
        p = p.contiguous()
        ia, ip = _i64(np.asarray(idx, dtype=np.int64).ravel())
        loss = C.c_double()
        go = gp = None
        if grad:
            go = torch.empty_like(o)
            gp = torch.empty_like(p)
        _check(L.lib().ptyc_amp_loss(self._ctx, o.data_ptr(), p.data_ptr(), ip, len(ia), float(scale),
                                     go.data_ptr() if grad else None, gp.data_ptr() if grad else None,
                                     C.byref(loss)), self._ctx)
        return (loss.value, go, gp) if grad else loss.value

    def amp_loss_async(self, obj, probe, idx, grad=True):
        """Loss (a float64 CUDA scalar tensor) and, with ``grad``, dL/dO and
        dL/dP as device tensors, all filled in when the enqueued work runs
        on the stream (nothing waits for it here).  The two gradients are
        views of one allocation (dL/dO, then dL/dP)."""
        loss, flat, go, gp = self._amp_loss_flat(obj, probe, idx, grad)
        return loss, go, gp

    def _amp_loss_flat(self, obj, probe, idx, grad):
        """amp_loss_async, also returning the one buffer that holds both
        gradients (so one scaling call covers them)."""
        o = obj.detach()
        p = probe.detach()
        if not (o.is_cuda and p.is_cuda) or o.dtype != torch.complex64 or p.dtype != torch.complex64:
            raise ValueError("obj and probe must be complex64 CUDA tensors")
        o = o.contiguous()
        p = p.contiguous()
        ia, ip = _i64(np.asarray(idx, dtype=np.int64).ravel())
        loss = torch.empty((), dtype=torch.float64, device=o.device)
        flat = go = gp = None
        if grad:
            flat = torch.empty(o.numel() + p.numel(), dtype=torch.complex64, device=o.device)
            go = flat[:o.numel()].view(o.shape)
            gp = flat[o.numel():].view(p.shape)
        _check(L.lib().ptyc_amp_loss_async(self._ctx, o.data_ptr(), p.data_ptr(), ip, len(ia),
                                           go.data_ptr() if grad else None, gp.data_ptr() if grad else None,
                                           loss.data_ptr()), self._ctx)
        # the inputs and outputs must outlive the enqueued work: torch's
        # caching allocator reuses freed blocks only in stream order
        return loss, flat, go, gp

    def scale_(self, data, scale_dev):
        """data (complex64 CUDA tensor) *= scale_dev (float64 CUDA scalar),
        in place, on the library's stream."""
        if not data.is_contiguous() or data.dtype != torch.complex64:
            raise ValueError("data must be a contiguous complex64 tensor")
        s = scale_dev.detach().to(torch.float64).contiguous()
        _check(L.lib().ptyc_scale_c64(self._ctx, data.data_ptr(), data.numel(), s.data_ptr()), self._ctx)
        return data

    # ------------------------------------------------------------ profiling
    def profile(self, enable=True):
        """Start (reset) or stop per-kernel event timing."""
        _check(L.lib().ptyc_profile(self._ctx, 1 if enable else 0), self._ctx)

    def profile_read(self):
        """{kernel name: (total ms, launches, position updates)}."""
        out = {}
        for k, name in L.KERNEL_NAMES.items():
            ms = C.c_double()
            n = C.c_int64()
            u = C.c_int64()
            _check(L.lib().ptyc_profile_read(self._ctx, k, C.byref(ms), C.byref(n), C.byref(u)), self._ctx)
            if n.value:
                out[name] = (ms.value, n.value, u.value)
        return out

    @property
    def tile(self) -> int:
        """Tile variant of the per-batch kernels (0 .. tile_count - 1)."""
        return int(L.lib().ptyc_get_tile(self._ctx))

    @tile.setter
    def tile(self, v):
        _check(L.lib().ptyc_set_tile(self._ctx, int(v)), self._ctx)

    @property
    def tile_count(self) -> int:
        return int(L.lib().ptyc_tile_count(self._ctx))

    def tune(self, reps=3):
        """Time every tile variant on one sweep of the loaded positions
        (state restored afterwards) and keep the fastest.  Returns (chosen
        variant, [best ms per sweep of each variant])."""
        t = C.c_int32()
        ms = (C.c_double * L.PTYC_TILE_MAX)()
        _check(L.lib().ptyc_tune(self._ctx, int(reps), C.byref(t), ms), self._ctx)
        return int(t.value), [float(ms[i]) for i in range(self.tile_count)]

    @property
    def form(self) -> str:
        f = int(L.lib().ptyc_get_form(self._ctx))
        return {L.PTYC_FORM_BATCH: "batch", L.PTYC_FORM_PERSISTENT: "persistent",
                L.PTYC_FORM_GRAPH: "graph"}.get(f, str(f))

    @form.setter
    def form(self, name):
        code = {"default": L.PTYC_FORM_DEFAULT, "batch": L.PTYC_FORM_BATCH,
                "persistent": L.PTYC_FORM_PERSISTENT, "graph": L.PTYC_FORM_GRAPH}[name]
        _check(L.lib().ptyc_set_form(self._ctx, code), self._ctx)

    @property
    def multi_variant(self) -> int:
        """How a sweep_multi call led by this engine runs (see tune_multi)."""
        return int(L.lib().ptyc_get_multi_variant(self._ctx))

    @multi_variant.setter
    def multi_variant(self, v):
        _check(L.lib().ptyc_set_multi_variant(self._ctx, int(v)), self._ctx)

    @property
    def num_positions(self) -> int:
        return int(L.lib().ptyc_num_positions(self._ctx))

    @property
    def sweeps_done(self) -> int:
        return int(L.lib().ptyc_sweep_count(self._ctx))

    def synchronize(self):
        _check(L.lib().ptyc_synchronize(self._ctx), self._ctx)

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            L.lib().ptyc_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sweep_multi(engines, n_sweeps=1, errors=False):
    """Run n_sweeps sweeps of several independent reconstructions together
    (one launch per stage and pattern size covers the current batch of all
    of them).  Same result as calling each engine's sweep(n_sweeps).
    Returns an [len(engines), n_sweeps] array of errors when ``errors``."""
    lib = L.lib()
    arr = (C.c_void_p * len(engines))(*[e._ctx.value for e in engines])
    err = np.zeros((len(engines), n_sweeps), dtype=np.float64) if errors else None
    ep = err.ctypes.data_as(C.POINTER(C.c_double)) if errors else None
    rc = lib.ptyc_sweep_multi(arr, len(engines), n_sweeps, ep)
    if rc != L.PTYC_OK:
        msgs = "; ".join(lib.ptyc_last_error(e._ctx).decode() for e in engines)
        raise L.PtycError(rc, msgs or "ptyc_sweep_multi failed")
    return err


def tune_multi(engines, reps=2):
    """Time every way ptyc_sweep_multi can run on one joint sweep of these
    engines (state restored afterwards) and keep the fastest on the first
    engine.  Returns (chosen variant, [best ms of each variant])."""
    lib = L.lib()
    arr = (C.c_void_p * len(engines))(*[e._ctx.value for e in engines])
    v = C.c_int32()
    ms = (C.c_double * L.PTYC_MULTI_VARIANTS)()
    rc = lib.ptyc_tune_multi(arr, len(engines), int(reps), C.byref(v), ms)
    if rc != L.PTYC_OK:
        msgs = "; ".join(lib.ptyc_last_error(e._ctx).decode() for e in engines)
        raise L.PtycError(rc, msgs or "ptyc_tune_multi failed")
    return int(v.value), [float(ms[i]) for i in range(lib.ptyc_multi_variant_count())]


def average(engines):
    """Replace object and probe of every engine by their mean over the
    engines (the synchronisation of the subset-parallel scheme)."""
    lib = L.lib()
    arr = (C.c_void_p * len(engines))(*[e._ctx.value for e in engines])
    rc = lib.ptyc_average(arr, len(engines))
    if rc != L.PTYC_OK:
        msgs = "; ".join(lib.ptyc_last_error(e._ctx).decode() for e in engines)
        raise L.PtycError(rc, msgs or "ptyc_average failed")


# ---------------------------------------------------------------- host helpers

def colour(positions, n, max_batch=0):
    """The library's greedy first-fit colouring (host only)."""
    pos = np.ascontiguousarray(positions, dtype=np.int32)
    out = np.zeros(len(pos), dtype=np.int32)
    nc = C.c_int32()
    _check(L.lib().ptyc_colour(len(pos), pos.ctypes.data, n, max_batch,
                               out.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(nc)))
    return out, nc.value


def check_batches(positions, n, order, batch_offsets) -> int:
    """The library's host validator; returns the status code."""
    pos = np.ascontiguousarray(positions, dtype=np.int32)
    o, op = _i64(order)
    b, bp = _i64(batch_offsets)
    return int(L.lib().ptyc_check_batches(len(pos), pos.ctypes.data, n, op, len(o), bp, len(b) - 1))
