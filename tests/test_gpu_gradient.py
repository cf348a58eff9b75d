"""Amplitude-loss forward and hand-written adjoint on the GPU (through the
C ABI) against the FP64 oracle's loss and adjoint; the autograd wrapper."""
import numpy as np
import pytest

import oracle
import sim

pytestmark = pytest.mark.gpu

RTOL = 1e-5


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_10674_amd import _lib
    _lib.lib()
    return torch


@pytest.fixture(scope="module")
def problem(torch_cuda):
    """128 px patterns, first 400 positions of the raster, an estimate near
    the truth (so the Fourier moduli are well above FP32 resolution)."""
    torch = torch_cuda
    from paper_2308_10674_amd import Engine
    wl = sim.make_config(1, n_positions=400)
    rng = np.random.default_rng(31)
    O = wl.object_true * np.exp(0.15j * rng.standard_normal(wl.object_true.shape))
    P = wl.probe_true * (1 + 0.05 * rng.standard_normal(wl.probe_true.shape))
    eng = Engine(wl.n, wl.h, wl.w, wl.probe0, wl.object0, mode="coloured", seed=wl.seed)
    eng.add_positions(wl.positions, wl.intensities)
    to = torch.from_numpy(O.astype(np.complex64)).cuda()
    tp = torch.from_numpy(P.astype(np.complex64)).cuda()
    idx = rng.choice(wl.count, 120, replace=False)
    return dict(wl=wl, eng=eng, O=O.astype(np.complex64), P=P.astype(np.complex64), to=to, tp=tp, idx=idx)


def _near_truth(wl, seed):
    """An estimate near the truth: the object with a 0.15 rad random phase
    error, the probe with 5 % random amplitude error (complex64)."""
    rng = np.random.default_rng(seed)
    O = wl.object_true * np.exp(0.15j * rng.standard_normal(wl.object_true.shape))
    P = wl.probe_true * (1 + 0.05 * rng.standard_normal(wl.probe_true.shape))
    return O.astype(np.complex64), P.astype(np.complex64)


def _compare(torch, eng, wl, O, P, idx):
    """Loss and both gradients of the GPU against the FP64 adjoint taken at
    the same complex64 estimate: (rel loss, rel-L2 grad O over the windows,
    rel-L2 grad P, grad O outside the windows all zero)."""
    to = torch.from_numpy(O).cuda()
    tp = torch.from_numpy(P).cuda()
    L, go, gp = eng.amp_loss(to, tp, idx, grad=True)
    Lo, go_o, gp_o = oracle.amplitude_loss_grad(O, P, wl.positions, wl.intensities, idx)
    mask = oracle.union_mask(wl.positions[idx], wl.n, wl.h, wl.w)
    go = go.cpu().numpy()
    gp = gp.cpu().numpy()
    return abs(L - Lo) / Lo, oracle.rel_l2(go, go_o, mask), oracle.rel_l2(gp, gp_o), bool(np.all(go[~mask] == 0))


@pytest.mark.parametrize("n", [16, 32, 64, 128, 256])
def test_gradient_every_size(n, torch_cuda):
    """Loss, dL/dO and dL/dP element-wise against the FP64 adjoint at every
    pattern size the library supports: a 5 x 5 raster with overlapping
    windows (step n/3), all 25 positions in one minibatch, so the adjoint's
    scatter-add runs over several colours."""
    from paper_2308_10674_amd import Engine
    step = max(1, n // 3)
    m = n + 4 * step + 8
    pos = sim.raster_positions(5, step, n, m, 1, 40 + n)
    wl = sim.make_workload(n, m, 0.3 * n, 0.5 / (0.3 * n), pos, 1e6, 40 + n)
    eng = Engine(wl.n, wl.h, wl.w, wl.probe0, wl.object0, mode="coloured", seed=wl.seed)
    eng.add_positions(wl.positions, wl.intensities)
    O, P = _near_truth(wl, 41 + n)
    idx = np.random.default_rng(n).permutation(wl.count)
    rl, ro, rp, zero_out = _compare(torch_cuda, eng, wl, O, P, idx)
    print(f"n={n} loss {rl:.2e} grad O {ro:.2e} grad P {rp:.2e}", flush=True)
    assert rl <= RTOL and ro <= RTOL and rp <= RTOL
    assert zero_out


def test_gradient_finite_difference_subproblem(torch_cuda):
    """The 32 px, 10-position subproblem on a 64^2 object on which the
    oracle's adjoint is pinned to FP64 central differences: the GPU's
    gradients against that adjoint (1e-5 relative L2), and the GPU's
    directional derivatives Re<grad, V> against FP64 central differences
    of the oracle's loss along random directions (bar 5e-5: the 2e-5 at
    which the oracle's own adjoint meets those differences plus the 1e-5
    parity bar)."""
    torch = torch_cuda
    from paper_2308_10674_amd import Engine
    wl = sim.make_workload(32, 64, 10.0, 0.05, sim.raster_positions(4, 8, 32, 64, 1, 21)[:10], 1e6, 21,
                           noise=True, dtype=np.float64)
    rng = np.random.default_rng(22)
    O = (wl.object_true * np.exp(0.2j * rng.standard_normal(wl.object_true.shape))).astype(np.complex64)
    P = (wl.probe0 + 0.1 * (rng.standard_normal(wl.probe0.shape) + 1j * rng.standard_normal(wl.probe0.shape))
         * np.abs(wl.probe0).max()).astype(np.complex64)
    eng = Engine(wl.n, wl.h, wl.w, wl.probe0, wl.object0, mode="coloured", seed=wl.seed)
    eng.add_positions(wl.positions, wl.intensities.astype(np.float32))
    wl.intensities = wl.intensities.astype(np.float32).astype(np.float64)   # what the GPU holds
    idx = np.arange(wl.count)
    rl, ro, rp, zero_out = _compare(torch, eng, wl, O, P, idx)
    print(f"fd subproblem: loss {rl:.2e} grad O {ro:.2e} grad P {rp:.2e}", flush=True)
    assert rl <= RTOL and ro <= RTOL and rp <= RTOL and zero_out
    _, go, gp = eng.amp_loss(torch.from_numpy(O).cuda(), torch.from_numpy(P).cuda(), idx, grad=True)
    go = go.cpu().numpy().astype(np.complex128)
    gp = gp.cpu().numpy().astype(np.complex128)
    O64, P64 = O.astype(np.complex128), P.astype(np.complex128)
    drng = np.random.default_rng(23)
    for _ in range(3):
        for which in ("O", "P"):
            base = O64 if which == "O" else P64
            V = drng.standard_normal(base.shape) + 1j * drng.standard_normal(base.shape)
            h = 1e-6 * (1.0 if which == "O" else np.abs(P64).max())
            if which == "O":
                fp = oracle.amplitude_loss(O64 + h * V, P64, wl.positions, wl.intensities)
                fm = oracle.amplitude_loss(O64 - h * V, P64, wl.positions, wl.intensities)
                ana = np.real(np.vdot(go, V))
            else:
                fp = oracle.amplitude_loss(O64, P64 + h * V, wl.positions, wl.intensities)
                fm = oracle.amplitude_loss(O64, P64 - h * V, wl.positions, wl.intensities)
                ana = np.real(np.vdot(gp, V))
            fd = (fp - fm) / (2 * h)
            print("fd", which, fd, ana, flush=True)
            assert abs(fd - ana) <= 5e-5 * abs(fd), (which, fd, ana)


def test_loss_matches_oracle(problem):
    pr = problem
    L = pr["eng"].amp_loss(pr["to"], pr["tp"], pr["idx"])
    Lo = oracle.amplitude_loss(pr["O"].astype(np.complex128), pr["P"].astype(np.complex128),
                               pr["wl"].positions, pr["wl"].intensities, pr["idx"])
    assert abs(L - Lo) <= RTOL * Lo, (L, Lo)


def test_gradient_matches_cpu_adjoint(problem):
    pr = problem
    wl = pr["wl"]
    L, go, gp = pr["eng"].amp_loss(pr["to"], pr["tp"], pr["idx"], grad=True)
    Lo, go_o, gp_o = oracle.amplitude_loss_grad(pr["O"], pr["P"], wl.positions, wl.intensities, pr["idx"])
    mask = oracle.union_mask(wl.positions[pr["idx"]], wl.n, wl.h, wl.w)
    go = go.cpu().numpy()
    gp = gp.cpu().numpy()
    ro = oracle.rel_l2(go, go_o, mask)
    rp = oracle.rel_l2(gp, gp_o)
    print("grad rel-L2 object", ro, "probe", rp)
    assert ro <= RTOL and rp <= RTOL
    assert np.all(go[~mask] == 0)
    assert abs(L - Lo) <= RTOL * Lo


def test_gradient_is_deterministic_and_scaled(problem):
    pr = problem
    _, a_o, a_p = pr["eng"].amp_loss(pr["to"], pr["tp"], pr["idx"], grad=True)
    _, b_o, b_p = pr["eng"].amp_loss(pr["to"], pr["tp"], pr["idx"], grad=True)
    _, c_o, c_p = pr["eng"].amp_loss(pr["to"], pr["tp"], pr["idx"], grad=True, scale=0.5)
    assert bool((a_o == b_o).all()) and bool((a_p == b_p).all())
    np.testing.assert_allclose(c_o.cpu().numpy(), 0.5 * a_o.cpu().numpy(), rtol=1e-6, atol=0)
    np.testing.assert_allclose(c_p.cpu().numpy(), 0.5 * a_p.cpu().numpy(), rtol=1e-6, atol=0)


def test_gradient_equals_scaled_epie_step(problem, torch_cuda):
    """For one position the ePIE object step is -alpha / (2 N^2 max|P|^2)
    times the loss gradient: two different GPU paths tied by a closed form."""
    torch = torch_cuda
    from paper_2308_10674_amd import Engine
    pr = problem
    wl = pr["wl"]
    j = int(pr["idx"][0])
    _, go, _ = pr["eng"].amp_loss(pr["to"], pr["tp"], [j], grad=True)
    e = Engine(wl.n, wl.h, wl.w, pr["P"], pr["O"], alpha=0.7, beta=0.0, mode="strict")
    e.add_positions(wl.positions, wl.intensities)
    e.sweep(1, order=[j])
    step = e.get_object().astype(np.complex128) - pr["O"].astype(np.complex128)
    scale = -0.7 / (2 * wl.n * wl.n * np.max(np.abs(pr["P"].astype(np.complex128)) ** 2))
    y, x = wl.positions[j]
    win = (slice(y, y + wl.n), slice(x, x + wl.n))
    r = oracle.rel_l2(step[win], scale * go.cpu().numpy().astype(np.complex128)[win])
    assert r <= 1e-4, r   # the step is a small difference of FP32 numbers near 1


def test_async_loss_equals_synchronous(problem, torch_cuda):
    """ptyc_amp_loss_async (device loss, no wait) gives the bytes of
    ptyc_amp_loss, and the library's in-place scale is a plain float
    multiply."""
    torch = torch_cuda
    pr = problem
    L, go, gp = pr["eng"].amp_loss(pr["to"], pr["tp"], pr["idx"], grad=True)
    Ld, god, gpd = pr["eng"].amp_loss_async(pr["to"], pr["tp"], pr["idx"], grad=True)
    Lo = pr["eng"].amp_loss_async(pr["to"], pr["tp"], pr["idx"], grad=False)[0]
    assert float(Ld) == L and float(Lo) == L
    assert bool((god == go).all()) and bool((gpd == gp).all())
    s = torch.tensor(0.37, dtype=torch.float64, device="cuda")
    ref = go.cpu().numpy() * np.float32(0.37)
    pr["eng"].scale_(god, s)
    np.testing.assert_array_equal(god.cpu().numpy(), ref)


def test_autograd_function(problem, torch_cuda):
    torch = torch_cuda
    from paper_2308_10674_amd import amplitude_loss
    pr = problem
    O = pr["to"].clone().requires_grad_(True)
    P = pr["tp"].clone().requires_grad_(True)
    loss = amplitude_loss(pr["eng"], O, P, pr["idx"])
    (3.0 * loss).backward()
    L1, go, gp = pr["eng"].amp_loss(pr["to"], pr["tp"], pr["idx"], grad=True)
    assert float(loss.detach()) == L1
    # the saved gradients times the upstream gradient (3), one float multiply
    np.testing.assert_array_equal(O.grad.cpu().numpy(), go.cpu().numpy() * np.float32(3.0))
    np.testing.assert_array_equal(P.grad.cpu().numpy(), gp.cpu().numpy() * np.float32(3.0))
    # the scaled-inside gradient of ptyc_amp_loss agrees to rounding
    _, go3, gp3 = pr["eng"].amp_loss(pr["to"], pr["tp"], pr["idx"], grad=True, scale=3.0)
    np.testing.assert_allclose(O.grad.cpu().numpy(), go3.cpu().numpy(), rtol=1e-5, atol=1e-6 * float(go3.abs().max()))


def test_directional_derivative(problem, torch_cuda):
    """Central differences of the GPU loss along random directions agree
    with Re<grad, V> (checks conjugation and factor conventions)."""
    torch = torch_cuda
    pr = problem
    eng = pr["eng"]
    L, go, gp = eng.amp_loss(pr["to"], pr["tp"], pr["idx"], grad=True)
    g = torch.Generator(device="cpu").manual_seed(5)
    for which in ("O", "P"):
        base = pr["to"] if which == "O" else pr["tp"]
        V = torch.complex(torch.randn(base.shape, generator=g), torch.randn(base.shape, generator=g)).cuda()
        # a perturbation shaped like the estimate keeps the curvature term small
        V = V * base.abs() / base.abs().max()
        h = 1e-3 * float(base.abs().max())
        if which == "O":
            fp = eng.amp_loss(pr["to"] + h * V, pr["tp"], pr["idx"])
            fm = eng.amp_loss(pr["to"] - h * V, pr["tp"], pr["idx"])
            ana = float(torch.real(torch.vdot(go.flatten(), V.flatten())))
        else:
            fp = eng.amp_loss(pr["to"], pr["tp"] + h * V, pr["idx"])
            fm = eng.amp_loss(pr["to"], pr["tp"] - h * V, pr["idx"])
            ana = float(torch.real(torch.vdot(gp.flatten(), V.flatten())))
        fd = (fp - fm) / (2 * h)
        print(which, fd, ana)
        assert abs(fd - ana) <= 2e-2 * abs(ana), (which, fd, ana)


def test_adam_descends(torch_cuda):
    """Gradient reconstruction with Adam on minibatches lowers the loss."""
    torch = torch_cuda
    from paper_2308_10674_amd import Engine, amplitude_loss
    wl = sim.make_config(1, n_positions=300)
    eng = Engine(wl.n, wl.h, wl.w, wl.probe0, wl.object0, mode="coloured", seed=wl.seed)
    eng.add_positions(wl.positions, wl.intensities)
    O = torch.from_numpy(wl.object0.astype(np.complex64)).cuda().requires_grad_(True)
    P = torch.from_numpy(wl.probe0.astype(np.complex64)).cuda().requires_grad_(True)
    opt = torch.optim.Adam([O, P], lr=1e-2)
    rng = np.random.default_rng(3)
    full = np.arange(wl.count)
    first = eng.amp_loss(O, P, full)
    for epoch in range(4):
        perm = rng.permutation(wl.count)
        for b in range(0, wl.count, 100):
            opt.zero_grad()
            amplitude_loss(eng, O, P, perm[b:b + 100]).backward()
            opt.step()
    last = eng.amp_loss(O, P, full)
    print("adam loss", first, "->", last)
    assert last < 0.8 * first


def test_bad_arguments(problem, torch_cuda):
    torch = torch_cuda
    from paper_2308_10674_amd import PtycError
    pr = problem
    with pytest.raises(PtycError):
        pr["eng"].amp_loss(pr["to"], pr["tp"], [10 ** 6])
    assert pr["eng"].amp_loss(pr["to"], pr["tp"], []) == 0.0


def _loss_into(torch, eng, to, tp, idx):
    """ptyc_amp_loss through the C ABI into gradient buffers filled with NaN
    beforehand, so an element the library leaves unwritten shows."""
    import ctypes as C

    from paper_2308_10674_amd import _lib
    go = torch.full_like(to, complex(float("nan"), float("nan")))
    gp = torch.full_like(tp, complex(float("nan"), float("nan")))
    ia = np.ascontiguousarray(np.asarray(idx, dtype=np.int64).ravel())
    loss = C.c_double()
    torch.cuda.synchronize()
    rc = _lib.lib().ptyc_amp_loss(eng._ctx, to.data_ptr(), tp.data_ptr(), ia.ctypes.data_as(C.POINTER(C.c_int64)),
                                  len(ia), 1.0, go.data_ptr(), gp.data_ptr(), C.byref(loss))
    assert rc == 0, rc
    return loss.value, go.cpu().numpy(), gp.cpu().numpy()


def test_gradient_edge_minibatches(problem, torch_cuda):
    """Every element of both gradients is written (the buffers hold NaN
    before the call): an empty minibatch gives loss 0 and zero gradients;
    a minibatch that lists one position twice counts its term twice, as
    the oracle's sum does; minibatches of 1, 16 and 17 positions (one
    partial sum of dL/dP, exactly one group of 16, one more) and of 120
    match the FP64 adjoint."""
    torch = torch_cuda
    pr = problem
    wl = pr["wl"]
    L, go, gp = _loss_into(torch, pr["eng"], pr["to"], pr["tp"], [])
    assert L == 0.0
    assert np.all(go == 0) and np.all(gp == 0)
    base = [int(j) for j in pr["idx"]]
    cases = {"one": base[:1], "sixteen": base[:16], "seventeen": base[:17], "repeat": base[:9] + base[3:5],
             "all": base}
    for name, idx in cases.items():
        L, go, gp = _loss_into(torch, pr["eng"], pr["to"], pr["tp"], idx)
        assert np.all(np.isfinite(go)) and np.all(np.isfinite(gp)), name
        Lo, go_o, gp_o = oracle.amplitude_loss_grad(pr["O"], pr["P"], wl.positions, wl.intensities, np.asarray(idx))
        mask = oracle.union_mask(wl.positions[np.asarray(idx)], wl.n, wl.h, wl.w)
        ro, rp = oracle.rel_l2(go, go_o, mask), oracle.rel_l2(gp, gp_o)
        print(name, len(idx), "loss", abs(L - Lo) / Lo, "grad O", ro, "grad P", rp)
        assert abs(L - Lo) <= RTOL * Lo, name
        assert ro <= RTOL and rp <= RTOL, (name, ro, rp)
        assert np.all(go[~mask] == 0), name


def test_gradient_full_size_minibatch(torch_cuda):
    """The benchmark's gradient workload at its full size: the 3600-position
    128 px raster on the 1024 x 1024 object, one shuffled minibatch of 512
    (the benchmark's minibatch), an estimate near the truth; loss and both
    gradients element-wise against the FP64 adjoint at 1e-5."""
    from paper_2308_10674_amd import Engine
    wl = sim.make_config(3)
    eng = Engine(wl.n, wl.h, wl.w, wl.probe0, wl.object0, mode="coloured", seed=wl.seed)
    eng.add_positions(wl.positions, wl.intensities)
    O, P = _near_truth(wl, 77)
    idx = np.random.default_rng([wl.seed, 9]).permutation(wl.count)[:512]
    rl, ro, rp, zero_out = _compare(torch_cuda, eng, wl, O, P, idx)
    print("full-size minibatch: loss", rl, "grad O", ro, "grad P", rp)
    assert rl <= RTOL and ro <= RTOL and rp <= RTOL, (rl, ro, rp)
    assert zero_out
    eng.close()
