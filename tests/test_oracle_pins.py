"""Pins of the FP64 oracle against facts it does not compute itself:
hand-worked examples, closed forms, textbook special cases, invariants,
brute force on tiny inputs.  CPU only."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import sim

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rand_c(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# ------------------------------------------------------------- transform

@pytest.mark.parametrize("n", [1, 2, 4, 8])
def test_fft_matches_bruteforce_dft(n):
    rng = np.random.default_rng([1, n])
    x = _rand_c(rng, (n, n))
    np.testing.assert_allclose(oracle.fft2(x), oracle.dft2_bruteforce(x), rtol=0, atol=1e-12 * n * n)


@pytest.mark.parametrize("n", [4, 32, 128])
def test_fft_closed_forms(n):
    # a unit impulse at (r0, c0) transforms to exp(-2 pi i (k r0 + l c0)/n)
    r0, c0 = 1, n - 1
    x = np.zeros((n, n), complex)
    x[r0, c0] = 1
    k, l = np.mgrid[0:n, 0:n]
    np.testing.assert_allclose(oracle.fft2(x), np.exp(-2j * np.pi * (k * r0 + l * c0) / n), atol=1e-12)
    # a constant transforms to n^2 at DC and zero elsewhere
    X = oracle.fft2(np.ones((n, n)))
    ref = np.zeros((n, n))
    ref[0, 0] = n * n
    np.testing.assert_allclose(X, ref, atol=1e-9)
    # the inverse carries 1/n^2
    np.testing.assert_allclose(oracle.ifft2(X), np.ones((n, n)), atol=1e-12)


@pytest.mark.parametrize("n", [16, 64])
def test_parseval_and_inverse(n):
    rng = np.random.default_rng([2, n])
    x = _rand_c(rng, (n, n))
    X = oracle.fft2(x)
    assert math.isclose(np.sum(np.abs(X) ** 2), n * n * np.sum(np.abs(x) ** 2), rel_tol=1e-12)
    np.testing.assert_allclose(oracle.ifft2(X), x, atol=1e-12)


# ------------------------------------------------------------- modulus

def test_modulus_projection_properties():
    rng = np.random.default_rng(3)
    Psi = _rand_c(rng, (16, 16))
    Psi[3, 4] = 0
    a = rng.random((16, 16)) * 5
    P1 = oracle.modulus_replace(Psi, a)
    nz = Psi != 0
    np.testing.assert_allclose(np.abs(P1[nz]), a[nz], rtol=1e-14)          # modulus imposed
    np.testing.assert_allclose(np.angle(P1[nz & (a > 0)]), np.angle(Psi[nz & (a > 0)]), atol=1e-12)
    assert P1[3, 4] == 0                                                       # sgn 0 = 0
    np.testing.assert_allclose(oracle.modulus_replace(P1, a), P1, atol=1e-14)  # idempotent


# ------------------------------------------------------------- one update

def test_hand_worked_n2_examples():
    with open(os.path.join(GOLD, "epie_n2_worked.json")) as f:
        gold = json.load(f)
    for c in gold["cases"]:
        P = np.array(c["probe_re"], float) + 1j * np.array(c["probe_im"], float)
        W = np.array(c["win_re"], float) + 1j * np.array(c["win_im"], float)
        I = np.array(c["intensity"], float)
        new_win, d, err = oracle.position_update(P, W, np.sqrt(I), alpha=1.0)
        np.testing.assert_allclose(new_win, np.array(c["new_win_re"]) + 1j * np.array(c["new_win_im"]), atol=1e-14)
        np.testing.assert_allclose(P + d, np.array(c["new_probe_re"]) + 1j * np.array(c["new_probe_im"]), atol=1e-14)
        assert math.isclose(err, c["err"], abs_tol=1e-12)
        # and through a full sequential sweep of one position
        O = np.ones((3, 3), complex) * 7
        O[1:3, 0:2] = W
        O2, P2, num, den = oracle.sweep_strict(O, P, np.array([[1, 0]]), I[None], [0])
        np.testing.assert_allclose(O2[1:3, 0:2], new_win, atol=1e-14)
        assert np.all(O2[0, :] == 7) and np.all(O2[:, 2] == 7)
        np.testing.assert_allclose(P2, P + d, atol=1e-14)
        assert math.isclose(den, c["sum_i"])


def test_error_reduction_special_case():
    """A constant probe c with beta = 0 turns the object step into the
    Gerchberg-Saxton / error-reduction projection: the new window w' obeys
    |F(c w')| = sqrt(I) with the phase of F(c w)."""
    n = 16
    rng = np.random.default_rng(4)
    c = 0.7 * np.exp(0.3j)
    W = _rand_c(rng, (n, n))
    I = rng.random((n, n)) * 10
    P = np.full((n, n), c)
    new_win, _, _ = oracle.position_update(P, W, np.sqrt(I), alpha=1.0)
    F_new = np.fft.fft2(c * new_win)
    F_old = np.fft.fft2(c * W)
    np.testing.assert_allclose(np.abs(F_new), np.sqrt(I), rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(F_new / np.abs(F_new), F_old / np.abs(F_old), atol=1e-10)


def test_probe_mirror_special_case():
    """A window of ones (any alpha) makes the probe step the error-reduction
    projection of the probe: |F P'| = sqrt(I) with the phase of F P."""
    n = 16
    rng = np.random.default_rng(5)
    P = _rand_c(rng, (n, n))
    I = rng.random((n, n)) * 10
    _, d, _ = oracle.position_update(P, np.ones((n, n), complex), np.sqrt(I), alpha=0.0)
    P2 = P + d
    np.testing.assert_allclose(np.abs(np.fft.fft2(P2)), np.sqrt(I), rtol=1e-10, atol=1e-10)
    FP = np.fft.fft2(P)
    np.testing.assert_allclose(np.fft.fft2(P2) / np.abs(np.fft.fft2(P2)), FP / np.abs(FP), atol=1e-10)


def test_step_sizes_scale_linearly():
    """alpha and beta enter linearly: half the strength gives half the step."""
    n = 8
    rng = np.random.default_rng(6)
    P = _rand_c(rng, (n, n))
    W = _rand_c(rng, (n, n))
    a = rng.random((n, n)) * 3
    w1, d, _ = oracle.position_update(P, W, a, alpha=1.0)
    w2, d2, _ = oracle.position_update(P, W, a, alpha=0.5)
    np.testing.assert_allclose(w2 - W, 0.5 * (w1 - W), atol=1e-13)
    np.testing.assert_allclose(d, d2, atol=0)


# ------------------------------------------------------------- whole sweep

def _tiny_problem(noise, dtype=np.float64, seed=11, side=6, n=16, step=4, m=48):
    pos = sim.raster_positions(side, step, n, m, 1, seed)
    return sim.make_workload(n, m, 4.0, 0.05, pos, 1e6, seed, noise=noise, dtype=dtype)


def test_fixed_point():
    """Noise-free data from the truth and a start at the truth: a sweep
    leaves object and probe unchanged (FP64 rounding only)."""
    wl = _tiny_problem(noise=False)
    order = np.arange(wl.count)[::-1]
    O, P, num, den = oracle.sweep_strict(wl.object_true, wl.probe_true, wl.positions, wl.intensities, order)
    mask = oracle.union_mask(wl.positions, wl.n, wl.h, wl.w)
    assert oracle.rel_l2(O, wl.object_true, mask) < 1e-13
    assert oracle.rel_l2(P, wl.probe_true) < 1e-13
    assert num / den < 1e-24
    off = np.arange(wl.count + 1)
    O2, P2, _, _ = oracle.sweep_coloured(wl.object_true, wl.probe_true, wl.positions, wl.intensities,
                                         np.arange(wl.count), off)
    assert oracle.rel_l2(O2, wl.object_true, mask) < 1e-13
    assert oracle.rel_l2(P2, wl.probe_true) < 1e-13


def test_fixed_point_breaks_when_perturbed():
    """The fixed point is not trivially satisfied: a perturbed start moves."""
    wl = _tiny_problem(noise=False)
    O0 = wl.object_true * np.exp(0.05j)
    O, P, num, den = oracle.sweep_strict(O0, wl.probe_true * 1.1, wl.positions, wl.intensities, np.arange(wl.count))
    assert num / den > 1e-4
    assert oracle.rel_l2(P, wl.probe_true * 1.1) > 1e-3


def test_untouched_pixels_keep_initial_value():
    wl = _tiny_problem(noise=True)
    O, P, _, _ = oracle.sweep_strict(wl.object0, wl.probe0, wl.positions, wl.intensities, np.arange(wl.count))
    mask = oracle.union_mask(wl.positions, wl.n, wl.h, wl.w)
    assert np.array_equal(O[~mask], wl.object0[~mask])
    assert not np.allclose(O[mask], wl.object0[mask])


def test_batches_of_one_equal_sequential():
    wl = _tiny_problem(noise=True)
    order = sim.sweep_order(wl.seed, 0, wl.count)
    Os, Ps, ns, ds = oracle.sweep_strict(wl.object0, wl.probe0, wl.positions, wl.intensities, order)
    Oc, Pc, nc, dc = oracle.sweep_coloured(wl.object0, wl.probe0, wl.positions, wl.intensities, order,
                                           np.arange(wl.count + 1))
    np.testing.assert_allclose(Oc, Os, rtol=0, atol=1e-14)
    np.testing.assert_allclose(Pc, Ps, rtol=0, atol=1e-12 * np.abs(Ps).max())
    assert math.isclose(nc, ns, rel_tol=1e-12) and math.isclose(dc, ds, rel_tol=1e-12)


def test_batch_members_commute():
    """Reordering positions inside a disjoint batch leaves the object
    unchanged and the probe equal up to summation order."""
    n = 16
    wl = _tiny_problem(noise=True, side=8, step=8, m=96)
    cols = oracle.greedy_colouring(wl.positions, n)
    order = np.argsort(cols, kind="stable")
    off = np.searchsorted(cols[order], np.arange(cols.max() + 2))
    assert max(np.diff(off)) > 4
    O1, P1, _, _ = oracle.sweep_coloured(wl.object0, wl.probe0, wl.positions, wl.intensities, order, off)
    rng = np.random.default_rng(8)
    order2 = order.copy()
    for b in range(len(off) - 1):
        seg = order2[off[b]:off[b + 1]]
        order2[off[b]:off[b + 1]] = rng.permutation(seg)
    O2, P2, _, _ = oracle.sweep_coloured(wl.object0, wl.probe0, wl.positions, wl.intensities, order2, off)
    # over a whole sweep the probe sums differ in rounding only ...
    np.testing.assert_allclose(O2, O1, rtol=0, atol=1e-13)
    np.testing.assert_allclose(P2, P1, rtol=0, atol=1e-13 * np.abs(P1).max())
    # ... and within one batch the object steps are bit-identical
    b = int(np.argmax(np.diff(off)))
    O3, _, _, _ = oracle.sweep_coloured(wl.object0, wl.probe0, wl.positions, wl.intensities,
                                        order[off[b]:off[b + 1]], [0, off[b + 1] - off[b]])
    O4, _, _, _ = oracle.sweep_coloured(wl.object0, wl.probe0, wl.positions, wl.intensities,
                                        order2[off[b]:off[b + 1]], [0, off[b + 1] - off[b]])
    np.testing.assert_array_equal(O3, O4)


def test_coloured_probe_step_is_batch_mean():
    """With alpha = 0 the object is frozen, so the probe after one batch is
    P + beta * mean of each member's single-position increment."""
    wl = _tiny_problem(noise=True, side=8, step=8, m=96)
    n = wl.n
    idx = np.array([0, 3, 6])
    assert all(not oracle.windows_overlap(wl.positions[a], wl.positions[b], n) for a in idx for b in idx if a != b)
    sq = np.sqrt(wl.intensities.astype(np.float64))
    incs = []
    for j in idx:
        y, x = wl.positions[j]
        _, d, _ = oracle.position_update(wl.probe0, wl.object0[y:y + n, x:x + n], sq[j], alpha=0.0)
        incs.append(d)
    _, P, _, _ = oracle.sweep_coloured(wl.object0, wl.probe0, wl.positions, wl.intensities, idx, [0, 3], alpha=0.0,
                                       beta=0.6)
    np.testing.assert_allclose(P, wl.probe0 + 0.6 * np.mean(incs, axis=0), atol=1e-12)


def test_restart_equals_uninterrupted():
    wl = _tiny_problem(noise=True)
    orders = [sim.sweep_order(wl.seed, s, wl.count) for s in range(4)]
    O, P, e_all = oracle.reconstruct(wl.object0, wl.probe0, wl.positions, wl.intensities, [(o, None) for o in orders])
    O1, P1, e1 = oracle.reconstruct(wl.object0, wl.probe0, wl.positions, wl.intensities,
                                    [(o, None) for o in orders[:2]])
    O2, P2, e2 = oracle.reconstruct(O1.copy(), P1.copy(), wl.positions, wl.intensities, [(o, None) for o in orders[2:]])
    np.testing.assert_array_equal(O, O2)
    np.testing.assert_array_equal(P, P2)
    assert e_all == e1 + e2


@pytest.mark.parametrize("noise", [False, True])
def test_error_descends_config0(noise):
    """Sequential ePIE on the small configuration (32 px patterns, 10x10
    raster, 10 sweeps): the running Fourier error falls by more than half
    and never blows up."""
    wl = sim.make_config(0, noise=noise, dtype=np.float64 if not noise else np.float32)
    orders = [(sim.sweep_order(wl.seed, s, wl.count), None) for s in range(10)]
    _, _, errs = oracle.reconstruct(wl.object0, wl.probe0, wl.positions, wl.intensities, orders)
    assert errs[-1] < 0.5 * errs[0], errs
    assert max(errs) <= errs[0] * 1.05
    assert all(np.isfinite(errs))


def test_error_descends_coloured_128():
    """Coloured batches at 128 px patterns (first 400 raster positions of the
    60x60 scan): the error falls as well."""
    wl = sim.make_config(1, n_positions=400)
    cols = oracle.greedy_colouring(wl.positions, wl.n)
    base = np.argsort(cols, kind="stable")
    off = np.searchsorted(cols[base], np.arange(cols.max() + 2))
    scheds = []
    for s in range(6):
        perm = np.random.default_rng([wl.seed, 7, s]).permutation(len(off) - 1)
        order = np.concatenate([base[off[b]:off[b + 1]] for b in perm])
        o2 = np.concatenate([[0], np.cumsum([off[b + 1] - off[b] for b in perm])])
        scheds.append((order, o2))
    _, _, errs = oracle.reconstruct(wl.object0, wl.probe0, wl.positions, wl.intensities, scheds)
    assert errs[-1] < 0.5 * errs[0], errs


# ------------------------------------------------------------- schedules

def test_overlap_rule_and_checker():
    n = 10
    assert oracle.windows_overlap((0, 0), (9, 9), n)
    assert not oracle.windows_overlap((0, 0), (10, 0), n)
    assert not oracle.windows_overlap((0, 0), (3, -10), n)
    pos = np.array([[0, 0], [5, 5], [10, 0], [0, 10]])
    oracle.check_schedule(pos, n, [0, 2, 3, 1], [0, 3, 4])
    with pytest.raises(ValueError):
        oracle.check_schedule(pos, n, [0, 1, 2, 3], [0, 2, 4])
    with pytest.raises(ValueError):
        oracle.check_schedule(pos, n, [0, 1, 2, 4], [0, 1, 4])
    with pytest.raises(ValueError):
        oracle.check_schedule(pos, n, [0, 1], [0, 1, 3])


def test_greedy_colouring_known_answers():
    n = 8
    # a row of windows spaced n/2 apart: neighbours overlap, next-but-one do not
    row = np.array([[0, 4 * k] for k in range(9)])
    assert list(oracle.greedy_colouring(row, n)) == [0, 1] * 4 + [0]
    # a k x k block of mutually overlapping windows needs k^2 colours
    blk = np.array([[i, j] for i in range(3) for j in range(3)])
    assert sorted(oracle.greedy_colouring(blk, n)) == list(range(9))
    # the cap splits a colour
    far = np.array([[0, 10 * k] for k in range(5)])
    assert list(oracle.greedy_colouring(far, n, max_batch=2)) == [0, 0, 1, 1, 2]


# ------------------------------------------------------------- gradient

def _fd_problem():
    wl = sim.make_workload(32, 64, 10.0, 0.05, sim.raster_positions(4, 8, 32, 64, 1, 21)[:10], 1e6, 21,
                           noise=True, dtype=np.float64)
    rng = np.random.default_rng(22)
    O = wl.object_true * np.exp(0.2j * rng.standard_normal(wl.object_true.shape))
    P = wl.probe0 + 0.1 * _rand_c(rng, wl.probe0.shape) * np.abs(wl.probe0).max()
    return wl, O, P


def test_gradient_matches_central_differences():
    wl, O, P = _fd_problem()
    L, gO, gP = oracle.amplitude_loss_grad(O, P, wl.positions, wl.intensities)
    rng = np.random.default_rng(23)
    for _ in range(3):
        VO = _rand_c(rng, O.shape)
        VP = _rand_c(rng, P.shape)
        for which in ("O", "P"):
            h = 1e-6 if which == "O" else 1e-6 * np.abs(P).max()
            if which == "O":
                fp = oracle.amplitude_loss(O + h * VO, P, wl.positions, wl.intensities)
                fm = oracle.amplitude_loss(O - h * VO, P, wl.positions, wl.intensities)
                ana = np.real(np.vdot(gO, VO))
            else:
                fp = oracle.amplitude_loss(O, P + h * VP, wl.positions, wl.intensities)
                fm = oracle.amplitude_loss(O, P - h * VP, wl.positions, wl.intensities)
                ana = np.real(np.vdot(gP, VP))
            fd = (fp - fm) / (2 * h)
            assert math.isclose(fd, ana, rel_tol=2e-5), (which, fd, ana)
    assert math.isclose(L, oracle.amplitude_loss(O, P, wl.positions, wl.intensities), rel_tol=1e-14)


def test_epie_object_step_is_scaled_gradient():
    """For one position the ePIE object step equals -alpha / (2 N^2 max|P|^2)
    times the amplitude-loss gradient: ties the two oracle functions."""
    wl, O, P = _fd_problem()
    j = 3
    y, x = wl.positions[j]
    n = wl.n
    win = O[y:y + n, x:x + n]
    new_win, _, _ = oracle.position_update(P, win, np.sqrt(wl.intensities[j]), alpha=0.8)
    _, gO, gP = oracle.amplitude_loss_grad(O, P, wl.positions, wl.intensities, idx=[j])
    scale = -0.8 / (2 * n * n * np.max(np.abs(P) ** 2))
    np.testing.assert_allclose(new_win - win, scale * gO[y:y + n, x:x + n], atol=1e-12 * np.abs(win).max())
    # and the probe step likewise with max|window|^2
    _, d, _ = oracle.position_update(P, win, np.sqrt(wl.intensities[j]), alpha=0.8)
    np.testing.assert_allclose(d, -gP / (2 * n * n * np.max(np.abs(win) ** 2)), atol=1e-9 * np.abs(d).max())


def test_strict_sweep_beta_and_alpha():
    """beta scales the probe step and alpha the object step in a sequential
    sweep; beta = 0 keeps the probe, alpha = 0 keeps the object."""
    wl = _tiny_problem(noise=True)
    n = wl.n
    j = 5
    y, x = wl.positions[j]
    sq = np.sqrt(wl.intensities[j].astype(np.float64))
    win = wl.object0[y:y + n, x:x + n]
    new_win, d, _ = oracle.position_update(wl.probe0, win, sq, alpha=0.7)
    O, P, _, _ = oracle.sweep_strict(wl.object0, wl.probe0, wl.positions, wl.intensities, [j], alpha=0.7, beta=0.3)
    np.testing.assert_allclose(P, wl.probe0 + 0.3 * d, atol=1e-12)
    np.testing.assert_allclose(O[y:y + n, x:x + n], new_win, atol=1e-14)
    _, P0, _, _ = oracle.sweep_strict(wl.object0, wl.probe0, wl.positions, wl.intensities, [0, 1, 2], beta=0.0)
    np.testing.assert_array_equal(P0, wl.probe0)
    O0, _, _, _ = oracle.sweep_strict(wl.object0, wl.probe0, wl.positions, wl.intensities, [0, 1, 2], alpha=0.0)
    np.testing.assert_array_equal(O0, wl.object0)


def test_coloured_sweep_alpha_scales_the_object_step():
    """In a coloured batch with beta = 0 the object step is linear in alpha
    (each window's step depends only on its own pre-update values and the
    batch's probe): alpha = 0 keeps the object, and the step at alpha = 0.4
    is 0.4 times the step at alpha = 1."""
    wl = _tiny_problem(noise=True)
    idx = []
    for j in range(wl.count):
        if all(not oracle.windows_overlap(wl.positions[j], wl.positions[k], wl.n) for k in idx):
            idx.append(j)
    assert len(idx) >= 2
    off = [0, len(idx)]
    O0, P0 = wl.object0, wl.probe0
    O1, P1, _, _ = oracle.sweep_coloured(O0, P0, wl.positions, wl.intensities, idx, off, alpha=1.0, beta=0.0)
    Oa, Pa, _, _ = oracle.sweep_coloured(O0, P0, wl.positions, wl.intensities, idx, off, alpha=0.4, beta=0.0)
    Oz, _, _, _ = oracle.sweep_coloured(O0, P0, wl.positions, wl.intensities, idx, off, alpha=0.0, beta=0.0)
    np.testing.assert_array_equal(Oz, O0)
    np.testing.assert_array_equal(P1, P0)
    step1 = O1 - O0
    assert np.max(np.abs(step1)) > 1e-3
    np.testing.assert_allclose(Oa - O0, 0.4 * step1, rtol=0, atol=1e-13 * np.max(np.abs(step1)) + 1e-15)


# ------------------------------------------------------------- subset-parallel scheme

def test_parallel_one_subset_is_plain_reconstruction():
    wl = _tiny_problem(noise=True)
    sched = [(sim.sweep_order(wl.seed, s, wl.count), None) for s in range(2)]
    O1, P1, _ = oracle.reconstruct(wl.object0, wl.probe0, wl.positions, wl.intensities, sched)
    O2, P2, _ = oracle.subset_round(wl.object0, wl.probe0, wl.positions, wl.intensities,
                                    [np.arange(wl.count)], [sched])
    np.testing.assert_array_equal(O1, O2)
    np.testing.assert_array_equal(P1, P2)


def test_parallel_separated_subsets_move_by_one_over_k():
    """beta = 0 and subsets whose windows never meet: each subset's region
    moves by exactly 1/K of what that subset alone does to it."""
    n = 16
    left = sim.raster_positions(3, 4, n, 40, 0, 1)                 # corners within [12, 20]
    right = left + np.array([0, 60], dtype=np.int32)
    pos = np.concatenate([left, right])
    wl = sim.make_workload(n, 48, 4.0, 0.05, pos, 1e6, 13, noise=True, h=48, w=110)
    subsets = [np.arange(9), np.arange(9, 18)]
    sched = [[(np.arange(9)[::-1], None)], [(np.arange(9), None)]]
    O, P, _ = oracle.subset_round(wl.object0, wl.probe0, wl.positions, wl.intensities, subsets, sched, beta=0.0)
    np.testing.assert_array_equal(P, wl.probe0)
    for sub, sc in zip(subsets, sched):
        Ok, _, _ = oracle.reconstruct(wl.object0, wl.probe0, wl.positions[sub], wl.intensities[sub], sc, beta=0.0)
        m = oracle.union_mask(wl.positions[sub], n, wl.h, wl.w)
        np.testing.assert_allclose(O[m], wl.object0[m] + (Ok[m] - wl.object0[m]) / 2, atol=1e-14)


def test_parallel_identical_subsets_average_to_one_run():
    wl = _tiny_problem(noise=True)
    sched = [(sim.sweep_order(wl.seed, 0, wl.count), None)]
    O1, P1, _ = oracle.reconstruct(wl.object0, wl.probe0, wl.positions, wl.intensities, sched)
    sub = np.arange(wl.count)
    O3, P3, _ = oracle.subset_round(wl.object0, wl.probe0, wl.positions, wl.intensities, [sub] * 4, [sched] * 4)
    np.testing.assert_allclose(O3, O1, rtol=0, atol=1e-15)
    np.testing.assert_allclose(P3, P1, rtol=0, atol=1e-13 * np.abs(P1).max())


def test_round_robin_split():
    subs = oracle.round_robin(10, 4)
    assert [list(s) for s in subs] == [[0, 4, 8], [1, 5, 9], [2, 6], [3, 7]]


# ------------------------------------------------------------- preprocessing and masks

@pytest.mark.parametrize("orient,expect", [
    (0, (3, 5)), (1, (5, 3)), (2, (4, 5)), (4, (3, 2)), (3, (2, 3)), (7, (2, 4)),
])
def test_preprocess_moves_a_single_pixel_where_stated(orient, expect):
    """A bright pixel at crop position (3, 5) of an 8 x 8 crop lands where
    transpose-then-flip-rows-then-flip-columns puts it (worked by hand)."""
    frame = np.zeros((1, 20, 30))
    frame[0, 6 + 3, 11 + 5] = 9.0
    I, _ = oracle.preprocess(frame, 8, crop=(6, 11), orient=orient, scale=2.0)
    assert I.shape == (1, 8, 8)
    assert np.argwhere(I[0] == 18.0).tolist() == [list(expect)]
    assert I.sum() == 18.0


def test_preprocess_centred_moves_dc_to_origin():
    frame = np.zeros((1, 8, 8))
    frame[0, 4, 4] = 1.0
    I, _ = oracle.preprocess(frame, 8, centred=True)
    assert I[0, 0, 0] == 1.0


def test_orientations_are_the_eight_symmetries():
    a = np.arange(16.0).reshape(4, 4)
    outs = {oracle.orient_crop(a, o, False).tobytes() for o in range(8)}
    assert len(outs) == 8
    np.testing.assert_array_equal(oracle.orient_crop(oracle.orient_crop(a, 1, False), 1, False), a)


def test_mask_follows_the_data_and_zeroes_masked_pixels():
    rng = np.random.default_rng(12)
    frames = rng.random((2, 12, 12)) + 1
    mask = np.ones((12, 12), bool)
    mask[4, 7] = False
    I, m = oracle.preprocess(frames, 8, crop=(2, 3), orient=5, centred=True, mask=mask)
    J, _ = oracle.preprocess(frames, 8, crop=(2, 3), orient=5, centred=True)
    assert (~m).sum() == 1
    assert np.all(I[:, ~m] == 0) and np.all(I[:, m] == J[:, m])
    marker = np.zeros((1, 12, 12))
    marker[0, 4, 7] = 1
    K, _ = oracle.preprocess(marker, 8, crop=(2, 3), orient=5, centred=True)
    assert np.array_equal(K[0] == 1, ~m)


def test_masked_modulus_projection():
    rng = np.random.default_rng(13)
    Psi = _rand_c(rng, (8, 8))
    a = rng.random((8, 8)) + 0.5
    m = rng.random((8, 8)) > 0.3
    out = oracle.modulus_replace(Psi, a, m)
    np.testing.assert_allclose(np.abs(out[m]), a[m], rtol=1e-14)
    np.testing.assert_array_equal(out[~m], Psi[~m])


def test_full_mask_is_no_mask_and_empty_mask_changes_nothing():
    wl = _tiny_problem(noise=True)
    order = sim.sweep_order(wl.seed, 0, wl.count)
    ones = np.ones((wl.n, wl.n), bool)
    O1, P1, n1, _ = oracle.sweep_strict(wl.object0, wl.probe0, wl.positions, wl.intensities, order)
    O2, P2, n2, _ = oracle.sweep_strict(wl.object0, wl.probe0, wl.positions, wl.intensities, order, mask=ones)
    np.testing.assert_array_equal(O1, O2)
    np.testing.assert_array_equal(P1, P2)
    O3, P3, n3, _ = oracle.sweep_strict(wl.object0, wl.probe0, wl.positions, wl.intensities, order, mask=~ones)
    np.testing.assert_allclose(O3, wl.object0, atol=1e-12)
    np.testing.assert_allclose(P3, wl.probe0, atol=1e-12 * np.abs(wl.probe0).max())
    assert n3 == 0.0
