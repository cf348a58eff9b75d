"""Host-side logic of bench.py: the roofline arithmetic of the dominant
kernel, the lookup of committed HBM-counter summaries by kernel source
hash, and the refusal of more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


class _WL:
    n = 128


def test_roofline_of_the_dominant_kernel():
    # 100 launches of the inverse stage updating 30 positions each in 1 ms in
    # total; the other kernels took less time
    r = {"wl": _WL(), "kernels": {"k_rows_fwd": (0.5, 100, 3000), "k_cols": (0.6, 100, 3000),
                                  "k_rows_inv": (1.0, 100, 3000)}}
    rf = bench.roofline_of(r)
    per_launch = 16 * 128 * 128 * 30
    assert rf["kernel"] == "k_rows_inv<128>"
    assert rf["algorithmic_bytes_per_launch"] == per_launch
    assert rf["avg_launch_us"] == pytest.approx(10.0)
    assert rf["achieved"] == pytest.approx(per_launch / 10e-6 / 1e9, rel=1e-4)
    assert rf["frac"] == pytest.approx(rf["achieved"] / bench.HBM_PEAK_GBS, rel=1e-3)
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    # every stage is reported too, each against its own algorithmic bytes
    st = {e["kernel"]: e for e in rf["stages"]}
    assert set(st) == {"k_rows_fwd<128>", "k_cols<128>", "k_rows_inv<128>"}
    assert st["k_cols<128>"]["algorithmic_bytes_per_launch"] == 4 * 128 * 128 * 30
    assert st["k_cols<128>"]["avg_launch_us"] == pytest.approx(6.0)
    assert st["k_rows_inv<128>"]["frac"] == rf["frac"]


def test_traffic_lookup_needs_the_current_kernel_source(monkeypatch):
    h = bench.kernel_source_hash()
    assert len(h) == 16
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0000000000000000")
    assert bench.load_traffic("k_rows_inv", 128) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_cpu_baseline_batches_compute_the_oracle_sweep():
    """The CPU baseline hands each oracle call only its batch's positions and
    patterns; a sweep of such calls equals the oracle's own coloured sweep
    over the whole workload, bit for bit."""
    import numpy as np

    import oracle
    import sim
    from paper_2308_10674_amd import colour

    wl = sim.make_config(0)
    col, nc = colour(wl.positions, wl.n)
    order = np.argsort(col, kind="stable")
    off = np.concatenate([[0], np.cumsum(np.bincount(col))])
    O_ref, P_ref, _, _ = oracle.sweep_coloured(wl.object0, wl.probe0, wl.positions, wl.intensities, order, off)
    O, P = wl.object0, wl.probe0
    for b in range(nc):
        O, P = bench._oracle_batch(oracle, O, P, wl, order[off[b]:off[b + 1]])
    np.testing.assert_array_equal(O, O_ref)
    np.testing.assert_array_equal(P, P_ref)
