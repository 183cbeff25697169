"""Host-side checks of bench.py (no GPU): its one-GPU contract, the
workloads it times, and that the committed HBM-traffic summary was taken on
the current kernel, layout and planner sources (bench.py reports
roofline.traffic only then)."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import workloads as W  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_headline_workload():
    """M = 32 complex64, L = 1000, 1..3 controls, 500 targets in bits 0..7
    and 500 in bits 8..31."""
    wl = bench.workload("m32")
    assert (wl["M"], wl["dtype"], wl["name"]) == (32, "c64", "m32_c64_L1000")
    tg, cm = wl["target"], wl["cmask"]
    assert len(tg) == 1000
    assert int((tg < 8).sum()) == 500 and int((tg >= 8).sum()) == 500 and int(tg.max()) < 32
    n_ctl = np.array([bin(int(c)).count("1") for c in cm])
    assert n_ctl.min() == 1 and n_ctl.max() == 3
    assert all(not (int(c) >> int(t)) & 1 for t, c in zip(tg, cm))
    again = bench.workload("m32")
    assert np.array_equal(again["target"], tg) and np.array_equal(again["cmask"], cm)


def test_served_and_batched_configurations():
    assert W.SERVED_REQUESTS == 1000 and W.SERVED_RATE == 122.0
    trace = W.served_trace(200, W.SERVED_RATE)
    ms = np.array([r.circuit.M for r in trace])
    assert ms.min() >= 12 and ms.max() <= 28
    arr = np.array([r.arrival_s for r in trace])
    assert np.all(np.diff(arr) > 0)
    # the circuits do not depend on the rate (only the arrival times do)
    other = W.served_trace(200, 2 * W.SERVED_RATE)
    assert all(a.circuit.M == b.circuit.M and np.array_equal(a.circuit.target, b.circuit.target)
               for a, b in zip(trace, other))
    circuits = W.batched_config()
    assert len(circuits) == 4096
    assert min(c.M for c in circuits) == 8 and max(c.M for c in circuits) == 20
    assert min(c.L for c in circuits) >= 10 and max(c.L for c in circuits) <= 500


def test_committed_traffic_summary_matches_the_sources():
    """profiles/k_tile_m32_c64_L1000_pmc.md records the hash of the sources
    that decide HBM traffic; a change to them needs a new counter run."""
    got = bench.stored_traffic("m32_c64_L1000")
    assert got is not None, f"counter summary taken on other sources than {bench.kernel_hash()}"
    algorithmic = 2 * (1 << 32) * 8
    assert 0.99 * algorithmic < got < 1.05 * algorithmic
