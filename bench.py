#!/usr/bin/env python3
"""Benchmark of the fused wiring-diagram path on one MI355X.

Workload (default): M = 32 address bits, complex64 entries (32 GiB per
buffer), a unit-norm Gaussian state generated on the device from a fixed
seed, and a wiring diagram of L = 1000 controlled-NOT steps with 1..3
controls (500 steps target bits 0..7, 500 target bits 8..31).  One "step" of
the benchmark applies the whole diagram to the state once (qsim_apply_steps:
validation, planning, upload and every pass).

Printed: one JSON line with the amplitude-step update rate (2^M * L per
applied diagram), the roofline of the dominant kernel (the fused tile pass,
HBM-bound) measured with HIP events over the timed region, and the CPU
oracle timed on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--workload m32|m26|small]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0   # MI355X published HBM3E bandwidth
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SRC = os.path.join(ROOT, "paper_quant_ph_0308158_amd", "csrc", "kernels.hip")


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def workload(name: str):
    import workloads as W
    if name == "m32":
        tg, cm = W.m32_config()
        return dict(name="m32_c64_L1000", M=32, dtype="c64", seed=W.SEED_M32, target=tg, cmask=cm,
                    desc=dict(controls="1-3", targets="500 in bits 0-7, 500 in bits 8-31",
                              input="unit-norm complex Gaussian"))
    if name == "m26":
        tg, cm = W.m26_config()
        return dict(name="m26_c128_L200", M=26, dtype="c128", seed=W.SEED_M26, target=tg, cmask=cm,
                    desc=dict(controls="0-4", targets="uniform over 26 bits",
                              input="unit-norm complex Gaussian"))
    if name == "small":
        tg, cm = W.small_config()
        return dict(name="m10_c128_L20", M=10, dtype="c128", seed=W.SEED_SMALL, target=tg, cmask=cm,
                    desc=dict(controls="1", targets="uniform", input="unit-norm complex Gaussian"))
    raise ValueError(name)


def stored_traffic(wl_name: str):
    """HBM bytes per tile-pass launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source."""
    path = os.path.join(PROFILES, f"k_tile_{wl_name}_pmc.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"^traffic_json:\s*(\{.*\})\s*$", text, flags=re.M)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("kernel_sha") != kernel_hash():
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(wl, k1_host, seconds: float):
    """The oracle's plain pair-swap loop on the host cores, on the first n
    steps of the same diagram over the same 2^M-entry input, n chosen so the
    sample takes about `seconds`."""
    import numpy as np
    import oracle
    M, tg, cm = wl["M"], wl["target"], wl["cmask"]
    threads = int(os.environ.get("QSIM_ORACLE_THREADS", min(os.cpu_count() or 1, 16)))
    buf = k1_host
    t0 = time.perf_counter()
    oracle.apply_inplace(M, buf, tg[:1], cm[:1], threads=threads)
    t1 = time.perf_counter() - t0
    n = int(max(1, min(len(tg) - 1, seconds / max(t1, 1e-6))))
    t0 = time.perf_counter()
    oracle.apply_inplace(M, buf, tg[1:1 + n], cm[1:1 + n], threads=threads)
    dt = time.perf_counter() - t0
    return {"value": float((1 << M) * n / dt), "unit": "amplitude-step updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"steps 2..{n + 1} of the same {len(tg)}-step diagram on the full 2^{M}-entry "
                      f"input (plain pair-swap loop, OpenMP over rows, {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="m32", choices=["m32", "m26", "small"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tuning", default=None, help="JSON dict of qsim_tuning fields")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(how it would shard is described in DESIGN.md).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_quant_ph_0308158_amd import qsim

    torch.cuda.set_device(0)
    wl = workload(args.workload)
    M, dt = wl["M"], wl["dtype"]
    tg, cm = wl["target"], wl["cmask"]
    L = len(tg)

    k1 = W.gaussian_state_torch(M, dt, seed=wl["seed"])
    other = torch.empty_like(k1)
    torch.cuda.synchronize()
    st = qsim.State(M, dt, buffers=(k1, other))
    if args.tuning:
        st.set_tuning(json.loads(args.tuning))
    tuning = json.loads(args.tuning) if args.tuning else None
    masks, lens, _ = qsim.plan_describe(M, dt, tg, cm, tuning)

    for _ in range(args.warmup):
        st.apply(tg, cm)
    torch.cuda.synchronize()

    st.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st.apply(tg, cm)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = st.profile_read()
    st.profile(False)

    updates = float(1 << M) * L * args.steps
    value = updates / elapsed
    ms_per_step = elapsed / args.steps * 1e3

    roofline = None
    if prof["tile_launches"]:
        per_launch_bytes = prof["tile_bytes"] / prof["tile_launches"]
        avg_ms = prof["tile_ms"] / prof["tile_launches"]
        achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": stored_traffic(wl["name"]),
                    "kernel": "k_tile", "algorithmic_bytes_per_launch": int(per_launch_bytes),
                    "avg_launch_ms": round(avg_ms, 4), "launches": int(prof["tile_launches"])}
    elif prof["other_launches"]:
        per_launch_bytes = 2.0 * (1 << M) * (8 if dt == "c64" else 16)
        avg_ms = prof["other_ms"] / prof["other_launches"]
        achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None, "kernel": "k_small",
                    "algorithmic_bytes_per_launch": int(per_launch_bytes), "avg_launch_ms": round(avg_ms, 4),
                    "launches": int(prof["other_launches"])}

    # Achievable-bandwidth reference: a plain copy between the same buffers.
    nbytes = (1 << M) * (8 if dt == "c64" else 16)
    qsim.copy_bytes(other.data_ptr(), k1.data_ptr(), nbytes)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(3):
        qsim.copy_bytes(other.data_ptr(), k1.data_ptr(), nbytes)
    ev1.record()
    torch.cuda.synchronize()
    copy_gbps = 3 * 2 * nbytes / (ev0.elapsed_time(ev1) * 1e-3) / 1e9

    cpu = None
    if not args.no_cpu_baseline:
        host = k1.cpu().numpy()   # the same input bytes (state after the timed steps)
        del k1, other
        st.close()
        torch.cuda.empty_cache()
        cpu = cpu_baseline(wl, host, args.cpu_seconds)
        del host
    else:
        st.close()

    out = {
        "metric": "amplitude-step updates/s (2^M x L per applied wiring diagram)",
        "value": value,
        "unit": "amplitude-step updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64" if dt == "c64" else "c128",
        "data": "synthetic",
        "config": {"workload": wl["name"], "M": M, "L": L, "passes": int(len(masks)),
                   "tile_bits": int(bin(int(masks[0])).count("1")) if len(masks) else M, **wl["desc"]},
        "roofline": roofline,
        "copy_probe_GBps": round(copy_gbps, 1),
        "cpu_baseline": cpu,
        "profile": {k: (round(v, 3) if isinstance(v, float) else v) for k, v in prof.items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
