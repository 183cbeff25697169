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
# Sources that decide the tile kernel's memory traffic: the kernels, and the
# host code that plans passes and lays out the state between them.
TRAFFIC_SRC = [os.path.join(ROOT, "paper_quant_ph_0308158_amd", "csrc", f)
               for f in ("kernels.hip", "qsim_internal.h", "abi.cpp", "planner.cpp")]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for path in TRAFFIC_SRC:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def workload(name: str):
    import workloads as W
    if name == "m32":
        tg, cm = W.m32_config()
        return dict(name="m32_c64_L1000", M=32, dtype="c64", seed=W.SEED_M32, target=tg, cmask=cm,
                    desc=dict(controls="1-3", targets="500 in bits 0-7, 500 in bits 8-31",
                              input="unit-norm complex Gaussian"))
    if name == "m34":
        tg, cm = W.m32_config(M=34, seed=34)
        return dict(name="m34_c64_L1000", M=34, dtype="c64", seed=34, target=tg, cmask=cm,
                    desc=dict(controls="1-3", targets="500 in bits 0-7, 500 in bits 8-33",
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


def stored_traffic(wl_name: str, kernel: str = "k_tile", alg_bytes=None):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source (and, given
    `alg_bytes`, on a launch with the same algorithmic bytes: batched
    mode's bytes depend on the parameters the autotuner picks)."""
    path = os.path.join(PROFILES, f"{kernel}_{wl_name}_pmc.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"^traffic_json:\s*(\{.*\})\s*$", text, flags=re.M)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("kernel_sha") != kernel_hash():
        return None
    if alg_bytes is not None and d.get("algorithmic_bytes") != int(alg_bytes):
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(wl, k1_host, seconds: float):
    """The oracle's plain pair-swap loop on the host cores, on the first n
    steps of the same diagram over the same 2^M-entry input, n chosen so the
    sample takes about `seconds`."""
    import numpy as np
    import oracle
    M, tg, cm = wl["M"], wl["target"], wl["cmask"]
    threads, why = oracle_threads()
    buf = k1_host
    t0 = time.perf_counter()
    oracle.apply_inplace(M, buf, tg[:1], cm[:1], threads=threads)
    t1 = time.perf_counter() - t0
    n = int(max(1, min(len(tg) - 2, seconds / max(t1, 1e-6))))
    t0 = time.perf_counter()
    oracle.apply_inplace(M, buf, tg[1:1 + n], cm[1:1 + n], threads=threads)
    dt = time.perf_counter() - t0
    # one more step on a single thread
    t0 = time.perf_counter()
    oracle.apply_inplace(M, buf, tg[1 + n:2 + n], cm[1 + n:2 + n], threads=1)
    d1 = time.perf_counter() - t0
    return {"value": float((1 << M) * n / dt), "unit": "amplitude-step updates/s", "cores": threads,
            "kind": "oracle", "cores_why": why, "host_cpus": os.cpu_count(), "model": cpu_model(),
            "sample": f"steps 2..{n + 1} of the same {len(tg)}-step diagram on the full 2^{M}-entry "
                      f"input (plain pair-swap loop, OpenMP over rows, {dt:.1f} s)",
            "single_thread": {"value": float((1 << M) / d1), "cores": 1,
                              "sample": f"step {n + 2} of the same diagram on one thread ({d1:.1f} s)"}}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_threads():
    """Threads for the oracle's OpenMP loop: every CPU this process may run
    on, unless OMP_NUM_THREADS (the share of the host's CPUs a one-GPU job
    is given) or QSIM_ORACLE_THREADS sets fewer."""
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    for var in ("QSIM_ORACLE_THREADS", "OMP_NUM_THREADS"):
        v = os.environ.get(var)
        if v and v.isdigit() and 0 < int(v) < avail:
            return int(v), f"{var}={v} (of {avail} CPUs this process may use)"
    return avail, f"all {avail} CPUs this process may use"


def cpu_configs(reps: int = 3):
    """The oracle on the two configurations small enough to run whole, best
    of `reps`: M=10 complex128 L=20 and M=26 complex128 L=200."""
    import numpy as np
    import oracle
    import workloads as W
    threads, _ = oracle_threads()
    out = {}
    for name, M, (tg, cm), k1 in (
            ("m10_c128_L20", 10, W.small_config(), W.alternating_state(10)),
            ("m26_c128_L200", 26, W.m26_config(), W.gaussian_state_torch(26, "c128", seed=W.SEED_M26).cpu().numpy())):
        best = None
        for _ in range(reps):
            t0 = time.perf_counter()
            oracle.apply(M, k1, tg, cm, threads=threads)
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        out[name] = {"best_of": reps, "ms": round(best * 1e3, 3), "cores": threads,
                     "value": float((1 << M) * len(tg) / best), "unit": "amplitude-step updates/s"}
        del k1
    return out


def bench_batched(reps: int = 3, plain_too: bool = True, autotune: bool = True):
    """The batched configuration: 4096 independent circuits (M uniform in
    8..20, L uniform in 10..500, 0..3 controls, complex64), all states
    resident on the device.  Timed two ways on the same states and
    circuits, each including host planning: plain (one qsim_apply_steps per
    circuit, serially on one stream, over `reps` rounds) and batched (one
    qsim_apply_batch per round, 20 rounds back to back).  The kernel's own
    time per launch comes from qsim_batch_last_info."""
    import torch
    import workloads as W
    from paper_quant_ph_0308158_amd import qsim
    circuits = W.batched_config()
    k1s, spares = W.gaussian_states_grouped_torch([c.M for c in circuits], "c64", seed=W.SEED_BATCHED)
    states = [qsim.State(c.M, "c64", buffers=(k1, sp)) for c, k1, sp in zip(circuits, k1s, spares)]
    steps = [(c.target, c.cmask) for c in circuits]
    packed = [qsim.pack_steps(t, cm) for t, cm in steps]
    batch = qsim.PackedBatch(steps)
    updates = float(sum((1 << c.M) * c.L for c in circuits))
    torch.cuda.synchronize()

    def plain():
        for st, pk in zip(states, packed):
            st.apply_packed(pk)

    def batched():
        qsim.apply_batch_packed(states, batch)

    # the batch autotuner picks the batched-mode parameters (states unchanged)
    tuned, tune_s = None, None
    if autotune:
        t0 = time.perf_counter()
        tuned = qsim.batch_autotune(states, batch)
        tune_s = time.perf_counter() - t0
    out = {"plain": None}
    # batches back to back (20 of them: the host plans each batch while the
    # device runs the one before, so one batch's host time is spread over
    # the run); the plain comparator over `reps` rounds
    for name, fn, k in (("plain", plain, reps), ("batched", batched, 20)):
        if name == "plain" and not plain_too:
            continue
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / k
        out[name] = {"ms": round(dt * 1e3, 3), "updates_per_s": updates / dt}
    # steady state: device time per batch with a batch already in flight, so
    # that every timed batch's host planning overlaps device work (the 20
    # batches above include the first one's host time)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    batched()
    e0.record()
    for _ in range(10):
        batched()
    e1.record()
    torch.cuda.synchronize()
    out["batched"]["steady_ms"] = round(e0.elapsed_time(e1) / 10, 3)
    qsim.batch_status()
    # the kernel's own time, launch by launch (HIP events on its stream)
    infos = []
    for _ in range(reps):
        batched()
        infos.append(qsim.batch_last_info())
    qsim.batch_status()
    info = infos[-1]
    kernel_ms = sum(i["kernel_ms"] for i in infos) / len(infos)
    achieved = info["algorithmic_bytes"] / (kernel_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": "k_batch", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                "traffic": stored_traffic("batched_4096", kernel="k_batch", alg_bytes=info["algorithmic_bytes"]),
                "algorithmic_bytes_per_launch": int(info["algorithmic_bytes"]), "avg_launch_ms": round(kernel_ms, 4),
                "launches": len(infos), "passes": info["passes"], "items": info["items"],
                "workgroups": info["workgroups"]}
    for st in states:
        st.close()
    # a plain copy of a known size in the same process: the reference that
    # scales rocprofv3's byte counters for the batched kernel
    cb = 1 << 31
    a = torch.empty(cb, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    qsim.copy_bytes(b.data_ptr(), a.data_ptr(), cb)
    torch.cuda.synchronize()
    del a, b
    return {"workload": "batched_4096_M8-20_L10-500_c64", "circuits": len(circuits),
            "amplitude_step_updates": updates, "plain": out["plain"], "batched": out["batched"],
            "roofline": roofline, "tuning": info["tuning"],
            "autotune": ({"chosen": {k: tuned[k] for k in qsim.BATCH_TUNING_FIELDS}, "from_cache": tuned["from_cache"],
                          "seconds": round(tune_s, 2), "batch_ms_chosen": round(tuned["best_ms"], 3),
                          "batch_ms_defaults": round(tuned["default_ms"], 3)} if tuned else None),
            "speedup_vs_plain": round(out["plain"]["ms"] / out["batched"]["ms"], 2) if out["plain"] else None}


def bench_rowmap(reps: int, warmup: int):
    """The materialised row array at M = 32, complex64: the row array x of
    the 1000-step headline diagram is built once (qsim_rowmap_build), then
    applied `reps` times (qsim_rowmap_apply: k2(i) = k1(x(i)), one gather).
    Algorithmic bytes per apply: 2^M x (4 B of x + 8 B read + 8 B written);
    the apply's duration comes from HIP events on its stream."""
    import torch
    import workloads as W
    from paper_quant_ph_0308158_amd import qsim
    M = 32
    tg, cm = W.m32_config()
    x = torch.empty(1 << M, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    qsim.rowmap_build(M, tg, cm, x)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    k1 = W.gaussian_state_torch(M, "c64", seed=W.SEED_M32)
    b1 = torch.empty_like(k1)
    st = qsim.State(M, "c64", buffers=(k1, b1))
    for _ in range(warmup):
        st.rowmap_apply(x.data_ptr())
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * reps)]
    t0 = time.perf_counter()
    for r in range(reps):
        ev[2 * r].record(stream)
        st.rowmap_apply(x.data_ptr())
        ev[2 * r + 1].record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    avg_ms = sum(ev[2 * r].elapsed_time(ev[2 * r + 1]) for r in range(reps)) / reps
    alg = float(1 << M) * (4 + 2 * 8)
    st.close()
    # a plain copy of a known size in the same process (scales rocprofv3's
    # byte counters)
    qsim.copy_bytes(b1.data_ptr(), k1.data_ptr(), 8 << M)
    torch.cuda.synchronize()
    del x, k1, b1
    torch.cuda.empty_cache()
    achieved = alg / (avg_ms * 1e-3) / 1e9
    return {"workload": "rowmap_m32_c64_L1000", "build_ms": round(build_ms, 2), "apply_ms": round(avg_ms, 3),
            "wall_ms_per_apply": round(wall * 1e3, 3), "updates_per_s": float(1 << M) * len(tg) / (avg_ms * 1e-3),
            "roofline": {"bound": "hbm", "kernel": "k_gather", "achieved": round(achieved, 1),
                         "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                         "algorithmic_bytes_per_launch": int(alg), "avg_launch_ms": round(avg_ms, 4)}}


def bench_served(n: int, rate: float, slots: int = 4, budget: float = 200e9, calibrate: bool = False):
    """The served configuration: Poisson arrivals of circuit requests (M
    log-uniform over [12, 29) floored, L uniform in 50..2000, 0..3 controls,
    complex64, the alternating input generated on the device), admitted into
    a 200 GB HBM arena.  Each result is read back in 2^20-row portions.
    Latency = arrival to the last portion on the host.  The same trace is
    served with continuous batching (`slots` requests on the device at once)
    and plain first-come-first-served (one at a time).  With calibrate, all
    requests arrive at t = 0 (measures service capacity)."""
    import workloads as W
    from paper_quant_ph_0308158_amd import qsim
    import torch
    trace = W.served_trace(n, rate)
    packed = [qsim.pack_steps(r.circuit.target, r.circuit.cmask) for r in trace]
    updates = float(sum((1 << r.circuit.M) * r.circuit.L for r in trace))
    readback = float(sum((1 << r.circuit.M) * 8 for r in trace))   # bytes of results sent to the host

    def run(fcfs: bool, digest: int = 0, at_once: bool = calibrate, only=None):
        srv = qsim.Server(budget_bytes=int(budget), max_slots=slots, fcfs=fcfs, digest=digest)
        w = srv.submit(12, "c64", [0], [0])   # warm the slot workers
        srv.drain()
        ids = []
        t0 = time.perf_counter()
        for k, (r, pk) in enumerate(zip(trace, packed)):
            if only is not None and k not in only:
                continue
            if not at_once:
                delay = t0 + r.arrival_s - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
            ids.append(srv.submit(r.circuit.M, "c64", pk["target"], pk["control_mask"]))
        srv.drain()
        infos = [srv.info(i) for i in ids]
        srv.close()
        if digest:
            return ids, infos
        if any(x["status"] != 0 for x in infos):
            raise RuntimeError("a served request failed")
        lat = sorted((x["t_done_ns"] - x["t_submit_ns"]) / 1e6 for x in infos)
        span = (max(x["t_done_ns"] for x in infos) - min(x["t_submit_ns"] for x in infos)) / 1e9
        pct = lambda p: lat[min(len(lat) - 1, int(round(p / 100.0 * (len(lat) - 1))))]
        return {"p50_ms": round(pct(50), 2), "p99_ms": round(pct(99), 2), "mean_ms": round(sum(lat) / len(lat), 2),
                "span_s": round(span, 3), "requests_per_s": round(len(infos) / span, 2),
                "updates_per_s": updates / span, "readback_GBps": round(readback / span / 1e9, 2)}

    def link_GBps():
        """Device-to-host rate of back-to-back 2^20-row (8 MiB) portion
        copies into pinned memory on one stream: the ceiling of the
        read-back every request ends with."""
        portion = 1 << 20
        src = torch.empty(256 * portion, dtype=torch.complex64, device="cuda")
        dst = [torch.empty(portion, dtype=torch.complex64, pin_memory=True) for _ in range(2)]
        for k in range(4):
            dst[k % 2].copy_(src[k * portion:(k + 1) * portion], non_blocking=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(256):
            dst[k % 2].copy_(src[k * portion:(k + 1) * portion], non_blocking=True)
        torch.cuda.synchronize()
        rate = 256 * portion * 8 / (time.perf_counter() - t0) / 1e9
        del src, dst
        torch.cuda.empty_cache()
        return round(rate, 1)

    cont = run(False)
    plain = run(True)
    # Check of the served results (untimed: digesting on the host would add
    # to the latencies): the whole trace again with continuous batching,
    # every `stride`-th request digested as it is read back, against the
    # same requests served one at a time.
    stride = 50
    ids, infos = run(False, digest=stride, at_once=True)
    picked = [k for k, i in enumerate(ids) if i % stride == 0]
    _, alone = run(True, digest=1, at_once=True, only=set(picked))
    bad = [k for k, a in zip(picked, alone) if a["digest"] != infos[k]["digest"] or a["bytes"] != infos[k]["bytes"]]
    if bad:
        raise RuntimeError(f"served requests {bad} differ in the mix and alone")
    check = {"requests_checked": len(picked), "mismatches": 0,
             "how": f"every {stride}th request of the trace: digest of its read-back portions with continuous "
                    f"batching equals its digest served alone"}
    link = link_GBps()
    return {"workload": f"served_poisson_{n}req_rate{rate:g}_M12-28_L50-2000_c64", "requests": n, "check": check,
            "rate_per_s": rate, "calibration": calibrate, "slots": slots, "budget_bytes": budget,
            "amplitude_step_updates": updates, "readback_bytes": readback,
            "link": {"bound": "pcie-d2h", "peak_GBps": link,
                     "frac": round(cont["readback_GBps"] / link, 3),
                     "how": "results read back per second of the continuous run over the device-to-host rate of "
                            "back-to-back 8 MiB portion copies into pinned memory"},
            "continuous": cont, "plain_fcfs": plain,
            "throughput_speedup_vs_plain": round(cont["updates_per_s"] / plain["updates_per_s"], 2),
            "p99_speedup_vs_plain": round(plain["p99_ms"] / cont["p99_ms"], 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="m32", choices=["m32", "m34", "m26", "small", "batched", "served", "rowmap"])
    ap.add_argument("--requests", type=int, default=None, help="served: requests in the trace (default 1000)")
    ap.add_argument("--rate", type=float, default=None, help="served: arrivals per second")
    ap.add_argument("--calibrate", action="store_true", help="served: all requests arrive at once")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-modes", action="store_true",
                    help="skip the batched and served comparisons of the default run")
    ap.add_argument("--skip-batched-served", action="store_true",
                    help="run the other modes (signed, blocked halves, product input, plain runs) only")
    ap.add_argument("--no-plain", action="store_true",
                    help="batched: time the batched launch only (no per-circuit plain run, no autotune)")
    ap.add_argument("--tuning", default=None, help="JSON dict of qsim_tuning fields")
    ap.add_argument("--autotune", action="store_true", help="pick the tuning with qsim_autotune first")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; "
              "run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_quant_ph_0308158_amd import qsim

    torch.cuda.set_device(0)
    if args.workload == "rowmap":
        print(json.dumps(bench_rowmap(max(1, args.steps), max(0, args.warmup))), flush=True)
        return
    if args.workload == "batched":
        print(json.dumps(bench_batched(max(1, args.steps), plain_too=not args.no_plain,
                                       autotune=not args.no_plain)), flush=True)
        return
    if args.requests is None:
        args.requests = W.SERVED_REQUESTS
    if args.workload == "served":
        rate = args.rate if args.rate is not None else W.SERVED_RATE
        print(json.dumps(bench_served(args.requests, rate, calibrate=args.calibrate)), flush=True)
        return
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
    autotune_s = None
    if args.autotune:
        t0 = time.perf_counter()
        tuned = st.autotune(tg, cm)
        autotune_s = round(time.perf_counter() - t0, 2)
        tuning = {k: tuned[k] for k in ("tile_bits", "low_bits", "mid_low_bits", "kernel_variant", "rows_per_thread",
                                        "plan_search")}
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

    modes = None
    if not args.no_modes and args.workload == "m32":
        # Signed diagram: the same steps with every fourth one a controlled
        # phase -1 instead of a NOT (phase steps join any pass).
        kd = (np.arange(L) % 4 == 3).astype(np.uint8)
        s_masks = qsim.plan_describe(M, dt, tg, cm, tuning, kind=kd)[0]
        st.apply(tg, cm, kind=kd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(2):
            st.apply(tg, cm, kind=kd)
        torch.cuda.synchronize()
        s_ms = (time.perf_counter() - t0) / 2 * 1e3
        signed = {"ms_per_step": round(s_ms, 3), "passes": int(len(s_masks)),
                  "value": float(1 << M) * L / (s_ms * 1e-3), "phase_steps": int(kd.sum()),
                  "vs_unsigned": round(ms_per_step / s_ms, 4)}
        # Blocked halves: the same kind of draws with the 500 low-target steps
        # first and the 500 high-target steps after them.
        tb_, cb_ = W.m32_config(blocked=True)
        b_masks = qsim.plan_describe(M, dt, tb_, cb_, tuning)[0]
        st.apply(tb_, cb_)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(2):
            st.apply(tb_, cb_)
        torch.cuda.synchronize()
        b_ms = (time.perf_counter() - t0) / 2 * 1e3
        blocked = {"ms_per_step": round(b_ms, 3), "passes": int(len(b_masks)),
                   "value": float(1 << M) * L / (b_ms * 1e-3)}
        # Product-state input (Appendix 1): the product kernel and then the
        # diagram, against the input formed inside the first pass.
        qq = W.unit_qubits(M, np.complex64 if dt == "c64" else np.complex128, seed=wl["seed"] + 1)

        def timed(fn, reps=2):
            fn()
            torch.cuda.synchronize()
            st.profile(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / reps * 1e3
            p = st.profile_read()
            st.profile(False)
            return ms, p

        def unfused():
            st.set_product(qq)
            st.apply(tg, cm)

        # Same-target runs in the plain path (Sec. 2(i)): the paper's parity
        # diagram (Sec. 4, M-1 steps on target a(1)) as one plain call (runs of
        # up to 16 steps share a launch), one plain call per step, and the
        # fused tile path.
        ptg, pcm = W.parity_circuit(M)

        def plain_steps():
            for s_ in range(len(ptg)):
                st.apply_plain(ptg[s_:s_ + 1], pcm[s_:s_ + 1])

        r_ms, _ = timed(lambda: st.apply_plain(ptg, pcm), reps=1)
        s_ms, _ = timed(plain_steps, reps=1)
        f_ms_p, _ = timed(lambda: st.apply(ptg, pcm), reps=1)
        plain_runs = {"diagram": f"parity of qubits 2..{M} onto qubit 1 ({len(ptg)} steps, one target)",
                      "plain_runs_ms": round(r_ms, 3), "plain_per_step_ms": round(s_ms, 3),
                      "fused_ms": round(f_ms_p, 3), "runs_speedup": round(s_ms / r_ms, 2)}
        # Device time per call: one call is in flight before the first event,
        # so the host planning of every timed call overlaps device work (from
        # an idle device the unfused path would hide its product kernel
        # behind the planning of its apply, the fused path nothing).  The two
        # paths alternate over three rounds and each keeps its median: the
        # difference (a few percent) is of the order of the drift between
        # blocks of calls.
        def device_ms(fn, reps=2):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            fn()
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps

        u_all, f_all = [], []
        for _ in range(3):
            u_all.append(device_ms(unfused))
            f_all.append(device_ms(lambda: st.apply_product(qq, tg, cm)))
        u_ms, f_ms = float(np.median(u_all)), float(np.median(f_all))
        _, fp = timed(lambda: st.apply_product(qq, tg, cm), reps=2)
        first = fp["other_ms"] / fp["other_launches"] if fp["other_launches"] else None
        product = {"unfused_ms": round(u_ms, 3), "fused_ms": round(f_ms, 3),
                   "speedup": round(u_ms / f_ms, 4), "passes": int(len(masks)),
                   "first_pass_ms": round(first, 3) if first else None,
                   "first_pass_write_GBps": round(nbytes / (first * 1e-3) / 1e9, 1) if first else None,
                   "value": float(1 << M) * L / (f_ms * 1e-3)}
        st.close()
        del k1, other
        torch.cuda.empty_cache()
        k1 = other = None
        modes = {"signed": signed, "blocked_halves": blocked, "product_input": product,
                 "plain_same_target_runs": plain_runs}
        if not args.skip_batched_served:
            modes = {"batched": bench_batched(5), "served": bench_served(args.requests, W.SERVED_RATE),
                     "served_capacity": bench_served(args.requests, W.SERVED_RATE, calibrate=True), **modes}
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        if k1 is None:   # the benchmark's input, regenerated from its seed
            k1 = W.gaussian_state_torch(M, dt, seed=wl["seed"])
        host = k1.cpu().numpy()
        st.close()
        del k1, other
        torch.cuda.empty_cache()
        cpu = cpu_baseline(wl, host, args.cpu_seconds)
        del host
        if args.workload == "m32":
            cpu["configs"] = cpu_configs()
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
                   "tile_bits": int(bin(int(masks[0])).count("1")) if len(masks) else M, **wl["desc"],
                   "tuning": tuning, "autotune_s": autotune_s},
        "roofline": roofline,
        "copy_probe_GBps": round(copy_gbps, 1),
        "cpu_baseline": cpu,
        "modes": modes,
        "profile": {k: (round(v, 3) if isinstance(v, float) else v) for k, v in prof.items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
