"""Host-side checks of libqsim that need no GPU: the library loads and exports
every symbol of include/qsim.h, argument validation, and the pass planner's
invariants (checked with the CPU oracle on the planner's reordered list)."""
import os
import re

import numpy as np
import pytest

import oracle
import workloads as W
from paper_quant_ph_0308158_amd import qsim

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "qsim.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qsim_[a-z_]+)\s*\(", text)))


def test_plain_c_caller(tmp_path):
    """The boundary is plain C: a C99 program that includes include/qsim.h
    and links libqsim.so plans the paper's Fig. 2 diagram on the host
    (qsim_plan_describe: no device work) and reads the library version."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lib = qsim.lib()._name
    prog = tmp_path / "caller.c"
    prog.write_text(r"""
#include <stdio.h>
#include "qsim.h"
int main(void) {
    /* Fig. 2: NOT a(2); NOT a(1) controlled by a(2); NOT a(2) */
    qsim_step st[3] = {{1, QSIM_STEP_NOT, 0}, {0, QSIM_STEP_NOT, 2}, {1, QSIM_STEP_NOT, 0}};
    uint32_t n = 0, len[8], order[8];
    uint64_t mask[8];
    int rc = qsim_plan_describe(12, QSIM_C64, st, 3, NULL, &n, mask, len, 8, order);
    if (rc != QSIM_OK) { printf("rc %d %s\n", rc, qsim_last_error()); return 1; }
    printf("%s passes %u steps %u\n", qsim_version(), n, len[0]);
    return 0;
}
""")
    exe = tmp_path / "caller"
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Werror", f"-I{os.path.join(ROOT, 'include')}", str(prog),
                        lib, f"-Wl,-rpath,{os.path.dirname(lib)}", "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "passes 1 steps 3" in r.stdout


def test_exports_every_header_symbol():
    syms = header_symbols()
    assert len(syms) >= 15
    lib = qsim.lib()
    for s in syms:
        assert hasattr(lib, s), f"libqsim.so does not export {s}"
    assert sorted(qsim.EXPORTS) == syms


def test_version_and_error_string():
    assert "gfx950" in qsim.version()
    assert isinstance(qsim.last_error(), str)


def test_step_layout_is_16_bytes():
    assert qsim.STEP_DTYPE.itemsize == 16


@pytest.mark.parametrize("bad", [
    dict(M=8, target=[8], cmask=[0]),
    dict(M=8, target=[2], cmask=[1 << 8]),
    dict(M=8, target=[2], cmask=[0b100]),
])
def test_invalid_steps_rejected(bad):
    with pytest.raises(qsim.QsimError) as ei:
        qsim.plan_describe(bad["M"], "c64", bad["target"], bad["cmask"])
    assert ei.value.code == qsim.ERR_INVALID


def test_invalid_m_and_dtype():
    with pytest.raises(qsim.QsimError):
        qsim.plan_describe(0, "c64", [], [])
    with pytest.raises(qsim.QsimError):
        qsim.plan_describe(qsim.MAX_M + 1, "c64", [], [])
    with pytest.raises(qsim.QsimError):
        qsim.plan_describe(8, "c64", [0], [0], tuning={"tile_bits": 20})
    with pytest.raises(qsim.QsimError):
        qsim.plan_describe(8, "c64", [0], [0], tuning={"plan_search": 4})
    with pytest.raises(qsim.QsimError):
        qsim.plan_describe(8, "c64", [0], [0], tuning={"product_stage": 4})
    qsim.plan_describe(8, "c64", [0], [0], tuning={"product_stage": 1})


def test_unknown_step_kind_rejected():
    st = qsim.pack_steps([1, 2], [0, 1], kind=[qsim.STEP_NOT, qsim.STEP_PHASE])
    n = qsim.ctypes.c_uint32(0)
    rc = qsim.lib().qsim_plan_describe(8, 0, st.ctypes.data, 2, None, qsim.ctypes.byref(n),
                                       None, None, 0, None)
    assert rc == 0
    st["kind"][1] = 7
    rc = qsim.lib().qsim_plan_describe(8, 0, st.ctypes.data, 2, None, qsim.ctypes.byref(n),
                                       None, None, 0, None)
    assert rc == qsim.ERR_INVALID
    assert "kind" in qsim.last_error()


def test_create_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(qsim.QsimError):
        qsim.State(10, "c64")


def _check_plan(M, dtype, tg, cm, tuning, kd=None):
    masks, lens, order = qsim.plan_describe(M, dtype, tg, cm, tuning, kind=kd)
    L = len(tg)
    assert sorted(order.tolist()) == list(range(L))
    assert int(lens.sum()) == L
    K = min(tuning.get("tile_bits", 13 if dtype == "c64" else 12), M)
    # the forced low bits leave a tile bit free when the state exceeds a tile
    low = min(tuning.get("low_bits", 5 if dtype == "c64" else 4), K - 1 if M > K else K)
    cap = tuning.get("max_seg_steps", 1024)
    mid = tuning.get("mid_low_bits", 2 if dtype == "c64" else 1)
    mid = low if (tuning.get("remap", True) is False or mid > low) else mid
    pos = 0
    for p, (I, n) in enumerate(zip(masks.tolist(), lens.tolist())):
        assert bin(I).count("1") == K, "a tile always has exactly K bits"
        need = low if p in (0, len(masks) - 1) else mid
        assert I & ((1 << need) - 1) == (1 << need) - 1, "tile must hold the low address bits"
        assert I < (1 << M)
        # only a final pass that restores the natural layout may be empty
        assert (1 <= n or p == len(masks) - 1) and n <= cap
        for s in order[pos:pos + n]:
            t, c = int(tg[s]), int(cm[s])
            if kd is not None and kd[s] == qsim.STEP_PHASE:
                continue                      # moves nothing: fits any tile
            assert (I >> t) & 1 or not (c & I), f"step {s} splits tiles of pass {p}"
        pos += n
    return masks, lens, order


@pytest.mark.parametrize("seed,M,dtype,tuning", [
    (0, 12, "c64", {"tile_bits": 6, "low_bits": 2}),
    (1, 14, "c128", {"tile_bits": 7, "low_bits": 3}),
    (2, 16, "c64", {"tile_bits": 8, "max_seg_steps": 9}),
    (3, 16, "c64", {"tile_bits": 8, "reorder": False}),
    (4, 13, "c64", {"tile_bits": 5, "low_bits": 1}),
    (5, 13, "c64", {"tile_bits": 5, "low_bits": 1, "min_overlap": 5}),
    (6, 16, "c128", {"tile_bits": 8, "min_overlap": 4, "mid_low_bits": 1}),
    (7, 14, "c64", {"tile_bits": 6, "low_bits": 2, "plan_search": 2}),
    (8, 16, "c128", {"tile_bits": 8, "max_seg_steps": 9, "plan_search": 2}),
    (9, 16, "c64", {"tile_bits": 8, "reorder": False, "plan_search": 2}),
    (10, 13, "c64", {"tile_bits": 5, "low_bits": 1, "min_overlap": 5, "plan_search": 2}),
    (11, 14, "c64", {"tile_bits": 6, "low_bits": 2, "plan_search": 3}),
    (12, 16, "c128", {"tile_bits": 8, "max_seg_steps": 9, "plan_search": 3}),
    (13, 16, "c64", {"tile_bits": 8, "reorder": False, "plan_search": 3}),
    (14, 13, "c64", {"tile_bits": 5, "low_bits": 1, "plan_search": 3}),
    (15, 18, "c128", {"tile_bits": 8, "mid_low_bits": 1, "plan_search": 3}),
])
def test_planner_reorder_is_exact(seed, M, dtype, tuning):
    """The planner's execution order has the same product as the original
    list (checked with the oracle on an address-tag state)."""
    rng = np.random.default_rng(seed)
    tg, cm = W.random_steps(rng, M, 150, (0, 3))
    masks, lens, order = _check_plan(M, dtype, tg, cm, tuning)
    assert len(masks) > 1
    k1 = W.tag_state(M)
    a = oracle.apply(M, k1, tg, cm)
    b = oracle.apply(M, k1, tg[order], cm[order])
    assert a.tobytes() == b.tobytes()
    if tuning.get("reorder") is False:
        assert order.tolist() == list(range(len(tg)))


def test_planner_on_benchmark_workloads():
    tg, cm = W.m32_config()
    masks, lens, order = _check_plan(32, "c64", tg, cm, {})
    assert len(masks) < 80
    # The mask search (on by default at this size) takes at least the greedy
    # scan's steps in each pass; on this workload that saves passes.
    off, _, _ = _check_plan(32, "c64", tg, cm, {"plan_search": 1})
    assert len(masks) <= len(off)
    climb, _, _ = _check_plan(32, "c64", tg, cm, {"plan_search": 2})
    assert len(climb) <= len(off)
    beam, _, order = _check_plan(32, "c64", tg, cm, {"plan_search": 3})
    assert len(beam) < len(climb)
    tg, cm = W.m26_config()
    _check_plan(26, "c128", tg, cm, {})


@pytest.mark.parametrize("seed,M,tile_bits,dtype", [
    (30, 14, 6, "c64"), (31, 20, 8, "c64"), (30, 18, 8, "c128"), (38, 14, 6, "c64"), (36, 18, 8, "c128"),
])
def test_beam_search_saves_passes(seed, M, tile_bits, dtype):
    """The beam search over whole plans (plan_search 3) finds plans with
    fewer passes than a climb per pass on these diagrams; its plans are
    valid, exact (oracle on address tags, the planner's order against the
    original) and the same on every call (seeded draws, any thread count)."""
    rng = np.random.default_rng(seed)
    tg, cm = W.random_steps(rng, M, 150, (0, 3))
    base = {"tile_bits": tile_bits, "mid_low_bits": 2}
    climb, _, _ = _check_plan(M, dtype, tg, cm, {**base, "plan_search": 2})
    masks, lens, order = _check_plan(M, dtype, tg, cm, {**base, "plan_search": 3})
    assert len(masks) < len(climb)
    k1 = W.tag_state(M)
    assert oracle.apply(M, k1, tg, cm).tobytes() == oracle.apply(M, k1, tg[order], cm[order]).tobytes()
    again = qsim.plan_describe(M, dtype, tg, cm, {**base, "plan_search": 3})
    assert again[0].tolist() == masks.tolist() and again[2].tolist() == order.tolist()


def test_beam_search_random_diagrams():
    """Beam-search plans of 24 seeded random diagrams (sizes, tiles, control
    counts, phase steps, no reordering) are valid plans, never longer than
    the climb's, and their order has the same product (oracle, tag state)."""
    rng = np.random.default_rng(77)
    for case in range(24):
        M = int(rng.integers(11, 16))
        K = int(rng.integers(5, min(M - 2, 9) + 1))
        L = int(rng.integers(20, 160))
        tg, cm = W.random_steps(rng, M, L, (0, int(rng.integers(1, 5))))
        kd = (rng.random(L) < 0.25).astype(np.uint8) if case % 3 == 0 else None
        tun = {"tile_bits": K, "low_bits": int(rng.integers(1, min(K, 5) + 1))}
        if case % 5 == 4:
            tun["reorder"] = False
        climb = qsim.plan_describe(M, "c64", tg, cm, dict(tun, plan_search=2), kind=kd)[0]
        masks, lens, order = _check_plan(M, "c64", tg, cm, dict(tun, plan_search=3), kd)
        assert len(masks) <= len(climb), (case, len(masks), len(climb))
        if kd is None:
            k1 = W.tag_state(M)
            assert oracle.apply(M, k1, tg, cm).tobytes() == oracle.apply(M, k1, tg[order], cm[order]).tobytes(), case
        else:
            k1 = (np.arange(1 << M) + 1j * np.arange(1 << M)[::-1]).astype(np.complex128)
            a = oracle.apply(M, k1, tg, cm, kind=kd)
            b = oracle.apply(M, k1, tg[order], cm[order], kind=kd[order])
            assert a.tobytes() == b.tobytes(), case


def test_beam_search_skipped_for_long_diagrams():
    """The beam search's host time grows with L times the passes: beyond
    4e6 the climb's plan is kept (same masks and order)."""
    tg, cm = W.m32_config(L=12000, seed=7)
    climb = qsim.plan_describe(32, "c64", tg, cm, {"plan_search": 2})
    beam = qsim.plan_describe(32, "c64", tg, cm, {"plan_search": 3})
    assert len(climb[0]) * len(tg) > 4e6
    assert beam[0].tolist() == climb[0].tolist() and beam[2].tolist() == climb[2].tolist()


def test_beam_search_with_phase_steps():
    rng = np.random.default_rng(25)
    M = 16
    tg, cm = W.random_steps(rng, M, 200, (0, 3))
    kd = (rng.random(200) < 0.3).astype(np.uint8)
    masks, lens, order = _check_plan(M, "c64", tg, cm, {"tile_bits": 7, "plan_search": 3}, kd)
    k1 = (np.arange(1 << M) + 1j * np.arange(1 << M)[::-1]).astype(np.complex128)
    a = oracle.apply(M, k1, tg, cm, kind=kd)
    b = oracle.apply(M, k1, tg[order], cm[order], kind=kd[order])
    assert a.tobytes() == b.tobytes()


def test_beam_search_beyond_32_address_bits():
    """At M = 36 middle passes may hold bits 32 and up; the beam's plans
    still start and end with tiles below bit 32 holding the low bits, and
    reorder only commuting steps."""
    tg, cm = W.m32_config(M=36, seed=36)
    masks, lens, order = _check_plan(36, "c64", tg, cm, {"plan_search": 3})
    m = [int(x) for x in masks]
    assert m[0] < (1 << 32) and m[-1] < (1 << 32)
    _order_commutes(tg, cm, None, order)
    climb = qsim.plan_describe(36, "c64", tg, cm, {"plan_search": 2})[0]
    assert len(m) <= len(climb)


def test_planner_same_target_run_is_one_pass():
    """Steps that share a target commute (Sec. 2(i)): a long run of them with
    controls spread over all bits fits in one pass."""
    rng = np.random.default_rng(9)
    M = 24
    tg = np.full(200, 20, dtype=np.uint32)
    cm = np.array([(1 << int(a)) | (1 << int(b)) for a, b in rng.integers(0, 20, size=(200, 2))],
                  dtype=np.uint64)
    masks, lens, order = _check_plan(M, "c64", tg, cm, {})
    assert len(masks) == 1


@pytest.mark.parametrize("seed,M,dtype,tuning", [
    (20, 12, "c64", {"tile_bits": 6, "low_bits": 2}),
    (21, 14, "c128", {"tile_bits": 7, "low_bits": 3, "plan_search": 2}),
    (22, 16, "c64", {"tile_bits": 8, "max_seg_steps": 9}),
    (23, 13, "c64", {"tile_bits": 5, "low_bits": 1, "min_overlap": 5}),
])
def test_planner_reorder_is_exact_with_phase_steps(seed, M, dtype, tuning):
    """Phase steps join any pass and move only past steps they commute with
    (no NOT of theirs targets one of their bits): the reordered list has the
    same signed product (oracle on integer-valued entries)."""
    rng = np.random.default_rng(seed)
    tg, cm = W.random_steps(rng, M, 150, (0, 3))
    kd = (rng.random(150) < 0.4).astype(np.uint8)
    masks, lens, order = _check_plan(M, dtype, tg, cm, tuning, kd)
    assert len(masks) > 1
    k1 = (np.arange(1 << M) + 1j * np.arange(1 << M)[::-1]).astype(np.complex128)
    a = oracle.apply(M, k1, tg, cm, kind=kd)
    b = oracle.apply(M, k1, tg[order], cm[order], kind=kd[order])
    assert a.tobytes() == b.tobytes()


def test_rowmap_rejects_phase_steps():
    with pytest.raises(qsim.QsimError) as ei:
        qsim.rowmap_build(8, [1], [0], 0, kind=[qsim.STEP_PHASE])
    assert ei.value.code == qsim.ERR_INVALID


def test_packed_batch_layout():
    """PackedBatch: circuit c's pointer addresses its own steps, packed as
    pack_steps would pack them, with its length; empty circuits included."""
    import ctypes
    rng = np.random.default_rng(40)
    steps = []
    for i in range(30):
        M = int(rng.integers(1, 12))
        L = 0 if i % 7 == 3 else int(rng.integers(1, 40))
        tg, cm = W.random_steps(rng, M, L, (0, 3))
        steps.append((tg, cm, (rng.random(L) < 0.3).astype(np.uint8)) if i % 2 else (tg, cm))
    pb = qsim.PackedBatch(steps)
    assert len(pb) == 30 and pb.ptrs.dtype == np.uint64 and pb.lens.dtype == np.uint64
    for i, sc in enumerate(steps):
        ref = qsim.pack_steps(*sc)
        assert int(pb.lens[i]) == len(ref)
        assert ctypes.string_at(int(pb.ptrs[i]), 16 * len(ref)) == ref.tobytes()


def _order_commutes(tg, cm, kd, order):
    """Every pair of steps whose relative order the plan swapped commutes:
    neither writes a bit the other reads (a NOT writes its target; reads its
    controls, a phase step reads its target and controls)."""
    pos = np.empty(len(order), dtype=np.int64)
    pos[np.asarray(order, dtype=np.int64)] = np.arange(len(order))
    kd = np.zeros(len(tg), dtype=np.uint8) if kd is None else kd
    W_ = [0 if kd[s] else 1 << int(tg[s]) for s in range(len(tg))]
    R_ = [int(cm[s]) | ((1 << int(tg[s])) if kd[s] else 0) for s in range(len(tg))]
    for i in range(len(tg)):
        for j in range(i + 1, len(tg)):
            if pos[j] < pos[i]:
                assert not (W_[i] & R_[j]) and not (W_[j] & R_[i]), f"steps {i} and {j} swapped but do not commute"


@pytest.mark.parametrize("M", [33, 34, 35, 36])
def test_planner_beyond_32_address_bits(M):
    """Tile offsets are 32-bit: the first and last pass (natural layout) keep
    their tile bits below bit 32, middle passes may hold higher bits (their
    layouts put the tile at the bottom); steps on bits 32 and up still find a
    pass, and the plan's reordering only swaps commuting steps."""
    tg, cm = W.m32_config(M=M, seed=M)
    kd = (np.arange(len(tg)) % 5 == 4).astype(np.uint8)
    for kind in (None, kd):
        masks, lens, order = _check_plan(M, "c64", tg, cm, {}, kind)
        m = [int(x) for x in masks]
        assert m[0] < (1 << 32) and m[-1] < (1 << 32)
        assert any(x >= (1 << 32) for x in m[1:-1]), "no middle pass used a high bit"
        _order_commutes(tg, cm, kind, order)


def test_planner_high_target_with_low_control_needs_tail_pass():
    """A step targeting bit 33 controlled by bit 0 (always in the tile) can
    only run in a middle pass; the plan then ends with a step-free pass that
    restores the natural layout."""
    M = 34
    tg = np.array([33, 3, 40 - 7], dtype=np.uint32)
    cm = np.array([0b1, 0, 1 << 20], dtype=np.uint64)
    masks, lens, order = _check_plan(M, "c64", tg, cm, {})
    assert int(lens[-1]) == 0 and int(masks[-1]) < (1 << 32)
    assert any(int(x) >> 33 & 1 for x in masks)


def test_batch_tiles_per_item_setting():
    """The batched kernel's tiles per queue item: validated, process-wide,
    0 restores the default (host only, no device work)."""
    default = qsim.batch_tiles_per_item()
    assert default == 32
    qsim.batch_set_tiles_per_item(8)
    assert qsim.batch_tiles_per_item() == 8
    with pytest.raises(qsim.QsimError) as ei:
        qsim.batch_set_tiles_per_item(257)
    assert ei.value.code == qsim.ERR_INVALID
    assert qsim.batch_tiles_per_item() == 8
    qsim.batch_set_tiles_per_item(0)
    assert qsim.batch_tiles_per_item() == default


def test_budget_rejects_state_creation(monkeypatch):
    """QSIM_HBM_BUDGET_BYTES caps what qsim_state_create may allocate: a
    state beyond it fails with QSIM_ERR_NOMEM before any device call (so
    this holds without a GPU too)."""
    monkeypatch.setenv("QSIM_HBM_BUDGET_BYTES", str(1 << 20))
    with pytest.raises(qsim.QsimError):
        qsim.State(20, "c64")                 # 2 x 8 MiB > 1 MiB
    assert "QSIM_HBM_BUDGET_BYTES" in qsim.last_error()


def test_batch_tuning_setting():
    """qsim_batch_set_tuning validates its fields and keeps one setting per
    dtype (host only)."""
    default = qsim.batch_get_tuning("c64")
    assert default == {"tiles_per_item": 32, "tile_bits": 13, "circuit_tiles": 64, "plan_search": 2, "order": 2}
    assert qsim.batch_get_tuning("c128")["tile_bits"] == 12
    qsim.batch_set_tuning("c128", {"tile_bits": 11, "order": 1})
    assert qsim.batch_get_tuning("c128")["tile_bits"] == 11 and qsim.batch_get_tuning("c64") == default
    for bad in ({"tile_bits": 9}, {"tile_bits": 14}, {"plan_search": 3}, {"order": 3}, {"tiles_per_item": 257},
                {"circuit_tiles": 300}):
        with pytest.raises(qsim.QsimError):
            qsim.batch_set_tuning("c64", bad)
    qsim.batch_set_tuning("c128", None)
    assert qsim.batch_get_tuning("c64") == default
    with pytest.raises(qsim.QsimError):
        qsim.batch_last_info()            # no batch has run in this process


def test_host_exception_becomes_an_error_code(monkeypatch):
    """A C++ exception on the host (here a failed allocation, forced with
    QSIM_FAULT_INJECT) ends at the C boundary as QSIM_ERR_NOMEM with a
    message, and the next call runs normally."""
    rng = np.random.default_rng(8200)
    tg, cm = W.random_steps(rng, 20, 300, (0, 3))
    want = qsim.plan_describe(20, "c64", tg, cm, {"tile_bits": 10, "small_bits": 5})
    monkeypatch.setenv("QSIM_FAULT_INJECT", "host:1")
    with pytest.raises(qsim.QsimError) as ei:
        qsim.plan_describe(20, "c64", tg, cm, {"tile_bits": 10, "small_bits": 5})
    assert ei.value.code == qsim.ERR_NOMEM
    assert "host memory allocation failed" in qsim.last_error()
    monkeypatch.delenv("QSIM_FAULT_INJECT")
    got = qsim.plan_describe(20, "c64", tg, cm, {"tile_bits": 10, "small_bits": 5})
    for a, b in zip(want, got):
        assert np.array_equal(a, b)
