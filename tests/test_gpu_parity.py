"""GPU parity of libqsim against the CPU oracle (bit-exact: entries are only
moved, so the tolerance is zero).  All calls go through the C ABI."""
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_quant_ph_0308158_amd import qsim
    return qsim


def run_gpu(q, M, k1, tg, cm, tuning=None, plain=False):
    dt = "c64" if k1.dtype == np.complex64 else "c128"
    with q.State(M, dt) as s:
        if tuning:
            s.set_tuning(tuning)
        s.write(k1)
        if plain:
            s.apply_plain(tg, cm, stream=0)
        else:
            s.apply(tg, cm, stream=0)
        return s.read()


def assert_same(a, b, what):
    if a.tobytes() != b.tobytes():
        ua = a.view(np.uint64)
        ub = b.view(np.uint64)
        bad = np.nonzero(ua != ub)[0]
        raise AssertionError(f"{what}: {len(bad)} words differ, first at {bad[:8].tolist()}")


# ------------------------------------------------------------------ small configuration

@pytest.mark.parametrize("inp", ["alternating", "random_phase"])
def test_small_config(q, inp):
    """M=10, complex128, L=20 steps with one control each."""
    M = 10
    tg, cm = W.small_config()
    k1 = W.alternating_state(M) if inp == "alternating" else \
        W.random_phase_state(np.random.default_rng(W.SEED_SMALL + 1), M)
    say("small config", inp)
    assert_same(run_gpu(q, M, k1, tg, cm), oracle.apply(M, k1, tg, cm), "small config")


def test_paper_worked_examples(q):
    from tests._golden import load_examples
    for ex in load_examples().values():
        if "expect_src" not in ex:
            continue
        M = ex["M"]
        say("paper example", ex["name"])
        got = run_gpu(q, M, W.tag_state(M), ex["target"], ex["cmask"])
        np.testing.assert_array_equal(got.view(np.uint64), ex["expect_src"])


# ------------------------------------------------------------------ every path, several sizes

@pytest.mark.parametrize("M", list(range(1, 17)) + [18, 20])
@pytest.mark.parametrize("dt", [np.complex64, np.complex128])
def test_sizes_default_tuning(q, M, dt):
    """M <= 4: direct kernel; up to 14 (c64) / 13 (c128): whole state in LDS;
    above: fused passes over 2^13 / 2^12-entry tiles."""
    rng = np.random.default_rng(100 + M)
    tg, cm = W.random_steps(rng, M, 60, (0, 4))
    k1 = W.gaussian_state(rng, M, dt)
    say("sizes", M, dt.__name__)
    assert_same(run_gpu(q, M, k1, tg, cm), oracle.apply(M, k1, tg, cm), f"M={M}")


@pytest.mark.parametrize("seed,M,dt,tuning", [
    (0, 12, np.complex64, {"tile_bits": 6, "low_bits": 2, "small_bits": 5}),
    (1, 12, np.complex128, {"tile_bits": 5, "low_bits": 1, "small_bits": 5}),
    (2, 15, np.complex64, {"tile_bits": 8, "max_seg_steps": 7, "small_bits": 5}),
    (3, 16, np.complex128, {"tile_bits": 9, "reorder": False, "small_bits": 5}),
    (4, 17, np.complex64, {"tile_bits": 14}),
    (5, 17, np.complex128, {"tile_bits": 13}),
    (6, 18, np.complex64, {"tile_bits": 12, "low_bits": 8}),
    (7, 19, np.complex64, {"tile_bits": 9, "remap": False, "small_bits": 5}),
    (8, 19, np.complex128, {"tile_bits": 8, "remap": True, "outer_order": 2, "small_bits": 5}),
    (9, 20, np.complex64, {"tile_bits": 13, "kernel_variant": 2}),
    (11, 21, np.complex64, {"tile_bits": 14, "kernel_variant": 3}),
    (12, 19, np.complex64, {"tile_bits": 10, "kernel_variant": 3, "wg_per_cu": 2}),
    (13, 18, np.complex128, {"tile_bits": 12, "kernel_variant": 1}),
    (14, 20, np.complex64, {"tile_bits": 13, "rows_per_thread": 8}),
    (15, 20, np.complex64, {"tile_bits": 13, "rows_per_thread": 16, "kernel_variant": 2}),
    (16, 19, np.complex128, {"tile_bits": 12, "rows_per_thread": 8}),
    (17, 19, np.complex128, {"tile_bits": 13, "rows_per_thread": 16, "kernel_variant": 2}),
    (18, 18, np.complex64, {"tile_bits": 9, "rows_per_thread": 8, "kernel_variant": 3, "small_bits": 5}),
    (10, 17, np.complex128, {"tile_bits": 11, "kernel_variant": 2, "wg_per_cu": 1, "remap": False}),
    (19, 20, np.complex64, {"tile_bits": 10, "xcd_swizzle": 1, "small_bits": 5}),
    (20, 21, np.complex128, {"tile_bits": 9, "xcd_swizzle": 2, "small_bits": 5}),
    (21, 20, np.complex64, {"tile_bits": 8, "plan_search": 3, "small_bits": 5}),
    (22, 18, np.complex128, {"tile_bits": 8, "plan_search": 3, "reorder": False, "small_bits": 5}),
    (23, 22, np.complex64, {"tile_bits": 10, "plan_search": 3, "mid_low_bits": 1}),
    (24, 20, np.complex128, {"tile_bits": 13, "kernel_variant": 3}),
    (25, 19, np.complex128, {"tile_bits": 12, "rows_per_thread": 16, "kernel_variant": 3}),
    (26, 21, np.complex128, {"tile_bits": 13, "kernel_variant": 2, "xcd_swizzle": 1}),
    (27, 22, np.complex64, {"tile_bits": 13, "kernel_variant": 2, "xcd_swizzle": 2}),
])
def test_many_passes(q, seed, M, dt, tuning):
    """Small tiles force many passes, outer steps and tile relabelling."""
    rng = np.random.default_rng(200 + seed)
    tg, cm = W.random_steps(rng, M, 300, (0, 4))
    k1 = W.gaussian_state(rng, M, dt)
    say("many passes", seed, M, tuning)
    assert_same(run_gpu(q, M, k1, tg, cm, tuning), oracle.apply(M, k1, tg, cm), str(tuning))


def test_tile_pass_entry(q):
    """qsim_apply_tile_pass: one pass with a caller-chosen tile mask."""
    rng = np.random.default_rng(12)
    M = 18
    I = 0x1F | (1 << 7) | (1 << 9) | (1 << 12) | (1 << 15) | (1 << 17) | (1 << 16) | (1 << 10) | (1 << 6)
    tg, cm = [], []
    while len(tg) < 40:
        t, c = W.random_steps(rng, M, 1, (0, 3))
        if (I >> int(t[0])) & 1 or not (int(c[0]) & I):
            tg.append(int(t[0])); cm.append(int(c[0]))
    tg = np.array(tg, dtype=np.uint32); cm = np.array(cm, dtype=np.uint64)
    k1 = W.gaussian_state(rng, M, np.complex64)
    say("tile pass entry")
    with q.State(M, "c64") as s:
        s.write(k1)
        s.apply_tile_pass(I, tg, cm, stream=0)
        assert_same(s.read(), oracle.apply(M, k1, tg, cm), "tile pass")
        with pytest.raises(q.QsimError):
            bad_t = [int(b) for b in range(M) if not (I >> b) & 1][0]
            s.apply_tile_pass(I, [bad_t], [1], stream=0)
        t0, c0 = W.empty_steps()
        s.apply_tile_pass(I, t0, c0, stream=0)
        assert_same(s.read(), oracle.apply(M, k1, tg, cm), "empty tile pass")


def test_special_values(q):
    rng = np.random.default_rng(5)
    for dt in (np.complex64, np.complex128):
        for M in (9, 17):
            k1 = W.special_values_state(rng, M, dt)
            tg, cm = W.random_steps(rng, M, 80, (0, 3))
            say("special values", M, dt.__name__)
            assert_same(run_gpu(q, M, k1, tg, cm), oracle.apply(M, k1, tg, cm), "special values")


def test_plain_path(q):
    rng = np.random.default_rng(6)
    for dt in (np.complex64, np.complex128):
        for M in (3, 12, 19):
            tg, cm = W.random_steps(rng, M, 40, (0, 3))
            k1 = W.gaussian_state(rng, M, dt)
            say("plain", M, dt.__name__)
            assert_same(run_gpu(q, M, k1, tg, cm, plain=True), oracle.apply(M, k1, tg, cm), "plain")


def run_plain_kinds(q, M, k1, tg, cm, kd):
    dt = "c64" if k1.dtype == np.complex64 else "c128"
    with q.State(M, dt) as s:
        s.write(k1)
        s.apply_plain(tg, cm, stream=0, kind=kd)
        return s.read()


def test_plain_same_target_runs(q):
    """Consecutive NOT steps on one target share one plain launch that
    interchanges a pair when an odd number of their conditions hold (Sec.
    2(i)): the paper's parity diagram (Sec. 4: M-1 steps on one target, two
    launches), runs of 1..40 steps (split every 16) with 0..4 controls and
    repeated masks (pairs toggled twice stay), interrupted by phase steps."""
    rng = np.random.default_rng(60)
    for M in (12, 20):
        tg, cm = W.parity_circuit(M)
        k1 = W.alternating_state(M)
        say("plain parity diagram", M)
        k2 = run_gpu(q, M, k1, tg, cm, plain=True)
        assert_same(k2, oracle.apply(M, k1, tg, cm), "plain parity diagram")
        want = np.array([(-1.0) ** bin(i).count("1") for i in range(1 << M)]) * 2.0 ** (-M / 2)
        assert np.array_equal(k2.real, want) and not k2.imag.any()
    for dt, M, seed in ((np.complex64, 17, 61), (np.complex128, 15, 62), (np.complex64, 19, 63)):
        r = np.random.default_rng(seed)
        tgs, cms = [], []
        while len(tgs) < 300:
            t = int(r.integers(0, M))
            run = int(r.integers(1, 41))
            t_run, c_run = W.random_steps(r, M, run, (0, 4), targets=[t] * run)
            if run > 3:
                c_run[2] = c_run[0]             # a repeated condition toggles a pair twice
            tgs += list(t_run)
            cms += list(c_run)
        tg = np.array(tgs, dtype=np.uint32)
        cm = np.array(cms, dtype=np.uint64)
        kd = (r.random(len(tg)) < 0.05).astype(np.uint8)
        k1 = W.gaussian_state(r, M, dt)
        say("plain runs", M, dt.__name__)
        assert_same(run_plain_kinds(q, M, k1, tg, cm, kd), oracle.apply(M, k1, tg, cm, kind=kd), "plain runs")
        assert_same(run_gpu(q, M, k1, tg, cm, plain=True), oracle.apply(M, k1, tg, cm), "plain runs, NOT only")


def test_empty_and_unconditional(q):
    rng = np.random.default_rng(7)
    M = 16
    k1 = W.gaussian_state(rng, M, np.complex64)
    t0, c0 = W.empty_steps()
    say("empty")
    assert_same(run_gpu(q, M, k1, t0, c0), k1, "L=0")
    tg = np.arange(M, dtype=np.uint32)
    cm = np.zeros(M, dtype=np.uint64)
    say("all unconditional")
    assert_same(run_gpu(q, M, k1, tg, cm), k1[::-1].copy(), "NOT on every bit reverses the vector")


def test_parity_experiment(q):
    """Sec. 4 wiring diagram on the alternating input: k2(i) = (-1)^popcount(i) |S|."""
    for M in (10, 16, 22):
        tg, cm = W.parity_circuit(M)
        say("parity", M)
        k2 = run_gpu(q, M, W.alternating_state(M), tg, cm)
        assert_same(k2, oracle.apply(M, W.alternating_state(M), tg, cm), "parity")


def test_portions(q):
    rng = np.random.default_rng(8)
    M = 18
    k1 = W.gaussian_state(rng, M, np.complex128)
    tg, cm = W.random_steps(rng, M, 50, (0, 3))
    ref = oracle.apply(M, k1, tg, cm)
    with q.State(M, "c128") as s:
        for off in range(0, 1 << M, 70001):   # ragged write portions
            s.write(k1[off:off + 70001], offset=off)
        s.apply(tg, cm, stream=0)
        for off, cnt in [(0, 1), (12345, 6789), ((1 << M) - 3, 3), (0, 1 << M), (77, 0)]:
            assert_same(s.read(off, cnt), ref[off:off + cnt], f"portion {off}+{cnt}")
        with pytest.raises(q.QsimError) as ei:
            s.read((1 << M) - 2, 3)
        assert ei.value.code == q.ERR_RANGE


def test_invalid_steps_leave_state(q):
    rng = np.random.default_rng(9)
    M = 15
    k1 = W.gaussian_state(rng, M, np.complex64)
    with q.State(M, "c64") as s:
        s.write(k1)
        tg = np.array([1, 2, M], dtype=np.uint32)
        cm = np.array([0, 1, 0], dtype=np.uint64)
        with pytest.raises(q.QsimError) as ei:
            s.apply(tg, cm, stream=0)
        assert ei.value.code == q.ERR_INVALID
        assert_same(s.read(), k1, "state after rejected apply")


def test_wrap_torch_buffers(q):
    import torch
    rng = np.random.default_rng(10)
    M = 20
    k1 = W.gaussian_state(rng, M, np.complex64)
    tg, cm = W.random_steps(rng, M, 100, (0, 3))
    b0 = torch.from_numpy(k1.copy()).cuda()
    b1 = torch.empty_like(b0)
    s = q.State(M, "c64", buffers=(b0, b1))
    s.apply(tg, cm)
    torch.cuda.synchronize()
    cur = b0 if s.current_ptr() == b0.data_ptr() else b1
    assert_same(cur.cpu().numpy(), oracle.apply(M, k1, tg, cm), "wrapped buffers")
    s.close()


@pytest.mark.parametrize("dt,n,mr,lr,seed", [
    (np.complex64, 24, (1, 18), (0, 120), 123),
    (np.complex128, 24, (1, 17), (0, 120), 124),
    (np.complex64, 300, (8, 16), (10, 200), 125),
])
def test_batch_matches_oracle(q, dt, n, mr, lr, seed):
    """One persistent launch over circuits of mixed size and depth: every
    circuit's result equals the oracle's, bit for bit."""
    rng = np.random.default_rng(seed)
    circuits = W.batched_config(n=n, seed=seed, m_range=mr, l_range=lr)
    states, ins = [], []
    code = "c64" if dt == np.complex64 else "c128"
    for c in circuits:
        k1 = W.gaussian_state(rng, c.M, dt)
        s = q.State(c.M, code)
        s.write(k1)
        states.append(s)
        ins.append(k1)
    say("batch", n, dt.__name__)
    q.apply_batch(states, [(c.target, c.cmask) for c in circuits], stream=0)
    q.batch_status()
    for c, s, k1 in zip(circuits, states, ins):
        assert_same(s.read(), oracle.apply(c.M, k1, c.target, c.cmask, threads=8), f"batch circuit M={c.M} L={c.L}")
        s.close()


def test_batch_config_matches_solo(q):
    """The batched configuration (4096 circuits, M 8..20, L 10..500, 0..3
    controls): every circuit of the single batched launch equals its solo
    qsim_apply_steps result bit for bit; a sample is also checked against
    the oracle."""
    import torch
    circuits = W.batched_config()
    say("batch config: setup")
    solo, batch, ins = [], [], []
    for i, c in enumerate(circuits):
        k1 = W.gaussian_state_torch(c.M, "c64", seed=1000 + i)
        a = q.State(c.M, "c64", buffers=(k1.clone(), torch.empty_like(k1)))
        b = q.State(c.M, "c64", buffers=(k1.clone(), torch.empty_like(k1)))
        solo.append(a); batch.append(b); ins.append(k1)
    say("batch config: solo applies")
    for c, a in zip(circuits, solo):
        a.apply(c.target, c.cmask)
    say("batch config: batched launch")
    q.apply_batch(batch, [(c.target, c.cmask) for c in circuits])
    q.batch_status()
    torch.cuda.synchronize()
    say("batch config: compare")
    for i, (c, a, b) in enumerate(zip(circuits, solo, batch)):
        ra = a._keep[0] if a.current_ptr() == a._keep[0].data_ptr() else a._keep[1]
        rb = b._keep[0] if b.current_ptr() == b._keep[0].data_ptr() else b._keep[1]
        assert torch.equal(ra.view(torch.int64), rb.view(torch.int64)), f"circuit {i} M={c.M} L={c.L}"
        if i % 256 == 0:
            ref = oracle.apply(c.M, ins[i].cpu().numpy(), c.target, c.cmask, threads=8)
            assert_same(rb.cpu().numpy(), ref, f"batch circuit {i} vs oracle")
    for a, b in zip(solo, batch):
        a.close(); b.close()


# ------------------------------------------------------------------ full-size configurations

def test_m26_config_full(q):
    """M=26, complex128 (1 GiB), L=200, 0..4 controls: whole-vector compare."""
    import torch
    M = 26
    tg, cm = W.m26_config()
    say("m26: generate")
    k1_dev = W.gaussian_state_torch(M, "c128", seed=W.SEED_M26)
    k1 = k1_dev.cpu().numpy()
    b1 = torch.empty_like(k1_dev)
    s = q.State(M, "c128", buffers=(k1_dev, b1))
    say("m26: apply")
    s.apply(tg, cm)
    k2 = s.read()
    s.close()
    say("m26: oracle")
    ref = oracle.apply(M, k1, tg, cm, threads=16, method="enum")
    assert_same(k2, ref, "m26 config")


# ------------------------------------------------------------------ serving

def _server_requests(seed, n, m_range, l_max):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        M = int(rng.integers(m_range[0], m_range[1] + 1))
        L = int(rng.integers(0, l_max + 1))
        tg, cm = W.random_steps(rng, M, L, (0, 3))
        k1 = W.gaussian_state(rng, M, np.complex64) if i % 3 else None
        reqs.append((M, tg, cm, k1))
    return reqs


def test_server_alone_and_in_mix(q):
    """Continuous batching: every request's read-back result is the same
    (digest of all its bytes) whether it runs alone or among others, and
    equals the oracle's result."""
    reqs = _server_requests(21, 24, (5, 16), 300)
    say("server: mix")
    with q.Server(budget_bytes=1 << 30, max_slots=8, portion_entries=1 << 12, digest=True) as srv:
        ids = [srv.submit(M, "c64", tg, cm, k1) for (M, tg, cm, k1) in reqs]
        srv.drain()
        mix = [srv.info(i) for i in ids]
    say("server: alone")
    alone = []
    with q.Server(budget_bytes=1 << 30, fcfs=True, portion_entries=1 << 12, digest=True) as srv:
        for (M, tg, cm, k1) in reqs:
            rid = srv.submit(M, "c64", tg, cm, k1)
            srv.drain()
            alone.append(srv.info(rid))
    for i, (a, b, (M, tg, cm, k1)) in enumerate(zip(alone, mix, reqs)):
        assert a["status"] == 0 and b["status"] == 0 and a["done"] and b["done"]
        assert a["bytes"] == b["bytes"] == 8 << M
        assert a["digest"] == b["digest"], f"request {i} differs alone and in the mix"
        k = k1 if k1 is not None else W.alternating_state(M, np.complex64)
        ref = oracle.apply(M, k, tg, cm)
        assert q.digest_bytes(ref.tobytes()) == b["digest"], f"request {i} differs from the oracle"


def test_server_small_budget_queues(q):
    """With an arena that holds two requests at a time, the others wait in the
    queue (admission never exceeds the budget) and all complete correctly."""
    reqs = _server_requests(22, 10, (16, 16), 100)   # 2 x 512 KiB each -> one 2 MiB granule
    say("server: small budget")
    with q.Server(budget_bytes=4 << 20, max_slots=8, portion_entries=1 << 12, digest=True) as srv:
        ids = [srv.submit(M, "c64", tg, cm, k1) for (M, tg, cm, k1) in reqs]
        peak = 0
        import time
        t_end = time.time() + 60
        while any(not srv.info(i)["done"] for i in ids) and time.time() < t_end:
            st = srv.stats()
            assert st["arena_used"] <= st["arena_bytes"]
            peak = max(peak, st["running"])
            time.sleep(0.001)
        srv.drain()
        infos = [srv.info(i) for i in ids]
        assert peak <= 2
        with pytest.raises(q.QsimError):
            srv.submit(20, "c64", [0], [0])        # 16 MiB of buffers > the whole arena
    for (M, tg, cm, k1), inf in zip(reqs, infos):
        assert inf["status"] == 0
        k = k1 if k1 is not None else W.alternating_state(M, np.complex64)
        assert q.digest_bytes(oracle.apply(M, k, tg, cm).tobytes()) == inf["digest"]


# ------------------------------------------------------------------ product-state input

@pytest.mark.parametrize("dt", [np.complex64, np.complex128])
def test_product_state_matches_oracle(q, dt):
    """qsim_state_set_product builds q_M x ... x q_1 (Appendix 1) bit-exactly
    as the oracle does, for every M from 1 to 20; then a diagram applied to it
    matches the oracle too."""
    rng = np.random.default_rng(31)
    code = "c64" if dt == np.complex64 else "c128"
    for M in list(range(1, 21)):
        qq = rng.standard_normal((M, 2)) + 1j * rng.standard_normal((M, 2))
        qq = (qq / np.linalg.norm(qq, axis=1, keepdims=True)).astype(dt)
        ref = oracle.product_state(M, qq)
        say("product state", M, code)
        with q.State(M, code) as s:
            s.set_product(qq, stream=0)
            assert_same(s.read(), ref, f"product state M={M}")
            if M in (8, 17):
                tg, cm = W.random_steps(rng, M, 50, (0, 3))
                s.apply(tg, cm, stream=0)
                assert_same(s.read(), oracle.apply(M, ref, tg, cm), f"product then apply M={M}")


def test_product_state_m32_sampled(q):
    """At M=32 (complex64): sampled rows against the oracle's product formula
    evaluated for those rows, and the 2-norm of a unit-norm product."""
    import torch
    M = 32
    rng = np.random.default_rng(32)
    qq = rng.standard_normal((M, 2)) + 1j * rng.standard_normal((M, 2))
    qq = (qq / np.linalg.norm(qq, axis=1, keepdims=True)).astype(np.complex64)
    b0 = torch.empty(1 << M, dtype=torch.complex64, device="cuda")
    b1 = torch.empty_like(b0)
    s = q.State(M, "c64", buffers=(b0, b1))
    say("product state m32")
    s.set_product(qq)
    torch.cuda.synchronize()
    rows = np.concatenate([rng.integers(0, 1 << M, size=300, dtype=np.uint64), [0, 1, (1 << M) - 1]])
    got = b0[torch.from_numpy(rows.astype(np.int64)).cuda()].cpu().numpy()
    for r, g in zip(rows.tolist(), got):
        assert g.tobytes() == oracle.product_entry(M, qq, r).tobytes(), f"row {r}"
    nrm = float(torch.linalg.vector_norm(b0.view(torch.float32).double()))
    assert abs(nrm - 1.0) < 1e-3
    s.close()



# ------------------------------------------------------------------ materialised row array

def test_rowmap_build_and_apply(q):
    """qsim_rowmap_build gives the paper's row array x of U_L...U_1 (the
    oracle's sparse-matrix bookkeeping folded over the reversed list), and
    qsim_rowmap_apply equals applying the diagram."""
    import torch
    rng = np.random.default_rng(41)
    for M, dt in ((1, np.complex128), (2, np.complex64), (3, np.complex64), (12, np.complex128),
                  (18, np.complex64), (20, np.complex128)):
        tg, cm = W.random_steps(rng, M, 150 if M > 2 else 9, (0, 3))
        x = torch.empty(1 << M, dtype=torch.int32, device="cuda")
        say("rowmap", M)
        q.rowmap_build(M, tg, cm, x)
        torch.cuda.synchronize()
        xr = oracle.rowmap(M, tg[::-1], cm[::-1])
        np.testing.assert_array_equal(x.cpu().numpy().view(np.uint32).astype(np.uint64), xr)
        k1 = W.gaussian_state(rng, M, dt)
        with q.State(M, "c64" if dt == np.complex64 else "c128") as s:
            s.write(k1)
            s.rowmap_apply(x.data_ptr(), stream=0)
            assert_same(s.read(), oracle.apply(M, k1, tg, cm), f"rowmap apply M={M}")



def test_autotune_keeps_state_and_result(q):
    """qsim_autotune leaves the state's contents unchanged and the tuning it
    picks gives the oracle's result."""
    rng = np.random.default_rng(51)
    for M, dt in ((17, np.complex64), (16, np.complex128)):
        tg, cm = W.random_steps(rng, M, 200, (0, 3))
        k1 = W.gaussian_state(rng, M, dt)
        with q.State(M, "c64" if dt == np.complex64 else "c128") as s:
            s.write(k1)
            say("autotune", M)
            t = s.autotune(tg, cm, stream=0)
            assert t["tile_bits"] in (12, 13, 14)
            assert_same(s.read(), k1, "state after autotune")
            s.apply(tg, cm, stream=0)
            assert_same(s.read(), oracle.apply(M, k1, tg, cm), "apply with the tuned parameters")


def test_autotune_cache(q, tmp_path, monkeypatch):
    """With QSIM_TUNING_CACHE set, qsim_autotune stores its choice under
    (architecture, dtype, M, band of L) and a later call takes it from
    there without measuring; an entry the library would reject is measured
    again and overwritten.  Every tuning gives the oracle's result."""
    import json
    rng = np.random.default_rng(52)
    M = 18
    tg, cm = W.random_steps(rng, M, 150, (0, 3))
    k1 = W.gaussian_state(rng, M, np.complex64)
    cache = tmp_path / "tuning.json"
    monkeypatch.setenv("QSIM_TUNING_CACHE", str(cache))
    with q.State(M, "c64") as s:
        s.write(k1)
        say("autotune with cache")
        t = s.autotune(tg, cm, stream=0)
        assert_same(s.read(), k1, "state after autotune")
        entries = json.loads(cache.read_text())["qsim_tuning"]
        (key, entry), = entries.items()
        assert key.endswith(":c64:M18:L128-256"), key
        assert all(entry[f] == t[f] for f in ("tile_bits", "kernel_variant", "mid_low_bits", "plan_search"))
        assert entry["best_ms"] > 0 and entry["best_ms"] <= entry["default_ms"]
    # a stored choice the measurement would not have made is taken as it is
    entry.update({"tile_bits": 10, "kernel_variant": 2, "mid_low_bits": 1, "plan_search": 2})
    cache.write_text(json.dumps({"qsim_tuning": {key: entry}}))
    with q.State(M, "c64") as s:
        s.write(k1)
        t = s.autotune(tg, cm, stream=0)
        assert (t["tile_bits"], t["kernel_variant"], t["mid_low_bits"], t["plan_search"]) == (10, 2, 1, 2)
        s.apply(tg, cm, stream=0)
        assert_same(s.read(), oracle.apply(M, k1, tg, cm), "apply with the cached tuning")
    # an entry out of range is measured again
    entry["tile_bits"] = 99
    cache.write_text(json.dumps({"qsim_tuning": {key: entry}}))
    with q.State(M, "c64") as s:
        s.write(k1)
        t = s.autotune(tg, cm, stream=0)
        assert t["tile_bits"] in (12, 13, 14)
        assert json.loads(cache.read_text())["qsim_tuning"][key]["tile_bits"] == t["tile_bits"]
        s.apply(tg, cm, stream=0)
        assert_same(s.read(), oracle.apply(M, k1, tg, cm), "apply after re-measuring")


def test_copy_bytes(q):
    """qsim_copy_bytes (the achievable-bandwidth reference of the benchmark)
    copies every byte, for sizes that leave a partial last workgroup."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(99)
    for nbytes in (16, 4096 + 48, (1 << 24) + 16 * 37):
        src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda", generator=g)
        dst = torch.zeros(nbytes + 64, dtype=torch.uint8, device="cuda")
        say("copy", nbytes)
        q.copy_bytes(dst.data_ptr(), src.data_ptr(), nbytes)
        torch.cuda.synchronize()
        assert torch.equal(dst[:nbytes], src)
        assert int(dst[nbytes:].count_nonzero()) == 0


def test_batches_back_to_back(q):
    """Batched launches queued one after another without waiting (the plan
    upload of one overlaps the kernel of the previous): batch 2 applies the
    reversed diagrams of batch 1, so every state returns to its input;
    batch 3 applies the diagrams again and must equal the oracle."""
    rng = np.random.default_rng(130)
    circuits = W.batched_config(n=60, seed=131, m_range=(3, 18), l_range=(0, 160))
    states, ins = [], []
    for c in circuits:
        k1 = W.gaussian_state(rng, c.M, np.complex64)
        s = q.State(c.M, "c64")
        s.write(k1)
        states.append(s)
        ins.append(k1)
    fwd = [(c.target, c.cmask) for c in circuits]
    rev = [(c.target[::-1].copy(), c.cmask[::-1].copy()) for c in circuits]
    say("batches back to back")
    q.apply_batch(states, fwd, stream=0)
    q.apply_batch_packed(states, q.PackedBatch(rev), stream=0)
    q.apply_batch(states, fwd, stream=0)
    q.batch_status()
    for c, s, k1 in zip(circuits, states, ins):
        assert_same(s.read(), oracle.apply(c.M, k1, c.target, c.cmask), f"third batch M={c.M} L={c.L}")
    q.apply_batch(states, rev, stream=0)
    q.batch_status()
    for c, s, k1 in zip(circuits, states, ins):
        assert_same(s.read(), k1, f"fourth batch undoes the third M={c.M} L={c.L}")
        s.close()


def test_batches_of_changing_size(q):
    """The host keeps its batch buffers (plans, pass and small-circuit
    descriptors, queue) from one call to the next: a large batch, then a
    batch of a few other circuits (fewer passes and descriptors than the
    buffers hold), then a batch with phase steps, then a subset of the
    first circuits again, queued back to back.  Every state equals the
    oracle's result of the diagrams applied to it, in order."""
    rng = np.random.default_rng(150)
    big = W.batched_config(n=80, seed=151, m_range=(3, 19), l_range=(0, 200))
    few = W.batched_config(n=5, seed=152, m_range=(14, 17), l_range=(1, 60))
    signed = W.batched_config(n=12, seed=153, m_range=(4, 16), l_range=(1, 90))
    groups = [big, few, signed, big[10:30]]
    states, ins, expect = {}, {}, {}
    for gi, g in enumerate(groups[:3]):
        for ci, c in enumerate(g):
            k1 = W.gaussian_state(rng, c.M, np.complex64)
            s = q.State(c.M, "c64")
            s.write(k1)
            states[(gi, ci)] = s
            ins[(gi, ci)] = k1
            expect[(gi, ci)] = k1
    kinds = [(rng.random(c.L) < 0.3).astype(np.uint8) for c in signed]
    say("batches of changing size")
    for gi, g in enumerate(groups):
        key_g = gi if gi < 3 else 0
        off = 10 if gi == 3 else 0
        sts, steps = [], []
        for ci, c in enumerate(g):
            key = (key_g, ci + off)
            sts.append(states[key])
            if gi == 2:
                steps.append((c.target, c.cmask, kinds[ci]))
                expect[key] = oracle.apply(c.M, expect[key], c.target, c.cmask, kind=kinds[ci])
            else:
                steps.append((c.target, c.cmask))
                expect[key] = oracle.apply(c.M, expect[key], c.target, c.cmask)
        q.apply_batch(sts, steps, stream=0)
    q.batch_status()
    for key, s in states.items():
        assert_same(s.read(), expect[key], f"circuit {key}")
        s.close()


def test_batch_invalid_step_runs_nothing(q):
    """A bad step in any circuit rejects the whole batch before anything is
    enqueued: every state keeps its contents."""
    rng = np.random.default_rng(140)
    circuits = W.batched_config(n=20, seed=141, m_range=(5, 16), l_range=(1, 80))
    states, ins = [], []
    for c in circuits:
        k1 = W.gaussian_state(rng, c.M, np.complex64)
        s = q.State(c.M, "c64")
        s.write(k1)
        states.append(s)
        ins.append(k1)
    steps = [(c.target, c.cmask) for c in circuits]
    bad_t = steps[13][0].copy()
    bad_t[-1] = circuits[13].M          # target beyond the address bits
    steps[13] = (bad_t, steps[13][1])
    say("batch with an invalid step")
    with pytest.raises(q.QsimError) as ei:
        q.apply_batch(states, steps, stream=0)
    assert ei.value.code == q.ERR_INVALID and "circuit 13" in q.last_error()
    q.batch_status()
    for s, k1 in zip(states, ins):
        assert_same(s.read(), k1, "state after a rejected batch")
        s.close()


def test_m32_complex128_sampled(q):
    """M=32 complex128 (64 GiB per buffer, byte offsets up to 2^36, 2^20
    tiles of 2^12 entries per pass): the headline diagram, sampled rows
    (including the first and last and those around 2^31) against the
    oracle's source rows, then the involution."""
    import torch
    torch.cuda.synchronize()
    torch.cuda.empty_cache()          # 128 GiB of buffers: return what earlier tests cached
    M = 32
    tg, cm = W.m32_config()
    say("m32 c128: generate")
    k1_dev = W.gaussian_state_torch(M, "c128", seed=3232)
    rng = np.random.default_rng(3232)
    rows = np.concatenate([rng.integers(0, 1 << M, size=1500, dtype=np.uint64),
                           np.arange(32, dtype=np.uint64), (1 << M) - 1 - np.arange(32, dtype=np.uint64),
                           (1 << 31) + np.arange(-16, 16, dtype=np.int64).astype(np.uint64)])
    src_rows = np.array([oracle.source_index(M, tg, cm, int(i)) for i in rows], dtype=np.int64)
    words = lambda t: t.view(torch.int64).view(-1, 2)
    expect = words(k1_dev)[torch.from_numpy(src_rows).cuda()].cpu().numpy()
    b1 = torch.empty_like(k1_dev)
    s = q.State(M, "c128", buffers=(k1_dev, b1))
    say("m32 c128: apply")
    s.apply(tg, cm)
    torch.cuda.synchronize()
    cur = k1_dev if s.current_ptr() == k1_dev.data_ptr() else b1
    got = words(cur)[torch.from_numpy(rows.astype(np.int64)).cuda()].cpu().numpy()
    np.testing.assert_array_equal(got, expect)
    say("m32 c128: involution")
    s.apply(tg[::-1].copy(), cm[::-1].copy())
    torch.cuda.synchronize()
    cur = k1_dev if s.current_ptr() == k1_dev.data_ptr() else b1
    s.close()
    del b1
    k1_again = W.gaussian_state_torch(M, "c128", seed=3232)
    same = torch.equal(cur.view(torch.int64), k1_again.view(torch.int64))
    del k1_again, cur, k1_dev
    torch.cuda.empty_cache()
    assert same


def test_m33_sampled_beyond_2_32_rows(q):
    """M=33 complex64 (2^33 rows, 64 GiB per buffer): row addresses and
    outer tile bits above bit 32.  Sampled rows (including the first and
    last) against the oracle's source rows, then the involution."""
    import torch
    torch.cuda.synchronize()
    torch.cuda.empty_cache()          # 128 GiB of buffers: return what earlier tests cached
    M = 33
    tg, cm = W.m32_config(M=33, seed=33)
    say("m33: generate")
    k1_dev = W.gaussian_state_torch(M, "c64", seed=33)
    rng = np.random.default_rng(3333)
    rows = np.concatenate([rng.integers(0, 1 << M, size=1500, dtype=np.uint64),
                           np.arange(32, dtype=np.uint64), (1 << M) - 1 - np.arange(32, dtype=np.uint64),
                           (1 << 32) + np.arange(-16, 16, dtype=np.int64).astype(np.uint64)])
    src_rows = np.array([oracle.source_index(M, tg, cm, int(i)) for i in rows], dtype=np.int64)
    assert (src_rows >= (1 << 32)).any() and (src_rows < (1 << 32)).any()
    expect = k1_dev.view(torch.int64)[torch.from_numpy(src_rows).cuda()].cpu().numpy()
    b1 = torch.empty_like(k1_dev)
    s = q.State(M, "c64", buffers=(k1_dev, b1))
    say("m33: apply")
    s.apply(tg, cm)
    torch.cuda.synchronize()
    cur = k1_dev if s.current_ptr() == k1_dev.data_ptr() else b1
    got = cur.view(torch.int64)[torch.from_numpy(rows.astype(np.int64)).cuda()].cpu().numpy()
    np.testing.assert_array_equal(got, expect)
    say("m33: involution")
    s.apply(tg[::-1].copy(), cm[::-1].copy())
    torch.cuda.synchronize()
    cur = k1_dev if s.current_ptr() == k1_dev.data_ptr() else b1
    s.close()
    del b1
    k1_again = W.gaussian_state_torch(M, "c64", seed=33)
    same = torch.equal(cur.view(torch.int64), k1_again.view(torch.int64))
    del k1_again, cur, k1_dev
    torch.cuda.empty_cache()
    assert same


@pytest.mark.parametrize("M,code", [(34, "c64"), (33, "c128")])
def test_largest_states_sampled(q, M, code):
    """The largest states one MI355X holds out of place (two 128 GiB
    buffers): M=34 complex64 and M=33 complex128.  Sampled rows (the first
    and last, those around 2^32 and 2^33, and random ones) against the
    oracle's source rows; then the reversed diagram, after which other
    sampled rows hold their original values (no second copy of the state
    fits beside the two buffers)."""
    import torch
    torch.cuda.synchronize()
    torch.cuda.empty_cache()          # 256 GiB of buffers: return what earlier tests cached
    tg, cm = W.m32_config(M=M, seed=M)
    say(f"M={M} {code}: generate")
    k1_dev = W.gaussian_state_torch(M, code, seed=M)
    rng = np.random.default_rng(100 * M + len(code))
    edges = np.concatenate([np.arange(32), (1 << M) - 1 - np.arange(32),
                            (1 << 32) + np.arange(-16, 16), (1 << (M - 1)) + np.arange(-16, 16)]).astype(np.uint64)
    rows = np.concatenate([rng.integers(0, 1 << M, size=1500, dtype=np.uint64), edges])
    src_rows = np.array([oracle.source_index(M, tg, cm, int(i)) for i in rows], dtype=np.int64)
    assert int(rows.max()) < (1 << M) and 0 <= int(src_rows.min()) and int(src_rows.max()) < (1 << M)
    assert (src_rows >= (1 << (M - 1))).any() and (src_rows < (1 << 32)).any()
    per = 1 if code == "c64" else 2          # 64-bit words per entry
    words = k1_dev.view(torch.int64).view(-1, per)
    expect = words[torch.from_numpy(src_rows).cuda()].cpu().numpy()
    back = np.concatenate([rng.integers(0, 1 << M, size=1500, dtype=np.uint64), edges])
    assert int(back.max()) < (1 << M)
    back_rows = torch.from_numpy(back.astype(np.int64)).cuda()
    before = words[back_rows].cpu().numpy()
    b1 = torch.empty_like(k1_dev)
    s = q.State(M, code, buffers=(k1_dev, b1))
    say(f"M={M} {code}: apply")
    s.apply(tg, cm)
    torch.cuda.synchronize()
    cur = k1_dev if s.current_ptr() == k1_dev.data_ptr() else b1
    got = cur.view(torch.int64).view(-1, per)[torch.from_numpy(rows.astype(np.int64)).cuda()].cpu().numpy()
    np.testing.assert_array_equal(got, expect)
    say(f"M={M} {code}: reversed diagram")
    s.apply(tg[::-1].copy(), cm[::-1].copy())
    torch.cuda.synchronize()
    cur = k1_dev if s.current_ptr() == k1_dev.data_ptr() else b1
    after = cur.view(torch.int64).view(-1, per)[back_rows].cpu().numpy()
    s.close()
    del b1, cur, k1_dev, words
    torch.cuda.empty_cache()
    np.testing.assert_array_equal(after, before)


def test_batch_autotune_keeps_states(q, tmp_path, monkeypatch):
    """qsim_batch_autotune times candidate settings with forward and reversed
    batches: the states are unchanged, the choice is stored in the tuning
    cache and read back from it by a second call, and a batch with it equals
    the oracle."""
    rng = np.random.default_rng(150)
    circuits = W.batched_config(n=48, seed=151, m_range=(6, 17), l_range=(0, 120))
    states, ins = [], []
    for c in circuits:
        k1 = W.gaussian_state(rng, c.M, np.complex64)
        s = q.State(c.M, "c64")
        s.write(k1)
        states.append(s)
        ins.append(k1)
    steps = [(c.target, c.cmask) for c in circuits]
    cache = tmp_path / "tuning.json"
    monkeypatch.setenv("QSIM_TUNING_CACHE", str(cache))
    say("batch autotune")
    try:
        t = q.batch_autotune(states, steps, stream=0)
        assert t["from_cache"] == 0 and t["best_ms"] > 0 and t["best_ms"] <= t["default_ms"]
        chosen = {k: t[k] for k in q.BATCH_TUNING_FIELDS}
        assert q.batch_get_tuning("c64") == chosen
        for s, k1 in zip(states, ins):
            assert_same(s.read(), k1, "state after batch autotune")
        import json
        entries = json.loads(cache.read_text())["qsim_batch_tuning"]
        (key, entry), = entries.items()
        assert ":c64:M" in key and all(entry[k] == v for k, v in chosen.items())
        q.batch_set_tuning("c64", None)
        t2 = q.batch_autotune(states, steps, stream=0)
        assert t2["from_cache"] == 1 and {k: t2[k] for k in q.BATCH_TUNING_FIELDS} == chosen
        q.apply_batch(states, steps, stream=0)
        q.batch_status()
        for c, s, k1 in zip(circuits, states, ins):
            assert_same(s.read(), oracle.apply(c.M, k1, c.target, c.cmask), f"tuned batch M={c.M} L={c.L}")
    finally:
        q.batch_set_tuning("c64", None)
        for s in states:
            s.close()


@pytest.mark.parametrize("dt,tuning", [
    ("c64", {"order": 1}),
    ("c64", {"order": 2, "tiles_per_item": 1}),
    ("c64", {"tile_bits": 12, "tiles_per_item": 8}),
    ("c64", {"tile_bits": 10, "circuit_tiles": 1}),
    ("c64", {"circuit_tiles": 64, "plan_search": 2}),
    ("c64", {"tile_bits": 11, "circuit_tiles": 4, "tiles_per_item": 64, "order": 1}),
    ("c128", {"tile_bits": 11}),
    ("c128", {"tile_bits": 12, "circuit_tiles": 1, "plan_search": 2, "tiles_per_item": 3}),
])
def test_batch_settings_match_oracle(q, dt, tuning):
    """Every batched-mode setting (queue order, tile size, whole-circuit
    cut-off, planning, item size) gives each circuit its oracle result,
    with and without phase steps; the launch reports its passes and
    algorithmic bytes."""
    npd = np.complex64 if dt == "c64" else np.complex128
    rng = np.random.default_rng(160 + len(str(tuning)))
    circuits = W.batched_config(n=40, seed=161, m_range=(3, 19), l_range=(0, 150))
    kinds = [(rng.random(c.L) < 0.15).astype(np.uint8) for c in circuits]
    states, ins = [], []
    for c in circuits:
        k1 = W.gaussian_state(rng, c.M, npd)
        s = q.State(c.M, dt)
        s.write(k1)
        states.append(s)
        ins.append(k1)
    say("batch settings", dt, tuning)
    try:
        q.batch_set_tuning(dt, tuning)
        assert all(q.batch_get_tuning(dt)[k] == v for k, v in tuning.items())
        q.apply_batch(states, [(c.target, c.cmask, kd) for c, kd in zip(circuits, kinds)], stream=0)
        q.batch_status()
        info = q.batch_last_info()
        assert info["circuits"] == len(circuits) and info["kernel_ms"] > 0
        assert all(info["tuning"][k] == v for k, v in tuning.items())
        assert info["algorithmic_bytes"] >= sum(2 * (npd().itemsize << c.M) for c in circuits if c.L)
        for c, s, k1, kd in zip(circuits, states, ins, kinds):
            assert_same(s.read(), oracle.apply(c.M, k1, c.target, c.cmask, kind=kd), f"M={c.M} L={c.L} {tuning}")
    finally:
        q.batch_set_tuning(dt, None)
        for s in states:
            s.close()
