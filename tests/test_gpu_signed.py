"""GPU parity for signed diagrams: controlled NOT steps mixed with controlled
phase -1 steps (the signed permutation matrices; the paper's first example
of a unitary matrix, Sec. 2(a), is one).  Bit-exact against the CPU oracle:
negation is a sign-bit flip, so the tolerance is zero.  All calls go through
the C ABI."""
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

NOT, PHASE = 0, 1


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


def signed_steps(rng, M, L, n_ctl=(0, 3), p_phase=0.35):
    tg, cm = W.random_steps(rng, M, L, n_ctl)
    kd = (rng.random(L) < p_phase).astype(np.uint8)
    return tg, cm, kd


def run_gpu(q, M, k1, tg, cm, kd, tuning=None, plain=False):
    dt = "c64" if k1.dtype == np.complex64 else "c128"
    with q.State(M, dt) as s:
        if tuning:
            s.set_tuning(tuning)
        s.write(k1)
        if plain:
            s.apply_plain(tg, cm, stream=0, kind=kd)
        else:
            s.apply(tg, cm, stream=0, kind=kd)
        return s.read()


def assert_same(a, b, what):
    if a.tobytes() != b.tobytes():
        ua, ub = a.view(np.uint64), b.view(np.uint64)
        bad = np.nonzero(ua != ub)[0]
        raise AssertionError(f"{what}: {len(bad)} words differ, first at {bad[:8].tolist()}")


# The paper's signed example matrix (Sec. 2(a)) as a diagram on bits 0, 1:
# three NOTs give the row map x = (3, 0, 2, 1), a phase step negates row 3.
EX_T = np.array([1, 0, 0, 0], dtype=np.uint32)
EX_C = np.array([0b01, 0b10, 0, 0b10], dtype=np.uint64)
EX_K = np.array([NOT, NOT, NOT, PHASE], dtype=np.uint8)
EX_G = np.array([[0, 0, 0, 1], [1, 0, 0, 0], [0, 0, 1, 0], [0, -1, 0, 0]])


@pytest.mark.parametrize("M", [2, 10, 18])
def test_signed_example_matrix(q, M):
    """On M bits the two-bit diagram acts as I (x) G on every block of four
    rows: direct walk (M=2), whole state in LDS (M=10), tiles (M=18)."""
    for dt in (np.complex64, np.complex128):
        i = np.arange(1 << M)
        k1 = (i + 1 + 1j * (7 * i + 3)).astype(dt)
        say("signed example", M, dt.__name__)
        got = run_gpu(q, M, k1, EX_T, EX_C, EX_K)
        expect = (k1.astype(np.complex128).reshape(-1, 4) @ EX_G.T).reshape(-1).astype(dt)
        assert_same(got, expect, "I x G")
        assert_same(got, oracle.apply(M, k1, EX_T, EX_C, kind=EX_K), "oracle")


@pytest.mark.parametrize("M", list(range(1, 17)) + [18, 20])
@pytest.mark.parametrize("dt", [np.complex64, np.complex128])
def test_signed_sizes_default_tuning(q, M, dt):
    rng = np.random.default_rng(7000 + M)
    tg, cm, kd = signed_steps(rng, M, 120)
    k1 = W.gaussian_state(rng, M, dt)
    say("signed size", M, dt.__name__)
    assert_same(run_gpu(q, M, k1, tg, cm, kd), oracle.apply(M, k1, tg, cm, kind=kd), f"M={M}")


@pytest.mark.parametrize("seed,M,dt,tuning", [
    (0, 12, np.complex64, {"tile_bits": 6, "low_bits": 2, "small_bits": 5}),
    (1, 12, np.complex128, {"tile_bits": 5, "low_bits": 1, "small_bits": 5}),
    (2, 15, np.complex64, {"tile_bits": 8, "max_seg_steps": 7, "small_bits": 5}),
    (3, 16, np.complex128, {"tile_bits": 9, "reorder": False, "small_bits": 5}),
    (4, 17, np.complex64, {"tile_bits": 14}),
    (5, 19, np.complex64, {"tile_bits": 9, "remap": False, "small_bits": 5}),
    (6, 20, np.complex64, {"tile_bits": 13, "kernel_variant": 2}),
    (7, 21, np.complex64, {"tile_bits": 14, "kernel_variant": 3}),
    (8, 20, np.complex64, {"tile_bits": 13, "rows_per_thread": 8}),
    (9, 19, np.complex128, {"tile_bits": 13, "rows_per_thread": 16, "kernel_variant": 2}),
    (10, 18, np.complex64, {"tile_bits": 9, "rows_per_thread": 8, "kernel_variant": 3, "small_bits": 5}),
    (11, 20, np.complex64, {"tile_bits": 10, "plan_search": 2, "small_bits": 5}),
    (12, 19, np.complex128, {"tile_bits": 8, "plan_search": 3, "small_bits": 5}),
])
def test_signed_many_passes(q, seed, M, dt, tuning):
    """Small tiles force phase steps with bits on both sides of the tile
    boundary (sign plane plus per-tile flags) in every kernel shape."""
    rng = np.random.default_rng(7100 + seed)
    tg, cm, kd = signed_steps(rng, M, 300, (0, 4))
    k1 = W.gaussian_state(rng, M, dt)
    say("signed many passes", seed, M, tuning)
    assert_same(run_gpu(q, M, k1, tg, cm, kd, tuning), oracle.apply(M, k1, tg, cm, kind=kd), str(tuning))


def test_signed_special_values(q):
    """NaN payloads, infinities, zeros and subnormals: only sign bits flip."""
    rng = np.random.default_rng(7200)
    for dt in (np.complex64, np.complex128):
        for M in (3, 9, 17):
            k1 = W.special_values_state(rng, M, dt)
            tg, cm, kd = signed_steps(rng, M, 80)
            say("signed special values", M, dt.__name__)
            assert_same(run_gpu(q, M, k1, tg, cm, kd), oracle.apply(M, k1, tg, cm, kind=kd), "special values")


def test_signed_only_phase_steps(q):
    """A diagram of phase steps only moves nothing: every entry keeps its row
    and flips sign once per phase step that selects it."""
    rng = np.random.default_rng(7300)
    M = 19
    tg, cm = W.random_steps(rng, M, 50, (0, 3))
    kd = np.ones(50, dtype=np.uint8)
    k1 = W.gaussian_state(rng, M, np.complex64)
    say("phase only")
    got = run_gpu(q, M, k1, tg, cm, kd)
    i = np.arange(1 << M, dtype=np.uint64)
    odd = np.zeros(1 << M, dtype=bool)
    for t, c in zip(tg, cm):
        m = np.uint64(int(c) | (1 << int(t)))
        odd ^= (i & m) == m
    np.testing.assert_array_equal(got, np.where(odd, -k1, k1))


def test_signed_plain_path(q):
    rng = np.random.default_rng(7400)
    for dt in (np.complex64, np.complex128):
        for M in (2, 12, 19):
            tg, cm, kd = signed_steps(rng, M, 40)
            k1 = W.gaussian_state(rng, M, dt)
            say("signed plain", M, dt.__name__)
            assert_same(run_gpu(q, M, k1, tg, cm, kd, plain=True), oracle.apply(M, k1, tg, cm, kind=kd), "plain")


def test_signed_tile_pass_entry(q):
    """qsim_apply_tile_pass: phase steps join the pass whatever their bits."""
    rng = np.random.default_rng(7500)
    M = 18
    I = 0x1F | (1 << 7) | (1 << 9) | (1 << 12) | (1 << 15) | (1 << 17) | (1 << 16) | (1 << 10) | (1 << 6)
    tg, cm, kd = [], [], []
    while len(tg) < 60:
        t, c = W.random_steps(rng, M, 1, (0, 3))
        ph = rng.random() < 0.5
        if ph or (I >> int(t[0])) & 1 or not (int(c[0]) & I):
            tg.append(int(t[0])); cm.append(int(c[0])); kd.append(PHASE if ph else NOT)
    tg = np.array(tg, dtype=np.uint32); cm = np.array(cm, dtype=np.uint64); kd = np.array(kd, dtype=np.uint8)
    assert (kd == PHASE).sum() > 10
    k1 = W.gaussian_state(rng, M, np.complex64)
    say("signed tile pass")
    with q.State(M, "c64") as s:
        s.write(k1)
        s.apply_tile_pass(I, tg, cm, stream=0, kind=kd)
        assert_same(s.read(), oracle.apply(M, k1, tg, cm, kind=kd), "tile pass")


def test_signed_batch(q):
    """One batched launch over signed circuits of every path (direct walk,
    whole state in LDS, tiled passes)."""
    rng = np.random.default_rng(7600)
    circuits = W.batched_config(n=40, seed=7601, m_range=(1, 18), l_range=(0, 150))
    states, ins, kinds = [], [], []
    for c in circuits:
        k1 = W.gaussian_state(rng, c.M, np.complex64)
        s = q.State(c.M, "c64")
        s.write(k1)
        states.append(s); ins.append(k1)
        kinds.append((rng.random(c.L) < 0.35).astype(np.uint8))
    say("signed batch")
    q.apply_batch(states, [(c.target, c.cmask, k) for c, k in zip(circuits, kinds)], stream=0)
    q.batch_status()
    for c, s, k1, kd in zip(circuits, states, ins, kinds):
        assert_same(s.read(), oracle.apply(c.M, k1, c.target, c.cmask, kind=kd), f"batch M={c.M} L={c.L}")
        s.close()


@pytest.mark.parametrize("dt,seed", [(np.complex64, 7610), (np.complex128, 7611)])
def test_signed_batch_mid_size_whole_circuits(q, dt, seed):
    """Mid-size circuits (passes of at most 16 tiles) run whole in one
    workgroup, mixed with tiled and in-LDS ones, deep diagrams (up to 600
    steps, many passes each), phase steps; every result against the oracle."""
    rng = np.random.default_rng(seed)
    circuits = W.batched_config(n=120, seed=seed, m_range=(11, 18), l_range=(100, 600))
    code = "c64" if dt == np.complex64 else "c128"
    states, ins, kinds = [], [], []
    for c in circuits:
        k1 = W.gaussian_state(rng, c.M, dt)
        s = q.State(c.M, code)
        s.write(k1)
        states.append(s); ins.append(k1)
        kinds.append((rng.random(c.L) < 0.2).astype(np.uint8))
    say("signed batch, mid-size whole circuits", code)
    q.apply_batch(states, [(c.target, c.cmask, k) for c, k in zip(circuits, kinds)], stream=0)
    q.batch_status()
    for c, s, k1, kd in zip(circuits, states, ins, kinds):
        assert_same(s.read(), oracle.apply(c.M, k1, c.target, c.cmask, kind=kd, threads=8), f"batch M={c.M} L={c.L}")
        s.close()


def test_signed_server(q):
    rng = np.random.default_rng(7700)
    reqs = []
    for i in range(12):
        M = int(rng.integers(3, 17))
        tg, cm, kd = signed_steps(rng, M, int(rng.integers(0, 200)))
        reqs.append((M, tg, cm, kd, W.gaussian_state(rng, M, np.complex64)))
    say("signed server")
    with q.Server(budget_bytes=1 << 30, max_slots=4, portion_entries=1 << 10, digest=True) as srv:
        ids = [srv.submit(M, "c64", tg, cm, k1, kind=kd) for (M, tg, cm, kd, k1) in reqs]
        srv.drain()
        infos = [srv.info(i) for i in ids]
    for (M, tg, cm, kd, k1), inf in zip(reqs, infos):
        assert inf["status"] == 0 and inf["done"]
        assert q.digest_bytes(oracle.apply(M, k1, tg, cm, kind=kd).tobytes()) == inf["digest"]


def test_signed_autotune_keeps_state(q):
    """The autotuner undoes each trial with the reversed diagram, which also
    holds for phase steps (each is its own inverse)."""
    rng = np.random.default_rng(7800)
    M = 17
    tg, cm, kd = signed_steps(rng, M, 150)
    k1 = W.gaussian_state(rng, M, np.complex64)
    with q.State(M, "c64") as s:
        s.write(k1)
        say("signed autotune")
        s.autotune(tg, cm, stream=0, kind=kd)
        assert_same(s.read(), k1, "state after autotune")
        s.apply(tg, cm, stream=0, kind=kd)
        assert_same(s.read(), oracle.apply(M, k1, tg, cm, kind=kd), "apply after autotune")


def test_signed_m32_sampled(q):
    """M=32 complex64 (32 GiB per buffer): the m32 configuration with one step
    in four turned into a phase step; sampled rows against the oracle's
    per-row source and sign, then the involution on the device."""
    import torch
    M = 32
    tg, cm = W.m32_config()
    kd = (np.arange(len(tg)) % 4 == 3).astype(np.uint8)
    say("signed m32: generate")
    k1_dev = W.gaussian_state_torch(M, "c64", seed=W.SEED_M32)
    rng = np.random.default_rng(3232)
    rows = np.concatenate([rng.integers(0, 1 << M, size=1500, dtype=np.uint64),
                           np.arange(32, dtype=np.uint64), (1 << M) - 1 - np.arange(32, dtype=np.uint64)])
    src, neg = zip(*(oracle.source_index_signed(M, tg, cm, kd, int(i)) for i in rows))
    expect = k1_dev.view(torch.int64)[torch.from_numpy(np.array(src, dtype=np.int64)).cuda()].cpu().numpy()
    sign_bits = np.array(0x8000000080000000, dtype=np.uint64).view(np.int64)   # both float32 sign bits
    expect = expect ^ np.where(np.array(neg), sign_bits, np.int64(0))
    b1 = torch.empty_like(k1_dev)
    s = q.State(M, "c64", buffers=(k1_dev, b1))
    say("signed m32: apply")
    s.apply(tg, cm, kind=kd)
    torch.cuda.synchronize()
    cur = k1_dev if s.current_ptr() == k1_dev.data_ptr() else b1
    got = cur.view(torch.int64)[torch.from_numpy(rows.astype(np.int64)).cuda()].cpu().numpy()
    np.testing.assert_array_equal(got, expect)
    say("signed m32: involution")
    s.apply(tg[::-1].copy(), cm[::-1].copy(), kind=kd[::-1].copy())
    torch.cuda.synchronize()
    cur = k1_dev if s.current_ptr() == k1_dev.data_ptr() else b1
    s.close()
    k1_again = W.gaussian_state_torch(M, "c64", seed=W.SEED_M32)
    assert torch.equal(cur.view(torch.int64), k1_again.view(torch.int64))
