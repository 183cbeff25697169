"""GPU parity of qsim_apply_steps_product: a diagram applied to the product
state q_M x ... x q_1 (Appendix 1) with the input formed inside the first
pass.  Bit-exact against the oracle (its product state, then its pair-swap
loop) and against the unfused device path (qsim_state_set_product, then
qsim_apply_steps).  All calls go through the C ABI."""
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


def assert_same(a, b, what):
    if a.tobytes() != b.tobytes():
        ua = a.view(np.uint32)
        ub = b.view(np.uint32)
        bad = np.nonzero(ua != ub)[0]
        raise AssertionError(f"{what}: {len(bad)} words differ, first at {bad[:8].tolist()}")


def unit_qubits(rng, M, dt):
    qq = rng.standard_normal((M, 2)) + 1j * rng.standard_normal((M, 2))
    return (qq / np.linalg.norm(qq, axis=1, keepdims=True)).astype(dt)


def signed_steps(rng, M, L, n_ctl):
    tg, cm = W.random_steps(rng, M, L, n_ctl)
    kd = (rng.random(L) < 0.3).astype(np.uint8)
    return tg, cm, kd


def run_both(q, M, dt, qq, tg, cm, kd, tuning):
    """(fused result, unfused result) on the device."""
    code = "c64" if dt == np.complex64 else "c128"
    with q.State(M, code) as s:
        if tuning:
            s.set_tuning(tuning)
        s.write(np.full(1 << M, np.nan, dtype=dt))   # the fused path ignores the current vector
        s.apply_product(qq, tg, cm, stream=0, kind=kd)
        fused = s.read()
        s.set_product(qq, stream=0)
        s.apply(tg, cm, stream=0, kind=kd)
        return fused, s.read()


@pytest.mark.parametrize("seed,M,dt,tuning,signed", [
    (0, 15, np.complex64, {"tile_bits": 8, "small_bits": 5}, False),
    (1, 16, np.complex128, {"tile_bits": 8, "small_bits": 5}, False),
    (2, 17, np.complex64, {"tile_bits": 13}, False),
    (3, 18, np.complex128, {"tile_bits": 12}, False),
    (4, 19, np.complex64, {"tile_bits": 10, "low_bits": 7, "small_bits": 5}, False),
    (5, 20, np.complex64, {"tile_bits": 9, "small_bits": 5, "xcd_swizzle": 1}, True),
    (6, 18, np.complex128, {"tile_bits": 9, "small_bits": 5}, True),
    (7, 21, np.complex64, {"tile_bits": 14}, False),
    (8, 20, np.complex64, {"tile_bits": 11, "plan_search": 3, "small_bits": 5}, True),
    (9, 16, np.complex64, {"tile_bits": 6, "low_bits": 3, "small_bits": 5}, False),
    (10, 19, np.complex128, {"tile_bits": 13, "kernel_variant": 2}, False),
    (11, 22, np.complex64, {}, False),
    # what the first pass stages in LDS: the whole tile, partials down to
    # bit 1 or to bit 2; tiles without address bit 1 fall back to the whole
    # tile or the partials down to bit 1
    (12, 17, np.complex64, {"tile_bits": 13, "product_stage": 1}, True),
    (13, 18, np.complex128, {"tile_bits": 12, "product_stage": 2}, True),
    (14, 20, np.complex64, {"tile_bits": 14, "product_stage": 2}, False),
    (15, 19, np.complex64, {"tile_bits": 9, "low_bits": 2, "small_bits": 5, "product_stage": 3}, True),
    (16, 18, np.complex64, {"tile_bits": 8, "low_bits": 1, "small_bits": 5, "product_stage": 3}, True),
    (17, 17, np.complex128, {"tile_bits": 7, "low_bits": 1, "small_bits": 5, "product_stage": 3}, False),
    (18, 21, np.complex128, {"tile_bits": 13, "kernel_variant": 2, "product_stage": 3}, True),
    (19, 16, np.complex64, {"tile_bits": 14, "product_stage": 1}, False),
    # 2^5-entry tiles (one thread): first tiles that hold the top address bit
    # (seeds 20-22: the product kernel runs first) and one that does not
    (20, 7, np.complex128, {"tile_bits": 5, "low_bits": 1, "small_bits": 5}, False),
    (21, 12, np.complex128, {"tile_bits": 5, "low_bits": 1, "small_bits": 5}, True),
    (22, 11, np.complex64, {"tile_bits": 5, "low_bits": 1, "small_bits": 5}, False),
    (23, 6, np.complex64, {"tile_bits": 5, "low_bits": 1, "small_bits": 4}, True),
])
def test_product_pass_matches_oracle(q, seed, M, dt, tuning, signed):
    rng = np.random.default_rng(900 + seed)
    qq = unit_qubits(rng, M, dt)
    if signed:
        tg, cm, kd = signed_steps(rng, M, 200, (0, 3))
    else:
        (tg, cm), kd = W.random_steps(rng, M, 200, (0, 3)), None
    say("product pass", seed, M, tuning, signed)
    fused, unfused = run_both(q, M, dt, qq, tg, cm, kd, tuning)
    ref = oracle.apply(M, oracle.product_state(M, qq), tg, cm, kind=kd)
    assert_same(fused, ref, f"fused M={M} {tuning}")
    assert_same(unfused, ref, f"unfused M={M} {tuning}")


def assert_same_up_to_nan_payload(a, b, what):
    """Every float part bit-equal, except that a NaN may meet a NaN of another
    payload or sign: IEEE 754 leaves the NaN an operation returns to the
    implementation (the host's x86 units and the GPU pick differently)."""
    fa = a.view(np.float32 if a.dtype == np.complex64 else np.float64)
    fb = b.view(fa.dtype)
    same = fa.view(np.uint32 if fa.dtype == np.float32 else np.uint64) == fb.view(
        np.uint32 if fa.dtype == np.float32 else np.uint64)
    both_nan = np.isnan(fa) & np.isnan(fb)
    bad = np.nonzero(~(same | both_nan))[0]
    if len(bad):
        raise AssertionError(f"{what}: {len(bad)} parts differ, first at {bad[:8].tolist()}")


def test_product_pass_special_values(q):
    """Qubits with infinities, NaN, signed zeros and subnormals: the fused
    first pass forms the same values as the product kernel and the oracle,
    bit for bit apart from NaN payloads; the signed zeros, infinities and
    subnormals that come out of the products match exactly."""
    rng = np.random.default_rng(910)
    M = 18
    qq = unit_qubits(rng, M, np.complex64)
    qq[0, 0] = complex(np.inf, 0.0)
    qq[5, 1] = complex(-0.0, 0.0)
    qq[9, 0] = complex(np.nan, 1.0)
    qq[11, 1] = complex(1e-40, -1e-41)
    qq[16, 0] = complex(-np.inf, np.inf)
    tg, cm = W.random_steps(rng, M, 120, (0, 3))
    fused, unfused = run_both(q, M, np.complex64, qq, tg, cm, None, {"tile_bits": 10, "small_bits": 5})
    ref = oracle.apply(M, oracle.product_state(M, qq), tg, cm)
    fr = ref.view(np.float32)
    assert np.isnan(fr).any() and np.isinf(fr).any() and (fr.view(np.uint32) == 0x80000000).any()
    assert_same_up_to_nan_payload(fused, ref, "fused special values")
    assert_same_up_to_nan_payload(unfused, ref, "unfused special values")
    assert_same_up_to_nan_payload(fused, unfused, "fused against unfused")


def test_product_pass_signed_zeros_and_subnormals(q):
    """Without NaN among the qubits every part matches bit for bit,
    including -0.0, infinities and subnormal products."""
    rng = np.random.default_rng(911)
    M = 17
    qq = unit_qubits(rng, M, np.complex64)
    qq[2, 1] = complex(-0.0, -0.0)
    qq[6, 0] = complex(3e-20, -2e-20)
    qq[7, 1] = complex(1e-19, 5e-20)
    qq[12, 0] = complex(1e15, -0.0)
    qq[14, 1] = complex(2e5, 1e6)
    tg, cm = W.random_steps(rng, M, 120, (0, 3))
    fused, unfused = run_both(q, M, np.complex64, qq, tg, cm, None, {"tile_bits": 9, "small_bits": 5})
    ref = oracle.apply(M, oracle.product_state(M, qq), tg, cm)
    fr = ref.view(np.float32)
    assert not np.isnan(fr).any() and (fr.view(np.uint32) == 0x80000000).any()
    assert ((np.abs(fr) < np.finfo(np.float32).tiny) & (fr != 0)).any(), "no subnormal product"
    assert_same(fused, ref, "fused")
    assert_same(unfused, ref, "unfused")


@pytest.mark.parametrize("M,dt,tuning,L", [
    (3, np.complex64, None, 10),                          # per-row walk
    (12, np.complex128, None, 40),                        # whole state in one workgroup
    (17, np.complex64, {"rows_per_thread": 16}, 60),      # 16 rows per thread: product kernel first
    (16, np.complex64, None, 0),                          # no steps: the product state itself
])
def test_product_unfused_paths(q, M, dt, tuning, L):
    """Where the first pass is not a one-tile-per-workgroup pass with 32 rows
    per thread the entry point runs the product kernel and then the diagram;
    the result is the same."""
    rng = np.random.default_rng(920 + M)
    qq = unit_qubits(rng, M, dt)
    tg, cm = W.random_steps(rng, M, L, (0, 3))
    say("product unfused", M, tuning, L)
    fused, unfused = run_both(q, M, dt, qq, tg, cm, None, tuning)
    ref = oracle.apply(M, oracle.product_state(M, qq), tg, cm)
    assert_same(fused, ref, "entry point")
    assert_same(unfused, ref, "set_product + apply")


def test_product_pass_rejects_bad_arguments(q):
    with q.State(16, "c64") as s:
        with pytest.raises(ValueError):
            s.apply_product(np.zeros((15, 2), dtype=np.complex64), [0], [0])
        with pytest.raises(q.QsimError):
            s.apply_product(np.zeros((16, 2), dtype=np.complex64), [16], [0])   # target >= M


@pytest.mark.parametrize("signed", [False, True])
def test_product_pass_m32_sampled(q, signed):
    """The M=32 complex64 diagram (L=1000) on a unit-norm product state:
    sampled rows against the oracle (source row of each sampled row, then
    the product formula for that row, negated where the signed walk says)."""
    import torch
    M = 32
    rng = np.random.default_rng(930 + int(signed))
    qq = unit_qubits(rng, M, np.complex64)
    tg, cm = W.m32_config()
    kd = (np.arange(len(tg)) % 4 == 3).astype(np.uint8) if signed else None
    torch.cuda.empty_cache()
    b0 = torch.empty(1 << M, dtype=torch.complex64, device="cuda")
    b1 = torch.empty_like(b0)
    s = q.State(M, "c64", buffers=(b0, b1))
    say("product pass m32", signed)
    s.apply_product(qq, tg, cm, kind=kd)
    torch.cuda.synchronize()
    cur = b0 if s.current_ptr() == b0.data_ptr() else b1
    rows = np.concatenate([rng.integers(0, 1 << M, size=200, dtype=np.uint64), [0, 1, (1 << M) - 1]])
    got = cur[torch.from_numpy(rows.astype(np.int64)).cuda()].cpu().numpy()
    for r, g in zip(rows.tolist(), got):
        if signed:
            x, neg = oracle.source_index_signed(M, tg, cm, kd, r)
        else:
            x, neg = oracle.source_index(M, tg, cm, r), False
        want = np.asarray(oracle.product_entry(M, qq, x), dtype=np.complex64).reshape(1)
        if neg:
            want = (want.view(np.uint32) ^ np.uint32(0x80000000)).view(np.complex64)
        assert g.tobytes() == want.tobytes(), f"row {r}"
    s.close()
    del b0, b1, cur
    torch.cuda.empty_cache()
