"""Property tests (hypothesis) over random wiring diagrams: M up to 12, L up
to 64, 0..4 controls per step, complex64 and complex128, with and without
phase steps, and the planner's edge cases forced (tiles as large as the
state, every step on the low bits, every step on the high bits).

CPU: the oracle's algebra (each step matrix is its own inverse, Sec. 2(a);
every step permutes the rows, and a phase step only flips signs) and the
planner's reordering (the plan's step order, applied by the oracle, gives
the result of the original order: only commuting steps change places,
Sec. 2(i)).  GPU: the library against the oracle, bit for bit, with the
fused tile path forced at these small sizes."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
import workloads as W

SETTINGS = dict(deadline=None, derandomize=True, database=None,
                suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])


@st.composite
def diagrams(draw, min_M=2, max_M=12, max_L=64):
    """(M, target, cmask, kind): the step targets and controls drawn from all
    bits, from the low half only or from the high half only."""
    M = draw(st.integers(min_M, max_M))
    L = draw(st.integers(0, max_L))
    region = draw(st.sampled_from(["all", "low", "high"]))
    lo, hi = {"all": (0, M), "low": (0, min(M, max(2, M // 2))), "high": (M // 2, M)}[region]
    if hi - lo < 2:
        lo, hi = 0, M
    tg = np.zeros(L, dtype=np.uint32)
    cm = np.zeros(L, dtype=np.uint64)
    for s in range(L):
        t = draw(st.integers(lo, hi - 1))
        ctl = draw(st.lists(st.integers(lo, hi - 1), max_size=4))
        mask = 0
        for c in ctl:
            if c != t:
                mask |= 1 << c
        tg[s], cm[s] = t, mask
    signed = draw(st.booleans())
    kind = np.array([draw(st.integers(0, 3)) == 0 for _ in range(L)], dtype=np.uint8) if signed else None
    return M, tg, cm, kind


@st.composite
def tile_sizes(draw, M, code):
    """log2 of the tile: most draws split the state into several tiles (and
    so several passes), some take a tile at least as large as the state."""
    cut = draw(st.integers(0, 7))
    top = 14 if code == "c64" else 13
    return top if cut == 0 else min(top, max(5, M - cut))


def _state(M, dt, seed):
    return W.gaussian_state(np.random.default_rng(seed), M, dt)


@settings(max_examples=150, **SETTINGS)
@given(diagrams(max_M=10), st.sampled_from([np.complex64, np.complex128]), st.integers(0, 2**31))
def test_oracle_diagram_then_reverse_is_identity(d, dt, seed):
    M, tg, cm, kd = d
    k1 = _state(M, dt, seed)
    k2 = oracle.apply(M, k1, tg, cm, kind=kd)
    back = oracle.apply(M, k2, tg[::-1].copy(), cm[::-1].copy(), kind=None if kd is None else kd[::-1].copy())
    assert back.tobytes() == k1.tobytes()


@settings(max_examples=150, **SETTINGS)
@given(diagrams(max_M=10), st.integers(0, 2**31))
def test_oracle_permutes_rows_up_to_sign(d, seed):
    """The result holds the input's entries, each once, some negated (and
    none negated without phase steps): sort by magnitude and compare."""
    M, tg, cm, kd = d
    k1 = _state(M, np.complex128, seed)
    k2 = oracle.apply(M, k1, tg, cm, kind=kd)
    key = lambda v: np.sort(np.abs(v.real) * 3 + np.abs(v.imag))
    assert np.array_equal(key(k2), key(k1))
    if kd is None or not kd.any():
        assert np.array_equal(np.sort_complex(k2), np.sort_complex(k1))


@settings(max_examples=150, **SETTINGS)
@given(diagrams(min_M=6), st.sampled_from(["c64", "c128"]), st.data(), st.integers(1, 5),
       st.sampled_from([1, 2, 3]), st.integers(0, 2**31))
def test_planner_order_is_exact(d, code, data, low_bits, search, seed):
    from paper_quant_ph_0308158_amd import qsim
    M, tg, cm, kd = d
    tile_bits = data.draw(tile_sizes(M, code))
    tuning = {"tile_bits": tile_bits, "low_bits": min(low_bits, tile_bits), "small_bits": 4, "plan_search": search}
    try:
        masks, lens, order = qsim.plan_describe(M, code, tg, cm, tuning, kind=kd)
    except qsim.QsimError:
        return   # a combination the library rejects outright (nothing to compare)
    L = len(tg)
    assert sorted(order[:L].tolist()) == list(range(L))
    assert sum(int(x) for x in lens) == L
    o = order[:L].astype(np.int64)
    k1 = _state(M, np.complex128, seed)
    want = oracle.apply(M, k1, tg, cm, kind=kd)
    got = oracle.apply(M, k1, tg[o], cm[o], kind=None if kd is None else kd[o])
    assert got.tobytes() == want.tobytes()


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_quant_ph_0308158_amd import qsim
    return qsim


@pytest.mark.gpu
def test_library_matches_oracle_property(q):
    """Random diagrams through the fused tile path (small_bits 4 forces it
    at every M above 4; tile sizes up to the whole state), on a Gaussian
    state and on a product state formed inside the first pass, against the
    oracle bit for bit."""

    @settings(max_examples=200, **SETTINGS)
    @given(diagrams(), st.sampled_from([np.complex64, np.complex128]), st.data(),
           st.integers(1, 5), st.integers(0, 2**31))
    def check(d, dt, data, low_bits, seed):
        M, tg, cm, kd = d
        code = "c64" if dt == np.complex64 else "c128"
        tile_bits = data.draw(tile_sizes(M, code))
        tuning = {"tile_bits": tile_bits, "low_bits": min(low_bits, tile_bits), "small_bits": 4}
        try:
            q.plan_describe(M, code, tg, cm, tuning, kind=kd)
        except q.QsimError:
            return
        k1 = _state(M, dt, seed)
        with q.State(M, code) as s:
            s.set_tuning(tuning)
            s.write(k1)
            s.apply(tg, cm, kind=kd, stream=0)
            got = s.read()
            assert got.tobytes() == oracle.apply(M, k1, tg, cm, kind=kd).tobytes()
            rng = np.random.default_rng(seed)
            qq = rng.standard_normal((M, 2)) + 1j * rng.standard_normal((M, 2))
            qq = (qq / np.linalg.norm(qq, axis=1, keepdims=True)).astype(dt)
            s.apply_product(qq, tg, cm, kind=kd, stream=0)
            got = s.read()
        ref = oracle.apply(M, oracle.product_state(M, qq), tg, cm, kind=kd)
        assert got.tobytes() == ref.tobytes()

    check()


@pytest.mark.gpu
def test_batch_matches_oracle_property(q):
    """Random batches (1..10 circuits of M = 1..15, L = 0..48, each circuit's
    steps on all, low or high bits) under random batched-mode settings, so
    that one batch mixes per-row circuits, circuits whole in LDS, whole
    multi-pass circuits and tile blocks: every circuit equals the oracle."""

    @settings(max_examples=100, **SETTINGS)
    @given(st.lists(diagrams(min_M=1, max_M=15, max_L=48), min_size=1, max_size=10),
           st.sampled_from(["c64", "c128"]), st.integers(10, 13), st.sampled_from([1, 2, 4, 8, 32]),
           st.sampled_from([1, 2, 64]), st.sampled_from([1, 2]), st.integers(0, 2**31))
    def check(batch, code, tile_bits, tpi, ctiles, order, seed):
        dt = np.complex64 if code == "c64" else np.complex128
        tuning = {"tile_bits": min(tile_bits, 13 if code == "c64" else 12), "tiles_per_item": tpi,
                  "circuit_tiles": ctiles, "order": order}
        rng = np.random.default_rng(seed)
        states, ins = [], []
        try:
            for M, tg, cm, kd in batch:
                k1 = W.gaussian_state(rng, M, dt)
                s = q.State(M, code)
                s.write(k1)
                states.append(s)
                ins.append(k1)
            q.batch_set_tuning(code, tuning)
            q.apply_batch(states, [(tg, cm, kd) for _, tg, cm, kd in batch], stream=0)
            q.batch_status()
            for (M, tg, cm, kd), s, k1 in zip(batch, states, ins):
                assert s.read().tobytes() == oracle.apply(M, k1, tg, cm, kind=kd).tobytes(), (M, len(tg), tuning)
        finally:
            q.batch_set_tuning(code, None)
            for s in states:
                s.close()

    check()
