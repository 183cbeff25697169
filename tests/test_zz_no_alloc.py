"""qsim_apply_steps_noalloc (the entry point for callers that cannot allocate
device memory) against qsim_apply_steps: the same result bit for bit, on
two calls in a row (the second on a smaller state, so it reuses scratch the
first one filled), on the small-state and direct paths, and a diagram whose
plan and tile records exceed the scratch is rejected with nothing run; and
the allocation-free apply captured into a HIP graph and replayed."""
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


def _pair(q, M, dt, k1, tg, cm, kind=None, tuning=None):
    """(regular result, allocation-free result) of one diagram on k1."""
    code = "c64" if dt == np.complex64 else "c128"
    out = []
    for noalloc in (False, True):
        with q.State(M, code) as s:
            if tuning:
                s.set_tuning(tuning)
            s.write(k1)
            if noalloc:
                s.apply_noalloc(tg, cm, stream=0, kind=kind)
            else:
                s.apply(tg, cm, stream=0, kind=kind)
            out.append(s.read())
    return out


def test_noalloc_matches_apply_twice_smaller_second(q):
    rng = np.random.default_rng(7001)
    cases = [(22, np.complex64, 400, None), (17, np.complex128, 150, {"tile_bits": 9, "small_bits": 5})]
    for M, dt, L, tuning in cases:
        tg, cm = W.random_steps(rng, M, L, (0, 3))
        kd = (rng.random(L) < 0.2).astype(np.uint8)
        k1 = W.gaussian_state(rng, M, dt)
        say("noalloc", M, dt.__name__, L, tuning)
        ref, got = _pair(q, M, dt, k1, tg, cm, kind=kd, tuning=tuning)
        assert ref.tobytes() == got.tobytes(), f"noalloc differs from apply at M={M}"
        assert got.tobytes() == oracle.apply(M, k1, tg, cm, kind=kd).tobytes(), f"noalloc vs oracle M={M}"


def test_noalloc_small_and_direct_paths(q):
    rng = np.random.default_rng(7002)
    for M, dt in ((13, np.complex64), (3, np.complex128)):
        tg, cm = W.random_steps(rng, M, 60, (0, 2))
        k1 = W.gaussian_state(rng, M, dt)
        say("noalloc small", M)
        ref, got = _pair(q, M, dt, k1, tg, cm)
        assert ref.tobytes() == got.tobytes()


def test_noalloc_same_stream_back_to_back(q):
    """Two allocation-free applies queued on one stream without waiting in
    between (the second diagram's plan overwrites the first's in the shared
    scratch only after the first's kernels in stream order): the second
    undoes the first."""
    rng = np.random.default_rng(7003)
    M = 21
    tg, cm = W.random_steps(rng, M, 300, (0, 3))
    k1 = W.gaussian_state(rng, M, np.complex64)
    with q.State(M, "c64") as s:
        s.write(k1)
        say("noalloc back to back")
        s.apply_noalloc(tg, cm, stream=0)
        s.apply_noalloc(tg[::-1].copy(), cm[::-1].copy(), stream=0)
        assert s.read().tobytes() == k1.tobytes()


def test_noalloc_rejects_plan_beyond_scratch(q):
    """M=28 with 32-entry tiles: 2^23 tiles of 8-byte records need more than
    the 64 MiB scratch; the call fails with QSIM_ERR_NOMEM and the state is
    unchanged (nothing was enqueued)."""
    import torch
    M = 28
    rng = np.random.default_rng(7004)
    tg, cm = W.random_steps(rng, M, 20, (1, 2))
    k1 = W.gaussian_state_torch(M, "c64", seed=7005)
    b1 = torch.empty_like(k1)
    keep = k1.clone()
    s = q.State(M, "c64", buffers=(k1, b1))
    s.set_tuning({"tile_bits": 5, "small_bits": 5})
    say("noalloc beyond scratch")
    with pytest.raises(q.QsimError) as ei:
        s.apply_noalloc(tg, cm)
    assert ei.value.code == q.ERR_NOMEM and "scratch" in q.last_error()
    torch.cuda.synchronize()
    assert s.current_ptr() == k1.data_ptr()
    assert torch.equal(k1.view(torch.int64), keep.view(torch.int64))
    s.close()


def test_noalloc_apply_replays_in_a_graph(q):
    """The allocation-free apply enqueues kernels only (the plan travels in
    kernel arguments into the scratch array; no copy, fill or wait), so it
    can be captured into a HIP graph and replayed.  Each replay applies the
    diagram again to the buffers the capture saw; with an even number of
    passes the result lands in the buffer the first pass reads, so replay r
    gives U^r k1.  Every replay is checked against the eager applies, with
    eager work and a synchronisation between replays."""
    import torch
    M = 20
    tg = cm = None
    for seed in range(100):
        t_, c_ = W.random_steps(np.random.default_rng(3000 + seed), M, 300, (0, 3))
        if len(q.plan_describe(M, "c64", t_, c_)[0]) % 2 == 0:
            tg, cm = t_, c_
            break
    assert tg is not None
    k1 = W.gaussian_state(np.random.default_rng(2020), M, np.complex64)
    with q.State(M, "c64") as s:
        s.write(k1)
        refs = []
        for _ in range(3):                      # eager (also resolves the scratch address)
            s.apply_noalloc(tg, cm, stream=0)
            refs.append(s.read())
        assert refs[0].tobytes() == oracle.apply(M, k1, tg, cm).tobytes()
        s.write(k1)
        torch.cuda.synchronize()
        say("graph capture")
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            s.apply_noalloc(tg, cm)             # on the capture stream; nothing runs yet
        torch.cuda.synchronize()
        for r in range(3):
            say("graph replay", r)
            g.replay()
            torch.cuda.synchronize()
            assert s.read().tobytes() == refs[r].tobytes(), f"replay {r} differs from eager apply {r + 1}"
            x = torch.randn(1 << 16, device="cuda")   # eager work between replays
            assert torch.isfinite(x.sum()).item()
            torch.cuda.synchronize()
        del g
