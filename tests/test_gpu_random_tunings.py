"""Seeded random combinations of the launch parameters (qsim_tuning: tile
size, rows per thread, forced low bits of the first/last and middle passes,
kernel shape, permuted layouts, planner search, XCD order, tile order,
small-state cut-off, what the product pass stages), each value inside the
range the library accepts, on random diagrams of M = 6..20 with and without
phase steps, complex64 and complex128.  Every combination applies its
diagram to a Gaussian state and to a product state (the input formed inside
the first pass) and must equal the oracle bit for bit.  Persistent kernels
and fewer than 32 rows per thread are drawn only with tiles of 2^9 entries
and more, the shapes those options are built for."""
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

N_CASES = 60


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


def draw(rng):
    dt = "c64" if rng.random() < 0.6 else "c128"
    kmax = 14 if dt == "c64" else 13
    M = int(rng.integers(6, 21))
    tb = int(rng.integers(5, kmax + 1))
    big = tb >= 9
    t = {"tile_bits": tb, "rows_per_thread": int(rng.choice([8, 16, 32])) if big else 32,
         "low_bits": int(rng.integers(1, min(tb, 7) + 1)),
         "kernel_variant": int(rng.choice([1, 2, 3])) if big else 1, "remap": int(rng.choice([1, 2])),
         "plan_search": int(rng.choice([1, 2, 3])), "xcd_swizzle": int(rng.choice([1, 2])),
         "outer_order": int(rng.choice([1, 2])), "small_bits": int(rng.integers(4, tb + 1)),
         "product_stage": int(rng.choice([1, 2, 3]))}
    t["mid_low_bits"] = int(rng.integers(1, t["low_bits"] + 1))
    return M, dt, t


def test_random_tunings_match_oracle(q):
    rng = np.random.default_rng(4242)
    ran = 0
    for case in range(N_CASES):
        M, dt, t = draw(rng)
        npdt = np.complex64 if dt == "c64" else np.complex128
        L = int(rng.integers(20, 250))
        tg, cm = W.random_steps(rng, M, L, (0, 3))
        kd = (rng.random(L) < 0.25).astype(np.uint8) if rng.random() < 0.5 else None
        try:
            q.plan_describe(M, dt, tg, cm, t, kind=kd)
        except q.QsimError:
            continue   # a combination the planner rejects (host only, nothing ran)
        k1 = W.gaussian_state(rng, M, npdt)
        qq = rng.standard_normal((M, 2)) + 1j * rng.standard_normal((M, 2))
        qq = (qq / np.linalg.norm(qq, axis=1, keepdims=True)).astype(npdt)
        say("case", case, M, dt, L, kd is not None, t)
        with q.State(M, dt) as s:
            s.set_tuning(t)
            s.write(k1)
            s.apply(tg, cm, kind=kd, stream=0)
            got = s.read()
            assert got.tobytes() == oracle.apply(M, k1, tg, cm, kind=kd).tobytes(), f"case {case}: apply"
            s.apply_product(qq, tg, cm, kind=kd, stream=0)
            got = s.read()
            ref = oracle.apply(M, oracle.product_state(M, qq), tg, cm, kind=kd)
            assert got.tobytes() == ref.tobytes(), f"case {case}: product-input apply"
        ran += 1
    assert ran >= N_CASES * 0.9, ran
