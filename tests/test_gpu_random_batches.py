"""Seeded random batched-mode settings (qsim_batch_tuning: tiles per queue
item, batch tile size, whole-circuit cut-off, planning, queue order), each
inside the range the library accepts, on random batches of circuits (M =
3..19, L = 0..150, complex64 and complex128, with and without phase steps):
every circuit's result equals the oracle's bit for bit."""
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

N_CASES = 16


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
    t = {"tiles_per_item": int(rng.choice([1, 2, 3, 5, 8, 16, 32, 64, 100, 256])),
         "tile_bits": int(rng.integers(10, 14 if dt == "c64" else 13)),
         "circuit_tiles": int(rng.choice([1, 2, 4, 8, 16, 32, 64, 128, 256])),
         "plan_search": int(rng.choice([1, 2])), "order": int(rng.choice([1, 2]))}
    return dt, t


def test_random_batch_settings_match_oracle(q):
    rng = np.random.default_rng(5151)
    for case in range(N_CASES):
        dt, t = draw(rng)
        npd = np.complex64 if dt == "c64" else np.complex128
        circuits = W.batched_config(n=30, seed=5200 + case, m_range=(3, 19), l_range=(0, 150))
        signed = rng.random() < 0.5
        kinds = [(rng.random(c.L) < 0.2).astype(np.uint8) if signed else None for c in circuits]
        states, ins = [], []
        for c in circuits:
            k1 = W.gaussian_state(rng, c.M, npd)
            s = q.State(c.M, dt)
            s.write(k1)
            states.append(s)
            ins.append(k1)
        say("batch case", case, dt, t, "signed" if signed else "")
        try:
            q.batch_set_tuning(dt, t)
            q.apply_batch(states, [(c.target, c.cmask, kd) for c, kd in zip(circuits, kinds)], stream=0)
            q.batch_status()
            for c, s, k1, kd in zip(circuits, states, ins, kinds):
                ref = oracle.apply(c.M, k1, c.target, c.cmask, kind=kd)
                assert s.read().tobytes() == ref.tobytes(), f"case {case} {t}: circuit M={c.M} L={c.L}"
        finally:
            q.batch_set_tuning(dt, None)
            for s in states:
                s.close()
