"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no part of the method's arithmetic: it only draws step lists
(target bit, control mask) and initial state vectors.  Both the CPU oracle and
the GPU library receive exactly what it produces.

Workloads (shapes follow the paper's problem statement: a 2^M-entry complex
state of arbitrary magnitude and phase, Sec. 1, and a wiring diagram of
controlled NOTs, Sec. 2):

* ``small``   M=10, complex128, L=20 steps with one control each; input either
               the paper's alternating +|S|, -|S| vector (Sec. 2(b), Sec. 4)
               or a random-phase vector of the same magnitude.
* ``m26``     M=26, complex128 unit-norm Gaussian, L=200, 0..4 controls.
* ``m32``     M=32, complex64 unit-norm Gaussian, L=1000, 1..3 controls; 500
               steps target bits 0..7 and 500 target bits 8..31, interleaved
               in a seeded random order.
* ``batched`` 4096 circuits, M uniform in 8..20, L uniform in 10..500,
               0..3 controls, complex64.
* ``served``  Poisson arrivals, M log-uniform over [12, 29) floored, L uniform
               in 50..2000, 0..3 controls, complex64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np

Steps = Tuple[np.ndarray, np.ndarray]  # (target uint32[L], cmask uint64[L])

SEED_SMALL = 10
SEED_M26 = 26
SEED_M32 = 32
SEED_BATCHED = 4096
SEED_SERVED = 2028
SERVED_RATE = 122.0  # requests per second: 0.8 x the one-at-a-time capacity on MI355X for the
                     # first 1000 requests of the trace (152.4-153.2 req/s)
SERVED_REQUESTS = 1000


def random_steps(rng: np.random.Generator, M: int, L: int, n_ctl: Tuple[int, int],
                 targets: Optional[Sequence[int]] = None) -> Steps:
    """L steps; step s targets ``targets[s]`` (or a uniform bit of [0, M)) and
    has a number of controls uniform in [n_ctl[0], n_ctl[1]], drawn without
    replacement from the other M-1 bits."""
    lo, hi = n_ctl
    hi = min(hi, M - 1)
    lo = min(lo, hi)
    tgt = np.empty(L, dtype=np.uint32)
    cm = np.zeros(L, dtype=np.uint64)
    for s in range(L):
        t = int(rng.integers(0, M)) if targets is None else int(targets[s])
        n = int(rng.integers(lo, hi + 1))
        others = np.array([b for b in range(M) if b != t], dtype=np.int64)
        picks = rng.choice(others, size=n, replace=False) if n > 0 else []
        c = 0
        for b in picks:
            c |= 1 << int(b)
        tgt[s] = t
        cm[s] = c
    return tgt, cm


def empty_steps() -> Steps:
    return np.zeros(0, dtype=np.uint32), np.zeros(0, dtype=np.uint64)


# ---------------------------------------------------------------- states (host)

def alternating_state(M: int, dtype=np.complex128) -> np.ndarray:
    """The paper's input k1 = |S| (1, -1, 1, -1, ...)' with |S| = 2^(-M/2)
    (Sec. 2(b), Sec. 4)."""
    s = 2.0 ** (-M / 2.0)
    v = np.empty(1 << M, dtype=dtype)
    v[0::2] = s
    v[1::2] = -s
    return v


def random_phase_state(rng: np.random.Generator, M: int, dtype=np.complex128) -> np.ndarray:
    """|S| e^{i theta_j} with theta_j uniform in [0, 2 pi)."""
    th = rng.uniform(0.0, 2.0 * math.pi, size=1 << M)
    return (2.0 ** (-M / 2.0) * np.exp(1j * th)).astype(dtype)


def gaussian_state(rng: np.random.Generator, M: int, dtype=np.complex64) -> np.ndarray:
    """i.i.d. standard complex Gaussian entries scaled to unit 2-norm."""
    n = 1 << M
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    v /= np.sqrt(np.sum(np.abs(v) ** 2))
    return v.astype(dtype)


def tag_state(M: int, dtype=np.complex64) -> np.ndarray:
    """Entry j carries the raw integer j in its bytes (an address tag), so any
    misplaced entry is visible exactly.  complex128 entries carry (j, ~j)."""
    n = 1 << M
    if dtype == np.complex64:
        return np.arange(n, dtype=np.uint64).view(np.complex64)
    w = np.empty(2 * n, dtype=np.uint64)
    w[0::2] = np.arange(n, dtype=np.uint64)
    w[1::2] = ~np.arange(n, dtype=np.uint64)
    return w.view(np.complex128)


def special_values_state(rng: np.random.Generator, M: int, dtype=np.complex64) -> np.ndarray:
    """Random raw bit patterns: NaN payloads, infinities, -0.0 and subnormals
    all occur; a path that moves entries through floating-point registers with
    canonicalisation would change some of them."""
    n = 1 << M
    words = rng.integers(0, 2**63, size=n * (1 if dtype == np.complex64 else 2),
                         dtype=np.uint64, endpoint=False)
    words ^= rng.integers(0, 2, size=words.shape, dtype=np.uint64) << np.uint64(63)
    return words.view(dtype)


# ---------------------------------------------------------------- states (device)

def unit_qubits(M: int, dtype=np.complex64, seed: int = SEED_M32) -> np.ndarray:
    """M seeded qubit pairs (q_b(0), q_b(1)), each a unit-norm complex
    Gaussian 2-vector, as an (M, 2) array: the factors of a product-state
    input (row b-1 holds q_b)."""
    rng = np.random.default_rng(seed)
    qq = rng.standard_normal((M, 2)) + 1j * rng.standard_normal((M, 2))
    return (qq / np.linalg.norm(qq, axis=1, keepdims=True)).astype(dtype)


def gaussian_state_torch(M: int, dtype: str, seed: int, device="cuda"):
    """Unit-norm complex Gaussian state generated where it will live (torch's
    seeded generator); used for sizes whose host generation would be slow.
    The bytes are read back when the oracle needs them."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    fdt = torch.float32 if dtype == "c64" else torch.float64
    n = 1 << M
    v = torch.empty(n, 2, dtype=fdt, device=device)
    chunk = 1 << 26
    for off in range(0, n, chunk):
        m = min(chunk, n - off)
        v[off:off + m].normal_(generator=g)
    nrm = torch.zeros((), dtype=torch.float64, device=device)
    for off in range(0, n, chunk):
        m = min(chunk, n - off)
        nrm += v[off:off + m].double().square().sum()
    v.div_(nrm.sqrt().to(fdt))
    return torch.view_as_complex(v)


def gaussian_states_grouped_torch(Ms: Sequence[int], dtype: str, seed: int, device="cuda"):
    """One unit-norm complex Gaussian state per entry of ``Ms`` (torch's seeded
    generator), drawn per distinct size as one (count, 2^M) tensor, so a
    batch of thousands of states takes a few dozen kernel launches.  Returns
    (states, spares): row views in the order of ``Ms`` and an uninitialised
    buffer of the same size for each."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    fdt = torch.float32 if dtype == "c64" else torch.float64
    states: List = [None] * len(Ms)
    spares: List = [None] * len(Ms)
    for m in sorted(set(int(x) for x in Ms)):
        idx = [i for i, x in enumerate(Ms) if int(x) == m]
        v = torch.empty(len(idx), 1 << m, 2, dtype=fdt, device=device)
        v.normal_(generator=g)
        nrm = v.double().square().sum(dim=(1, 2), keepdim=True).sqrt()
        v.div_(nrm.to(fdt))
        c = torch.view_as_complex(v)
        sp = torch.empty_like(c)
        for r, i in enumerate(idx):
            states[i] = c[r]
            spares[i] = sp[r]
    return states, spares


# ---------------------------------------------------------------- configurations

def small_config(seed: int = SEED_SMALL, M: int = 10, L: int = 20) -> Steps:
    """L steps, each a NOT on a uniform target with exactly one distinct control."""
    return random_steps(np.random.default_rng(seed), M, L, (1, 1))


def m26_config(seed: int = SEED_M26, M: int = 26, L: int = 200) -> Steps:
    return random_steps(np.random.default_rng(seed), M, L, (0, 4))


def m32_config(seed: int = SEED_M32, M: int = 32, L: int = 1000, n_low_bits: int = 8,
               blocked: bool = False) -> Steps:
    """Half the steps target bits [0, n_low_bits), the rest [n_low_bits, M),
    interleaved in a seeded random order; 1..3 controls.  blocked=True: the
    same draws with the low-target half first, then the high-target half."""
    rng = np.random.default_rng(seed)
    half = L // 2
    kinds = np.array([0] * half + [1] * (L - half))
    rng.shuffle(kinds)
    if blocked:
        kinds = np.sort(kinds, kind="stable")
    targets = [int(rng.integers(0, n_low_bits)) if k == 0 else int(rng.integers(n_low_bits, M))
               for k in kinds]
    return random_steps(rng, M, L, (1, 3), targets=targets)


@dataclass
class Circuit:
    M: int
    target: np.ndarray
    cmask: np.ndarray
    seed: int

    @property
    def L(self) -> int:
        return int(len(self.target))


def batched_config(n: int = 4096, seed: int = SEED_BATCHED, m_range=(8, 20),
                   l_range=(10, 500), n_ctl=(0, 3)) -> List[Circuit]:
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        M = int(rng.integers(m_range[0], m_range[1] + 1))
        L = int(rng.integers(l_range[0], l_range[1] + 1))
        cs = int(rng.integers(0, 2**31))
        t, c = random_steps(np.random.default_rng(cs), M, L, n_ctl)
        out.append(Circuit(M, t, c, cs))
    return out


@dataclass
class Request:
    arrival_s: float
    circuit: Circuit


def served_trace(n: int, rate_per_s: float, seed: int = SEED_SERVED, m_range=(12, 28),
                 l_range=(50, 2000), n_ctl=(0, 3)) -> List[Request]:
    """Poisson arrivals at ``rate_per_s``; M drawn log-uniformly over
    [m_lo, m_hi + 1) and floored, i.e. P(M = m) proportional to ln((m+1)/m)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    lo, hi = m_range
    for _ in range(n):
        t += float(rng.exponential(1.0 / rate_per_s))
        M = int(math.floor(math.exp(rng.uniform(math.log(lo), math.log(hi + 1)))))
        M = max(lo, min(hi, M))
        L = int(rng.integers(l_range[0], l_range[1] + 1))
        cs = int(rng.integers(0, 2**31))
        tg, cm = random_steps(np.random.default_rng(cs), M, L, n_ctl)
        out.append(Request(t, Circuit(M, tg, cm, cs)))
    return out


def parity_circuit(M: int) -> Steps:
    """The wiring diagram of the paper's computational example (Sec. 4): the
    parity of qubits 2..M targeted to the bottom qubit, one controlled NOT per
    qubit j = 2..M with control a(j) and target a(1)."""
    tgt = np.zeros(M - 1, dtype=np.uint32)
    cm = np.array([1 << j for j in range(1, M)], dtype=np.uint64)
    return tgt, cm
