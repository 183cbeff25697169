"""Pins of the CPU oracle to facts other than itself (CPU only).

* the paper's printed worked examples (tests/golden/paper_examples.txt);
* a dense brute force that builds every step matrix from Kronecker products
  (bit order fixed by the Appendix 1 example) and multiplies them;
* invariants: involution, conservation of the multiset of entries and of the
  norm, split associativity, commutation of non-interfering steps;
* the closed form of the paper's own computational example (Sec. 4);
* signed steps (controlled phase -1): the paper's printed signed example
  matrix (Sec. 2(a)) reproduced by a four-step diagram, dense brute force
  with signed step matrices, involution and sign-bit exactness;
* mutation checks: plausible mistakes, planted in pure-Python variants of the
  oracle's loop, each fail at least one of the pins above.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from tests._golden import load_examples

EXAMPLES = load_examples()


def tags_of(state: np.ndarray) -> np.ndarray:
    return state.view(np.uint64) if state.dtype == np.complex64 else state.view(np.uint64)[0::2]


# ------------------------------------------------------------------ paper examples

@pytest.mark.parametrize("name", sorted(EXAMPLES))
def test_paper_example(name):
    ex = EXAMPLES[name]
    M, tg, cm = ex["M"], ex["target"], ex["cmask"]
    if "expect_src" in ex:
        for dt in (np.complex64, np.complex128):
            k2 = oracle.apply(M, W.tag_state(M, dt), tg, cm)
            np.testing.assert_array_equal(tags_of(k2), ex["expect_src"], err_msg=ex["cite"])
            k2e = oracle.apply(M, W.tag_state(M, dt), tg, cm, method="enum")
            np.testing.assert_array_equal(tags_of(k2e), ex["expect_src"], err_msg=ex["cite"])
    if "expect_sign" in ex:
        assert ex["input"] == "alt"
        k1 = W.alternating_state(M)
        k2 = oracle.apply(M, k1, tg, cm)
        s = 2.0 ** (-M / 2)
        np.testing.assert_array_equal(k2.real, ex["expect_sign"] * s)
        np.testing.assert_array_equal(k2.imag, 0.0)
    if "pairs" in ex:
        assert len(tg) == 1
        src = tags_of(oracle.apply(M, W.tag_state(M), tg, cm))
        pairs = sorted((int(i), int(src[i])) for i in range(1 << M) if src[i] > i)
        assert pairs == ex["pairs"], ex["cite"]
    if "rowmap_1based_prefix" in ex:
        x = oracle.rowmap(M, tg, cm)
        pre = ex["rowmap_1based_prefix"]
        assert [int(v) + 1 for v in x[:len(pre)]] == pre, ex["cite"]
        # The paper folds x <- y(x) in step order, which is the row map of
        # U_1 U_2 ... U_n; k2 = U_n ... U_1 k1 therefore equals k1 gathered
        # through the row map of the reversed list.
        xr = oracle.rowmap(M, tg[::-1], cm[::-1])
        k2 = oracle.apply(M, W.tag_state(M), tg, cm)
        np.testing.assert_array_equal(tags_of(k2), xr)


def test_fig2_order_matters_off_palindrome():
    """A non-palindromic two-step circuit separates the two composition orders
    (reading of Sec. 2(a)/(h): steps[0] acts first)."""
    M = 2
    tg = np.array([1, 0], dtype=np.uint32)
    cm = np.array([0b01, 0b10], dtype=np.uint64)
    src = tags_of(oracle.apply(M, W.tag_state(M), tg, cm))
    # (a, b, c, d) -> (a, d, b, c): worked by hand from the two step matrices.
    np.testing.assert_array_equal(src, [0, 3, 1, 2])
    src_rev = tags_of(oracle.apply(M, W.tag_state(M), tg[::-1], cm[::-1]))
    np.testing.assert_array_equal(src_rev, [0, 2, 3, 1])


# ------------------------------------------------------------------ dense brute force

def kron_all(factors):
    out = np.array([[1]], dtype=np.int64)
    for f in factors:
        out = np.kron(out, f)
    return out


def test_kron_bit_order_appendix1():
    """Appendix 1: k1 = q_M x ... x q_1 and k1(5) = q3(1) q2(0) q1(1), so bit b
    of the row index selects the component of the rightmost-but-b factor."""
    primes = [2, 3, 5, 7, 11, 13]
    q = {i: np.array([primes[2 * (i - 1)], primes[2 * (i - 1) + 1]], dtype=np.int64) for i in (1, 2, 3)}
    k1 = kron_all([q[3][None, :], q[2][None, :], q[1][None, :]])[0]
    assert k1[5] == q[3][1] * q[2][0] * q[1][1]
    for i in range(8):
        assert k1[i] == q[3][(i >> 2) & 1] * q[2][(i >> 1) & 1] * q[1][i & 1]


def dense_step(M, t, cmask):
    """U_s = (I - P) + P X: P projects onto rows whose control bits are 1,
    X is the NOT on bit t; both are Kronecker products with bit M-1 leftmost."""
    I2 = np.eye(2, dtype=np.int64)
    P1 = np.array([[0, 0], [0, 1]], dtype=np.int64)
    X = np.array([[0, 1], [1, 0]], dtype=np.int64)
    P = kron_all([P1 if (cmask >> b) & 1 else I2 for b in range(M - 1, -1, -1)])
    Xt = kron_all([X if b == t else I2 for b in range(M - 1, -1, -1)])
    Id = np.eye(1 << M, dtype=np.int64)
    return (Id - P) + P @ Xt


@pytest.mark.parametrize("seed", range(12))
def test_dense_bruteforce(seed):
    rng = np.random.default_rng(1000 + seed)
    M = int(rng.integers(1, 8))
    L = int(rng.integers(0, 26))
    tg, cm = W.random_steps(rng, M, L, (0, 4))
    n = 1 << M
    U = np.eye(n, dtype=np.int64)
    for s in range(L):
        Us = dense_step(M, int(tg[s]), int(cm[s]))
        assert (Us == Us.T).all()                       # symmetric (Sec. 2(a))
        assert (Us @ Us == np.eye(n, dtype=np.int64)).all()
        assert (Us.sum(axis=1) == 1).all() and (Us.sum(axis=0) == 1).all()
        assert set(np.unique(Us)) <= {0, 1}
        U = Us @ U                                      # k2 = U_L ... U_1 k1
    assert (U.T @ U == np.eye(n, dtype=np.int64)).all()  # U+U = I (Sec. 2(a))
    expect = U @ np.arange(n, dtype=np.int64)
    for dt in (np.complex64, np.complex128):
        for method in ("plain", "enum"):
            got = tags_of(oracle.apply(M, W.tag_state(M, dt), tg, cm, method=method))
            np.testing.assert_array_equal(got.astype(np.int64), expect)
    xr = oracle.rowmap(M, tg[::-1], cm[::-1])
    np.testing.assert_array_equal(xr.astype(np.int64), expect)
    for i in range(n):
        assert oracle.source_index(M, tg, cm, i) == expect[i]
    idx = rng.integers(0, n, size=17)
    k1 = W.gaussian_state(rng, M, np.complex128)
    np.testing.assert_array_equal(oracle.sample_rows(M, k1, tg, cm, idx), k1[expect[idx]])


# ------------------------------------------------------------------ invariants

@pytest.mark.parametrize("seed", range(6))
def test_involution(seed):
    """Each step matrix is its own inverse, so the reversed diagram undoes it."""
    rng = np.random.default_rng(2000 + seed)
    M = int(rng.integers(1, 13))
    L = int(rng.integers(0, 120))
    tg, cm = W.random_steps(rng, M, L, (0, 4))
    for dt in (np.complex64, np.complex128):
        k1 = W.gaussian_state(rng, M, dt)
        k2 = oracle.apply(M, k1, tg, cm)
        back = oracle.apply(M, k2, tg[::-1], cm[::-1])
        assert back.tobytes() == k1.tobytes()


@pytest.mark.parametrize("seed", range(4))
def test_multiset_and_norm(seed):
    """Entries are only moved: the sorted raw words agree exactly and the
    2-norm agrees to rounding (it is 1 for a normalised input, Sec. 2(b))."""
    rng = np.random.default_rng(3000 + seed)
    M = int(rng.integers(4, 14))
    tg, cm = W.random_steps(rng, M, 64, (0, 3))
    k1 = W.gaussian_state(rng, M, np.complex128)
    k2 = oracle.apply(M, k1, tg, cm)
    a = np.sort(k1.view(np.uint64).reshape(-1, 2).view([("re", "u8"), ("im", "u8")]).ravel())
    b = np.sort(k2.view(np.uint64).reshape(-1, 2).view([("re", "u8"), ("im", "u8")]).ravel())
    assert a.tobytes() == b.tobytes()
    assert abs(np.linalg.norm(k2) - 1.0) < 1e-12
    assert np.sum(np.sort(np.abs(k1) ** 2)) == np.sum(np.sort(np.abs(k2) ** 2))


@pytest.mark.parametrize("M", [2, 3, 5, 8, 12, 16])
def test_parity_closed_form(M):
    """Sec. 4: parity of qubits 2..M targeted to the bottom qubit on the
    alternating input.  Bit 0 of the source row becomes bit 0 XOR the other
    bits, so k2(i) = (-1)^popcount(i) |S|."""
    tg, cm = W.parity_circuit(M)
    k2 = oracle.apply(M, W.alternating_state(M), tg, cm)
    i = np.arange(1 << M, dtype=np.uint64)
    pop = np.zeros_like(i)
    for b in range(M):
        pop += (i >> np.uint64(b)) & np.uint64(1)
    expect = np.where(pop % 2 == 0, 1.0, -1.0) * 2.0 ** (-M / 2)
    np.testing.assert_array_equal(k2.real, expect)
    if M == 3:
        np.testing.assert_array_equal(np.sign(k2.real), [1, -1, -1, 1, -1, 1, 1, -1])


@pytest.mark.parametrize("seed", range(3))
def test_split_associativity(seed):
    rng = np.random.default_rng(4000 + seed)
    M = 9
    tg, cm = W.random_steps(rng, M, 40, (0, 3))
    k1 = W.gaussian_state(rng, M, np.complex64)
    full = oracle.apply(M, k1, tg, cm)
    for m in (0, 1, 7, 20, 39, 40):
        part = oracle.apply(M, oracle.apply(M, k1, tg[:m], cm[:m]), tg[m:], cm[m:])
        assert part.tobytes() == full.tobytes()


def test_commutation():
    """Steps (t1, C1), (t2, C2) commute when neither target is a control of
    the other (the premise of the same-target shortcut, Sec. 2(i)); when one
    target controls the other they do not."""
    rng = np.random.default_rng(5)
    M = 7
    k1 = W.tag_state(M)
    seen_commute = seen_not = 0
    for _ in range(300):
        tg, cm = W.random_steps(rng, M, 2, (0, 3))
        a = oracle.apply(M, k1, tg, cm)
        b = oracle.apply(M, k1, tg[::-1], cm[::-1])
        commute = not ((int(cm[1]) >> int(tg[0])) & 1) and not ((int(cm[0]) >> int(tg[1])) & 1)
        if commute:
            seen_commute += 1
            assert a.tobytes() == b.tobytes()
        else:
            seen_not += 1
            assert a.tobytes() != b.tobytes()
    assert seen_commute > 50 and seen_not > 20


# ------------------------------------------------------------------ exactness / edges

def test_special_values_preserved():
    rng = np.random.default_rng(6)
    for dt in (np.complex64, np.complex128):
        k1 = W.special_values_state(rng, 10, dt)
        tg, cm = W.random_steps(rng, 10, 50, (0, 3))
        k2 = oracle.apply(10, k1, tg, cm)
        back = oracle.apply(10, k2, tg[::-1], cm[::-1])
        assert back.tobytes() == k1.tobytes()
        assert sorted(k2.view(np.uint64).tolist()) == sorted(k1.view(np.uint64).tolist())


def test_empty_and_degenerate():
    k1 = W.gaussian_state(np.random.default_rng(7), 6, np.complex64)
    t0, c0 = W.empty_steps()
    assert oracle.apply(6, k1, t0, c0).tobytes() == k1.tobytes()
    # M = 1: only the unconditional NOT exists.
    k = np.array([1 + 2j, 3 + 4j], dtype=np.complex64)
    np.testing.assert_array_equal(oracle.apply(1, k, [0], [0]), k[::-1])
    # every other bit a control: only the last pair moves.
    M = 5
    src = tags_of(oracle.apply(M, W.tag_state(M), [2], [0b11011]))
    expect = np.arange(32, dtype=np.uint64)
    expect[[27, 31]] = [31, 27]
    np.testing.assert_array_equal(src, expect)


@pytest.mark.parametrize("bad", [
    dict(M=4, target=[4], cmask=[0]),        # target beyond the address bits
    dict(M=4, target=[1], cmask=[1 << 4]),   # control beyond the address bits
    dict(M=4, target=[1], cmask=[0b10]),     # target among its own controls
    dict(M=0, target=[], cmask=[]),
    dict(M=41, target=[], cmask=[]),
])
def test_invalid_rejected(bad):
    k = np.zeros(1 << max(bad["M"], 0), dtype=np.complex64) if bad["M"] <= 20 else np.zeros(2, np.complex64)
    with pytest.raises(ValueError):
        if bad["M"] in (0, 41):
            oracle.rowmap(bad["M"], bad["target"], bad["cmask"])
        else:
            oracle.apply(bad["M"], k, bad["target"], bad["cmask"])


def test_threads_agree():
    rng = np.random.default_rng(8)
    M = 16
    tg, cm = W.random_steps(rng, M, 30, (0, 3))
    k1 = W.gaussian_state(rng, M, np.complex128)
    a = oracle.apply(M, k1, tg, cm, threads=1)
    b = oracle.apply(M, k1, tg, cm, threads=4)
    c = oracle.apply(M, k1, tg, cm, threads=4, method="enum")
    assert a.tobytes() == b.tobytes() == c.tobytes()
    idx = rng.integers(0, 1 << M, size=1000)
    np.testing.assert_array_equal(oracle.sample_rows(M, k1, tg, cm, idx, threads=4), a[idx])


# ------------------------------------------------------------------ mutation checks

def _py_apply(M, src, tg, cm, mutant=None):
    """Pure-Python pair-swap loop with an optional planted mistake."""
    v = list(src)
    order = range(len(tg)) if mutant != "reverse_order" else range(len(tg) - 1, -1, -1)
    for s in order:
        t, C = int(tg[s]), int(cm[s])
        if mutant == "target_off_by_one":
            t = (t + 1) % M
            C &= ~(1 << t)
        if mutant == "drop_controls":
            C = C & (C - 1) if C else 0  # forgets one control
        if mutant == "or_controls" and C:
            T = 1 << t
            for i in range(1 << M):
                if not i & T and i & C:
                    v[i], v[i | T] = v[i | T], v[i]
            continue
        T = 1 << t
        for i in range(1 << M):
            cond = (i & C) == C
            if mutant == "controls_inverted":
                cond = (i & C) == 0
            if not i & T and cond:
                v[i], v[i | T] = v[i | T], v[i]
    return v


def _failing_pins(apply_fn):
    """Which pin families a candidate implementation fails."""
    failed = set()
    for ex in EXAMPLES.values():
        if "expect_src" not in ex:
            continue
        got = apply_fn(ex["M"], list(range(1 << ex["M"])), ex["target"], ex["cmask"])
        if list(got) != [int(x) for x in ex["expect_src"]]:
            failed.add("paper")
    rng = np.random.default_rng(77)
    for _ in range(6):
        M = int(rng.integers(2, 6))
        tg, cm = W.random_steps(rng, M, 8, (0, 3))
        U = np.eye(1 << M, dtype=np.int64)
        for s in range(len(tg)):
            U = dense_step(M, int(tg[s]), int(cm[s])) @ U
        if list(apply_fn(M, list(range(1 << M)), tg, cm)) != list(U @ np.arange(1 << M)):
            failed.add("dense")
    return failed


def test_pins_accept_correct_loop():
    assert _failing_pins(lambda M, v, tg, cm: _py_apply(M, v, tg, cm)) == set()


@pytest.mark.parametrize("mutant", ["reverse_order", "target_off_by_one", "drop_controls",
                                    "or_controls", "controls_inverted"])
def test_pins_catch_planted_mistake(mutant):
    failed = _failing_pins(lambda M, v, tg, cm: _py_apply(M, v, tg, cm, mutant))
    assert failed, f"planted mistake {mutant} passed every pin"


# ------------------------------------------------------------------ product-state input (Appendix 1)

def test_product_state_appendix1_example():
    """k1(5) = q3(1) q2(0) q1(1): with distinct primes as the qubit components
    every product is exact and the whole vector equals the integer Kronecker
    product q_M x ... x q_1 (bit order of Appendix 1)."""
    primes = [2, 3, 5, 7, 11, 13, 17, 19]
    for M, dt in ((3, np.complex128), (3, np.complex64), (4, np.complex128)):
        q = np.array([[primes[2 * b], primes[2 * b + 1]] for b in range(M)], dtype=dt)
        k1 = oracle.product_state(M, q)
        kron = np.array([1], dtype=np.int64)
        for b in range(M - 1, -1, -1):
            kron = np.kron(kron, q[b].real.astype(np.int64))
        np.testing.assert_array_equal(k1.real, kron)
        np.testing.assert_array_equal(k1.imag, 0)
        if M == 3:
            assert k1[5] == q[2][1] * q[1][0] * q[0][1]


def test_product_state_complex_and_norm():
    """Complex components (exact small Gaussian integers) multiply as complex
    numbers; unit-norm qubits give a unit-norm state (Sec. 2(b) normalisation)."""
    q = np.array([[1 + 2j, 3 - 1j], [2 - 1j, 1j], [1 + 1j, -2 + 0j]], dtype=np.complex128)
    k1 = oracle.product_state(3, q)
    for i in range(8):
        expect = q[2][(i >> 2) & 1] * q[1][(i >> 1) & 1] * q[0][i & 1]
        assert k1[i] == expect
    rng = np.random.default_rng(3)
    for dt, tol in ((np.complex128, 1e-12), (np.complex64, 1e-5)):
        qq = rng.standard_normal((12, 2)) + 1j * rng.standard_normal((12, 2))
        qq /= np.linalg.norm(qq, axis=1, keepdims=True)
        k = oracle.product_state(12, qq.astype(dt))
        assert abs(np.linalg.norm(k.astype(np.complex128)) - 1.0) < tol
        # the alternating input of Sec. 2(b) is the product of H|1> on the bottom qubit
        # and H|0> on the others
    s = 2 ** -0.5
    qh = np.array([[s, -s]] + [[s, s]] * 9, dtype=np.complex128)
    np.testing.assert_allclose(oracle.product_state(10, qh), W.alternating_state(10), rtol=0, atol=1e-15)


def test_product_entry_matches_product_state():
    rng = np.random.default_rng(4)
    for dt in (np.complex64, np.complex128):
        qq = (rng.standard_normal((11, 2)) + 1j * rng.standard_normal((11, 2))).astype(dt)
        full = oracle.product_state(11, qq)
        for i in (0, 1, 5, 777, 2047):
            assert oracle.product_entry(11, qq, i).tobytes() == full[i].tobytes()


# ------------------------------------------------------------------ signed steps (Sec. 2(a) example matrix)

NOT, PHASE = 0, 1


def dense_phase(M, t, cmask):
    """Controlled phase -1: I - 2 P, P projecting onto the rows whose bits t
    and C are all 1 (a Kronecker product, bit M-1 leftmost)."""
    I2 = np.eye(2, dtype=np.int64)
    P1 = np.array([[0, 0], [0, 1]], dtype=np.int64)
    m = cmask | (1 << t)
    P = kron_all([P1 if (m >> b) & 1 else I2 for b in range(M - 1, -1, -1)])
    return np.eye(1 << M, dtype=np.int64) - 2 * P


def dense_signed(M, tg, cm, kd):
    U = np.eye(1 << M, dtype=np.int64)
    for s in range(len(tg)):
        f = dense_phase if kd[s] == PHASE else dense_step
        U = f(M, int(tg[s]), int(cm[s])) @ U
    return U


def int_state(M, dt):
    """Small integers in both parts: exact under negation and under a 0/+-1
    matrix product in float64."""
    i = np.arange(1 << M)
    return (i + 1 + 1j * (1000 + 3 * i)).astype(dt)


def random_signed(rng, M, L, p_phase=0.35):
    tg, cm = W.random_steps(rng, M, L, (0, 3))
    kd = (rng.random(L) < p_phase).astype(np.uint8)
    return tg, cm, kd


# Construction (not printed in the paper): on two bits (b1 b0), the NOTs
# [b0 controls b1, b1 controls b0, NOT b0] move the entry at (b1, b0) to
# (b0 ^ b1, b1 ^ 1), i.e. k2(i) = k1(x(i)) with x = (3, 0, 2, 1); a phase
# step on bit 0 controlled by bit 1 then negates row 3.
SIGNED_EXAMPLE = (np.array([1, 0, 0, 0], dtype=np.uint32),
                  np.array([0b01, 0b10, 0, 0b10], dtype=np.uint64),
                  np.array([NOT, NOT, NOT, PHASE], dtype=np.uint8))


def test_paper_signed_example_matrix():
    ex = EXAMPLES["sec2a_signed_example"]
    M, G = ex["M"], ex["matrix"]
    tg, cm, kd = SIGNED_EXAMPLE
    U = dense_signed(M, tg, cm, kd)
    np.testing.assert_array_equal(U, G, err_msg=ex["cite"])
    assert (G.T @ G == np.eye(4, dtype=np.int64)).all()        # unitary (Sec. 2(a))
    for dt in (np.complex64, np.complex128):
        k1 = int_state(M, dt)
        k2 = oracle.apply(M, k1, tg, cm, kind=kd)
        np.testing.assert_array_equal(k2, (G @ k1.astype(np.complex128)).astype(dt))
        np.testing.assert_array_equal(oracle.sample_rows(M, k1, tg, cm, np.arange(4), kind=kd), k2)
    # Without the phase step the same diagram is the 0/1 matrix |G|.
    k2 = oracle.apply(M, int_state(M, np.complex128), tg[:3], cm[:3])
    np.testing.assert_array_equal(k2, np.abs(G) @ int_state(M, np.complex128))


@pytest.mark.parametrize("seed", range(10))
def test_signed_dense_bruteforce(seed):
    rng = np.random.default_rng(9000 + seed)
    M = int(rng.integers(1, 8))
    L = int(rng.integers(0, 26))
    tg, cm, kd = random_signed(rng, M, L)
    U = dense_signed(M, tg, cm, kd)
    n = 1 << M
    assert (U.T @ U == np.eye(n, dtype=np.int64)).all()
    assert (np.abs(U).sum(axis=1) == 1).all()                   # a signed permutation
    for dt in (np.complex64, np.complex128):
        k1 = int_state(M, dt)
        expect = (U @ k1.astype(np.complex128)).astype(dt)
        got = oracle.apply(M, k1, tg, cm, kind=kd)
        np.testing.assert_array_equal(got, expect)
        idx = rng.integers(0, n, size=13)
        np.testing.assert_array_equal(oracle.sample_rows(M, k1, tg, cm, idx, kind=kd), expect[idx])
    for i in range(n):
        x, neg = oracle.source_index_signed(M, tg, cm, kd, i)
        assert U[i, x] == (-1 if neg else 1)
    # all-NOT kinds reduce to the unsigned oracle
    k1 = W.gaussian_state(rng, M, np.complex64)
    z = np.zeros(L, dtype=np.uint8)
    assert oracle.apply(M, k1, tg, cm, kind=z).tobytes() == oracle.apply(M, k1, tg, cm).tobytes()


@pytest.mark.parametrize("seed", range(4))
def test_signed_involution_and_sign_bits(seed):
    """Every signed step is its own inverse, negation flips only sign bits
    (NaN payloads, zeros and infinities included), and the magnitudes are
    only moved."""
    rng = np.random.default_rng(9100 + seed)
    M = int(rng.integers(2, 12))
    tg, cm, kd = random_signed(rng, M, 80)
    for dt in (np.complex64, np.complex128):
        k1 = W.special_values_state(rng, M, dt)
        k2 = oracle.apply(M, k1, tg, cm, kind=kd)
        back = oracle.apply(M, k2, tg[::-1], cm[::-1], kind=kd[::-1])
        assert back.tobytes() == k1.tobytes()
        sign = np.uint64(0x8000000080000000) if dt == np.complex64 else np.uint64(1 << 63)
        a = np.sort(k1.view(np.uint64) & ~sign)
        b = np.sort(k2.view(np.uint64) & ~sign)
        assert a.tobytes() == b.tobytes()
    # one phase step on bit t, no controls: rows with bit t set flip both signs
    t = int(rng.integers(0, M))
    k1 = W.special_values_state(rng, M, np.complex64)
    k2 = oracle.apply(M, k1, [t], [0], kind=[PHASE])
    rows = (np.arange(1 << M) >> t) & 1
    flip = np.where(rows == 1, np.uint64(0x8000000080000000), np.uint64(0))
    np.testing.assert_array_equal(k2.view(np.uint64), k1.view(np.uint64) ^ flip)


def test_signed_commutation():
    """A phase step commutes with a NOT step exactly when the NOT's target is
    not among the phase step's bits; phase steps always commute."""
    rng = np.random.default_rng(9200)
    M = 6
    k1 = int_state(M, np.complex128)
    seen = [0, 0]
    for _ in range(300):
        tg, cm, kd = random_signed(rng, M, 2, 0.5)
        a = oracle.apply(M, k1, tg, cm, kind=kd)
        b = oracle.apply(M, k1, tg[::-1], cm[::-1], kind=kd[::-1])
        def tm(s): return 0 if kd[s] else 1 << int(tg[s])
        def rm(s): return int(cm[s]) | ((1 << int(tg[s])) if kd[s] else 0)
        commute = not (tm(0) & rm(1)) and not (tm(1) & rm(0))
        seen[commute] += 1
        assert (a.tobytes() == b.tobytes()) == commute
    assert min(seen) > 30


def _py_apply_signed(M, v, tg, cm, kd, mutant=None):
    v = list(v)
    for s in range(len(tg)):
        t, C, T = int(tg[s]), int(cm[s]), 1 << int(tg[s])
        if kd[s] == PHASE and mutant != "phase_as_not":
            if mutant == "phase_ignored":
                continue
            m = C if mutant == "phase_controls_only" else C | T
            for i in range(1 << M):
                hit = (i & m) != 0 if mutant == "phase_or" else (i & m) == m
                if hit:
                    v[i] = -v[i]
            continue
        for i in range(1 << M):
            if not i & T and (i & C) == C:
                v[i], v[i | T] = v[i | T], v[i]
    return v


def _failing_signed_pins(apply_fn):
    failed = set()
    ex = EXAMPLES["sec2a_signed_example"]
    tg, cm, kd = SIGNED_EXAMPLE
    if list(apply_fn(2, [1, 2, 3, 4], tg, cm, kd)) != list(ex["matrix"] @ np.array([1, 2, 3, 4])):
        failed.add("paper")
    rng = np.random.default_rng(78)
    for _ in range(8):
        M = int(rng.integers(2, 6))
        tg, cm, kd = random_signed(rng, M, 8, 0.5)
        x = np.arange(1, (1 << M) + 1)
        if list(apply_fn(M, list(x), tg, cm, kd)) != list(dense_signed(M, tg, cm, kd) @ x):
            failed.add("dense")
    return failed


def test_signed_pins_accept_correct_loop():
    assert _failing_signed_pins(lambda M, v, tg, cm, kd: _py_apply_signed(M, v, tg, cm, kd)) == set()


@pytest.mark.parametrize("mutant", ["phase_as_not", "phase_ignored", "phase_controls_only", "phase_or"])
def test_signed_pins_catch_planted_mistake(mutant):
    failed = _failing_signed_pins(lambda M, v, tg, cm, kd: _py_apply_signed(M, v, tg, cm, kd, mutant))
    assert failed, f"planted mistake {mutant} passed every pin"
