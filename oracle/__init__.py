"""CPU oracle for k2 = U_L ... U_1 k1 over a wiring diagram of controlled-NOT steps.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library or its binding.  It
shares no code with the GPU path.

The arithmetic lives in ``oracle.c`` (plain C, built into ``liboracle.so``);
this module only marshals numpy arrays into it.  Steps are given as two
arrays: ``target`` (address bit of the NOT, 0-based, bit b is the paper's
a(b+1)) and ``cmask`` (bit mask of the controlling bits, all of which must be
1 for the step to fire).  ``steps[0]`` acts first (Sec. 2(a): k2 = U_L k1 with
U_L the product of the step matrices).  An optional ``kind`` array adds
controlled phase -1 steps (kind 1) beside the controlled NOTs (kind 0).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# QSIM_ORACLE_LIB names another build of oracle.c to load (the sanitizer
# check runs the pins against one built with AddressSanitizer and UBSan).
_LIB = os.environ.get("QSIM_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP on)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-Wall", "-Wextra", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def library_path() -> str:
    """Path of the oracle library this process loads."""
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    for name in ("oracle_apply", "oracle_apply_enum"):
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p, u32p, u64p,
                      ctypes.c_uint64, ctypes.c_int]
    lib.oracle_rowmap.restype = ctypes.c_int
    lib.oracle_rowmap.argtypes = [ctypes.c_uint32, u32p, u64p, ctypes.c_uint64, u64p]
    lib.oracle_source_index.restype = ctypes.c_uint64
    lib.oracle_source_index.argtypes = [ctypes.c_uint32, u32p, u64p, ctypes.c_uint64,
                                        ctypes.c_uint64]
    lib.oracle_sample_rows.restype = ctypes.c_int
    lib.oracle_sample_rows.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p,
                                       u32p, u64p, ctypes.c_uint64, u64p, ctypes.c_uint64,
                                       ctypes.c_void_p, ctypes.c_int]
    lib.oracle_product_state.restype = ctypes.c_int
    lib.oracle_product_state.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]
    lib.oracle_product_entry.restype = ctypes.c_int
    lib.oracle_product_entry.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint64,
                                         ctypes.c_void_p]
    u8p = ctypes.POINTER(ctypes.c_uint8)
    lib.oracle_apply_signed.restype = ctypes.c_int
    lib.oracle_apply_signed.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p, u32p, u64p, u8p,
                                        ctypes.c_uint64, ctypes.c_int]
    lib.oracle_sample_rows_signed.restype = ctypes.c_int
    lib.oracle_sample_rows_signed.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p, u32p, u64p,
                                              u8p, ctypes.c_uint64, u64p, ctypes.c_uint64, ctypes.c_void_p,
                                              ctypes.c_int]
    lib.oracle_source_index_signed.restype = ctypes.c_uint64
    lib.oracle_source_index_signed.argtypes = [ctypes.c_uint32, u32p, u64p, u8p, ctypes.c_uint64,
                                               ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)]
    lib.oracle_max_threads.restype = ctypes.c_int
    lib.oracle_max_threads.argtypes = []
    _lib = lib
    return lib


def _steps_arrays(target, cmask):
    t = np.ascontiguousarray(np.asarray(target, dtype=np.uint32))
    c = np.ascontiguousarray(np.asarray(cmask, dtype=np.uint64))
    if t.shape != c.shape or t.ndim != 1:
        raise ValueError("target and cmask must be 1-D arrays of equal length")
    return t, c


def _ptrs(t, c):
    return (t.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
            c.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))


def _elem_bytes(state: np.ndarray) -> int:
    if state.dtype == np.complex64:
        return 8
    if state.dtype == np.complex128:
        return 16
    raise ValueError(f"state dtype must be complex64 or complex128, got {state.dtype}")


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"{what}: oracle rejected the arguments (code {rc})")


def _kinds(kind, n):
    k = np.ascontiguousarray(np.asarray(kind, dtype=np.uint8))
    if k.shape != (n,):
        raise ValueError("kind must be a 1-D array with one entry per step")
    return k, k.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def apply(M: int, state: np.ndarray, target, cmask, threads: int = 1,
          method: str = "plain", kind=None) -> np.ndarray:
    """Return U_L ... U_1 state (a new array), by the plain pair-swap loop
    (``method="plain"``) or by intelligent looping (``method="enum"``).
    ``kind`` (optional, one entry per step): 0 = controlled NOT, 1 =
    controlled phase -1 on the rows whose target and control bits are all
    1 (plain loop only)."""
    eb = _elem_bytes(state)
    if state.shape != (1 << M,):
        raise ValueError("state must hold 2^M entries")
    out = np.array(state, copy=True, order="C")
    t, c = _steps_arrays(target, cmask)
    tp, cp = _ptrs(t, c)
    if kind is not None:
        if method != "plain":
            raise ValueError("signed steps use the plain loop")
        k, kp = _kinds(kind, len(t))
        _check(_load().oracle_apply_signed(M, eb, out.ctypes.data, tp, cp, kp, len(t), int(threads)),
               "apply_signed")
        return out
    fn = _load().oracle_apply if method == "plain" else _load().oracle_apply_enum
    _check(fn(M, eb, out.ctypes.data, tp, cp, len(t), int(threads)), "apply")
    return out


def apply_inplace(M: int, state: np.ndarray, target, cmask, threads: int = 1) -> None:
    """Plain pair-swap loop applied to ``state`` in place."""
    eb = _elem_bytes(state)
    if state.shape != (1 << M,) or not state.flags.c_contiguous:
        raise ValueError("state must be a contiguous array of 2^M entries")
    t, c = _steps_arrays(target, cmask)
    tp, cp = _ptrs(t, c)
    _check(_load().oracle_apply(M, eb, state.ctypes.data, tp, cp, len(t), int(threads)),
           "apply_inplace")


def rowmap(M: int, target, cmask) -> np.ndarray:
    """The paper's row array x after folding the steps in the given order with
    x(i) <- y(x(i)) (Sec. 2(h)); x is the row map of U_{s_1} U_{s_2} ... U_{s_n}."""
    if not 1 <= M <= 40:
        raise ValueError("M must lie in [1, 40]")
    t, c = _steps_arrays(target, cmask)
    tp, cp = _ptrs(t, c)
    x = np.empty(1 << M, dtype=np.uint64)
    _check(_load().oracle_rowmap(M, tp, cp, len(t),
                                 x.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))), "rowmap")
    return x


def source_index(M: int, target, cmask, i: int) -> int:
    """x(i) of U_L ... U_1 for one row: k2(i) = k1(x(i))."""
    t, c = _steps_arrays(target, cmask)
    tp, cp = _ptrs(t, c)
    return int(_load().oracle_source_index(M, tp, cp, len(t), int(i)))


def source_index_signed(M: int, target, cmask, kind, i: int):
    """(x(i), negated) of U_L ... U_1 with signed steps: k2(i) = +-k1(x(i))."""
    t, c = _steps_arrays(target, cmask)
    tp, cp = _ptrs(t, c)
    k, kp = _kinds(kind, len(t))
    neg = ctypes.c_int(0)
    x = _load().oracle_source_index_signed(M, tp, cp, kp, len(t), int(i), ctypes.byref(neg))
    return int(x), bool(neg.value)


def sample_rows(M: int, k1: np.ndarray, target, cmask, idx, threads: int = 1, kind=None) -> np.ndarray:
    """k2 at the rows ``idx`` without forming the whole of k2 (``kind`` as
    in apply)."""
    eb = _elem_bytes(k1)
    if k1.shape != (1 << M,) or not k1.flags.c_contiguous:
        raise ValueError("k1 must be a contiguous array of 2^M entries")
    t, c = _steps_arrays(target, cmask)
    tp, cp = _ptrs(t, c)
    ix = np.ascontiguousarray(np.asarray(idx, dtype=np.uint64))
    out = np.empty(len(ix), dtype=k1.dtype)
    if kind is not None:
        k, kp = _kinds(kind, len(t))
        _check(_load().oracle_sample_rows_signed(M, eb, k1.ctypes.data, tp, cp, kp, len(t),
                                                 ix.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                                 len(ix), out.ctypes.data, int(threads)), "sample_rows_signed")
        return out
    _check(_load().oracle_sample_rows(M, eb, k1.ctypes.data, tp, cp, len(t),
                                      ix.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                      len(ix), out.ctypes.data, int(threads)), "sample_rows")
    return out


def product_state(M: int, qubits: np.ndarray) -> np.ndarray:
    """k1 = q_M (x) ... (x) q_1 (Appendix 1) from qubits[b-1] = (q_b(0), q_b(1)),
    an (M, 2) complex64 or complex128 array; the product runs from q_M down
    to q_1 in the array's precision without fused multiply-adds."""
    q = np.ascontiguousarray(qubits)
    if q.shape != (M, 2):
        raise ValueError("qubits must have shape (M, 2)")
    eb = _elem_bytes(q.reshape(-1))
    out = np.empty(1 << M, dtype=q.dtype)
    _check(_load().oracle_product_state(M, eb, q.ctypes.data, out.ctypes.data), "product_state")
    return out


def product_entry(M: int, qubits: np.ndarray, i: int):
    """k1(i) of product_state(M, qubits), computed for one row."""
    q = np.ascontiguousarray(qubits)
    if q.shape != (M, 2):
        raise ValueError("qubits must have shape (M, 2)")
    eb = _elem_bytes(q.reshape(-1))
    out = np.empty(1, dtype=q.dtype)
    _check(_load().oracle_product_entry(M, eb, q.ctypes.data, int(i), out.ctypes.data), "product_entry")
    return out[0]


def max_threads() -> int:
    return int(_load().oracle_max_threads())
