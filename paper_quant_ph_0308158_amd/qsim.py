"""ctypes binding of libqsim (include/qsim.h): argument marshalling only.

Every step of the computation runs in the HIP kernels of libqsim.so; this
module converts numpy / torch arguments into the C ABI's plain pointers and
sizes.  If libqsim.so is missing the import fails: there is no fallback.

Steps are passed as a pair of arrays ``(target, cmask)``: ``target[s]`` is
the 0-based address bit that step s flips (the paper's a(target+1)),
``cmask[s]`` the mask of its controlling bits, all of which must be 1 for
the step to fire (Sec. 2(b)-(g)).  ``steps[0]`` acts first, so applying
a diagram computes k2 = U_L ... U_1 k1 (Sec. 2(a), 2(h)).
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libqsim.so")

QSIM_C64 = 0
QSIM_C128 = 1
OK, ERR_INVALID, ERR_NOMEM, ERR_DEVICE, ERR_RANGE = 0, -1, -2, -3, -4
MAX_M = 36

STEP_DTYPE = np.dtype([("target", "<u4"), ("kind", "<u4"), ("control_mask", "<u8")])
STEP_NOT, STEP_PHASE = 0, 1   # qsim_step_kind

# Every symbol declared in include/qsim.h.
EXPORTS = (
    "qsim_state_create", "qsim_state_wrap", "qsim_state_destroy", "qsim_state_qubits",
    "qsim_state_elem_bytes", "qsim_state_current", "qsim_write_portion", "qsim_apply_steps",
    "qsim_apply_steps_plain", "qsim_read_portion", "qsim_read_portion_async", "qsim_apply_batch",
    "qsim_state_set_tuning", "qsim_plan_describe", "qsim_copy_bytes", "qsim_last_error",
    "qsim_version", "qsim_state_profile", "qsim_state_profile_read", "qsim_apply_tile_pass",
    "qsim_batch_last_status", "qsim_server_create", "qsim_server_submit", "qsim_server_drain",
    "qsim_server_request_info", "qsim_server_stats", "qsim_server_destroy", "qsim_state_set_product", "qsim_apply_steps_product",
    "qsim_rowmap_build", "qsim_rowmap_apply", "qsim_autotune", "qsim_batch_set_tiles_per_item",
    "qsim_batch_tiles_per_item", "qsim_batch_autotune", "qsim_apply_steps_noalloc",
    "qsim_batch_set_tuning", "qsim_batch_get_tuning", "qsim_batch_last_info",
)


class QsimError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"qsim error {code}: {msg}")
        self.code = code


class Profile(ctypes.Structure):
    _fields_ = [("tile_launches", ctypes.c_uint64), ("tile_ms", ctypes.c_double),
                ("tile_bytes", ctypes.c_uint64), ("map_launches", ctypes.c_uint64),
                ("map_ms", ctypes.c_double), ("other_launches", ctypes.c_uint64),
                ("other_ms", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_slots", ctypes.c_uint32),
                ("portion_entries", ctypes.c_uint32), ("fcfs", ctypes.c_uint32),
                ("max_bypass", ctypes.c_uint32), ("digest", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("done", ctypes.c_int32), ("t_submit_ns", ctypes.c_uint64),
                ("t_admit_ns", ctypes.c_uint64), ("t_done_ns", ctypes.c_uint64), ("digest", ctypes.c_uint64),
                ("bytes", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class Tuning(ctypes.Structure):
    _fields_ = [("tile_bits", ctypes.c_uint32), ("low_bits", ctypes.c_uint32),
                ("max_seg_steps", ctypes.c_uint32), ("reorder", ctypes.c_uint32),
                ("small_bits", ctypes.c_uint32), ("kernel_variant", ctypes.c_uint32),
                ("wg_per_cu", ctypes.c_uint32), ("outer_order", ctypes.c_uint32),
                ("remap", ctypes.c_uint32), ("mid_low_bits", ctypes.c_uint32),
                ("min_overlap", ctypes.c_uint32), ("rows_per_thread", ctypes.c_uint32),
                ("plan_search", ctypes.c_uint32), ("xcd_swizzle", ctypes.c_uint32),
                ("product_stage", ctypes.c_uint32)]


class BatchTuning(ctypes.Structure):
    _fields_ = [("tiles_per_item", ctypes.c_uint32), ("tile_bits", ctypes.c_uint32),
                ("circuit_tiles", ctypes.c_uint32), ("plan_search", ctypes.c_uint32),
                ("order", ctypes.c_uint32), ("from_cache", ctypes.c_uint32),
                ("best_ms", ctypes.c_float), ("default_ms", ctypes.c_float)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class BatchInfo(ctypes.Structure):
    _fields_ = [("circuits", ctypes.c_uint32), ("items", ctypes.c_uint32), ("passes", ctypes.c_uint32),
                ("workgroups", ctypes.c_uint32), ("algorithmic_bytes", ctypes.c_uint64),
                ("kernel_ms", ctypes.c_double), ("tuning", BatchTuning)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "tuning"}
        d["tuning"] = self.tuning.as_dict()
        return d


def _load() -> ctypes.CDLL:
    # PyTorch ships its own HIP runtime under the soname libamdhip64.so.7.
    # Loading torch first makes libqsim.so bind to that same runtime, so
    # device pointers and streams from torch are valid in libqsim; loading
    # libqsim first would pull in a second copy of the runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_quant_ph_0308158_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    sig = {
        "qsim_state_create": (vp, [u32, i32]),
        "qsim_state_wrap": (vp, [u32, i32, vp, vp]),
        "qsim_state_destroy": (None, [vp]),
        "qsim_state_qubits": (u32, [vp]),
        "qsim_state_elem_bytes": (u32, [vp]),
        "qsim_state_current": (vp, [vp]),
        "qsim_write_portion": (i32, [vp, u64, u64, vp]),
        "qsim_apply_steps": (i32, [vp, vp, u64, vp]),
        "qsim_apply_steps_plain": (i32, [vp, vp, u64, vp]),
        "qsim_read_portion": (i32, [vp, u64, u64, vp]),
        "qsim_read_portion_async": (i32, [vp, u64, u64, vp, vp]),
        "qsim_apply_batch": (i32, [vp, vp, vp, u32, vp]),
        "qsim_state_set_tuning": (i32, [vp, vp]),
        "qsim_plan_describe": (i32, [u32, i32, vp, u64, vp, vp, vp, vp, u32, vp]),
        "qsim_copy_bytes": (i32, [vp, vp, u64, vp]),
        "qsim_last_error": (ctypes.c_char_p, []),
        "qsim_version": (ctypes.c_char_p, []),
        "qsim_state_profile": (i32, [vp, i32]),
        "qsim_apply_tile_pass": (i32, [vp, u64, vp, u64, vp]),
        "qsim_batch_last_status": (i32, []),
        "qsim_server_create": (vp, [vp]),
        "qsim_server_submit": (ctypes.c_int64, [vp, u32, i32, vp, vp, u64]),
        "qsim_server_drain": (i32, [vp]),
        "qsim_server_request_info": (i32, [vp, ctypes.c_int64, vp]),
        "qsim_server_stats": (i32, [vp, vp, vp, vp, vp]),
        "qsim_server_destroy": (None, [vp]),
        "qsim_state_set_product": (i32, [vp, vp, vp]),
        "qsim_apply_steps_product": (i32, [vp, vp, vp, u64, vp]),
        "qsim_rowmap_build": (i32, [u32, vp, u64, vp, vp]),
        "qsim_rowmap_apply": (i32, [vp, vp, vp]),
        "qsim_autotune": (i32, [vp, vp, u64, vp, vp]),
        "qsim_state_profile_read": (i32, [vp, vp]),
        "qsim_batch_set_tiles_per_item": (i32, [u32]),
        "qsim_batch_tiles_per_item": (u32, []),
        "qsim_batch_autotune": (i32, [vp, vp, vp, u32, vp, vp]),
        "qsim_apply_steps_noalloc": (i32, [vp, vp, u64, vp]),
        "qsim_batch_set_tuning": (i32, [i32, vp]),
        "qsim_batch_get_tuning": (i32, [i32, vp]),
        "qsim_batch_last_info": (i32, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()


def lib() -> ctypes.CDLL:
    return _lib


def last_error() -> str:
    return _lib.qsim_last_error().decode()


def version() -> str:
    return _lib.qsim_version().decode()


def _check(rc: int):
    if rc != OK:
        raise QsimError(rc, last_error())


def dtype_code(dtype) -> int:
    if dtype in ("c64", np.complex64, QSIM_C64):
        return QSIM_C64
    if dtype in ("c128", np.complex128, QSIM_C128):
        return QSIM_C128
    try:
        import torch
        if dtype == torch.complex64:
            return QSIM_C64
        if dtype == torch.complex128:
            return QSIM_C128
    except ImportError:
        pass
    raise ValueError(f"unsupported dtype {dtype!r}")


def np_dtype(code: int):
    return np.complex64 if code == QSIM_C64 else np.complex128


def pack_steps(target, cmask, kind=None) -> np.ndarray:
    """qsim_step array; ``kind`` (optional, per step): STEP_NOT (controlled
    NOT, the default) or STEP_PHASE (controlled phase -1)."""
    t = np.asarray(target, dtype=np.uint32).ravel()
    c = np.asarray(cmask, dtype=np.uint64).ravel()
    if t.shape != c.shape:
        raise ValueError("target and cmask differ in length")
    st = np.zeros(len(t), dtype=STEP_DTYPE)
    st["target"] = t
    st["control_mask"] = c
    if kind is not None:
        k = np.asarray(kind, dtype=np.uint32).ravel()
        if k.shape != t.shape:
            raise ValueError("kind and target differ in length")
        st["kind"] = k
    return st


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return torch.cuda.current_stream().cuda_stream or None
        except ImportError:
            pass
        return None
    if isinstance(stream, int):
        return stream or None
    return stream.cuda_stream or None


def _tuning_struct(tuning: Optional[dict]) -> Optional[Tuning]:
    if tuning is None:
        return None
    t = Tuning()
    for k, v in tuning.items():
        if k in ("reorder", "remap") and isinstance(v, bool):
            v = 1 if v else 2
        setattr(t, k, int(v))
    return t


class State:
    """A 2^M-entry state on the current HIP device (two ping-pong buffers)."""

    def __init__(self, M: int, dtype="c64", buffers=None):
        self.M = int(M)
        self.code = dtype_code(dtype)
        self._keep = None
        if buffers is None:
            h = _lib.qsim_state_create(self.M, self.code)
        else:
            b0, b1 = buffers
            self._keep = (b0, b1)
            h = _lib.qsim_state_wrap(self.M, self.code, ctypes.c_void_p(_ptr(b0)), ctypes.c_void_p(_ptr(b1)))
        if not h:
            raise QsimError(ERR_INVALID, last_error())
        self._h = ctypes.c_void_p(h)

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None):
            _lib.qsim_state_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    @property
    def elem_bytes(self) -> int:
        return int(_lib.qsim_state_elem_bytes(self._h))

    @property
    def n(self) -> int:
        return 1 << self.M

    def current_ptr(self) -> int:
        return int(_lib.qsim_state_current(self._h))

    # -- data movement
    def write(self, host: np.ndarray, offset: int = 0):
        a = np.ascontiguousarray(host)
        if a.dtype != np_dtype(self.code):
            raise ValueError(f"expected {np_dtype(self.code)}, got {a.dtype}")
        _check(_lib.qsim_write_portion(self._h, offset, a.size, a.ctypes.data))

    def read(self, offset: int = 0, count: Optional[int] = None) -> np.ndarray:
        if count is None:
            count = self.n - offset
        out = np.empty(count, dtype=np_dtype(self.code))
        _check(_lib.qsim_read_portion(self._h, offset, count, out.ctypes.data))
        return out

    def read_into(self, out: np.ndarray, offset: int = 0):
        if out.dtype != np_dtype(self.code) or not out.flags.c_contiguous:
            raise ValueError("out must be a contiguous array of the state's dtype")
        _check(_lib.qsim_read_portion(self._h, offset, out.size, out.ctypes.data))

    def read_async(self, offset: int, count: int, host_ptr: int, stream=None):
        _check(_lib.qsim_read_portion_async(self._h, offset, count, ctypes.c_void_p(host_ptr),
                                            ctypes.c_void_p(_stream_ptr(stream))))

    # -- compute
    def apply(self, target, cmask, stream=None, kind=None):
        st = pack_steps(target, cmask, kind)
        _check(_lib.qsim_apply_steps(self._h, st.ctypes.data if len(st) else None, len(st),
                                     ctypes.c_void_p(_stream_ptr(stream))))

    def apply_packed(self, steps: np.ndarray, stream=None):
        _check(_lib.qsim_apply_steps(self._h, steps.ctypes.data if len(steps) else None, len(steps),
                                     ctypes.c_void_p(_stream_ptr(stream))))

    def apply_noalloc(self, target, cmask, stream=None, kind=None):
        """qsim_apply_steps_noalloc: the same result, with the plan and tile
        records in the library's per-device scratch (no device allocation)."""
        st = pack_steps(target, cmask, kind)
        _check(_lib.qsim_apply_steps_noalloc(self._h, st.ctypes.data if len(st) else None, len(st),
                                             ctypes.c_void_p(_stream_ptr(stream))))

    def set_product(self, qubits: np.ndarray, stream=None):
        """k1 = q_M (x) ... (x) q_1 from qubits[b-1] = (q_b(0), q_b(1)) (shape (M, 2))."""
        q = np.ascontiguousarray(qubits, dtype=np_dtype(self.code))
        if q.shape != (self.M, 2):
            raise ValueError("qubits must have shape (M, 2)")
        _check(_lib.qsim_state_set_product(self._h, q.ctypes.data, ctypes.c_void_p(_stream_ptr(stream))))

    def apply_product(self, qubits: np.ndarray, target, cmask, stream=None, kind=None):
        """current <- U_L ... U_1 (q_M (x) ... (x) q_1), the product input formed
        inside the first pass (qsim_apply_steps_product)."""
        q = np.ascontiguousarray(qubits, dtype=np_dtype(self.code))
        if q.shape != (self.M, 2):
            raise ValueError("qubits must have shape (M, 2)")
        st = pack_steps(target, cmask, kind)
        _check(_lib.qsim_apply_steps_product(self._h, q.ctypes.data, st.ctypes.data if len(st) else None, len(st),
                                             ctypes.c_void_p(_stream_ptr(stream))))

    def rowmap_apply(self, x_ptr: int, stream=None):
        """current <- k1(x(i)) with a device row array from rowmap_build."""
        _check(_lib.qsim_rowmap_apply(self._h, ctypes.c_void_p(_ptr(x_ptr)), ctypes.c_void_p(_stream_ptr(stream))))

    def apply_tile_pass(self, tile_mask: int, target, cmask, stream=None, kind=None):
        st = pack_steps(target, cmask, kind)
        _check(_lib.qsim_apply_tile_pass(self._h, int(tile_mask), st.ctypes.data if len(st) else None,
                                         len(st), ctypes.c_void_p(_stream_ptr(stream))))

    def apply_plain(self, target, cmask, stream=None, kind=None):
        st = pack_steps(target, cmask, kind)
        _check(_lib.qsim_apply_steps_plain(self._h, st.ctypes.data if len(st) else None, len(st),
                                           ctypes.c_void_p(_stream_ptr(stream))))

    def profile(self, enable: bool = True):
        _check(_lib.qsim_state_profile(self._h, 1 if enable else 0))

    def profile_read(self) -> dict:
        p = Profile()
        _check(_lib.qsim_state_profile_read(self._h, ctypes.byref(p)))
        return p.as_dict()

    def autotune(self, target, cmask, stream=None, kind=None) -> dict:
        """Measure candidate tunings for this diagram on this state (contents
        unchanged) and keep the fastest; returns it."""
        st = pack_steps(target, cmask, kind)
        t = Tuning()
        _check(_lib.qsim_autotune(self._h, st.ctypes.data if len(st) else None, len(st),
                                  ctypes.c_void_p(_stream_ptr(stream)), ctypes.byref(t)))
        return {k: getattr(t, k) for k, _ in Tuning._fields_}

    def set_tuning(self, tuning: Optional[dict]):
        t = _tuning_struct(tuning)
        _check(_lib.qsim_state_set_tuning(self._h, ctypes.byref(t) if t is not None else None))


def _ptr(buf) -> int:
    if isinstance(buf, int):
        return buf
    return int(buf.data_ptr())


def apply_batch(states: Sequence[State], steps: Sequence[Tuple], stream=None):
    """steps[c] = (target, cmask) or (target, cmask, kind) for circuit c."""
    n = len(states)
    packed = [pack_steps(*sc) for sc in steps]
    hs = (ctypes.c_void_p * n)(*[s.handle.value for s in states])
    ps = (ctypes.c_void_p * n)(*[p.ctypes.data if len(p) else None for p in packed])
    ls = (ctypes.c_uint64 * n)(*[len(p) for p in packed])
    _check(_lib.qsim_apply_batch(ctypes.cast(hs, ctypes.c_void_p), ctypes.cast(ps, ctypes.c_void_p),
                                 ctypes.cast(ls, ctypes.c_void_p), n, ctypes.c_void_p(_stream_ptr(stream))))


class PackedBatch:
    """The step lists of a batch in one contiguous qsim_step buffer, with the
    per-circuit pointer and length arrays qsim_apply_batch takes, so a
    batched call marshals three arrays instead of one object per circuit.
    steps[c] = (target, cmask) or (target, cmask, kind)."""

    def __init__(self, steps: Sequence[Tuple]):
        parts = [pack_steps(*sc) for sc in steps]
        self.lens = np.array([len(p) for p in parts], dtype=np.uint64)
        self.buf = np.concatenate(parts) if parts else np.zeros(0, dtype=STEP_DTYPE)
        if len(self.buf) == 0:
            self.buf = np.zeros(1, dtype=STEP_DTYPE)     # a valid base address
        offsets = np.concatenate([[0], np.cumsum(self.lens)[:-1]]).astype(np.uint64) if parts else self.lens
        self.ptrs = np.uint64(self.buf.ctypes.data) + offsets * np.uint64(STEP_DTYPE.itemsize)

    def __len__(self):
        return len(self.lens)


def _handles(states: Sequence[State]) -> np.ndarray:
    return np.fromiter((s._h.value for s in states), dtype=np.uint64, count=len(states))


def apply_batch_packed(states: Sequence[State], packed, stream=None):
    """apply_batch with the steps already packed: a PackedBatch, or a list of
    arrays from pack_steps."""
    n = len(states)
    if not isinstance(packed, PackedBatch):
        hs = (ctypes.c_void_p * n)(*[s.handle.value for s in states])
        ps = (ctypes.c_void_p * n)(*[p.ctypes.data if len(p) else None for p in packed])
        ls = (ctypes.c_uint64 * n)(*[len(p) for p in packed])
        _check(_lib.qsim_apply_batch(ctypes.cast(hs, ctypes.c_void_p), ctypes.cast(ps, ctypes.c_void_p),
                                     ctypes.cast(ls, ctypes.c_void_p), n, ctypes.c_void_p(_stream_ptr(stream))))
        return
    if len(packed) != n:
        raise ValueError("one step list per state")
    hs = _handles(states)
    _check(_lib.qsim_apply_batch(ctypes.c_void_p(hs.ctypes.data), ctypes.c_void_p(packed.ptrs.ctypes.data),
                                 ctypes.c_void_p(packed.lens.ctypes.data), n, ctypes.c_void_p(_stream_ptr(stream))))


def rowmap_build(M: int, target, cmask, x_dev, stream=None, kind=None):
    """Write the row array x of the diagram (k2(i) = k1(x(i))) into x_dev: a
    device buffer of 2^M uint32 (a torch tensor or a raw pointer).  Phase
    steps are rejected: a row array holds no signs."""
    st = pack_steps(target, cmask, kind)
    _check(_lib.qsim_rowmap_build(M, st.ctypes.data if len(st) else None, len(st), ctypes.c_void_p(_ptr(x_dev)),
                                  ctypes.c_void_p(_stream_ptr(stream))))


def batch_set_tiles_per_item(tiles: int):
    """Tiles of one pass per queue item of the batched kernel (0 = default)."""
    _check(_lib.qsim_batch_set_tiles_per_item(int(tiles)))


def batch_tiles_per_item() -> int:
    return int(_lib.qsim_batch_tiles_per_item())


BATCH_TUNING_FIELDS = ("tiles_per_item", "tile_bits", "circuit_tiles", "plan_search", "order")


def batch_set_tuning(dtype, tuning: Optional[dict]):
    """Batched-mode parameters for states of `dtype` (None: defaults)."""
    t = None
    if tuning is not None:
        t = BatchTuning()
        for k, v in tuning.items():
            if k not in BATCH_TUNING_FIELDS:
                raise ValueError(f"unknown batch tuning field {k!r}")
            setattr(t, k, int(v))
    _check(_lib.qsim_batch_set_tuning(dtype_code(dtype), ctypes.byref(t) if t is not None else None))


def batch_get_tuning(dtype) -> dict:
    t = BatchTuning()
    _check(_lib.qsim_batch_get_tuning(dtype_code(dtype), ctypes.byref(t)))
    return {k: getattr(t, k) for k in BATCH_TUNING_FIELDS}


def batch_autotune(states: Sequence[State], steps, stream=None) -> dict:
    """Choose the batched-mode parameters for this batch by measurement (the
    states' contents are unchanged) and keep them for its dtype; returns the
    choice with the measured times (and from_cache = 1 when the tuning cache
    named by QSIM_TUNING_CACHE supplied it).  steps: a PackedBatch or a list
    of (target, cmask[, kind])."""
    n = len(states)
    pb = steps if isinstance(steps, PackedBatch) else PackedBatch(steps)
    if len(pb) != n:
        raise ValueError("one step list per state")
    hs = _handles(states)
    out = BatchTuning()
    _check(_lib.qsim_batch_autotune(ctypes.c_void_p(hs.ctypes.data), ctypes.c_void_p(pb.ptrs.ctypes.data),
                                    ctypes.c_void_p(pb.lens.ctypes.data), n, ctypes.c_void_p(_stream_ptr(stream)),
                                    ctypes.byref(out)))
    return out.as_dict()


def batch_last_info() -> dict:
    """What the last batched launch did: circuits, items, passes, workgroups,
    algorithmic bytes, kernel time (ms) and its parameters."""
    out = BatchInfo()
    _check(_lib.qsim_batch_last_info(ctypes.byref(out)))
    return out.as_dict()


def batch_status():
    """Wait for the last batched launch; raise if it did not complete cleanly."""
    _check(_lib.qsim_batch_last_status())


def plan_describe(M: int, dtype, target, cmask, tuning: Optional[dict] = None, kind=None):
    """Host-only pass plan: (masks, lens, order)."""
    st = pack_steps(target, cmask, kind)
    L = len(st)
    n_passes = ctypes.c_uint32(0)
    t = _tuning_struct(tuning)
    order = np.zeros(max(L, 1), dtype=np.uint32)
    cap = max(L, 1)
    masks = np.zeros(cap, dtype=np.uint64)
    lens = np.zeros(cap, dtype=np.uint32)
    _check(_lib.qsim_plan_describe(M, dtype_code(dtype), st.ctypes.data if L else None, L,
                                   ctypes.byref(t) if t is not None else None, ctypes.byref(n_passes),
                                   masks.ctypes.data, lens.ctypes.data, cap, order.ctypes.data))
    p = n_passes.value
    return masks[:p].copy(), lens[:p].copy(), order[:L].copy()


def copy_bytes(dst_ptr: int, src_ptr: int, nbytes: int, stream=None):
    _check(_lib.qsim_copy_bytes(ctypes.c_void_p(dst_ptr), ctypes.c_void_p(src_ptr), nbytes,
                                ctypes.c_void_p(_stream_ptr(stream))))


class Server:
    """Request server (qsim_server_*): continuous batching over slot streams
    with an HBM arena, or one request at a time with ``fcfs=True``."""

    def __init__(self, budget_bytes: int = 0, max_slots: int = 0, portion_entries: int = 0,
                 fcfs: bool = False, max_bypass: int = 0, digest=False):
        cfg = ServerConfig()
        cfg.hbm_budget_bytes = int(budget_bytes)
        cfg.max_slots = int(max_slots)
        cfg.portion_entries = int(portion_entries)
        cfg.fcfs = 1 if fcfs else 0
        cfg.max_bypass = int(max_bypass)
        cfg.digest = int(digest)     # True / 1: every request; k > 1: every k-th request by id
        h = _lib.qsim_server_create(ctypes.byref(cfg))
        if not h:
            raise QsimError(ERR_NOMEM, "qsim_server_create failed")
        self._h = ctypes.c_void_p(h)

    def submit(self, M: int, dtype, target, cmask, k1: Optional[np.ndarray] = None, kind=None) -> int:
        st = pack_steps(target, cmask, kind)
        ptr = None
        if k1 is not None:
            k1 = np.ascontiguousarray(k1)
            if k1.dtype != np_dtype(dtype_code(dtype)) or k1.size != (1 << M):
                raise ValueError("k1 must hold 2^M entries of the request's dtype")
            ptr = k1.ctypes.data
        rid = _lib.qsim_server_submit(self._h, M, dtype_code(dtype), ptr, st.ctypes.data if len(st) else None,
                                      len(st))
        if rid < 0:
            raise QsimError(int(rid), "submit rejected")
        return int(rid)

    def drain(self):
        _check(_lib.qsim_server_drain(self._h))

    def info(self, rid: int) -> dict:
        r = RequestInfo()
        _check(_lib.qsim_server_request_info(self._h, rid, ctypes.byref(r)))
        return r.as_dict()

    def stats(self) -> dict:
        a, u = ctypes.c_uint64(0), ctypes.c_uint64(0)
        qd, rn = ctypes.c_uint32(0), ctypes.c_uint32(0)
        _check(_lib.qsim_server_stats(self._h, ctypes.byref(a), ctypes.byref(u), ctypes.byref(qd),
                                      ctypes.byref(rn)))
        return {"arena_bytes": a.value, "arena_used": u.value, "queued": qd.value, "running": rn.value}

    def close(self):
        if getattr(self, "_h", None):
            _lib.qsim_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


_MIX1 = np.uint64(0xBF58476D1CE4E5B9)
_MIX2 = np.uint64(0x94D049BB133111EB)
_DIGEST_KEY = np.uint64(0x9E3779B97F4A7C15)


def _mix(z: np.ndarray) -> np.ndarray:
    """SplitMix64's finaliser on a uint64 array (products wrap mod 2^64)."""
    z = (z ^ (z >> np.uint64(30))) * _MIX1
    z = (z ^ (z >> np.uint64(27))) * _MIX2
    return z ^ (z >> np.uint64(31))


class Digest:
    """Host-side copy of the server's result digest (qsim_request_info.digest),
    for checking a result read back some other way: the sum mod 2^64 over
    the result's 8-byte words w_j of mix(w_j ^ mix(j + key)), then mixed
    with the byte count.  Portions are added in row order."""

    def __init__(self):
        self.sum = 0
        self.n = 0

    def add(self, data, chunk_words: int = 1 << 21, threads: int = 8):
        w = np.frombuffer(data, dtype=np.uint64) if isinstance(data, (bytes, bytearray, memoryview)) \
            else np.ascontiguousarray(data).view(np.uint64).ravel()
        j0 = self.n // 8

        def part_sum(off):
            part = w[off:off + chunk_words]
            with np.errstate(over="ignore"):
                j = np.arange(j0 + off, j0 + off + len(part), dtype=np.uint64) + _DIGEST_KEY
                return int(_mix(part ^ _mix(j)).sum(dtype=np.uint64))

        offs = range(0, len(w), chunk_words)
        if len(offs) > 1 and threads > 1:
            from concurrent.futures import ThreadPoolExecutor
            with ThreadPoolExecutor(max_workers=threads) as ex:   # numpy releases the GIL
                total = sum(ex.map(part_sum, offs))
        else:
            total = sum(part_sum(o) for o in offs)
        self.sum = (self.sum + total) & ((1 << 64) - 1)
        self.n += 8 * len(w)
        return self

    def value(self) -> int:
        with np.errstate(over="ignore"):
            n = _mix(np.array([self.n], dtype=np.uint64))[0]
            return int(_mix(np.array([np.uint64(self.sum) ^ n], dtype=np.uint64))[0])


def digest_bytes(data) -> int:
    """The server's digest of a whole result (bytes or a numpy array)."""
    return Digest().add(data).value()
