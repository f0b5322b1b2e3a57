"""ctypes binding of libdiaq_hip (the C ABI in ``include/diaq.h``).

Argument marshalling only: every step of the hot path runs in the HIP
kernels of ``libdiaq_hip.so``.  PyTorch supplies device memory (tensors'
``data_ptr``) and the HIP stream (torch's current stream).  There is no CPU
fallback: if the library or a GPU is missing, calls raise.

Function names follow the C ABI: ``from_gate``, ``from_pauli_sum``,
``spmv``, ``fuse``, ``apply_circuit``, ``expect``, ``adjoint_grad``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Sequence

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdiaq_hip.so")

C64, C128 = 0, 1
TRANSPOSE, CONJUGATE, ADJOINT = 1, 2, 3

GATE_KINDS = {"I": 0, "H": 1, "X": 2, "Y": 3, "Z": 4, "S": 5, "SDG": 6, "T": 7, "TDG": 8, "SX": 9,
              "RX": 10, "RY": 11, "RZ": 12, "P": 13, "U3": 14, "SWAP": 15, "RXX": 16, "RYY": 17,
              "RZZ": 18, "MATRIX": 19}

STATUS = {0: "ok", 1: "invalid argument", 2: "not multiplyable", 3: "out of memory",
          4: "device error", 5: "unsupported"}


class DiaqError(RuntimeError):
    """A libdiaq_hip call returned a non-zero status."""

    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS.get(status, "status %d" % status), message))
        self.status = status


class diaq_gate_t(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("ntargets", ctypes.c_int32), ("ncontrols", ctypes.c_int32),
                ("targets", ctypes.c_int32 * 3), ("controls", ctypes.c_int32 * 3),
                ("params", ctypes.c_double * 3), ("param_index", ctypes.c_int32),
                ("param_scale", ctypes.c_double), ("matrix", ctypes.POINTER(ctypes.c_double))]


class diaq_plan_t(ctypes.Structure):
    _fields_ = [("fuse", ctypes.c_int32), ("max_fused_qubits", ctypes.c_int32), ("kron", ctypes.c_int32),
                ("rows_per_thread", ctypes.c_int32), ("block", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 3)]


class diaq_tuning_t(ctypes.Structure):
    _fields_ = [("spmv_rows", ctypes.c_int32), ("spmv_group_bits", ctypes.c_int32), ("spmv_chunk", ctypes.c_int32),
                ("spmv_nontemporal", ctypes.c_int32), ("spmv_group_min_qubit", ctypes.c_int32),
                ("expand_nontemporal", ctypes.c_int32), ("diag_pad", ctypes.c_int32),
                ("spmv_xcd_runs", ctypes.c_int32), ("spmv_group_qubits", ctypes.c_uint64),
                ("kron_stage_qubit", ctypes.c_int32), ("kron_split", ctypes.c_int32),
                ("kron_nontemporal", ctypes.c_int32), ("kron_small_qubits", ctypes.c_int32),
                ("kron_order", ctypes.c_int32), ("spmv_order", ctypes.c_int32),
                ("spmv_pack", ctypes.c_int32)]


class diaq_spmv_shape_t(ctypes.Structure):
    _fields_ = [("in_place", ctypes.c_int32), ("rows_per_lane", ctypes.c_int32), ("group", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("nontemporal", ctypes.c_int32), ("tile_log2", ctypes.c_int32),
                ("group_qubits", ctypes.c_int32 * 3), ("xcd_run_log2", ctypes.c_int32),
                ("pair_bit", ctypes.c_int32), ("tile_order", ctypes.c_int32), ("blocks", ctypes.c_int64),
                ("packed", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class diaq_chain_step_t(ctypes.Structure):
    _fields_ = [("ndiag", ctypes.c_int32), ("reserved", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("nvalues", ctypes.c_int64)]


class diaq_profile_t(ctypes.Structure):
    _fields_ = [("expand_launches", ctypes.c_int64), ("expand_ms", ctypes.c_double),
                ("expand_bytes", ctypes.c_double), ("spmv_launches", ctypes.c_int64),
                ("spmv_ms", ctypes.c_double), ("spmv_bytes", ctypes.c_double)]


_lib = None

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_U32 = ctypes.c_uint32
_D = ctypes.c_double

# name -> argtypes (restype is int status unless noted)
_SIGS = {
    "diaq_create": [_I32, _P, ctypes.POINTER(_P)],
    "diaq_set_stream": [_P, _P],
    "diaq_synchronize": [_P],
    "diaq_destroy": [_P],
    "diaq_dia_create": [_P, _I32, _I32, _I32, ctypes.POINTER(_I64), _P, ctypes.POINTER(_P)],
    "diaq_dia_info": [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                      ctypes.POINTER(_I64), ctypes.POINTER(_P)],
    "diaq_dia_offsets": [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64)],
    "diaq_dia_transpose": [_P, _I32, ctypes.POINTER(_P)],
    "diaq_dia_copy_values": [_P, _P, _P, _I32],
    "diaq_dia_free": [_P],
    "diaq_from_gate_query": [ctypes.POINTER(diaq_gate_t), _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I64),
                             ctypes.POINTER(_I64)],
    "diaq_from_gate": [_P, ctypes.POINTER(diaq_gate_t), _I32, _I32, ctypes.POINTER(_P)],
    "diaq_from_pauli_sum": [_P, _I32, _I32, _I32, ctypes.POINTER(ctypes.c_uint64),
                            ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(_D), ctypes.POINTER(_P)],
    "diaq_spmv": [_P, _P, _P, _P, _U32],
    "diaq_fuse": [_P, _P, _P, _D, ctypes.POINTER(_P)],
    "diaq_apply_circuit": [_P, ctypes.POINTER(diaq_gate_t), _I64, _I64, _I64, _I32, _I32, _P, _P,
                           ctypes.POINTER(diaq_plan_t)],
    "diaq_expect": [_P, _P, _P, _P, ctypes.POINTER(_D)],
    "diaq_expect_noalloc": [_P, _P, _P, _P, _P],
    "diaq_adjoint_grad": [_P, ctypes.POINTER(diaq_gate_t), _I64, _I32, _I32, _P, _P, _P, _I64,
                          ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(diaq_plan_t)],
    "diaq_set_tuning": [_P, ctypes.POINTER(diaq_tuning_t)],
    "diaq_get_tuning": [_P, ctypes.POINTER(diaq_tuning_t)],
    "diaq_spmv_shape": [ctypes.POINTER(diaq_gate_t), _I32, _I32, ctypes.POINTER(diaq_tuning_t),
                        ctypes.POINTER(diaq_spmv_shape_t)],
    "diaq_plan_count": [ctypes.POINTER(diaq_gate_t), _I64, _I32, _I32, ctypes.POINTER(diaq_plan_t),
                        ctypes.POINTER(_I64), ctypes.POINTER(_D)],
    "diaq_batch_create": [_P, _P, _I32, _U32, ctypes.POINTER(_P)],
    "diaq_batch_run": [_P, ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_D)],
    "diaq_batch_free": [_P],
    "diaq_autotune": [_P, _I32, _I32, ctypes.c_char_p, ctypes.POINTER(diaq_tuning_t)],
    "diaq_autotune_plan": [_P, ctypes.POINTER(diaq_gate_t), _I64, _I32, _I32, _I32, _I32, ctypes.POINTER(diaq_plan_t)],
    "diaq_dia_nnz": [_P, _P, _D, ctypes.POINTER(_I64)],
    "diaq_trace_product": [_P, _P, _P, ctypes.POINTER(_D)],
    "diaq_unitary": [_P, ctypes.POINTER(diaq_gate_t), _I64, _I32, _I32, _P, _D, ctypes.POINTER(diaq_chain_step_t),
                     ctypes.POINTER(_P)],
    "diaq_density_evolve": [_P, ctypes.POINTER(diaq_gate_t), _I64, _P, _D, ctypes.POINTER(diaq_chain_step_t),
                            ctypes.POINTER(_P)],
    "diaq_circuit_graph_create": [_P, ctypes.POINTER(diaq_gate_t), _I64, _I32, _I32, _P, _P,
                                  ctypes.POINTER(diaq_plan_t), ctypes.POINTER(_P)],
    "diaq_circuit_graph_launch": [_P, _P],
    "diaq_circuit_graph_nodes": [_P, ctypes.POINTER(_I64)],
    "diaq_circuit_graph_free": [_P],
    "diaq_copy": [_P, _P, _P, ctypes.c_size_t],
    "diaq_profile_start": [_P],
    "diaq_profile_stop": [_P, ctypes.POINTER(diaq_profile_t)],
}

EXPORTED = sorted(_SIGS) + ["diaq_last_error", "diaq_status_string"]


def load(path: str = LIB_PATH):
    """Open libdiaq_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError("libdiaq_hip.so not built at %s; run __graft_entry__.build()" % path)
        lib = ctypes.CDLL(path)
        for name, args in _SIGS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        lib.diaq_last_error.restype = ctypes.c_char_p
        lib.diaq_last_error.argtypes = []
        lib.diaq_status_string.restype = ctypes.c_char_p
        lib.diaq_status_string.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def _check(status: int):
    if status != 0:
        raise DiaqError(status, load().diaq_last_error().decode(errors="replace"))


# --------------------------------------------------------------------------
# Contexts (one per device and torch stream)
# --------------------------------------------------------------------------

_contexts: dict = {}


class Context:
    def __init__(self, device: int = 0, stream: int | None = None):
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device).cuda_stream
        h = _P()
        _check(load().diaq_create(device, _P(self.stream), ctypes.byref(h)))
        self.handle = h

    def synchronize(self):
        _check(load().diaq_synchronize(self.handle))

    def close(self):
        if self.handle:
            load().diaq_destroy(self.handle)
            self.handle = None


def context(device: int | None = None) -> Context:
    """The context bound to torch's current stream on `device`."""
    if not torch.cuda.is_available():
        raise RuntimeError("libdiaq_hip needs a HIP GPU; none is visible")
    if device is None:
        device = torch.cuda.current_device()
    stream = torch.cuda.current_stream(device).cuda_stream
    key = (device, stream)
    ctx = _contexts.get(key)
    if ctx is None:
        ctx = Context(device, stream)
        _contexts[key] = ctx
    return ctx


# --------------------------------------------------------------------------
# Gates
# --------------------------------------------------------------------------

def _dtype_code(dtype) -> int:
    if dtype in (torch.complex128, np.complex128, "c128", C128):
        return C128
    if dtype in (torch.complex64, np.complex64, "c64", C64):
        return C64
    raise ValueError("unsupported dtype %r (complex64 or complex128)" % (dtype,))


def _torch_dtype(code: int):
    return torch.complex128 if code == C128 else torch.complex64


def gate_struct(g, keep: list) -> diaq_gate_t:
    """Marshal one gate object (kind, targets, controls, params,
    param_index, param_scale, matrix)."""
    s = diaq_gate_t()
    s.kind = GATE_KINDS[g.kind]
    t = tuple(g.targets)
    c = tuple(getattr(g, "controls", ()) or ())
    if len(t) > 3 or len(c) > 3:
        raise DiaqError(1, "a gate takes at most 3 targets and 3 controls")
    s.ntargets, s.ncontrols = len(t), len(c)
    for j, q in enumerate(t):
        s.targets[j] = q
    for j, q in enumerate(c):
        s.controls[j] = q
    for j, p in enumerate(tuple(getattr(g, "params", ()) or ())):
        s.params[j] = float(p)
    s.param_index = int(getattr(g, "param_index", -1))
    s.param_scale = float(getattr(g, "param_scale", 1.0))
    m = getattr(g, "matrix", None)
    if m is not None:
        arr = np.ascontiguousarray(np.asarray(m, dtype=np.complex128))
        keep.append(arr)
        s.matrix = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return s


def gate_array(gates: Sequence):
    keep: list = []
    arr = (diaq_gate_t * max(1, len(gates)))()
    for i, g in enumerate(gates):
        arr[i] = gate_struct(g, keep)
    return arr, keep


# --------------------------------------------------------------------------
# DiaQ matrices
# --------------------------------------------------------------------------

class DiaqMatrix:
    """Handle to a DiaQ matrix living in device memory (Sec. IV)."""

    def __init__(self, handle, ctx: Context, owner=None):
        self.handle = handle
        self.ctx = ctx
        self._owner = owner  # keeps shared storage alive (transpose views)

    def __del__(self):
        try:
            if self.handle and _lib is not None:
                _lib.diaq_dia_free(self.handle)
        except Exception:
            pass
        self.handle = None

    def info(self):
        n, nd, dt, nv = _I32(), _I32(), _I32(), _I64()
        vp = _P()
        _check(load().diaq_dia_info(self.handle, ctypes.byref(n), ctypes.byref(nd), ctypes.byref(dt),
                                    ctypes.byref(nv), ctypes.byref(vp)))
        return n.value, nd.value, dt.value, nv.value, vp.value

    @property
    def nqubits(self) -> int:
        return self.info()[0]

    @property
    def ndiag(self) -> int:
        return self.info()[1]

    @property
    def dtype(self):
        return _torch_dtype(self.info()[2])

    def offsets(self) -> np.ndarray:
        nd = self.ndiag
        o = np.zeros(max(nd, 1), dtype=np.int64)
        s = np.zeros(nd + 1, dtype=np.int64)
        _check(load().diaq_dia_offsets(self.handle, o.ctypes.data_as(ctypes.POINTER(_I64)),
                                       s.ctypes.data_as(ctypes.POINTER(_I64))))
        return o[:nd]

    def stored_offsets(self):
        return self.offsets()

    def values(self) -> np.ndarray:
        """Host copy of the stored (packed) diagonals."""
        n, nd, dt, nv, _ = self.info()
        out = np.zeros(nv, dtype=np.complex128 if dt == C128 else np.complex64)
        if nv:
            _check(load().diaq_dia_copy_values(self.ctx.handle, self.handle, _P(out.ctypes.data), 1))
        return out

    def diagonals(self) -> dict:
        """{dIndex: compact diagonal} as applied (transposed views relabelled)."""
        n, nd, dt, nv, _ = self.info()
        vals = self.values()
        o = np.zeros(max(nd, 1), dtype=np.int64)
        s = np.zeros(nd + 1, dtype=np.int64)
        _check(load().diaq_dia_offsets(self.handle, o.ctypes.data_as(ctypes.POINTER(_I64)),
                                       s.ctypes.data_as(ctypes.POINTER(_I64))))
        N = 1 << n
        out = {}
        for k in range(nd):
            d = int(o[k])
            out[d] = vals[s[k]:s[k] + N - abs(d)]
        return out

    def transpose(self, conjugate: bool = False) -> "DiaqMatrix":
        h = _P()
        _check(load().diaq_dia_transpose(self.handle, 1 if conjugate else 0, ctypes.byref(h)))
        return DiaqMatrix(h, self.ctx, owner=self)


def dia_create(n: int, offsets: Iterable[int], values: torch.Tensor | None = None, dtype=torch.complex128,
               ctx: Context | None = None) -> DiaqMatrix:
    """Wrap caller-filled packed diagonals (a device tensor, kept alive by
    the returned handle) or allocate zeroed ones."""
    ctx = ctx or context()
    offs = np.ascontiguousarray(np.asarray(list(offsets), dtype=np.int64))
    h = _P()
    vp = None
    if values is not None:
        if not values.is_cuda or not values.is_contiguous():
            raise ValueError("values must be a contiguous device tensor")
        dtype = values.dtype
        vp = _P(values.data_ptr())
    _check(load().diaq_dia_create(ctx.handle, n, _dtype_code(dtype), len(offs),
                                  offs.ctypes.data_as(ctypes.POINTER(_I64)), vp, ctypes.byref(h)))
    return DiaqMatrix(h, ctx, owner=values)


def from_dense_diagonals(n: int, diags: dict, dtype=torch.complex128, ctx: Context | None = None) -> DiaqMatrix:
    """numpy -> DiaQ converter: {dIndex: compact diagonal} to a device matrix."""
    offs = sorted(diags)
    packed = np.concatenate([np.asarray(diags[d]) for d in offs]) if offs else np.zeros(0)
    t = torch.from_numpy(np.ascontiguousarray(packed.astype(np.complex128 if dtype == torch.complex128
                                                            else np.complex64))).to("cuda")
    return dia_create(n, offs, t if t.numel() else None, dtype, ctx)


def from_dense(A: np.ndarray, dtype=torch.complex128, ctx: Context | None = None) -> DiaqMatrix:
    """numpy dense -> DiaQ converter: the diagonals holding a non-zero."""
    A = np.asarray(A)
    N = A.shape[0]
    if A.shape != (N, N) or N & (N - 1) or N < 2:
        raise ValueError("need a square 2^n x 2^n matrix")
    diags = {d: np.diagonal(A, d) for d in range(-(N - 1), N) if np.any(np.diagonal(A, d) != 0)}
    return from_dense_diagonals(N.bit_length() - 1, diags, dtype, ctx)


def to_dense(M: DiaqMatrix) -> np.ndarray:
    """DiaQ -> numpy dense converter (host copy of the applied matrix)."""
    n, _, dt, _, _ = M.info()
    N = 1 << n
    A = np.zeros((N, N), dtype=np.complex128 if dt == C128 else np.complex64)
    for d, v in M.diagonals().items():
        t = np.arange(N - abs(d))
        A[t + max(0, -d), t + max(0, d)] = v
    return A


def from_gate_query(gate, n: int):
    keep: list = []
    s = gate_struct(gate, keep)
    nd = _I32()
    offs = np.zeros(27, dtype=np.int64)
    nv = _I64()
    _check(load().diaq_from_gate_query(ctypes.byref(s), n, ctypes.byref(nd),
                                       offs.ctypes.data_as(ctypes.POINTER(_I64)), ctypes.byref(nv)))
    return offs[:nd.value].copy(), nv.value


def from_gate(gate, n: int, dtype=torch.complex128, ctx: Context | None = None) -> DiaqMatrix:
    ctx = ctx or context()
    keep: list = []
    s = gate_struct(gate, keep)
    h = _P()
    _check(load().diaq_from_gate(ctx.handle, ctypes.byref(s), n, _dtype_code(dtype), ctypes.byref(h)))
    return DiaqMatrix(h, ctx)


def from_pauli_sum(n: int, terms, dtype=torch.complex128, ctx: Context | None = None) -> DiaqMatrix:
    """terms = [(xmask, zmask, coef)], term = coef * i^{|x&z|} X^x Z^z."""
    ctx = ctx or context()
    xs = np.ascontiguousarray(np.array([t[0] for t in terms], dtype=np.uint64))
    zs = np.ascontiguousarray(np.array([t[1] for t in terms], dtype=np.uint64))
    cs = np.ascontiguousarray(np.array([t[2] for t in terms], dtype=np.float64))
    h = _P()
    _check(load().diaq_from_pauli_sum(ctx.handle, n, _dtype_code(dtype), len(terms),
                                      xs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                      zs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                      cs.ctypes.data_as(ctypes.POINTER(_D)), ctypes.byref(h)))
    return DiaqMatrix(h, ctx)


# --------------------------------------------------------------------------
# Kernels
# --------------------------------------------------------------------------

def _vec(t: torch.Tensor, n: int, dtype_code: int, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous() or t.numel() != (1 << n) or _dtype_code(t.dtype) != dtype_code:
        raise ValueError("%s must be a contiguous %s vector of 2^%d elements" % (name, _torch_dtype(dtype_code), n))
    return _P(t.data_ptr())


def spmv(A: DiaqMatrix, x: torch.Tensor, y: torch.Tensor | None = None, flags: int = 0) -> torch.Tensor:
    """y <- op(A) x (Alg. 2)."""
    n, _, dt, _, _ = A.info()
    if y is None:
        y = torch.empty_like(x)
    _check(load().diaq_spmv(A.ctx.handle, A.handle, _vec(x, n, dt, "x"), _vec(y, n, dt, "y"), flags))
    return y


def fuse(first: DiaqMatrix, second: DiaqMatrix, drop_tol: float = 0.0) -> DiaqMatrix:
    """second * first (Alg. 1)."""
    h = _P()
    _check(load().diaq_fuse(first.ctx.handle, first.handle, second.handle, drop_tol, ctypes.byref(h)))
    return DiaqMatrix(h, first.ctx)


def make_plan(fuse: bool = False, max_fused_qubits: int = 0, kron: bool = False, rows_per_thread: int = 0,
              block: int = 0) -> diaq_plan_t:
    p = diaq_plan_t()
    p.fuse, p.max_fused_qubits, p.kron = int(fuse), max_fused_qubits, int(kron)
    p.rows_per_thread, p.block = rows_per_thread, block
    return p


def apply_circuit(gates: Sequence, state: torch.Tensor, n: int | None = None, scratch: torch.Tensor | None = None,
                  plan: diaq_plan_t | None = None, begin: int = 0, end: int | None = None,
                  ctx: Context | None = None, marshalled=None) -> torch.Tensor:
    """In place: state <- U_{end-1} ... U_begin state."""
    ctx = ctx or context(state.device.index)
    if n is None:
        n = int(state.numel()).bit_length() - 1
    dt = _dtype_code(state.dtype)
    if scratch is None:
        scratch = torch.empty_like(state)
    arr, keep = marshalled if marshalled is not None else gate_array(gates)
    ng = len(gates)
    e = ng if end is None else end
    _check(load().diaq_apply_circuit(ctx.handle, arr, ng, begin, e, n, dt, _vec(state, n, dt, "state"),
                                     _vec(scratch, n, dt, "scratch"),
                                     ctypes.byref(plan) if plan is not None else None))
    return state


class CircuitGraph:
    """One application of `gates` to `state` (with `scratch`) under `plan`,
    recorded once as a HIP graph; ``launch()`` replays it on the context's
    stream.  The graph keeps `state` and `scratch` alive."""

    def __init__(self, gates: Sequence, state: torch.Tensor, scratch: torch.Tensor | None = None,
                 n: int | None = None, plan: diaq_plan_t | None = None, ctx: Context | None = None):
        self.ctx = ctx or context(state.device.index)
        if n is None:
            n = int(state.numel()).bit_length() - 1
        dt = _dtype_code(state.dtype)
        self.state = state
        self.scratch = scratch if scratch is not None else torch.empty_like(state)
        arr, keep = gate_array(gates)
        h = _P()
        _check(load().diaq_circuit_graph_create(self.ctx.handle, arr, len(gates), n, dt,
                                                _vec(state, n, dt, "state"), _vec(self.scratch, n, dt, "scratch"),
                                                ctypes.byref(plan) if plan is not None else None, ctypes.byref(h)))
        self.handle = h

    def launch(self) -> torch.Tensor:
        _check(load().diaq_circuit_graph_launch(self.ctx.handle, self.handle))
        return self.state

    def nodes(self) -> int:
        v = _I64()
        _check(load().diaq_circuit_graph_nodes(self.handle, ctypes.byref(v)))
        return int(v.value)

    def close(self):
        if getattr(self, "handle", None):
            _check(load().diaq_circuit_graph_free(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def copy(src: torch.Tensor, dst: torch.Tensor, ctx: Context | None = None) -> torch.Tensor:
    """dst <- src on the device (same size, contiguous, 16-byte aligned)."""
    if src.numel() * src.element_size() != dst.numel() * dst.element_size():
        raise ValueError("copy needs equal sizes")
    if not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("copy needs contiguous tensors")
    ctx = ctx or context(src.device.index)
    _check(load().diaq_copy(ctx.handle, _P(src.data_ptr()), _P(dst.data_ptr()), src.numel() * src.element_size()))
    return dst


def expect(H: DiaqMatrix, psi: torch.Tensor, phi: torch.Tensor | None = None) -> complex:
    """<psi|H|phi> (phi defaults to psi); synchronises the stream."""
    n, _, dt, _, _ = H.info()
    out = (_D * 2)()
    _check(load().diaq_expect(H.ctx.handle, H.handle, _vec(psi, n, dt, "psi"),
                              _vec(phi, n, dt, "phi") if phi is not None else None, out))
    return complex(out[0], out[1])


def expect_noalloc(H: DiaqMatrix, psi: torch.Tensor, out: torch.Tensor, phi: torch.Tensor | None = None) -> torch.Tensor:
    """<psi|H|phi> written into out (float64 device tensor of 2 elements:
    real, imaginary) without any allocation or synchronisation (for graph
    capture and serving loops); returns out."""
    n, _, dt, _, _ = H.info()
    if out.dtype != torch.float64 or out.numel() < 2 or not out.is_cuda or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 device tensor of 2 elements")
    _check(load().diaq_expect_noalloc(H.ctx.handle, H.handle, _vec(psi, n, dt, "psi"),
                                      _vec(phi, n, dt, "phi") if phi is not None else None, _P(out.data_ptr())))
    return out


def adjoint_grad(gates: Sequence, H: DiaqMatrix, psi0: torch.Tensor, nparams: int,
                 work: torch.Tensor | None = None, plan: diaq_plan_t | None = None, marshalled=None):
    """(E, dE/dtheta) by the adjoint reverse sweep; synchronises.  marshalled:
    gate_array(gates) from an earlier call, reused as it is."""
    n, _, dt, _, _ = H.info()
    if work is None:
        work = torch.empty(3 << n, dtype=psi0.dtype, device=psi0.device)
    if work.numel() < (3 << n) or work.dtype != psi0.dtype or not work.is_contiguous():
        raise ValueError("work must hold 3 * 2^n contiguous elements of the state dtype")
    arr, keep = marshalled if marshalled is not None else gate_array(gates)
    e = _D()
    grad = np.zeros(max(nparams, 1), dtype=np.float64)
    _check(load().diaq_adjoint_grad(H.ctx.handle, arr, len(gates), n, dt, H.handle, _vec(psi0, n, dt, "psi0"),
                                    _P(work.data_ptr()), nparams, ctypes.byref(e),
                                    grad.ctypes.data_as(ctypes.POINTER(_D)),
                                    ctypes.byref(plan) if plan is not None else None))
    return e.value, grad[:nparams]


def set_tuning(ctx: Context | None = None, **knobs):
    """Set product-kernel knobs (the fields of diaq_tuning_t: spmv_rows,
    spmv_group_bits, spmv_chunk, spmv_nontemporal, spmv_group_min_qubit,
    expand_nontemporal, diag_pad, spmv_xcd_runs, spmv_group_qubits);
    unnamed knobs keep their current value."""
    ctx = ctx or context()
    t = diaq_tuning_t()
    _check(load().diaq_get_tuning(ctx.handle, ctypes.byref(t)))
    for k, v in knobs.items():
        setattr(t, k, int(v))
    _check(load().diaq_set_tuning(ctx.handle, ctypes.byref(t)))


def get_tuning(ctx: Context | None = None) -> dict:
    ctx = ctx or context()
    t = diaq_tuning_t()
    _check(load().diaq_get_tuning(ctx.handle, ctypes.byref(t)))
    return {f: getattr(t, f) for f, _ in diaq_tuning_t._fields_ if not f.endswith("reserved")}


def profile_start(ctx: Context | None = None):
    """Start timing apply_circuit's kernels with HIP events."""
    ctx = ctx or context()
    _check(load().diaq_profile_start(ctx.handle))


def profile_stop(ctx: Context | None = None) -> dict:
    """Stop timing; returns launch counts, milliseconds and algorithmic
    bytes of the expansion and product kernels (synchronises)."""
    ctx = ctx or context()
    p = diaq_profile_t()
    _check(load().diaq_profile_stop(ctx.handle, ctypes.byref(p)))
    return {f: getattr(p, f) for f, _ in diaq_profile_t._fields_}


class DiaqExpectation(torch.autograd.Function):
    """E(theta) = <psi(theta)|H|psi(theta)> with the adjoint backward.

    ``build(theta_list) -> gates`` rebuilds the circuit from the parameter
    values (gates carry param_index / param_scale)."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, build, H: DiaqMatrix, psi0: torch.Tensor):
        th = theta.detach().cpu().double().numpy()
        gates = build(th)
        e, g = adjoint_grad(gates, H, psi0, th.size)
        # the value and the saved gradient live where theta lives
        ctx.save_for_backward(torch.from_numpy(g).to(device=theta.device, dtype=theta.dtype))
        return torch.tensor(e, dtype=theta.dtype, device=theta.device)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out * g, None, None, None


def spmv_shape(gate, n: int, dtype=torch.complex128, **knobs) -> dict:
    """Launch shape of the product kernel for gate's expansion at n qubits
    under the tuning knobs (fields of diaq_tuning_t; unnamed ones 0 =
    defaults).  Host-only, no GPU needed."""
    t = diaq_tuning_t()
    for k, v in knobs.items():
        setattr(t, k, int(v))
    keep: list = []
    g = gate_struct(gate, keep)
    out = diaq_spmv_shape_t()
    _check(load().diaq_spmv_shape(ctypes.byref(g), n, _dtype_code(dtype), ctypes.byref(t), ctypes.byref(out)))
    d = {f: getattr(out, f) for f, _ in diaq_spmv_shape_t._fields_ if f != "reserved"}
    d["group_qubits"] = [q for q in out.group_qubits if q >= 0]
    return d


def plan_count(gates: Sequence, n: int, plan: diaq_plan_t | None = None, dtype=torch.complex128):
    """(operations, algorithmic bytes) diaq_apply_circuit issues for `gates`
    under `plan` (host-only, no GPU needed)."""
    arr, keep = gate_array(gates)
    nops = _I64()
    b = _D()
    _check(load().diaq_plan_count(arr, len(gates), n, _dtype_code(dtype),
                                  ctypes.byref(plan) if plan is not None else None, ctypes.byref(nops),
                                  ctypes.byref(b)))
    return nops.value, b.value


# --------------------------------------------------------------------------
# Batched circuits (one persistent launch, optional hipGraph replay)
# --------------------------------------------------------------------------

class diaq_circuit_t(ctypes.Structure):
    _fields_ = [("nqubits", ctypes.c_int32), ("nparams", ctypes.c_int32), ("ngates", ctypes.c_int64),
                ("gates", ctypes.POINTER(diaq_gate_t)), ("nterms", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("zmask", ctypes.POINTER(ctypes.c_uint64)), ("coef", ctypes.POINTER(ctypes.c_double))]


BATCH_GRAPH = 1


class Batch:
    """Circuits uploaded once and run together: ``run(theta)`` returns the
    expectation values and the per-circuit adjoint gradients.

    ``circuits`` is a list of (nqubits, gates, terms, nparams) where terms
    are diagonal Pauli strings (xmask must be 0)."""

    def __init__(self, circuits, graph: bool = False, ctx: Context | None = None):
        self.ctx = ctx or context()
        self._keep = []
        arr = (diaq_circuit_t * max(1, len(circuits)))()
        self.nparams = []
        for i, (n, gates, terms, nparams) in enumerate(circuits):
            garr, keep = gate_array(gates)
            if any(t[0] for t in terms):
                raise ValueError("batched observables must be diagonal (xmask = 0)")
            zm = np.ascontiguousarray(np.array([t[1] for t in terms], dtype=np.uint64))
            cf = np.ascontiguousarray(np.array([t[2] for t in terms], dtype=np.float64))
            self._keep += [garr, keep, zm, cf]
            c = arr[i]
            c.nqubits, c.nparams, c.ngates = n, nparams, len(gates)
            c.gates = ctypes.cast(garr, ctypes.POINTER(diaq_gate_t))
            c.nterms = len(terms)
            c.zmask = zm.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
            c.coef = cf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            self.nparams.append(nparams)
        self.ncirc = len(circuits)
        h = _P()
        _check(load().diaq_batch_create(self.ctx.handle, arr, len(circuits), BATCH_GRAPH if graph else 0,
                                        ctypes.byref(h)))
        self.handle = h
        self._keep = []  # the library copied everything

    def run(self, theta=None):
        ev = np.zeros(max(1, self.ncirc))
        gr = np.zeros(max(1, sum(self.nparams)))
        tp = None
        if theta is not None:
            th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
            if th.size != sum(self.nparams):
                raise ValueError("theta needs %d entries" % sum(self.nparams))
            tp = th.ctypes.data_as(ctypes.POINTER(_D))
        _check(load().diaq_batch_run(self.handle, tp, ev.ctypes.data_as(ctypes.POINTER(_D)),
                                     gr.ctypes.data_as(ctypes.POINTER(_D))))
        out, k = [], 0
        for p in self.nparams:
            out.append(gr[k:k + p].copy())
            k += p
        return ev[:self.ncirc].copy(), out

    def __del__(self):
        try:
            if getattr(self, "handle", None) and _lib is not None:
                _lib.diaq_batch_free(self.handle)
        except Exception:
            pass
        self.handle = None


# --------------------------------------------------------------------------
# Autotuning
# --------------------------------------------------------------------------

def autotune(n: int, dtype=torch.complex128, cache_path: str | None = None, ctx: Context | None = None) -> dict:
    """Time the product kernel's candidate knobs at 2^n elements, install
    the fastest in the context and return it (cached in a JSON file)."""
    ctx = ctx or context()
    t = diaq_tuning_t()
    _check(load().diaq_autotune(ctx.handle, n, _dtype_code(dtype),
                                cache_path.encode() if cache_path else None, ctypes.byref(t)))
    return {f: getattr(t, f) for f, _ in diaq_tuning_t._fields_ if not f.endswith("reserved")}


def autotune_plan(gates: Sequence, n: int, dtype=torch.complex128, allow_kron: bool = False, measure: int = 3,
                  ctx: Context | None = None) -> diaq_plan_t:
    """Plan (fusion depth, DiaQ or Alg. 3 products) for one circuit, ranked
    by bytes and decided by timing the leaders on its first gates."""
    ctx = ctx or context()
    arr, keep = gate_array(gates)
    p = diaq_plan_t()
    _check(load().diaq_autotune_plan(ctx.handle, arr, len(gates), n, _dtype_code(dtype), int(allow_kron), measure,
                                     ctypes.byref(p)))
    return p


# --------------------------------------------------------------------------
# Matrix-level simulation: unitary and density-matrix evolution
# --------------------------------------------------------------------------

def dia_nnz(A: DiaqMatrix, tol: float = 0.0) -> int:
    """Stored elements with |v| > tol (v != 0 when tol = 0)."""
    out = _I64()
    _check(load().diaq_dia_nnz(A.ctx.handle, A.handle, float(tol), ctypes.byref(out)))
    return out.value


def trace_product(A: DiaqMatrix, B: DiaqMatrix) -> complex:
    """Tr(A B) (e.g. Tr(H rho), or the purity Tr(rho rho))."""
    out = (_D * 2)()
    _check(load().diaq_trace_product(A.ctx.handle, A.handle, B.handle, out))
    return complex(out[0], out[1])


def _steps_array(steps, count: int) -> np.ndarray:
    rec = np.zeros(count, dtype=[("ndiag", np.int32), ("nnz", np.int64), ("nvalues", np.int64)])
    for t in range(count):
        rec[t] = (steps[t].ndiag, steps[t].nnz, steps[t].nvalues)
    return rec


def unitary(gates: Sequence, n: int, dtype=torch.complex128, start: DiaqMatrix | None = None,
            drop_tol: float = 0.0, track: bool = True, ctx: Context | None = None):
    """Unitary simulation: (U, per-gate records of ndiag / nnz / nvalues)
    with U = G_last ... G_first * start (identity when start is None)."""
    ctx = ctx or context()
    arr, keep = gate_array(gates)
    steps = (diaq_chain_step_t * max(1, len(gates)))() if track else None
    h = _P()
    _check(load().diaq_unitary(ctx.handle, arr, len(gates), n, _dtype_code(dtype),
                               start.handle if start is not None else None, float(drop_tol), steps,
                               ctypes.byref(h)))
    return DiaqMatrix(h, ctx), (_steps_array(steps, len(gates)) if track else None)


def density_evolve(gates: Sequence, rho: DiaqMatrix, drop_tol: float = 0.0, track: bool = True):
    """rho <- G rho G^dagger for each gate: (rho_out, per-gate records)."""
    arr, keep = gate_array(gates)
    steps = (diaq_chain_step_t * max(1, len(gates)))() if track else None
    h = _P()
    _check(load().diaq_density_evolve(rho.ctx.handle, arr, len(gates), rho.handle, float(drop_tol), steps,
                                      ctypes.byref(h)))
    return DiaqMatrix(h, rho.ctx), (_steps_array(steps, len(gates)) if track else None)
