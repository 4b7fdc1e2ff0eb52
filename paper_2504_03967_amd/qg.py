"""ctypes binding of libqg.so (the C ABI declared in include/qg.h).

Argument marshalling only: every step of the simulation runs in the library's
HIP kernels.  PyTorch supplies device memory and the stream.  The module fails
loudly when the built library is missing; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch  # loads the HIP runtime the library binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqg.so")

QG_OK, QG_EINVAL, QG_ENOMEM, QG_EDEVICE, QG_EUNSUPPORTED, QG_EINTERNAL = 0, -1, -2, -3, -4, -5
C64, C128 = 0, 1
FUSE_NONE, FUSE_GREEDY, FUSE_LEARNED = 0, 1, 2
OBS_ZZ_CHAIN, OBS_CSR = 0, 1

EXPORTS = (
    "qg_state_alloc", "qg_state_free", "qg_state_reset", "qg_state_set_stream", "qg_state_info",
    "qg_apply_circuit", "qg_apply_from_zero", "qg_probs", "qg_sample", "qg_expval", "qg_adjoint_grad", "qg_batch_expval",
    "qg_plan_passes", "qg_plan_kernels", "qg_last_error", "qg_version", "qg_set_tuning", "qg_get_tuning",
    "qg_batch_create", "qg_batch_set_params", "qg_batch_launch", "qg_batch_free",
    "qg_mlp_create", "qg_mlp_n_params", "qg_mlp_set_params", "qg_mlp_get_params", "qg_mlp_forward",
    "qg_mlp_grad", "qg_mlp_adam_step", "qg_mlp_train", "qg_mlp_free", "qg_pass_features", "qg_set_cost_model",
    "qg_autotune", "qg_expval_noalloc", "qg_plan_bytes",
)
PASS_FEATURES = 24
PASS_CONFIGS = 5
PASS_DENSE = 4


class QGError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"qg status {status}: {msg}")
        self.status = status


class _Circuit(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_gates", ctypes.c_int32),
                ("gate_type", ctypes.c_void_p), ("gate_param", ctypes.c_void_p),
                ("param_idx", ctypes.c_void_p)]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(python -m paper_2504_03967_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    sig = {
        "qg_state_alloc": [ctypes.c_int, ctypes.c_int, P, ctypes.c_size_t, P, P],
        "qg_state_free": [P],
        "qg_state_reset": [P],
        "qg_state_set_stream": [P, P],
        "qg_state_info": [P, P, P, P],
        "qg_apply_circuit": [P, P, ctypes.c_int],
        "qg_apply_from_zero": [P, P, ctypes.c_int],
        "qg_probs": [P, P, I64, P],
        "qg_sample": [P, I64, U64, P],
        "qg_expval": [P, P, P, ctypes.c_int, P, P],
        "qg_expval_noalloc": [P, P, P, ctypes.c_int, P, P],
        "qg_adjoint_grad": [P, ctypes.c_int, P, P, ctypes.c_int, ctypes.c_int, P, P, P],
        "qg_batch_expval": [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P, P, P],
        "qg_plan_passes": [P, ctypes.c_int, ctypes.c_int, P, P],
        "qg_plan_kernels": [P, ctypes.c_int, ctypes.c_int, P, ctypes.c_int32, P],
        "qg_plan_bytes": [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P],
        "qg_batch_create": [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P, P, P, P],
        "qg_batch_set_params": [P, P],
        "qg_batch_launch": [P],
        "qg_batch_free": [P],
        "qg_mlp_create": [ctypes.c_int, ctypes.c_int, U64, P, P],
        "qg_mlp_n_params": [P, P],
        "qg_mlp_set_params": [P, P],
        "qg_mlp_get_params": [P, P],
        "qg_mlp_forward": [P, P, ctypes.c_int, P],
        "qg_mlp_grad": [P, P, P, ctypes.c_int, P, P],
        "qg_mlp_adam_step": [P, P, ctypes.c_float],
        "qg_mlp_train": [P, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_float, U64, P],
        "qg_mlp_free": [P],
        "qg_pass_features": [P, ctypes.c_int, ctypes.c_int, P, P],
        "qg_set_cost_model": [P],
        "qg_autotune": [P, ctypes.c_int, P],
        "qg_set_tuning": [ctypes.c_char_p, I64],
        "qg_get_tuning": [ctypes.c_char_p, P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.qg_last_error.restype = ctypes.c_char_p
    lib.qg_last_error.argtypes = []
    lib.qg_version.restype = ctypes.c_char_p
    lib.qg_version.argtypes = []
    return lib


lib = _load()


def _check(st: int) -> None:
    if st != QG_OK:
        raise QGError(st, lib.qg_last_error().decode())


def version() -> str:
    return lib.qg_version().decode()


def set_tuning(key: str, value: int) -> None:
    _check(lib.qg_set_tuning(key.encode(), int(value)))


def get_tuning(key: str) -> int:
    v = ctypes.c_int64()
    _check(lib.qg_get_tuning(key.encode(), ctypes.byref(v)))
    return int(v.value)


def _stream_handle(stream: Optional[torch.cuda.Stream]) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class CircuitArgs:
    """Keeps the numpy arrays of one circuit alive while the C struct points at them."""

    def __init__(self, circ):
        self.gt = np.ascontiguousarray(circ.gate_type, dtype=np.int32).reshape(-1, 3)
        self.gp = np.ascontiguousarray(circ.gate_param, dtype=np.float64).reshape(-1, 3)
        pidx = getattr(circ, "param_idx", None)
        self.pi = None if pidx is None else np.ascontiguousarray(pidx, dtype=np.int32)
        self.c = _Circuit(int(circ.n_qubits), int(self.gt.shape[0]), self.gt.ctypes.data, self.gp.ctypes.data,
                          None if self.pi is None else self.pi.ctypes.data)

    @property
    def ptr(self):
        return ctypes.byref(self.c)


def _dtype_code(dtype) -> int:
    if dtype in (C64, "c64", torch.complex64):
        return C64
    if dtype in (C128, "c128", torch.complex128):
        return C128
    raise ValueError(f"unknown dtype {dtype!r}")


class State:
    """A 2^n-amplitude state in a torch-owned device buffer (borrowed by the library)."""

    def __init__(self, n: int, dtype="c128", device: str = "cuda", stream: Optional[torch.cuda.Stream] = None):
        self.n = int(n)
        self.code = _dtype_code(dtype)
        tdt = torch.complex64 if self.code == C64 else torch.complex128
        self.tensor = torch.empty(1 << self.n, dtype=tdt, device=device)
        self._stream = stream
        h = ctypes.c_void_p()
        _check(lib.qg_state_alloc(self.n, self.code, ctypes.c_void_p(self.tensor.data_ptr()),
                                  self.tensor.numel() * self.tensor.element_size(), _stream_handle(stream),
                                  ctypes.byref(h)))
        self.handle = h

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib.qg_state_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def autotune(self, reps: int = 3) -> np.ndarray:
        """Runs the library's autotuner on this state; returns the (tile, reg, swz) table [5, 3]."""
        t = np.zeros((5, 3), np.int32)
        _check(lib.qg_autotune(self.handle, int(reps), t.ctypes.data))
        return t

    def set_stream(self, stream: Optional[torch.cuda.Stream]) -> None:
        self._stream = stream
        _check(lib.qg_state_set_stream(self.handle, _stream_handle(stream)))

    def reset(self) -> "State":
        _check(lib.qg_state_reset(self.handle))
        return self

    def apply(self, circ, fusion: int = FUSE_GREEDY) -> "State":
        ca = CircuitArgs(circ)
        _check(lib.qg_apply_circuit(self.handle, ca.ptr, int(fusion)))
        return self

    def apply_from_zero(self, circ, fusion: int = FUSE_GREEDY) -> "State":
        """Reset to |0...0> and apply circ (qg_apply_from_zero: passes skip tiles still zero)."""
        ca = CircuitArgs(circ)
        _check(lib.qg_apply_from_zero(self.handle, ca.ptr, int(fusion)))
        return self

    def probs(self, idx: Optional[Sequence[int]] = None) -> torch.Tensor:
        if idx is None:
            out = torch.empty(1 << self.n, dtype=torch.float64, device=self.tensor.device)
            _check(lib.qg_probs(self.handle, None, 0, ctypes.c_void_p(out.data_ptr())))
            return out
        ix = np.ascontiguousarray(idx, dtype=np.uint64)
        out = torch.empty(ix.size, dtype=torch.float64, device=self.tensor.device)
        _check(lib.qg_probs(self.handle, ix.ctypes.data, ix.size, ctypes.c_void_p(out.data_ptr())))
        return out

    def sample(self, shots: int, seed: int) -> torch.Tensor:
        """Shot indices (int64 tensor holding the uint64 values)."""
        out = torch.empty(max(int(shots), 0), dtype=torch.int64, device=self.tensor.device)
        _check(lib.qg_sample(self.handle, int(shots), int(seed) & ((1 << 64) - 1), ctypes.c_void_p(out.data_ptr())))
        return out

    def expval(self, masks: Sequence[int], coeffs: Optional[Sequence[float]] = None):
        m = np.ascontiguousarray(masks, dtype=np.uint64)
        terms = torch.empty(m.size, dtype=torch.float64, device=self.tensor.device)
        total = torch.empty(1, dtype=torch.float64, device=self.tensor.device)
        c = None if coeffs is None else np.ascontiguousarray(coeffs, dtype=np.float64)
        _check(lib.qg_expval(self.handle, m.ctypes.data, None if c is None else c.ctypes.data, m.size,
                             ctypes.c_void_p(terms.data_ptr()),
                             None if c is None else ctypes.c_void_p(total.data_ptr())))
        return terms, (None if c is None else total[0])

    def expval_noalloc(self, masks: Sequence[int], coeffs: Optional[Sequence[float]],
                       out_terms: Optional[torch.Tensor], out_sum: Optional[torch.Tensor]) -> None:
        """qg_expval_noalloc into caller-allocated float64 device tensors (either may be None);
        the library allocates nothing (at most 256 masks)."""
        m = np.ascontiguousarray(masks, dtype=np.uint64)
        c = None if coeffs is None else np.ascontiguousarray(coeffs, dtype=np.float64)
        for t, k in ((out_terms, m.size), (out_sum, 1)):
            if t is not None and (t.dtype != torch.float64 or not t.is_contiguous() or t.numel() < k):
                raise ValueError("outputs must be contiguous float64 tensors of n_terms and 1 elements")
        _check(lib.qg_expval_noalloc(self.handle, m.ctypes.data, None if c is None else c.ctypes.data, m.size,
                                     None if out_terms is None else ctypes.c_void_p(out_terms.data_ptr()),
                                     None if out_sum is None else ctypes.c_void_p(out_sum.data_ptr())))


def adjoint_grad(circ, masks, coeffs, n_params: int, dtype="c128", stream=None):
    """(value, grad) tensors of f = sum_m coeff_m <Z_m> by the library's adjoint sweep."""
    ca = CircuitArgs(circ)
    m = np.ascontiguousarray(masks, dtype=np.uint64)
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    val = torch.empty(1, dtype=torch.float64, device="cuda")
    grad = torch.empty(max(n_params, 1), dtype=torch.float64, device="cuda")
    _check(lib.qg_adjoint_grad(ca.ptr, _dtype_code(dtype), m.ctypes.data, c.ctypes.data, m.size, int(n_params),
                               _stream_handle(stream), ctypes.c_void_p(val.data_ptr()),
                               ctypes.c_void_p(grad.data_ptr())))
    return val[0], grad[:n_params]


class _CircuitArray:
    def __init__(self, circs):
        self.args = [CircuitArgs(c) for c in circs]
        self.arr = (_Circuit * max(len(circs), 1))(*[a.c for a in self.args])

    @property
    def ptr(self):
        return ctypes.cast(self.arr, ctypes.c_void_p)


def _obs_csr(obs):
    """obs: None (ZZ chain) or a list of (masks, coeffs) per circuit."""
    if obs is None:
        return OBS_ZZ_CHAIN, None, None, None
    off = np.zeros(len(obs) + 1, dtype=np.int64)
    for i, (m, _) in enumerate(obs):
        off[i + 1] = off[i] + len(m)
    masks = np.ascontiguousarray(np.concatenate([np.asarray(m, np.uint64) for m, _ in obs]) if obs else
                                 np.zeros(0, np.uint64), dtype=np.uint64)
    coeffs = np.ascontiguousarray(np.concatenate([np.asarray(c, np.float64) for _, c in obs]) if obs else
                                  np.zeros(0), dtype=np.float64)
    return OBS_CSR, off, masks, coeffs


class Batch:
    """Reusable batched launch (graph-captured when the stream is not the NULL stream)."""

    def __init__(self, circs, dtype="c128", obs=None, stream: Optional[torch.cuda.Stream] = None):
        self.n = len(circs)
        self.code = _dtype_code(dtype)
        self.out = torch.zeros(max(self.n, 1), dtype=torch.float64, device="cuda")
        self._ca = _CircuitArray(circs)
        kind, off, masks, coeffs = _obs_csr(obs)
        self._obs = (off, masks, coeffs)
        h = ctypes.c_void_p()
        _check(lib.qg_batch_create(self._ca.ptr, self.n, self.code, kind,
                                   None if off is None else off.ctypes.data,
                                   None if masks is None else masks.ctypes.data,
                                   None if coeffs is None else coeffs.ctypes.data,
                                   _stream_handle(stream), ctypes.c_void_p(self.out.data_ptr()), ctypes.byref(h)))
        self.handle = h

    def set_params(self, circs) -> None:
        ca = _CircuitArray(circs)
        _check(lib.qg_batch_set_params(self.handle, ca.ptr))

    def launch(self) -> torch.Tensor:
        _check(lib.qg_batch_launch(self.handle))
        return self.out[:self.n]

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib.qg_batch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_expval(circs, dtype="c128", obs=None, stream=None) -> torch.Tensor:
    """One-shot batched expectations (qg_batch_expval)."""
    ca = _CircuitArray(circs)
    kind, off, masks, coeffs = _obs_csr(obs)
    out = torch.zeros(max(len(circs), 1), dtype=torch.float64, device="cuda")
    _check(lib.qg_batch_expval(ca.ptr, len(circs), _dtype_code(dtype), kind,
                               None if off is None else off.ctypes.data,
                               None if masks is None else masks.ctypes.data,
                               None if coeffs is None else coeffs.ctypes.data,
                               _stream_handle(stream), ctypes.c_void_p(out.data_ptr())))
    return out[:len(circs)]


class MLP:
    """The library's cost-model MLP (FP32, three ReLU hidden layers of width 64)."""

    def __init__(self, n_in: int = PASS_FEATURES, seed: int = 0, stream=None):
        h = ctypes.c_void_p()
        _check(lib.qg_mlp_create(int(n_in), 64, int(seed) & ((1 << 64) - 1), _stream_handle(stream),
                                 ctypes.byref(h)))
        self.handle = h
        self.n_in = int(n_in)
        n = ctypes.c_int64()
        _check(lib.qg_mlp_n_params(h, ctypes.byref(n)))
        self.n_params = int(n.value)

    def get_params(self) -> np.ndarray:
        out = np.empty(self.n_params, np.float32)
        _check(lib.qg_mlp_get_params(self.handle, out.ctypes.data))
        return out

    def set_params(self, theta) -> None:
        th = np.ascontiguousarray(theta, dtype=np.float32)
        assert th.size == self.n_params
        _check(lib.qg_mlp_set_params(self.handle, th.ctypes.data))

    def forward(self, X) -> np.ndarray:
        X = np.ascontiguousarray(X, dtype=np.float32).reshape(-1, self.n_in)
        y = np.empty(X.shape[0], np.float32)
        _check(lib.qg_mlp_forward(self.handle, X.ctypes.data, X.shape[0], y.ctypes.data))
        return y

    def grad(self, X, t):
        X = np.ascontiguousarray(X, dtype=np.float32).reshape(-1, self.n_in)
        t = np.ascontiguousarray(t, dtype=np.float32)
        g = np.empty(self.n_params, np.float32)
        loss = ctypes.c_double()
        _check(lib.qg_mlp_grad(self.handle, X.ctypes.data, t.ctypes.data, X.shape[0], ctypes.byref(loss),
                               g.ctypes.data))
        return float(loss.value), g

    def adam_step(self, g, lr: float) -> None:
        g = np.ascontiguousarray(g, dtype=np.float32)
        _check(lib.qg_mlp_adam_step(self.handle, g.ctypes.data, float(lr)))

    def train(self, X, t, epochs: int, batch: int, lr: float, seed: int = 0) -> np.ndarray:
        X = np.ascontiguousarray(X, dtype=np.float32).reshape(-1, self.n_in)
        t = np.ascontiguousarray(t, dtype=np.float32)
        losses = np.zeros(max(epochs, 1), np.float64)
        _check(lib.qg_mlp_train(self.handle, X.ctypes.data, t.ctypes.data, X.shape[0], int(epochs), int(batch),
                                float(lr), int(seed), losses.ctypes.data))
        return losses[:epochs]

    def install(self) -> None:
        _check(lib.qg_set_cost_model(self.handle))

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib.qg_mlp_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def clear_cost_model() -> None:
    _check(lib.qg_set_cost_model(None))


def pass_features(circ, dtype="c128", config: int = 1):
    """(features of the whole circuit as one pass under candidate config, greedy pass count)."""
    ca = CircuitArgs(circ)
    f = np.empty(PASS_FEATURES, np.float32)
    npass = ctypes.c_int32()
    _check(lib.qg_pass_features(ca.ptr, _dtype_code(dtype), int(config), f.ctypes.data, ctypes.byref(npass)))
    return f, int(npass.value)


def plan_passes(circ, dtype="c128", fusion: int = FUSE_GREEDY):
    """(pass index of each gate, number of passes) of the library's plan (host only)."""
    ca = CircuitArgs(circ)
    pog = np.zeros(max(ca.gt.shape[0], 1), dtype=np.int32)
    npass = ctypes.c_int32()
    _check(lib.qg_plan_passes(ca.ptr, _dtype_code(dtype), int(fusion), pog.ctypes.data, ctypes.byref(npass)))
    return pog[:ca.gt.shape[0]], int(npass.value)


FORM_APPLY, FORM_ADJOINT, FORM_BATCHED, FORM_FROM_ZERO = 0, 1, 2, 3


def plan_bytes(circ, dtype="c128", form: int = FORM_APPLY, fusion: int = FUSE_GREEDY):
    """(passes, HBM bytes the plan moves) of qg_apply_circuit (form FORM_APPLY, with
    `fusion`), qg_apply_from_zero (FORM_FROM_ZERO, with `fusion`), qg_adjoint_grad
    (FORM_ADJOINT) or one batched circuit (FORM_BATCHED)."""
    ca = CircuitArgs(circ)
    npass = ctypes.c_int32()
    b = ctypes.c_double()
    _check(lib.qg_plan_bytes(ca.ptr, _dtype_code(dtype), int(form), int(fusion), ctypes.byref(npass),
                             ctypes.byref(b)))
    return int(npass.value), float(b.value)


KERNEL_NAMES = ("tile", "dense", "swap_half", "swap_lane", "lane_gate")


def plan_kernels(circ, dtype="c128", fusion: int = FUSE_GREEDY):
    """Kernel family of each pass of the library's plan, as names from KERNEL_NAMES (host only)."""
    ca = CircuitArgs(circ)
    npass = ctypes.c_int32()
    _check(lib.qg_plan_kernels(ca.ptr, _dtype_code(dtype), int(fusion), None, 0, ctypes.byref(npass)))
    k = np.zeros(max(npass.value, 1), dtype=np.int32)
    _check(lib.qg_plan_kernels(ca.ptr, _dtype_code(dtype), int(fusion), k.ctypes.data, k.size,
                               ctypes.byref(npass)))
    return [KERNEL_NAMES[v] for v in k[:npass.value]]


class QGExpval(torch.autograd.Function):
    """f(params) = sum_m coeff_m <Z_{mask_m}> of ``circ`` with its trainable angles
    (``circ.param_idx`` slots) taken from ``params`` (float64, one value per slot).

    Forward and the gradient come from one call of the library's adjoint sweep
    (qg_adjoint_grad) when a gradient is needed; otherwise the forward is an
    apply + expval on a fresh state.
    """

    @staticmethod
    def forward(ctx, params: torch.Tensor, circ, masks, coeffs, dtype: str = "c128"):
        p = params.detach().to("cpu", torch.float64).numpy()
        c = circ.copy()
        sel = c.param_idx >= 0
        c.gate_param[sel, 0] = p[c.param_idx[sel]]
        if params.requires_grad:
            val, grad = adjoint_grad(c, masks, coeffs, int(p.size), dtype)
            ctx.save_for_backward(grad.to(params.device))
            return val.to(params.device)
        st = State(c.n_qubits, dtype)
        st.apply(c, FUSE_GREEDY)
        _, total = st.expval(masks, coeffs)
        st.close()
        return total.to(params.device)

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return g * grad, None, None, None, None
