"""FP64 CPU oracle for the state-vector circuit simulation (arXiv 2504.03967, App. A).

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only users.  It shares no code with the
GPU library and never imports it.

The arithmetic lives in ``qg_oracle.c`` (plain gate-by-gate pair loops, see the
header of that file); this module only marshals numpy arrays into it.  The MLP
reference of the fusion cost model is in ``oracle/mlp.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qg_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP, -O2)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=gnu11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.qgo_init.argtypes = [ctypes.c_int, P]
        lib.qgo_apply_circuit.argtypes = [ctypes.c_int, P, ctypes.c_int64, P, P]
        lib.qgo_apply_circuit.restype = ctypes.c_int
        lib.qgo_apply_circuit_dagger.argtypes = [ctypes.c_int, P, ctypes.c_int64, P, P]
        lib.qgo_apply_circuit_dagger.restype = ctypes.c_int
        lib.qgo_probs.argtypes = [ctypes.c_int, P, P]
        lib.qgo_expval.argtypes = [ctypes.c_int, P, ctypes.c_int, P, P]
        lib.qgo_philox4x32_10.argtypes = [P, P, P]
        lib.qgo_shot_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.qgo_shot_uniform.restype = ctypes.c_double
        lib.qgo_sample.argtypes = [ctypes.c_int, P, ctypes.c_int64, ctypes.c_uint64, P]
        lib.qgo_sample.restype = ctypes.c_int
        lib.qgo_adjoint_grad.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, P, ctypes.c_int,
                                         ctypes.c_int, P, P, P, P]
        lib.qgo_adjoint_grad.restype = ctypes.c_int
        lib.qgo_batch_zz_chain.argtypes = [ctypes.c_int, P, P, P, P, P]
        lib.qgo_batch_zz_chain.restype = ctypes.c_int
        lib.qgo_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> ctypes.c_void_p:
    return ctypes.c_void_p(a.ctypes.data)


def _gates(circ):
    gt = np.ascontiguousarray(circ.gate_type, dtype=np.int32).reshape(-1, 3)
    gp = np.ascontiguousarray(circ.gate_param, dtype=np.float64).reshape(-1, 3)
    return gt, gp


def num_threads() -> int:
    return _load().qgo_num_threads()


def zero_state(n: int) -> np.ndarray:
    psi = np.empty(1 << n, dtype=np.complex128)
    _load().qgo_init(n, _ptr(psi))
    return psi


def apply(circ, psi: np.ndarray | None = None, dagger: bool = False) -> np.ndarray:
    """Apply ``circ`` gate by gate to ``psi`` (default |0...0>), in place; returns the state."""
    lib = _load()
    n = int(circ.n_qubits)
    if psi is None:
        psi = zero_state(n)
    assert psi.dtype == np.complex128 and psi.flags.c_contiguous and psi.size == (1 << n)
    gt, gp = _gates(circ)
    fn = lib.qgo_apply_circuit_dagger if dagger else lib.qgo_apply_circuit
    rc = fn(n, _ptr(psi), gt.shape[0], _ptr(gt), _ptr(gp))
    if rc != 0:
        raise ValueError(f"oracle: malformed gate {-1 - rc}")
    return psi


def simulate(circ) -> np.ndarray:
    return apply(circ)


def probs(psi: np.ndarray) -> np.ndarray:
    n = int(psi.size).bit_length() - 1
    out = np.empty(psi.size, dtype=np.float64)
    _load().qgo_probs(n, _ptr(psi), _ptr(out))
    return out


def expval(psi: np.ndarray, masks) -> np.ndarray:
    n = int(psi.size).bit_length() - 1
    m = np.ascontiguousarray(masks, dtype=np.uint64)
    out = np.empty(m.size, dtype=np.float64)
    _load().qgo_expval(n, _ptr(psi), m.size, _ptr(m), _ptr(out))
    return out


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, dtype=np.uint32)
    _load().qgo_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def shot_uniform(seed: int, s: int) -> float:
    return _load().qgo_shot_uniform(seed, s)


def sample(psi: np.ndarray, shots: int, seed: int) -> np.ndarray:
    n = int(psi.size).bit_length() - 1
    out = np.empty(shots, dtype=np.uint64)
    if _load().qgo_sample(n, _ptr(psi), shots, seed, _ptr(out)) != 0:
        raise MemoryError("oracle: sample allocation failed")
    return out


def batch_zz_chain(circs) -> np.ndarray:
    """sum_q <Z_q Z_{q+1}> of each circuit's final state (independent circuits in parallel)."""
    n = np.array([c.n_qubits for c in circs], dtype=np.int32)
    goff = np.zeros(len(circs) + 1, dtype=np.int64)
    goff[1:] = np.cumsum([c.n_gates for c in circs])
    gt = np.ascontiguousarray(np.concatenate([_gates(c)[0] for c in circs]), dtype=np.int32)
    gp = np.ascontiguousarray(np.concatenate([_gates(c)[1] for c in circs]), dtype=np.float64)
    out = np.empty(len(circs), dtype=np.float64)
    rc = _load().qgo_batch_zz_chain(len(circs), _ptr(n), _ptr(goff), _ptr(gt), _ptr(gp), _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle: batch failed ({rc})")
    return out


def adjoint_grad(circ, n_params: int, masks, coeffs):
    """(f, grad) of f = sum_m coeff_m <Z_{mask_m}> by the adjoint recursion."""
    lib = _load()
    gt, gp = _gates(circ)
    pidx = np.ascontiguousarray(circ.param_idx, dtype=np.int32)
    m = np.ascontiguousarray(masks, dtype=np.uint64)
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    val = np.zeros(1, dtype=np.float64)
    grad = np.zeros(max(n_params, 1), dtype=np.float64)
    rc = lib.qgo_adjoint_grad(int(circ.n_qubits), gt.shape[0], _ptr(gt), _ptr(gp), _ptr(pidx),
                              n_params, m.size, _ptr(m), _ptr(c), _ptr(val), _ptr(grad))
    if rc != 0:
        raise ValueError(f"oracle: adjoint failed ({rc})")
    return float(val[0]), grad[:n_params]
