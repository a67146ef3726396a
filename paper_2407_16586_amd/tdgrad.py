"""ctypes binding of libtdgrad.so (the C ABI in include/tdgrad.h).

Argument marshalling only: every step of the gradient runs in the HIP library.
Importing this module does not touch the GPU; loading the library fails loudly
when it has not been built (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtdgrad.so")

TDG_OK, TDG_EINVAL, TDG_EUNSUPPORTED, TDG_ENOMEM, TDG_EDEVICE, TDG_ESTATE = 0, -1, -2, -3, -4, -5
TERMS_J, TERMS_K, TERMS_KLR, TERMS_ALL = 1, 2, 4, 7
NUM_CLASSES = 21
# class order of the library: (la, lb | lc, ld), bra pair class >= ket pair class
PAIR_CLASSES = ((0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2))
CLASSES = tuple(PAIR_CLASSES[b] + PAIR_CLASSES[k] for b in range(6) for k in range(b + 1))

EXPORTED = ("tdg_plan_create", "tdg_grad_jk", "tdg_plan_destroy", "tdg_plan_dims",
            "tdg_plan_schwarz", "tdg_rys_rule", "tdg_last_error")


class TdgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"tdgrad error {status}: {msg}")
        self.status = status


class Basis(C.Structure):
    _fields_ = [("n_atoms", C.c_int32), ("coords", C.c_void_p),
                ("n_shells", C.c_int32), ("shell_atom", C.c_void_p), ("shell_l", C.c_void_p),
                ("shell_nprim", C.c_void_p), ("shell_prim_off", C.c_void_p),
                ("shell_ao_off", C.c_void_p), ("n_prims", C.c_int32),
                ("exps", C.c_void_p), ("coefs", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("omega", C.c_double), ("alpha", C.c_double), ("beta", C.c_double),
                ("schwarz_tol", C.c_double), ("precision", C.c_int32), ("terms", C.c_int32),
                ("autotune", C.c_int32), ("kernel_variant", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("quartets", C.c_int64), ("prim_quartets", C.c_int64), ("candidates", C.c_int64),
                ("class_quartets", C.c_int64 * NUM_CLASSES),
                ("class_prim_quartets", C.c_int64 * NUM_CLASSES),
                ("class_ms", C.c_double * NUM_CLASSES),
                ("class_variant", C.c_int32 * NUM_CLASSES), ("ms_total", C.c_double),
                ("ms_kernels", C.c_double)]

    def as_dict(self):
        return {"quartets": self.quartets, "prim_quartets": self.prim_quartets,
                "candidates": self.candidates, "class_quartets": list(self.class_quartets),
                "class_prim_quartets": list(self.class_prim_quartets),
                "class_ms": list(self.class_ms), "class_variant": list(self.class_variant),
                "ms_total": self.ms_total,
                "ms_kernels": self.ms_kernels}


_lib = None


def lib():
    """Load libtdgrad.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2407_16586_amd.build.build()")
        # torch's HIP runtime must be the process's runtime before the library loads: the two
        # exchange device pointers and streams, which are only valid inside one runtime
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.tdg_plan_create.argtypes = [C.POINTER(Basis), C.POINTER(Params), C.c_int, C.POINTER(vp)]
        L.tdg_grad_jk.argtypes = [vp, vp, vp, vp, C.c_int32, vp, vp, C.POINTER(Stats)]
        L.tdg_plan_destroy.argtypes = [vp]
        L.tdg_plan_dims.argtypes = [vp, vp, vp, vp]
        L.tdg_plan_schwarz.argtypes = [vp, vp]
        L.tdg_rys_rule.argtypes = [C.c_int32, C.c_double, vp, vp]
        L.tdg_last_error.restype = C.c_char_p
        for f in EXPORTED[:-1]:
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != TDG_OK:
        raise TdgError(rc, lib().tdg_last_error().decode())


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p).value


class Plan:
    """A plan for one molecule (geometry + basis); see tdg_plan_create."""

    def __init__(self, mol, omega=None, alpha=None, beta=None, schwarz_tol=1e-10, terms=TERMS_ALL,
                 precision=0, device=0, autotune=True, kernel_variant=-1):
        self._keep = [np.ascontiguousarray(mol.coords, dtype=np.float64)]
        for name in ("shell_atom", "shell_l", "shell_nprim", "shell_prim_off", "shell_ao_off"):
            self._keep.append(np.ascontiguousarray(getattr(mol, name), dtype=np.int32))
        self._keep.append(np.ascontiguousarray(mol.exps, dtype=np.float64))
        self._keep.append(np.ascontiguousarray(mol.coefs, dtype=np.float64))
        k = self._keep
        b = Basis(mol.n_atoms, _ptr(k[0]), mol.n_shells, _ptr(k[1]), _ptr(k[2]), _ptr(k[3]),
                  _ptr(k[4]), _ptr(k[5]), mol.n_prims, _ptr(k[6]), _ptr(k[7]))
        self.params = Params(mol.omega if omega is None else omega, mol.alpha if alpha is None else alpha,
                             mol.beta if beta is None else beta, schwarz_tol, precision, terms,
                             1 if autotune else 0, kernel_variant)
        h = C.c_void_p()
        _check(lib().tdg_plan_create(C.byref(b), C.byref(self.params), device, C.byref(h)))
        self._h = h
        nbf, nat, ns = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().tdg_plan_dims(h, C.byref(nbf), C.byref(nat), C.byref(ns)))
        self.n_bf, self.n_atoms, self.n_shells = nbf.value, nat.value, ns.value

    def close(self):
        if getattr(self, "_h", None):
            lib().tdg_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def schwarz(self):
        out = np.zeros(self.n_shells * (self.n_shells + 1) // 2)
        _check(lib().tdg_plan_schwarz(self._h, _ptr(out)))
        return out

    def grad(self, P0, PD, R, stats=False):
        """Host numpy densities -> host gradient [n_atoms, 3] (synchronous)."""
        c = lambda x: np.ascontiguousarray(x, dtype=np.float64)
        P0, PD, R = c(P0), c(PD), c(R)
        n = self.n_bf
        for x in (P0, PD, R):
            if x.shape != (n, n):
                raise ValueError(f"density must be {n}x{n}, got {x.shape}")
        out = np.zeros((self.n_atoms, 3))
        st = Stats()
        _check(lib().tdg_grad_jk(self._h, _ptr(P0), _ptr(PD), _ptr(R), 0, None, _ptr(out),
                                 C.byref(st) if stats else None))
        return (out, st.as_dict()) if stats else out

    def grad_device(self, P0, PD, R, out, stream=None, stats=False):
        """torch CUDA/HIP tensors (float64, contiguous) on the plan's device; asynchronous
        on `stream` (default: torch's current stream) unless stats are requested."""
        import torch
        n = self.n_bf
        for x in (P0, PD, R):
            if x.dtype != torch.float64 or not x.is_contiguous() or tuple(x.shape) != (n, n) or not x.is_cuda:
                raise ValueError("densities must be contiguous float64 device tensors of shape (n_bf, n_bf)")
        if out.dtype != torch.float64 or not out.is_contiguous() or tuple(out.shape) != (self.n_atoms, 3):
            raise ValueError("out must be a contiguous float64 device tensor (n_atoms, 3)")
        s = (stream or torch.cuda.current_stream()).cuda_stream
        st = Stats()
        _check(lib().tdg_grad_jk(self._h, P0.data_ptr(), PD.data_ptr(), R.data_ptr(), 1, s,
                                 out.data_ptr(), C.byref(st) if stats else None))
        return st.as_dict() if stats else None


def rys_rule(n, T):
    u = np.zeros(n)
    w = np.zeros(n)
    _check(lib().tdg_rys_rule(n, float(T), _ptr(u), _ptr(w)))
    return u, w
