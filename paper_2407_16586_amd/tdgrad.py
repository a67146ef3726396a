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

EXPORTED = ("tdg_plan_create", "tdg_grad_jk", "tdg_grad_jk_batch", "tdg_plan_destroy", "tdg_plan_dims",
            "tdg_plan_schwarz", "tdg_rys_rule", "tdg_plan_set_screen_model", "tdg_collect",
            "tdg_plan_update_coords", "tdg_screen_list", "tdg_quartet_contribs", "tdg_grad_jk_noalloc", "tdg_plan_set_streams",
            "tdg_fock", "tdg_zvector",
            "tdg_mlp_create", "tdg_mlp_destroy", "tdg_mlp_nweights", "tdg_mlp_set_weights",
            "tdg_mlp_get_weights", "tdg_mlp_forward", "tdg_mlp_grad", "tdg_mlp_train_step",
            "tdg_last_error")


class TdgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"tdgrad error {status}: {msg}")
        self.status = status


class Basis(C.Structure):
    _fields_ = [("n_atoms", C.c_int32), ("coords", C.c_void_p),
                ("n_shells", C.c_int32), ("shell_atom", C.c_void_p), ("shell_l", C.c_void_p),
                ("shell_nprim", C.c_void_p), ("shell_prim_off", C.c_void_p),
                ("shell_ao_off", C.c_void_p), ("n_prims", C.c_int32),
                ("exps", C.c_void_p), ("coefs", C.c_void_p), ("spherical", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("omega", C.c_double), ("alpha", C.c_double), ("beta", C.c_double),
                ("schwarz_tol", C.c_double), ("precision", C.c_int32), ("terms", C.c_int32),
                ("autotune", C.c_int32), ("kernel_variant", C.c_int32),
                ("mixed_tau64", C.c_double), ("mixed_p64", C.c_double), ("max_tasks", C.c_int64),
                ("screening", C.c_int32), ("deterministic", C.c_int32), ("ml_min_components", C.c_int32),
                ("streams", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("quartets", C.c_int64), ("prim_quartets", C.c_int64), ("candidates", C.c_int64),
                ("class_quartets", C.c_int64 * NUM_CLASSES),
                ("class_prim_quartets", C.c_int64 * NUM_CLASSES),
                ("class_ms", C.c_double * NUM_CLASSES),
                ("class_variant", C.c_int32 * NUM_CLASSES),
                ("fp32_quartets", C.c_int64), ("ml_skipped", C.c_int64), ("chunks", C.c_int64),
                ("class_fp32_quartets", C.c_int64 * NUM_CLASSES),
                ("ms_total", C.c_double),
                ("ms_kernels", C.c_double)]

    def as_dict(self):
        return {"quartets": self.quartets, "prim_quartets": self.prim_quartets,
                "candidates": self.candidates, "class_quartets": list(self.class_quartets),
                "class_prim_quartets": list(self.class_prim_quartets),
                "class_ms": list(self.class_ms), "class_variant": list(self.class_variant),
                "fp32_quartets": self.fp32_quartets, "ml_skipped": self.ml_skipped,
                "chunks": self.chunks,
                "class_fp32_quartets": list(self.class_fp32_quartets),
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
        L.tdg_grad_jk_batch.argtypes = [C.c_int32, vp, vp, vp, vp, C.c_int32, vp, vp, C.POINTER(Stats)]
        L.tdg_plan_destroy.argtypes = [vp]
        L.tdg_plan_dims.argtypes = [vp, vp, vp, vp]
        L.tdg_plan_schwarz.argtypes = [vp, vp]
        L.tdg_rys_rule.argtypes = [C.c_int32, C.c_double, vp, vp]
        L.tdg_plan_set_screen_model.argtypes = [vp, vp, C.c_double, C.c_double]
        L.tdg_collect.argtypes = [vp, vp, vp, vp, C.c_int32, vp, vp, vp, C.c_int64, C.c_int64,
                                  C.POINTER(C.c_int64)]
        L.tdg_grad_jk_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, C.POINTER(Stats)]
        L.tdg_plan_update_coords.argtypes = [vp, vp]
        L.tdg_plan_set_streams.argtypes = [vp, C.c_int32]
        L.tdg_screen_list.argtypes = [vp, vp, vp, vp, C.c_int32, vp, vp, C.c_int64, C.c_int64,
                                      C.POINTER(C.c_int64)]
        L.tdg_quartet_contribs.argtypes = [vp, vp, vp, vp, C.c_int32, vp, C.c_int64, vp, C.c_int32, vp]
        L.tdg_fock.argtypes = [vp, vp, C.c_int32, vp, C.c_double, C.c_double, C.c_double, C.c_int32, vp,
                               C.POINTER(Stats)]
        L.tdg_zvector.argtypes = [vp, C.c_int32, C.c_int32, vp, vp, vp, vp, vp, C.c_double, C.c_double,
                                  C.c_double, C.c_int32, C.c_double, C.c_int32, vp, C.POINTER(C.c_int32),
                                  C.POINTER(C.c_double)]
        L.tdg_mlp_create.argtypes = [C.c_int, C.c_uint64, C.POINTER(vp)]
        L.tdg_mlp_destroy.argtypes = [vp]
        L.tdg_mlp_nweights.argtypes = []
        L.tdg_mlp_set_weights.argtypes = [vp, vp]
        L.tdg_mlp_get_weights.argtypes = [vp, vp]
        L.tdg_mlp_forward.argtypes = [vp, vp, C.c_int64, vp, vp]
        L.tdg_mlp_grad.argtypes = [vp, vp, vp, C.c_int64, vp, vp, vp]
        L.tdg_mlp_train_step.argtypes = [vp, vp, vp, C.c_int64, C.c_float, vp, vp]
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
                 precision=0, device=0, autotune=True, kernel_variant=-1, mixed_tau64=0.1,
                 mixed_p64=1e4, max_tasks=0, screening=0, deterministic=False, streams=0,
                 ml_min_components=0):
        self._keep = [np.ascontiguousarray(mol.coords, dtype=np.float64)]
        for name in ("shell_atom", "shell_l", "shell_nprim", "shell_prim_off", "shell_ao_off"):
            self._keep.append(np.ascontiguousarray(getattr(mol, name), dtype=np.int32))
        self._keep.append(np.ascontiguousarray(mol.exps, dtype=np.float64))
        self._keep.append(np.ascontiguousarray(mol.coefs, dtype=np.float64))
        k = self._keep
        b = Basis(mol.n_atoms, _ptr(k[0]), mol.n_shells, _ptr(k[1]), _ptr(k[2]), _ptr(k[3]),
                  _ptr(k[4]), _ptr(k[5]), mol.n_prims, _ptr(k[6]), _ptr(k[7]),
                  int(getattr(mol, "spherical", 0)))
        self.params = Params(mol.omega if omega is None else omega, mol.alpha if alpha is None else alpha,
                             mol.beta if beta is None else beta, schwarz_tol, precision, terms,
                             1 if autotune else 0, kernel_variant, mixed_tau64, mixed_p64, max_tasks,
                             screening, 1 if deterministic else 0, ml_min_components, streams)
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

    def set_streams(self, n):
        """Spread the class kernels of later calls over n streams (1 .. the plan's streams)."""
        _check(lib().tdg_plan_set_streams(self._h, int(n)))

    def update_coords(self, coords):
        """Move the plan to new coordinates [n_atoms, 3] (bohr); see tdg_plan_update_coords."""
        c = np.ascontiguousarray(coords, dtype=np.float64)
        if c.shape != (self.n_atoms, 3):
            raise ValueError(f"coords must be ({self.n_atoms}, 3), got {c.shape}")
        _check(lib().tdg_plan_update_coords(self._h, _ptr(c)))

    def screen_list(self, P0, PD, R, cap=None, stride=1):
        """Every stride-th surviving shell quartet [n, 4] (caller shell indices, library
        orientation) and the total number of survivors."""
        c = lambda x: np.ascontiguousarray(x, dtype=np.float64)
        P0, PD, R = c(P0), c(PD), c(R)
        n = C.c_int64()
        if cap is None:
            _check(lib().tdg_screen_list(self._h, _ptr(P0), _ptr(PD), _ptr(R), 0, None, None, 0, stride,
                                         C.byref(n)))
            cap = (n.value + stride - 1) // stride
        out = np.zeros((max(cap, 1), 4), dtype=np.int32)
        _check(lib().tdg_screen_list(self._h, _ptr(P0), _ptr(PD), _ptr(R), 0, None, _ptr(out), cap, stride,
                                     C.byref(n)))
        return out[:min((n.value + stride - 1) // stride, cap)], n.value

    def quartet_contribs(self, P0, PD, R, quartets, precision=0):
        """Contributions [n, 4, 3] of listed shell quartets [n, 4] to the atoms of the listed shells."""
        c = lambda x: np.ascontiguousarray(x, dtype=np.float64)
        P0, PD, R = c(P0), c(PD), c(R)
        q = np.ascontiguousarray(quartets, dtype=np.int32).reshape(-1, 4)
        out = np.zeros((q.shape[0], 4, 3))
        _check(lib().tdg_quartet_contribs(self._h, _ptr(P0), _ptr(PD), _ptr(R), 0, None, q.shape[0],
                                          _ptr(q), precision, _ptr(out)))
        return out

    def fock(self, B, cJ=1.0, cK=0.0, cKlr=0.0, relative=False, stats=False):
        """Host numpy B [n_bf, n_bf] -> host Fock-type matrix (synchronous); see tdg_fock
        (relative: screening of B scaled to a largest element of one)."""
        B = np.ascontiguousarray(B, dtype=np.float64)
        n = self.n_bf
        if B.shape != (n, n):
            raise ValueError(f"B must be {n}x{n}, got {B.shape}")
        out = np.zeros((n, n))
        st = Stats()
        _check(lib().tdg_fock(self._h, _ptr(B), 0, None, float(cJ), float(cK), float(cKlr), int(bool(relative)),
                              _ptr(out), C.byref(st) if stats else None))
        return (out, st.as_dict()) if stats else out

    def fock_device(self, B, out, cJ=1.0, cK=0.0, cKlr=0.0, relative=False, stream=None, stats=False):
        """torch float64 device tensors B and out [n_bf, n_bf]; queued on `stream` (default:
        torch's current stream), with one wait on it for the screening counts."""
        import torch
        n = self.n_bf
        for x in (B, out):
            if x.dtype != torch.float64 or not x.is_contiguous() or tuple(x.shape) != (n, n) or not x.is_cuda:
                raise ValueError("B and out must be contiguous float64 device tensors of shape (n_bf, n_bf)")
        s = (stream or torch.cuda.current_stream()).cuda_stream
        st = Stats()
        _check(lib().tdg_fock(self._h, B.data_ptr(), 1, s, float(cJ), float(cK), float(cKlr), int(bool(relative)),
                              out.data_ptr(), C.byref(st) if stats else None))
        return st.as_dict() if stats else None

    def zvector(self, C_occ, C_vir, eps_occ, eps_vir, L, cJ=4.0, cK=None, cKlr=None, relative=True, tol=1e-10,
                max_iter=50):
        """Z of (d - A) Z = L (tdg_zvector; host numpy arrays); returns (Z [n_vir, n_occ],
        products evaluated, final relative residual).  cK, cKlr default to eq zfock's
        -2 alpha and -2 beta of the plan's parameters."""
        c = lambda x: np.ascontiguousarray(x, dtype=np.float64)
        Co, Cv, eo, ev, Lm = c(C_occ), c(C_vir), c(eps_occ), c(eps_vir), c(L)
        no, nv = Co.shape[1], Cv.shape[1]
        if Co.shape[0] != self.n_bf or Cv.shape[0] != self.n_bf or Lm.shape != (nv, no):
            raise ValueError("shape mismatch")
        cK = -2.0 * self.params.alpha if cK is None else cK
        cKlr = -2.0 * self.params.beta if cKlr is None else cKlr
        Z = np.zeros((nv, no))
        it, res = C.c_int32(), C.c_double()
        _check(lib().tdg_zvector(self._h, no, nv, _ptr(Co), _ptr(Cv), _ptr(eo), _ptr(ev), _ptr(Lm), float(cJ),
                                 float(cK), float(cKlr), int(bool(relative)), float(tol), int(max_iter), _ptr(Z),
                                 C.byref(it), C.byref(res)))
        return Z, it.value, res.value

    def set_screen_model(self, model, log10_threshold=-12.0, tau_hi=1e-6):
        """Attach a trained Estimator (or None); it vetoes quartets after the Schwarz
        screening in plans created with screening=1."""
        self._model = model
        _check(lib().tdg_plan_set_screen_model(self._h, model._h if model is not None else None,
                                               log10_threshold, tau_hi))

    def collect(self, P0, PD, R, feat, target, stride=1, stream=None):
        """Device densities (torch, float64) -> features/targets written into the device tensors
        feat [cap, 16] and target [cap] (float32); returns the number of samples."""
        import torch
        n = C.c_int64()
        s = (stream or torch.cuda.current_stream()).cuda_stream
        _check(lib().tdg_collect(self._h, P0.data_ptr(), PD.data_ptr(), R.data_ptr(), 1, s,
                                 feat.data_ptr(), target.data_ptr(), feat.shape[0], stride,
                                 C.byref(n)))
        return n.value

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


    def grad_device_noalloc(self, P0, PD, R, out, stream=None, stats=False):
        """As grad_device, through tdg_grad_jk_noalloc (no device allocation in the call)."""
        import torch
        n = self.n_bf
        for x in (P0, PD, R):
            if x.dtype != torch.float64 or not x.is_contiguous() or tuple(x.shape) != (n, n) or not x.is_cuda:
                raise ValueError("densities must be contiguous float64 device tensors of shape (n_bf, n_bf)")
        if out.dtype != torch.float64 or not out.is_contiguous() or tuple(out.shape) != (self.n_atoms, 3):
            raise ValueError("out must be a contiguous float64 device tensor (n_atoms, 3)")
        s = (stream or torch.cuda.current_stream()).cuda_stream
        st = Stats()
        _check(lib().tdg_grad_jk_noalloc(self._h, P0.data_ptr(), PD.data_ptr(), R.data_ptr(), s,
                                         out.data_ptr(), C.byref(st) if stats else None))
        return st.as_dict() if stats else None


class Estimator:
    """The quartet-contribution network (tdg_mlp_*): BF16 matrix-core forward/backward,
    FP32 master weights, Adam."""

    def __init__(self, seed=0, device=0):
        h = C.c_void_p()
        _check(lib().tdg_mlp_create(device, seed, C.byref(h)))
        self._h = h
        self.nweights = lib().tdg_mlp_nweights()

    def close(self):
        if getattr(self, "_h", None):
            lib().tdg_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def weights(self):
        w = np.zeros(self.nweights, dtype=np.float32)
        _check(lib().tdg_mlp_get_weights(self._h, _ptr(w)))
        return w

    def set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        assert w.shape == (self.nweights,)
        _check(lib().tdg_mlp_set_weights(self._h, _ptr(w)))

    def forward(self, X, out=None, stream=None):
        import torch
        out = out if out is not None else torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        s = (stream or torch.cuda.current_stream()).cuda_stream
        _check(lib().tdg_mlp_forward(self._h, X.data_ptr(), X.shape[0], out.data_ptr(), s))
        return out

    def grad(self, X, Y, stream=None):
        import torch
        g = np.zeros(self.nweights, dtype=np.float32)
        loss = np.zeros(1, dtype=np.float32)
        s = (stream or torch.cuda.current_stream()).cuda_stream
        _check(lib().tdg_mlp_grad(self._h, X.data_ptr(), Y.data_ptr(), X.shape[0], _ptr(g), _ptr(loss), s))
        return float(loss[0]), g

    def train_step(self, X, Y, lr, want_loss=False, stream=None):
        import torch
        loss = np.zeros(1, dtype=np.float32)
        s = (stream or torch.cuda.current_stream()).cuda_stream
        _check(lib().tdg_mlp_train_step(self._h, X.data_ptr(), Y.data_ptr(), X.shape[0], lr,
                                        _ptr(loss) if want_loss else None, s))
        return float(loss[0]) if want_loss else None


def grad_batch(plans, dens, stats=False):
    """Host numpy densities [(P0, PD, R), ...] for plans [...] -> list of host gradients,
    evaluated in one batched pass (tdg_grad_jk_batch)."""
    n = len(plans)
    keep = []
    ptrs = [(C.c_void_p * n)() for _ in range(3)]
    outs = []
    for m, (p, d) in enumerate(zip(plans, dens)):
        for k in range(3):
            x = np.ascontiguousarray(d[k], dtype=np.float64)
            if x.shape != (p.n_bf, p.n_bf):
                raise ValueError("density shape mismatch")
            keep.append(x)
            ptrs[k][m] = _ptr(x)
        outs.append(np.zeros((p.n_atoms, 3)))
    hp = (C.c_void_p * n)(*[p._h.value for p in plans])
    go = (C.c_void_p * n)(*[_ptr(o) for o in outs])
    st = Stats()
    _check(lib().tdg_grad_jk_batch(n, hp, ptrs[0], ptrs[1], ptrs[2], 0, None, go,
                                   C.byref(st) if stats else None))
    return (outs, st.as_dict()) if stats else outs


def grad_batch_device(plans, dens, outs, stream=None, stats=False):
    """torch device tensors: dens [(P0, PD, R), ...], outs [(n_atoms, 3), ...]; asynchronous."""
    import torch
    n = len(plans)
    ptrs = [(C.c_void_p * n)() for _ in range(3)]
    for m, d in enumerate(dens):
        for k in range(3):
            ptrs[k][m] = d[k].data_ptr()
    hp = (C.c_void_p * n)(*[p._h.value for p in plans])
    go = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
    s = (stream or torch.cuda.current_stream()).cuda_stream
    st = Stats()
    _check(lib().tdg_grad_jk_batch(n, hp, ptrs[0], ptrs[1], ptrs[2], 1, s, go,
                                   C.byref(st) if stats else None))
    return st.as_dict() if stats else None


def rys_rule(n, T):
    u = np.zeros(n)
    w = np.zeros(n)
    _check(lib().tdg_rys_rule(n, float(T), _ptr(u), _ptr(w)))
    return u, w
