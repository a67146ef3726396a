"""CPU FP64 oracle for the two-electron TDA-TDDFT gradient (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It wraps ``liboracle.so`` (built from ``tdg_oracle.c`` with gcc,
OpenMP, plain scalar code) through ctypes and shares no code with the HIP
library.  See ``tdg_oracle.c`` for what is computed and which passages of the
paper each piece follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tdg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc -O2 -fopenmp (plain C, no intrinsics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-D_DEFAULT_SOURCE", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Basis(C.Structure):
    _fields_ = [("n_atoms", C.c_int32), ("coords", C.c_void_p),
                ("n_shells", C.c_int32), ("shell_atom", C.c_void_p), ("shell_l", C.c_void_p),
                ("shell_nprim", C.c_void_p), ("shell_prim_off", C.c_void_p),
                ("shell_ao_off", C.c_void_p),
                ("n_prims", C.c_int32), ("exps", C.c_void_p), ("coefs", C.c_void_p),
                ("n_bf", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("omega", C.c_double), ("alpha", C.c_double), ("beta", C.c_double),
                ("tau", C.c_double), ("terms", C.c_int32), ("nthreads", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("quartets", C.c_int64), ("prim_quartets", C.c_int64),
                ("skipped", C.c_int64), ("one_center", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        vp, i64 = C.c_void_p, C.c_int64
        L.orc_grad.argtypes = [C.POINTER(Basis), vp, vp, vp, C.POINTER(Params), vp, C.POINTER(Stats)]
        L.orc_grad_brute.argtypes = [C.POINTER(Basis), vp, vp, vp, C.POINTER(Params), vp]
        L.orc_energy.argtypes = [C.POINTER(Basis), vp, vp, vp, C.POINTER(Params), vp]
        L.orc_quartet_contribs.argtypes = [C.POINTER(Basis), vp, vp, vp, C.POINTER(Params), i64, vp, vp]
        L.orc_quartet_bounds.argtypes = [C.POINTER(Basis), vp, vp, vp, i64, vp, vp]
        L.orc_screen_select.argtypes = [C.POINTER(Basis), vp, vp, vp, C.c_double, C.c_int, C.c_int, i64, vp,
                                        vp, C.POINTER(i64)]
        L.orc_fock_blocks.argtypes = [C.POINTER(Basis), vp, C.c_double, C.c_double, C.c_double, C.c_double,
                                      C.c_int, i64, vp, vp]
        L.orc_schwarz.argtypes = [C.POINTER(Basis), vp]
        L.orc_eri_tensor.argtypes = [C.POINTER(Basis), C.c_int, C.c_double, vp]
        L.orc_norm_coefs.argtypes = [C.POINTER(Basis), vp]
        L.orc_prim_eri.argtypes = [vp, vp, vp, C.c_int, C.c_double]
        L.orc_prim_eri.restype = C.c_double
        L.orc_boys.argtypes = [C.c_int, C.c_double, vp]
        for f in ("orc_grad", "orc_grad_brute", "orc_energy", "orc_quartet_contribs",
                  "orc_quartet_bounds", "orc_screen_select", "orc_fock_blocks", "orc_schwarz", "orc_eri_tensor", "orc_norm_coefs"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def sph_transform(mol):
    """T [n_functions, n_cart] mapping the unit-normalised Cartesian functions of every shell to
    the caller's functions: identity for s, p and Cartesian d; for a d shell of a spherical
    basis the five real solid harmonics r^2 Y_2m (m = -2..2) in the order xy, yz, z^2, xz,
    x^2 - y^2, each scaled to unit norm.  With unit-normalised Cartesian components
    (order xx, xy, xz, yy, yz, zz) the squared components overlap as <xx|yy> = 1/3, so
    (xx - yy) has norm^2 4/3 and (2zz - xx - yy) norm^2 4."""
    ls = np.asarray(mol.shell_l)
    ncart = (ls + 1) * (ls + 2) // 2
    sph = bool(getattr(mol, "spherical", False))
    nfun = np.where((ls == 2) & sph, 5, ncart)
    T = np.zeros((int(nfun.sum()), int(ncart.sum())))
    r, c = 0, 0
    for l, nf, nc in zip(ls, nfun, ncart):
        if sph and l == 2:
            xx, xy, xz, yy, yz, zz = range(6)
            blk = np.zeros((5, 6))
            blk[0, xy] = 1.0
            blk[1, yz] = 1.0
            blk[2, [zz, xx, yy]] = [1.0, -0.5, -0.5]
            blk[3, xz] = 1.0
            blk[4, [xx, yy]] = [np.sqrt(3.0) / 2.0, -np.sqrt(3.0) / 2.0]
        else:
            blk = np.eye(nc)
        T[r:r + nf, c:c + nc] = blk
        r, c = r + nf, c + nc
    return T


def _cart_view(mol):
    """(Cartesian molecule, T, caller's function offsets): for a spherical basis the same shells
    with Cartesian AO offsets in shell order (the caller's functions are assumed in shell
    order, as the stored generators write them); for a Cartesian basis the molecule itself."""
    if not getattr(mol, "spherical", False):
        return mol, None
    import dataclasses
    ls = np.asarray(mol.shell_l)
    ncart = (ls + 1) * (ls + 2) // 2
    nfun = np.where(ls == 2, 5, ncart)
    if not np.array_equal(np.asarray(mol.shell_ao_off), np.concatenate([[0], np.cumsum(nfun)[:-1]])):
        raise ValueError("spherical oracle basis: functions must be in shell order")
    off = np.ascontiguousarray(np.concatenate([[0], np.cumsum(ncart)[:-1]]), dtype=np.int32)
    cm = dataclasses.replace(mol, shell_ao_off=off, spherical=False, P0=None, PD=None, R=None)
    return cm, sph_transform(mol)


class _Bound:
    """Keeps the numpy arrays behind a Basis struct alive (Cartesian functions)."""

    def __init__(self, mol, coords=None):
        mol = _cart_view(mol)[0]
        c = np.ascontiguousarray(mol.coords if coords is None else coords, dtype=np.float64)
        self.keep = [c, mol.shell_atom, mol.shell_l, mol.shell_nprim, mol.shell_prim_off,
                     mol.shell_ao_off, mol.exps, mol.coefs]
        self.b = Basis(mol.n_atoms, _p(c).value, mol.n_shells, _p(mol.shell_atom).value,
                       _p(mol.shell_l).value, _p(mol.shell_nprim).value,
                       _p(mol.shell_prim_off).value, _p(mol.shell_ao_off).value,
                       mol.n_prims, _p(mol.exps).value, _p(mol.coefs).value, mol.n_bf)


def _params(mol, tau=0.0, terms=7, nthreads=0, omega=None, alpha=None, beta=None):
    return Params(mol.omega if omega is None else omega, mol.alpha if alpha is None else alpha,
                  mol.beta if beta is None else beta, tau, terms, nthreads)


def _dens(mol, P0=None, PD=None, R=None):
    """The densities on the Cartesian functions: X_cart = T^T X T for a spherical basis (each
    density is a bilinear form in the functions of its two indices)."""
    f = lambda x, d: np.ascontiguousarray(d if x is None else x, dtype=np.float64)
    out = f(P0, mol.P0), f(PD, mol.PD), f(R, mol.R)
    T = _cart_view(mol)[1]
    if T is None:
        return out
    return tuple(np.ascontiguousarray(T.T @ x @ T) for x in out)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def grad(mol, tau=0.0, terms=7, nthreads=0, coords=None, P0=None, PD=None, R=None,
         omega=None, alpha=None, beta=None, return_stats=False):
    """Gradient [n_atoms, 3] (hartree/bohr), unique quartets with symmetrised Gamma."""
    bb = _Bound(mol, coords)
    P0, PD, R = _dens(mol, P0, PD, R)
    prm = _params(mol, tau, terms, nthreads, omega, alpha, beta)
    out = np.zeros((mol.n_atoms, 3))
    st = Stats()
    _check(lib().orc_grad(C.byref(bb.b), _p(P0), _p(PD), _p(R), C.byref(prm), _p(out), C.byref(st)),
           "grad")
    if return_stats:
        return out, {"quartets": st.quartets, "prim_quartets": st.prim_quartets,
                     "skipped": st.skipped, "one_center": st.one_center}
    return out


def grad_brute(mol, terms=7, nthreads=0, P0=None, PD=None, R=None, omega=None, alpha=None,
               beta=None):
    """Gradient over every ordered shell quartet with the literal Gamma (tiny bases)."""
    bb = _Bound(mol)
    P0, PD, R = _dens(mol, P0, PD, R)
    prm = _params(mol, 0.0, terms, nthreads, omega, alpha, beta)
    out = np.zeros((mol.n_atoms, 3))
    _check(lib().orc_grad_brute(C.byref(bb.b), _p(P0), _p(PD), _p(R), C.byref(prm), _p(out)),
           "grad_brute")
    return out


def energy(mol, terms=7, nthreads=0, coords=None, P0=None, PD=None, R=None, omega=None,
           alpha=None, beta=None):
    """Pseudo-energy sum Gamma (mu nu|lam sig) + Gamma^lr (mu nu|lam sig)_lr."""
    bb = _Bound(mol, coords)
    P0, PD, R = _dens(mol, P0, PD, R)
    prm = _params(mol, 0.0, terms, nthreads, omega, alpha, beta)
    e = np.zeros(1)
    _check(lib().orc_energy(C.byref(bb.b), _p(P0), _p(PD), _p(R), C.byref(prm), _p(e)), "energy")
    return float(e[0])


def quartet_contribs(mol, quartets, terms=7, nthreads=0):
    """Per-quartet contributions [nq, 4, 3] for shell quartets given as [nq, 4] int32."""
    bb = _Bound(mol)
    P0, PD, R = _dens(mol)
    q = np.ascontiguousarray(quartets, dtype=np.int32)
    out = np.zeros((q.shape[0], 4, 3))
    prm = _params(mol, 0.0, terms, nthreads)
    _check(lib().orc_quartet_contribs(C.byref(bb.b), _p(P0), _p(PD), _p(R), C.byref(prm),
                                      q.shape[0], _p(q), _p(out)), "quartet_contribs")
    return out


def quartet_bounds(mol, quartets):
    bb = _Bound(mol)
    P0, PD, R = _dens(mol)
    q = np.ascontiguousarray(quartets, dtype=np.int32)
    out = np.zeros(q.shape[0])
    _check(lib().orc_quartet_bounds(C.byref(bb.b), _p(P0), _p(PD), _p(R), q.shape[0], _p(q),
                                    _p(out)), "quartet_bounds")
    return out


def screen_select(mol, tau, keep=True, nthreads=0, cap=None, P0=None, PD=None, R=None):
    """Unique shell quartets [n, 4] (a>=b, c>=d, pair ab >= pair cd; one-atom quartets left out)
    whose screening bound is >= tau (keep) or < tau (not keep), and their bounds [n]."""
    bb = _Bound(mol)
    P0, PD, R = _dens(mol, P0, PD, R)
    n = C.c_int64()
    if cap is None:
        _check(lib().orc_screen_select(C.byref(bb.b), _p(P0), _p(PD), _p(R), tau, int(keep), nthreads, 0,
                                       None, None, C.byref(n)), "screen_select")
        cap = n.value
    q = np.zeros((max(cap, 1), 4), dtype=np.int32)
    bnd = np.zeros(max(cap, 1))
    _check(lib().orc_screen_select(C.byref(bb.b), _p(P0), _p(PD), _p(R), tau, int(keep), nthreads, cap,
                                   _p(q), _p(bnd), C.byref(n)), "screen_select")
    m = min(n.value, cap)
    return q[:m], bnd[:m]


def fock_blocks(mol, B, pairs, cJ=1.0, cK=0.0, cKlr=0.0, omega=None, nthreads=0):
    """Blocks F[a, b] of the Fock-type matrix for shell pairs [n, 2]; list of arrays (in the
    caller's functions: for a spherical basis T_a F_cart T_b^T with B_cart = T^T B T)."""
    cm, T = _cart_view(mol)
    if T is not None:
        Bc = T.T @ np.asarray(B, dtype=np.float64) @ T
        blocks = fock_blocks(cm, Bc, pairs, cJ, cK, cKlr, mol.omega if omega is None else omega, nthreads)
        ls = np.asarray(mol.shell_l)
        ncart = (ls + 1) * (ls + 2) // 2
        nfun = np.where(ls == 2, 5, ncart)
        fo, co = np.concatenate([[0], np.cumsum(nfun)]), np.concatenate([[0], np.cumsum(ncart)])
        Tb = lambda s: T[fo[s]:fo[s + 1], co[s]:co[s + 1]]
        pr = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
        return [Tb(a) @ blk @ Tb(b).T for (a, b), blk in zip(pr, blocks)]
    bb = _Bound(mol)
    B = np.ascontiguousarray(B, dtype=np.float64)
    pr = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    nc = (mol.shell_l + 1) * (mol.shell_l + 2) // 2
    sizes = nc[pr[:, 0]] * nc[pr[:, 1]]
    out = np.zeros(int(sizes.sum()))
    _check(lib().orc_fock_blocks(C.byref(bb.b), _p(B), cJ, cK, cKlr, mol.omega if omega is None else omega,
                                 nthreads, pr.shape[0], _p(pr), _p(out)), "fock_blocks")
    res, o = [], 0
    for (a, b_), s in zip(pr, sizes):
        res.append(out[o:o + s].reshape(nc[a], nc[b_]))
        o += s
    return res


def fock(mol, B, cJ=1.0, cK=0.0, cKlr=0.0, omega=None, nthreads=0):
    """The full Fock-type matrix [n_bf, n_bf] (small bases)."""
    ns = mol.n_shells
    pairs = np.array([(a, b) for a in range(ns) for b in range(ns)], dtype=np.int32)
    blocks = fock_blocks(mol, B, pairs, cJ, cK, cKlr, omega, nthreads)
    F = np.zeros((mol.n_bf, mol.n_bf))
    nc = np.array([blk.shape[0] for blk in blocks[::ns]])
    for (a, b), blk in zip(pairs, blocks):
        oa, ob = mol.shell_ao_off[a], mol.shell_ao_off[b]
        F[oa:oa + nc[a], ob:ob + nc[b]] = blk
    return F


def cphf_matrix(mol, C_occ, C_vir, omega=None, alpha=None, beta=None):
    """A of eq cphf_a (section II.B) without the exchange-correlation kernel term, written out
    from its definition in the molecular orbitals:
      A_{ai,bj} = 4 (ia|jb) - alpha [(ij|ab) + (ib|aj)] - beta [(ij|ab)_lr + (ib|aj)_lr],
    rows (a, i) and columns (b, j) in row-major (virtual, occupied) order."""
    al = mol.alpha if alpha is None else alpha
    be = mol.beta if beta is None else beta
    Co, Cv = np.asarray(C_occ, dtype=np.float64), np.asarray(C_vir, dtype=np.float64)

    def mo(T, X1, X2, X3, X4):
        return np.einsum("pqrs,pi,qj,rk,sl->ijkl", T, X1, X2, X3, X4, optimize=True)

    I = eri_tensor(mol, 0)
    Il = eri_tensor(mol, 1, omega)
    ovov = lambda T: mo(T, Co, Cv, Co, Cv)      # (ia|jb)[i, a, j, b]
    oovv = lambda T: mo(T, Co, Co, Cv, Cv)      # (ij|ab)[i, j, a, b]
    ovvo = lambda T: mo(T, Co, Cv, Cv, Co)      # (ib|aj)[i, b, a, j]
    A = (4.0 * np.einsum("iajb->aibj", ovov(I))
         - al * (np.einsum("ijab->aibj", oovv(I)) + np.einsum("ibaj->aibj", ovvo(I)))
         - be * (np.einsum("ijab->aibj", oovv(Il)) + np.einsum("ibaj->aibj", ovvo(Il))))
    no, nv = Co.shape[1], Cv.shape[1]
    return A.reshape(nv * no, nv * no)


def zvector(mol, C_occ, C_vir, eps_occ, eps_vir, L, omega=None, alpha=None, beta=None):
    """Z of eq cphf, (d - A) Z = L with d_ai = eps_i - eps_a, by a direct dense solve."""
    A = cphf_matrix(mol, C_occ, C_vir, omega, alpha, beta)
    eo, ev = np.asarray(eps_occ), np.asarray(eps_vir)
    d = (eo[None, :] - ev[:, None]).reshape(-1)
    Z = np.linalg.solve(np.diag(d) - A, np.asarray(L, dtype=np.float64).reshape(-1))
    return Z.reshape(len(ev), len(eo))


def schwarz(mol):
    bb = _Bound(mol)
    ns = mol.n_shells
    out = np.zeros(ns * (ns + 1) // 2)
    _check(lib().orc_schwarz(C.byref(bb.b), _p(out)), "schwarz")
    return out


def eri_tensor(mol, op=0, omega=None):
    cm, T = _cart_view(mol)
    if T is not None:  # (mu nu|lam sig) in the caller's functions
        Tc = eri_tensor(cm, op, mol.omega if omega is None else omega)
        return np.einsum("ai,bj,ck,dl,ijkl->abcd", T, T, T, T, Tc, optimize=True)
    bb = _Bound(mol)
    n = mol.n_bf
    out = np.zeros((n, n, n, n))
    _check(lib().orc_eri_tensor(C.byref(bb.b), op, mol.omega if omega is None else omega,
                                _p(out)), "eri_tensor")
    return out


def norm_coefs(mol):
    bb = _Bound(mol)
    out = np.zeros(mol.n_prims)
    _check(lib().orc_norm_coefs(C.byref(bb.b), _p(out)), "norm_coefs")
    return out


def prim_eri(lxyz, zeta, centers, op=0, omega=0.3):
    l = np.ascontiguousarray(lxyz, dtype=np.int32).reshape(4, 3)
    z = np.ascontiguousarray(zeta, dtype=np.float64).reshape(4)
    c = np.ascontiguousarray(centers, dtype=np.float64).reshape(4, 3)
    return float(lib().orc_prim_eri(_p(l), _p(z), _p(c), op, omega))


def boys(mmax, T):
    out = np.zeros(mmax + 1)
    lib().orc_boys(mmax, float(T), _p(out))
    return out
