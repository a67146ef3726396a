"""Seeded synthetic workloads for the two-electron TDA-TDDFT gradient.

This module builds inputs only: geometries, shell/primitive tables and the
three density matrices (ground state P0, relaxed difference PDelta and
transition R).  It contains none of the method's arithmetic (no integrals, no
normalisation, no screening) and is shared by the HIP path's tests, the
benchmark and the CPU oracle's tests as their common source of inputs.

Shapes follow the paper's workload class (section III.A): protein-like
first-row/hydrogen systems with a contracted core s shell, split valence and
one d polarisation shell on heavy atoms, Cartesian functions, l <= 2.

Basis recipe per atom (the contraction pattern of the paper's def2-SVP runs,
section III.A: [3s2p1d] on heavy atoms, [2s1p] on H), in two variants:
  "stated" (default; the recipe the workloads are defined with): exponents
      log-uniform in [0.1, 5000] for every shell, sorted descending within a
      shell; contraction coefficients N(0, 1), normalised by the consumer;
  "svp": exponent ranges per shell shaped like def2-SVP and positive
      coefficients exp(N(0, 0.5)):
        heavy s(6) [3, 5000]  s(1) [0.3, 1.0]  s(1) [0.08, 0.3]
              p(3) [0.4, 15]  p(1) [0.1, 0.3]  d(1) [0.4, 1.5]
        H     s(3) [0.4, 15]  s(1) [0.1, 0.25] p(1) [0.6, 1.2]
  heavy : s(6) s(1) s(1) p(3) p(1) d(1)  -> 6 shells, 13 prims, 15 Cartesian functions
  H     : s(3) s(1) p(1)                 -> 3 shells,  5 prims,  5 functions

Densities (definitions of section II.A): P0 = occ * C_o C_o^T,
R = C_o X C_v^T with X an n_occ x n_vir amplitude matrix of unit Frobenius
norm, PDelta a random symmetric matrix of Frobenius norm 0.1.  C is the Q
factor of a Gaussian random matrix (Euclidean-orthonormal; synthetic data,
not an SCF result).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BASE_SEED = 20240716

# (l, primitives, exponent range) per shell, per recipe; coefficient law per recipe
_WIDE = (0.1, 5000.0)
RECIPES = {
    "stated": {
        "heavy": ((0, 6, _WIDE), (0, 1, _WIDE), (0, 1, _WIDE), (1, 3, _WIDE), (1, 1, _WIDE), (2, 1, _WIDE)),
        "H": ((0, 3, _WIDE), (0, 1, _WIDE), (1, 1, _WIDE)),
        "coef": lambda rng, k: rng.standard_normal(k),
    },
    "svp": {
        "heavy": ((0, 6, (3.0, 5000.0)), (0, 1, (0.3, 1.0)), (0, 1, (0.08, 0.3)),
                  (1, 3, (0.4, 15.0)), (1, 1, (0.1, 0.3)), (2, 1, (0.4, 1.5))),
        "H": ((0, 3, (0.4, 15.0)), (0, 1, (0.1, 0.25)), (1, 1, (0.6, 1.2))),
        "coef": lambda rng, k: np.exp(0.5 * rng.standard_normal(k)),
    },
}

# range-separated hybrid parameters of the paper's production functional
OMEGA = 0.3
ALPHA_SR = 0.157706
ALPHA_LR = 1.0


def ncart(l: int) -> int:
    return (l + 1) * (l + 2) // 2


@dataclasses.dataclass
class Molecule:
    """One molecule: geometry, Cartesian Gaussian basis and densities.

    Arrays (all C-contiguous):
      coords      [n_atoms, 3] float64, bohr
      Z           [n_atoms] int32 nuclear charge (1 = H, else heavy)
      shell_atom, shell_l, shell_nprim, shell_prim_off, shell_ao_off [n_shells] int32
      exps, coefs [n_prims] float64 (coefs multiply unnormalised primitives)
      P0, PD, R   [n_bf, n_bf] float64 row-major
    """
    name: str
    coords: np.ndarray
    Z: np.ndarray
    shell_atom: np.ndarray
    shell_l: np.ndarray
    shell_nprim: np.ndarray
    shell_prim_off: np.ndarray
    shell_ao_off: np.ndarray
    exps: np.ndarray
    coefs: np.ndarray
    n_occ: int
    P0: np.ndarray | None = None
    PD: np.ndarray | None = None
    R: np.ndarray | None = None
    omega: float = OMEGA
    alpha: float = ALPHA_SR
    beta: float = ALPHA_LR - ALPHA_SR
    spherical: bool = False     # d shells as 5 real solid harmonics (shell_ao_off counts 5)

    @property
    def n_atoms(self) -> int:
        return int(self.coords.shape[0])

    @property
    def n_shells(self) -> int:
        return int(self.shell_l.shape[0])

    @property
    def n_prims(self) -> int:
        return int(self.exps.shape[0])

    @property
    def n_bf(self) -> int:
        nf = lambda l: 5 if (self.spherical and l == 2) else ncart(l)
        return int(max(o + nf(int(l)) for o, l in zip(self.shell_ao_off, self.shell_l)))

    def subset_check(self) -> None:
        assert self.coords.dtype == np.float64 and self.coords.shape[1] == 3
        for a in ("shell_atom", "shell_l", "shell_nprim", "shell_prim_off", "shell_ao_off"):
            assert getattr(self, a).dtype == np.int32
        if self.P0 is not None:
            n = self.n_bf
            assert self.P0.shape == (n, n) and self.PD.shape == (n, n) and self.R.shape == (n, n)


def _build_basis(rng: np.random.Generator, Z: np.ndarray, recipe: str = "stated"):
    rec = RECIPES[recipe]
    sh_atom, sh_l, sh_np, sh_po, sh_ao = [], [], [], [], []
    exps, coefs = [], []
    ao = 0
    for ia, z in enumerate(Z):
        for l, k, (elo, ehi) in (rec["H"] if z == 1 else rec["heavy"]):
            e = np.sort(np.exp(rng.uniform(math.log(elo), math.log(ehi), size=k)))[::-1]
            c = rec["coef"](rng, k)
            sh_atom.append(ia)
            sh_l.append(l)
            sh_np.append(k)
            sh_po.append(len(exps))
            sh_ao.append(ao)
            exps.extend(e.tolist())
            coefs.extend(c.tolist())
            ao += ncart(l)
    i32 = lambda v: np.ascontiguousarray(np.asarray(v, dtype=np.int32))
    return (i32(sh_atom), i32(sh_l), i32(sh_np), i32(sh_po), i32(sh_ao),
            np.ascontiguousarray(np.asarray(exps, dtype=np.float64)),
            np.ascontiguousarray(np.asarray(coefs, dtype=np.float64)))


def _densities(rng: np.random.Generator, n_bf: int, n_occ: int, occ_factor: float = 2.0):
    A = rng.standard_normal((n_bf, n_bf))
    Qm, Rm = np.linalg.qr(A)
    Qm = Qm * np.sign(np.diag(Rm))[None, :]          # sign-fixed: diag(R) > 0
    Co, Cv = Qm[:, :n_occ], Qm[:, n_occ:]
    P0 = occ_factor * Co @ Co.T
    P0 = 0.5 * (P0 + P0.T)
    S = rng.standard_normal((n_bf, n_bf))
    S = 0.5 * (S + S.T)
    PD = 0.1 * S / np.linalg.norm(S)
    X = rng.standard_normal((n_occ, n_bf - n_occ))
    X /= np.linalg.norm(X)
    R = Co @ X @ Cv.T
    c = np.ascontiguousarray
    return c(P0), c(PD), c(R), c(Qm), c(X)


def _min_sep_ok(xyz: np.ndarray, new: np.ndarray, dmin: float) -> bool:
    if xyz.shape[0] == 0:
        return True
    return bool(np.min(np.linalg.norm(xyz - new[None, :], axis=1)) >= dmin)


def _box_geometry(rng, n_atoms, box, dmin=1.8, max_tries=200000):
    pts = np.zeros((0, 3))
    tries = 0
    while pts.shape[0] < n_atoms:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place atoms at the requested separation")
        p = rng.uniform(0.0, box, size=3)
        if _min_sep_ok(pts, p, dmin):
            pts = np.vstack([pts, p])
    return pts


def _sphere_geometry(rng, n_atoms, density=0.1, dmin=1.8, max_tries=10_000_000):
    radius = (3.0 * n_atoms / (4.0 * math.pi * density)) ** (1.0 / 3.0)
    pts = np.zeros((n_atoms, 3))
    n = 0
    tries = 0
    cell = dmin
    grid: dict = {}
    while n < n_atoms:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("droplet packing failed")
        p = rng.uniform(-radius, radius, size=3)
        if p @ p > radius * radius:
            continue
        key = tuple(np.floor(p / cell).astype(int))
        ok = True
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    for j in grid.get((key[0] + dx, key[1] + dy, key[2] + dz), ()):
                        if np.sum((pts[j] - p) ** 2) < dmin * dmin:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            pts[n] = p
            grid.setdefault(key, []).append(n)
            n += 1
    return pts


def _assemble(name, rng, coords, Z, n_occ=None, occ_frac=0.1, with_dens=True, recipe="stated"):
    basis = _build_basis(rng, Z, recipe)
    sh_atom, sh_l, sh_np, sh_po, sh_ao, exps, coefs = basis
    n_bf = int(sh_ao[-1] + ncart(int(sh_l[-1])))
    if n_occ is None:
        n_occ = max(1, int(round(occ_frac * n_bf)))
    mol = Molecule(name=name, coords=np.ascontiguousarray(coords, dtype=np.float64),
                   Z=np.ascontiguousarray(Z, dtype=np.int32), shell_atom=sh_atom,
                   shell_l=sh_l, shell_nprim=sh_np, shell_prim_off=sh_po,
                   shell_ao_off=sh_ao, exps=exps, coefs=coefs, n_occ=int(n_occ))
    if with_dens:
        mol.P0, mol.PD, mol.R, _, _ = _densities(rng, n_bf, n_occ)
    mol.subset_check()
    return mol


def config0(seed_offset: int = 0) -> Molecule:
    """6 atoms (2 heavy + 4 H) in a 6 bohr box, min separation 1.8 bohr; n_occ = 8."""
    rng = np.random.default_rng(BASE_SEED + 0 + seed_offset)
    coords = _box_geometry(rng, 6, 6.0)
    Z = np.array([6, 6, 1, 1, 1, 1], dtype=np.int32)
    return _assemble("six-atom box (50 functions)", rng, coords, Z, n_occ=8)


def chain(n_heavy: int = 20, seed: int = BASE_SEED + 1, n_occ: int | None = 50, recipe: str = "stated") -> Molecule:
    """Alkane-like chain: heavy atoms every 2.9 bohr along x with +-0.2 bohr jitter,
    two H per heavy atom at 2.06 bohr."""
    rng = np.random.default_rng(seed)
    pts, Z = [], []
    for i in range(n_heavy):
        c = np.array([2.9 * i, 0.0, 0.0]) + rng.uniform(-0.2, 0.2, size=3)
        pts.append(c)
        Z.append(6)
        for s in (+1.0, -1.0):
            d = np.array([0.0, s * 0.816, 0.577 * (-1.0) ** i])
            d = d / np.linalg.norm(d) * 2.06
            pts.append(c + d + rng.uniform(-0.2, 0.2, size=3) * 0.25)
            Z.append(1)
    coords = np.array(pts)
    dm = np.linalg.norm(coords[:, None] - coords[None], axis=-1) + np.eye(len(coords)) * 1e9
    assert dm.min() >= 1.8, dm.min()
    if n_occ is None:
        n_occ = 5 * n_heavy // 2
    return _assemble(f"{3 * n_heavy}-atom chain", rng, coords, np.array(Z), n_occ=n_occ, recipe=recipe)


def config1(recipe: str = "stated") -> Molecule:
    """60-atom alkane-like chain (20 heavy + 40 H, 500 functions), n_occ = 50."""
    m = chain(20, BASE_SEED + 1, 50, recipe)
    m.name = "60-atom chain (500 functions)" + ("" if recipe == "stated" else f", {recipe} exponents")
    return m


def droplet(n_atoms: int, seed: int, heavy_frac: float = 1.0 / 3.0, occ_frac: float = 0.1,
            with_dens: bool = True) -> Molecule:
    rng = np.random.default_rng(seed)
    coords = _sphere_geometry(rng, n_atoms)
    n_heavy = int(round(heavy_frac * n_atoms))
    Z = np.array([6] * n_heavy + [1] * (n_atoms - n_heavy), dtype=np.int32)
    rng.shuffle(Z)
    return _assemble(f"{n_atoms}-atom droplet", rng, coords, Z, occ_frac=occ_frac,
                     with_dens=with_dens)


def config2(n_mol: int = 64, with_dens: bool = True) -> list[Molecule]:
    """64 independent molecules, 10-120 atoms each (1/3 heavy), droplet geometry at
    0.1 atoms/bohr^3, n_occ = round(0.1 n_bf)."""
    rng = np.random.default_rng(BASE_SEED + 2)
    sizes = rng.integers(10, 121, size=n_mol)
    return [droplet(int(n), BASE_SEED + 2 + 1000 * (i + 1), with_dens=with_dens)
            for i, n in enumerate(sizes)]


def config2_molecule(i: int, with_dens: bool = True) -> Molecule:
    """Molecule i of config2() alone (the same seeds, without building the others)."""
    sizes = np.random.default_rng(BASE_SEED + 2).integers(10, 121, size=64)
    return droplet(int(sizes[i]), BASE_SEED + 2 + 1000 * (i + 1), with_dens=with_dens)


def water_cluster(n_waters: int, seed: int, with_dens: bool = True, recipe: str = "stated") -> Molecule:
    """n waters on the sites of a 6x6x4 cubic lattice (5.9 bohr) nearest its centroid, +-0.4 bohr
    jitter, O-H 1.81 bohr, HOH 104.5 degrees, random orientations; 5 occupied orbitals per water."""
    rng = np.random.default_rng(seed)
    g = np.array([(i, j, k) for i in range(6) for j in range(6) for k in range(4)], float) * 5.9
    cen = g.mean(axis=0)
    order = np.argsort(np.linalg.norm(g - cen, axis=1), kind="stable")
    sites = g[order[:n_waters]]
    roh, ang = 1.81, math.radians(104.5)
    body = np.array([[0.0, 0.0, 0.0],
                     [roh * math.sin(ang / 2), 0.0, roh * math.cos(ang / 2)],
                     [-roh * math.sin(ang / 2), 0.0, roh * math.cos(ang / 2)]])
    pts, Z = [], []
    for s_ in sites:
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        q = q * np.sign(np.diag(r))[None, :]
        o = s_ + rng.uniform(-0.4, 0.4, size=3)
        for a, z in zip(body, (8, 1, 1)):
            pts.append(o + q @ a)
            Z.append(z)
    return _assemble(f"{n_waters} waters", rng, np.array(pts), np.array(Z), n_occ=5 * n_waters,
                     with_dens=with_dens, recipe=recipe)


def config3(with_dens: bool = True) -> Molecule:
    """133 waters on a 5.9 bohr cubic lattice with +-0.4 bohr jitter, random orientations."""
    return water_cluster(133, BASE_SEED + 3, with_dens)


def config4(with_dens: bool = True) -> Molecule:
    """1500-atom protein-like droplet, H735 C480 O150 N135, 0.1 atoms/bohr^3."""
    rng = np.random.default_rng(BASE_SEED + 4)
    coords = _sphere_geometry(rng, 1500)
    Z = np.array([1] * 735 + [6] * 480 + [8] * 150 + [7] * 135, dtype=np.int32)
    rng.shuffle(Z)
    electrons = int(Z.sum())
    return _assemble("1500-atom droplet", rng, coords, Z, n_occ=electrons // 2,
                     with_dens=with_dens)


def spherical_copy(mol: Molecule, seed: int = 0) -> Molecule:
    """The same geometry and shells with d shells as 5 real solid harmonics (functions in shell
    order) and fresh seeded densities of the smaller size: P0 = 2 C_o C_o^T from random
    orthonormal orbitals, a symmetric PDelta and a general R, of the magnitudes the
    Cartesian generators use."""
    ls = np.asarray(mol.shell_l)
    nf = np.where(ls == 2, 5, (ls + 1) * (ls + 2) // 2)
    off = np.ascontiguousarray(np.concatenate([[0], np.cumsum(nf)[:-1]]), dtype=np.int32)
    out = dataclasses.replace(mol, name=mol.name + " (spherical d)", shell_ao_off=off, spherical=True,
                              P0=None, PD=None, R=None)
    n = int(nf.sum())
    rng = np.random.default_rng(seed)
    n_occ = max(1, min(mol.n_occ, n // 2))
    P0, PD, R = _densities(rng, n, n_occ)[:3]
    out.P0, out.PD, out.R = P0, PD, R
    return out


def random_molecule(n_heavy: int, n_h: int, seed: int, box: float | None = None,
                    n_occ: int | None = None) -> Molecule:
    """Small random molecule in a box (test helper for edge cases)."""
    rng = np.random.default_rng(seed)
    n = n_heavy + n_h
    if box is None:
        box = max(3.0, 2.2 * n ** (1.0 / 3.0) * 1.8)
    coords = _box_geometry(rng, n, box)
    Z = np.array([6] * n_heavy + [1] * n_h, dtype=np.int32)
    return _assemble(f"random {n_heavy}+{n_h}", rng, coords, Z,
                     n_occ=n_occ if n_occ is not None else None, occ_frac=0.15)


CONFIGS = {0: config0, 1: config1, 3: config3, 4: config4}
