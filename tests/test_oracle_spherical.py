"""Pins of the oracle's spherical (real solid-harmonic) d functions (section II.C names both
Cartesian and spherical functions; eq cartG gives the Cartesian ones):

- through a tight s charge far away, (mu nu|cc) R -> <mu|nu>: the five functions of a d
  shell are orthonormal, and orthogonal to the s-type combination xx + yy + zz that the six
  Cartesian components also contain -- a wrong coefficient in any of them fails this;
- the gradient in the spherical basis equals Richardson central differences of the
  pseudo-energy in that basis, and equals the Cartesian computation with the densities
  transformed as T^T P T (by the definition of the functions)."""
import numpy as np

from paper_2407_16586_amd import synth
from tests import molecules


def _far_charge_molecule(spherical):
    Rf = 2000.0
    shells = [(0, 2, [1.1, 0.35], [0.6, 0.5]), (0, 2, [0.7], [1.0]), (1, 0, [500.0], [1.0])]
    m = molecules.make([[0, 0, 0], [Rf, 0, 0]], shells)
    if spherical:
        m = synth.spherical_copy(m)
    return m, Rf


def test_solid_harmonics_orthonormal(oracle_lib):
    m, Rf = _far_charge_molecule(True)
    T = oracle_lib.eri_tensor(m, 0)
    n = m.n_bf
    S = T[:n - 1, :n - 1, n - 1, n - 1] * Rf         # overlaps of the two d shells' functions
    for blk in (slice(0, 5), slice(5, 10)):
        assert np.abs(S[blk, blk] - np.eye(5)).max() < 1e-6, S[blk, blk]
    # the s-type combination of the Cartesian components is orthogonal to all five
    mc, _ = _far_charge_molecule(False)
    Tc = oracle_lib.eri_tensor(mc, 0)
    Sc = Tc[:6, :6, 12, 12] * Rf                     # Cartesian overlaps of the first d shell
    r2 = np.array([1.0, 0, 0, 1.0, 0, 1.0])
    Tr = oracle_lib.sph_transform(m)[:5, :6]
    assert np.abs(Tr @ Sc @ r2).max() < 1e-6 * np.abs(Sc @ r2).max()


def test_spherical_gradient_vs_fd_and_transformed_densities(oracle_lib):
    m = synth.spherical_copy(molecules.small_mixed(), seed=3)
    g = oracle_lib.grad(m)
    # the Cartesian computation with transformed densities
    T = oracle_lib.sph_transform(m)
    mc = molecules.small_mixed()
    gc = oracle_lib.grad(mc, P0=T.T @ m.P0 @ T, PD=T.T @ m.PD @ T, R=T.T @ m.R @ T)
    assert np.abs(g - gc).max() <= 1e-13 * np.abs(g).max()
    # Richardson central differences of the spherical pseudo-energy (atom 2, x and z)
    for atom, d in ((2, 0), (3, 2)):
        def e(hh):
            x = m.coords.copy()
            x[atom, d] += hh
            return oracle_lib.energy(m, coords=x)
        h = 2e-3
        d1 = (e(h) - e(-h)) / (2 * h)
        d2 = (e(h / 2) - e(-h / 2)) / h
        fd = (4 * d2 - d1) / 3
        assert abs(fd - g[atom, d]) <= 1e-8 * max(1.0, abs(g[atom, d])), (atom, d, fd, g[atom, d])
