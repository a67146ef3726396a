"""Pins of the oracle's Fock-type matrix (section II.B, eqs G_2e and zfock, two-electron
part), F = cJ J(Bs) + cK K(Bs) + cKlr K_lr(Bs) with Bs = (B + B^T)/2,
  J_{mu nu} = sum (mu nu|lam sig) Bs_{lam sig},   K_{mu nu} = sum (mu lam|nu sig) Bs_{lam sig},
checked against what the mathematics fixes rather than against the oracle itself:

- s functions only: every integral is the closed form erf(sqrt(a) R)/R of unit-charge
  Gaussians (a = pq/(p+q), and 1/a = 1/p + 1/q + 1/omega^2 for the long-range kernel),
  written out here with the textbook normalisation, and J, K, K_lr are contracted from
  that tensor; a swapped index pair (J for K, or (mu nu|lam sig) for (mu lam|nu sig))
  fails it;
- with p and d shells: the pseudo-energy of a ground-state-like density B (the oracle's
  eq gamma contraction, pinned separately by finite differences and by the MO forms) is
  the quadratic form tr(B F(B)) with (cJ, cK, cKlr) = (1/2, -alpha/4, -beta/4); by
  polarisation tr(B1 F(B2)) = [E(B1 + B2) - E(B1 - B2)] / 4 for every symmetric B1,
  which fixes every element of F(B2);
- J, K and K_lr are positive semidefinite forms (the Coulomb and erf kernels have
  positive Fourier transforms): tr(B X(B)) >= 0 for any B;
- F is symmetric, linear in B and in the coefficients, and depends on B only through Bs.
"""
import math

import numpy as np
import pytest
from scipy.special import erf

from tests import molecules


def _s_molecule(seed=5):
    rng = np.random.default_rng(seed)
    coords = np.array([[0.0, 0.0, 0.0], [1.4, 0.2, -0.1], [-0.3, 1.7, 0.4], [0.5, -0.6, 1.9]])
    coords += rng.uniform(-0.1, 0.1, coords.shape)
    shells = [
        (0, 0, [30.0, 5.0, 1.1], [0.2, 0.5, 0.5]),
        (0, 0, [0.35], [1.0]),
        (1, 0, [4.0, 0.7], [0.4, 0.7]),
        (2, 0, [2.2, 0.5], [0.6, 0.5]),
        (3, 0, [0.9], [1.0]),
        (3, 0, [12.0, 2.0], [0.5, 0.6]),
    ]
    return molecules.make(coords, shells, seed=seed)


def _s_functions(m):
    """Per basis function: exponents, coefficients with the primitive normalisation
    (2 a / pi)^(3/4) and the contraction renormalised to unit self-overlap, centre."""
    funcs = []
    for s in range(m.n_shells):
        o, k = m.shell_prim_off[s], m.shell_nprim[s]
        z = np.array(m.exps[o:o + k])
        c = np.array(m.coefs[o:o + k]) * (2 * z / math.pi) ** 0.75
        S = sum(c[i] * c[j] * (math.pi / (z[i] + z[j])) ** 1.5 for i in range(k) for j in range(k))
        funcs.append((z, c / math.sqrt(S), m.coords[m.shell_atom[s]]))
    return funcs


def _ss_prim(za, zb, zc, zd, A, B, C, D, omega=None):
    p, q = za + zb, zc + zd
    P, Q = (za * A + zb * B) / p, (zc * C + zd * D) / q
    Kab = math.exp(-za * zb / p * float(np.sum((A - B) ** 2)))
    Kcd = math.exp(-zc * zd / q * float(np.sum((C - D) ** 2)))
    a = p * q / (p + q) if omega is None else 1.0 / (1.0 / p + 1.0 / q + 1.0 / omega ** 2)
    R = math.sqrt(float(np.sum((P - Q) ** 2)))
    pre = Kab * Kcd * (math.pi ** 2 / (p * q)) ** 1.5
    if R < 1e-12:
        return pre * 2.0 * math.sqrt(a / math.pi)
    return pre * erf(math.sqrt(a) * R) / R


def _s_tensor(m, omega=None):
    f = _s_functions(m)
    n = len(f)
    T = np.zeros((n, n, n, n))
    for i in range(n):
        for j in range(n):
            for k in range(n):
                for l in range(n):
                    (za, ca, A), (zb, cb, B), (zc, cc, C), (zd, cd, D) = f[i], f[j], f[k], f[l]
                    v = 0.0
                    for a in range(len(za)):
                        for b in range(len(zb)):
                            for c in range(len(zc)):
                                for d in range(len(zd)):
                                    v += (ca[a] * cb[b] * cc[c] * cd[d] *
                                          _ss_prim(za[a], zb[b], zc[c], zd[d], A, B, C, D, omega))
                    T[i, j, k, l] = v
    return T


def test_fock_s_only_closed_form(oracle_lib):
    m = _s_molecule()
    n = m.n_bf
    rng = np.random.default_rng(2)
    B = rng.standard_normal((n, n))
    Bs = 0.5 * (B + B.T)
    I = _s_tensor(m)
    Il = _s_tensor(m, m.omega)
    J = np.einsum("mnls,ls->mn", I, Bs)
    K = np.einsum("mlns,ls->mn", I, Bs)
    Kl = np.einsum("mlns,ls->mn", Il, Bs)
    for (cj, ck, cl), ref in (((1.0, 0.0, 0.0), J), ((0.0, 1.0, 0.0), K), ((0.0, 0.0, 1.0), Kl),
                              ((2.0, -m.alpha, -m.beta), 2 * J - m.alpha * K - m.beta * Kl)):
        F = oracle_lib.fock(m, B, cj, ck, cl)
        err = np.abs(F - ref).max()
        assert err <= 1e-12 * np.abs(ref).max(), ((cj, ck, cl), err)


def _sym(rng, n):
    A = rng.standard_normal((n, n))
    return 0.5 * (A + A.T)


def test_fock_energy_quadratic_form(oracle_lib):
    m = molecules.small_mixed()
    n = m.n_bf
    rng = np.random.default_rng(4)
    Z = np.zeros((n, n))
    cf = (0.5, -m.alpha / 4, -m.beta / 4)
    E = lambda X: oracle_lib.energy(m, P0=X, PD=Z, R=Z)
    B2 = _sym(rng, n)
    F2 = oracle_lib.fock(m, B2, *cf)
    e2 = E(B2)
    assert abs(np.sum(B2 * F2) - e2) <= 1e-11 * abs(e2)
    for _ in range(3):
        B1 = _sym(rng, n)
        ref = (E(B1 + B2) - E(B1 - B2)) / 4.0
        v = np.sum(B1 * F2)
        assert abs(v - ref) <= 1e-11 * max(abs(ref), abs(e2)), (v, ref)


def test_fock_positive_forms(oracle_lib):
    m = molecules.small_mixed()
    n = m.n_bf
    rng = np.random.default_rng(6)
    for _ in range(3):
        B = rng.standard_normal((n, n))
        Bs = 0.5 * (B + B.T)
        for cf in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
            assert np.sum(Bs * oracle_lib.fock(m, B, *cf)) >= 0.0, cf


def test_fock_symmetry_and_linearity(oracle_lib):
    m = molecules.small_mixed()
    n = m.n_bf
    rng = np.random.default_rng(8)
    B1, B2 = rng.standard_normal((n, n)), rng.standard_normal((n, n))
    cf = (2.0, -m.alpha, -m.beta)
    F1, F2 = oracle_lib.fock(m, B1, *cf), oracle_lib.fock(m, B2, *cf)
    scale = np.abs(F1).max()
    assert np.abs(F1 - F1.T).max() <= 1e-13 * scale
    assert np.abs(oracle_lib.fock(m, B1.T, *cf) - F1).max() <= 1e-13 * scale
    F12 = oracle_lib.fock(m, 0.7 * B1 - 1.3 * B2, *cf)
    assert np.abs(F12 - (0.7 * F1 - 1.3 * F2)).max() <= 1e-12 * scale
    parts = [oracle_lib.fock(m, B1, *c) for c in ((1, 0, 0), (0, 1, 0), (0, 0, 1))]
    assert np.abs(cf[0] * parts[0] + cf[1] * parts[1] + cf[2] * parts[2] - F1).max() <= 1e-12 * scale


def test_fock_blocks_subset(oracle_lib):
    m = molecules.small_mixed()
    rng = np.random.default_rng(9)
    B = rng.standard_normal((m.n_bf, m.n_bf))
    F = oracle_lib.fock(m, B, 2.0, -m.alpha, -m.beta)
    pairs = np.array([[2, 6], [6, 2], [0, 0], [7, 4]], dtype=np.int32)
    blocks = oracle_lib.fock_blocks(m, B, pairs, 2.0, -m.alpha, -m.beta)
    nc = (m.shell_l + 1) * (m.shell_l + 2) // 2
    for (a, b), blk in zip(pairs, blocks):
        oa, ob = m.shell_ao_off[a], m.shell_ao_off[b]
        assert np.array_equal(blk, F[oa:oa + nc[a], ob:ob + nc[b]])
