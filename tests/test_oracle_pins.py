"""Pins of the CPU oracle against what mathematics and the paper fix.

Every check here uses a source of truth other than the oracle's own code:
independent library routines (mpmath, scipy, torch autograd), closed forms,
limits, finite differences, invariants and a brute-force sum.  A plausible
mistake in the oracle (a dropped recursion term, a wrong sign, a transposed
density, a wrong degeneracy) fails at least one of them.
"""
import math

import numpy as np
import pytest

from tests import molecules


# ---------------------------------------------------------------- Boys function
def test_boys_against_mpmath(oracle_lib):
    """F_m(T) = 1F1(m+1/2; m+3/2; -T)/(2m+1) (Boys function; confluent hypergeometric form)."""
    import mpmath
    mpmath.mp.dps = 40
    for T in [0.0, 1e-12, 1e-6, 0.03, 0.5, 1.0, 2.7, 7.9, 12.0, 19.9, 29.99, 30.01, 45.0, 80.0,
              150.0, 400.0, 2500.0]:
        F = oracle_lib.boys(10, T)
        for m in range(11):
            ref = float(mpmath.hyp1f1(m + 0.5, m + 1.5, -T) / (2 * m + 1))
            assert abs(F[m] - ref) <= 2e-14 * abs(ref) + 1e-300, (m, T, F[m], ref)


def test_boys_special_values(oracle_lib):
    from scipy.special import gammainc, gamma
    F0 = oracle_lib.boys(9, 0.0)
    assert np.allclose(F0, [1.0 / (2 * m + 1) for m in range(10)], rtol=1e-15, atol=0)
    # F_m(T) = Gamma(m+1/2) P(m+1/2, T) / (2 T^(m+1/2)) (regularised lower incomplete gamma)
    for T in (0.7, 5.0, 33.0):
        F = oracle_lib.boys(6, T)
        for m in range(7):
            ref = gamma(m + 0.5) * gammainc(m + 0.5, T) / (2 * T ** (m + 0.5))
            assert abs(F[m] - ref) < 1e-13 * ref


# ------------------------------------------------------------- s-type integrals
def _ss_closed(za, zb, zc, zd, A, B, C, D, omega=None):
    """Closed form evaluated at 40 digits (the inputs are exact doubles), so the reference's
    own rounding (exp of arguments of several hundred) does not enter the comparison."""
    import mpmath
    mp = mpmath.mp
    mp.dps = 40
    f = mpmath.mpf
    za, zb, zc, zd = f(za), f(zb), f(zc), f(zd)
    A, B, C, D = ([f(x) for x in v] for v in (A, B, C, D))
    p, q = za + zb, zc + zd
    P = [(za * a + zb * b) / p for a, b in zip(A, B)]
    Q = [(zc * c + zd * d) / q for c, d in zip(C, D)]
    Kab = mpmath.exp(-za * zb / p * sum((a - b) ** 2 for a, b in zip(A, B)))
    Kcd = mpmath.exp(-zc * zd / q * sum((c - d) ** 2 for c, d in zip(C, D)))
    R = mpmath.sqrt(sum((x - y) ** 2 for x, y in zip(P, Q)))
    a = p * q / (p + q)
    if omega is not None:
        a = 1 / (1 / p + 1 / q + 1 / f(omega) ** 2)
    pre = Kab * Kcd * (mpmath.pi ** 2 / (p * q)) ** f(1.5)
    if R < f(1e-12):
        return float(pre * 2 * mpmath.sqrt(a / mpmath.pi))
    return float(pre * mpmath.erf(mpmath.sqrt(a) * R) / R)


def test_ss_closed_form(oracle_lib):
    """Unit-charge Gaussians interact as erf(sqrt(a) R)/R with a = pq/(p+q) (1/r) and
    1/a = 1/p + 1/q + 1/omega^2 (erf(omega r)/r): eqs eri_j and lreri_k for s functions."""
    rng = np.random.default_rng(11)
    z0 = np.zeros(12, dtype=np.int32)
    for _ in range(40):
        z = np.exp(rng.uniform(math.log(0.1), math.log(5000.0), 4))
        cen = rng.uniform(-2, 2, (4, 3))
        for op, om in ((0, None), (1, 0.3), (1, 2.5)):
            v = oracle_lib.prim_eri(z0, z, cen, op, om if om else 0.0)
            ref = _ss_closed(*z, *cen, omega=om)
            assert abs(v - ref) <= 1e-13 * abs(ref) + 1e-300, (op, v, ref)


def test_ss_derivative_closed_form(oracle_lib):
    """d/dR [erf(aR)/R] = 2a/sqrt(pi) exp(-a^2R^2)/R - erf(aR)/R^2 pins the 2 zeta factor,
    the sign and the eta scaling of the p-type (raised) integrals: for two unit-charge
    s Gaussians on the x axis, (p_x s|s s) = dI/dA_x / (2 za)."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        za, zc = np.exp(rng.uniform(math.log(0.2), math.log(50.0), 2))
        Ax, Cx = rng.uniform(-1, 1), rng.uniform(2, 4)
        A = np.array([Ax, 0.0, 0.0]); C = np.array([Cx, 0.0, 0.0])
        for om in (None, 0.3):
            a = za * zc / (za + zc) if om is None else 1.0 / (1 / za + 1 / zc + 1 / om ** 2)
            R = Cx - Ax
            s = math.sqrt(a)
            dIdR = 2 * s / math.sqrt(math.pi) * math.exp(-a * R * R) / R - math.erf(s * R) / R ** 2
            pre = (math.pi ** 2 / (za * zc)) ** 1.5
            dIdAx = -pre * dIdR                     # R = Cx - Ax
            lx = np.array([1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0], dtype=np.int32)
            v = oracle_lib.prim_eri(lx, [za, 1e-300, zc, 1e-300], np.stack([A, A, C, C]),
                                    0 if om is None else 1, om or 0.0)
            assert abs(v - dIdAx / (2 * za)) < 1e-12 * abs(dIdAx / (2 * za)), (v, dIdAx / (2 * za))


# ------------------------------------------------- higher l by autograd of (ss|ss)
def _hermite_expansion(n):
    """(x-A)^n g = sum_k coef_k a^(-(n+k)/2) d^k g/dA^k  for g = exp(-a (x-A)^2).
    From t^n = n!/2^n sum_m H_{n-2m}(t)/(m!(n-2m)!) and d^k g/dA^k = a^(k/2) H_k g."""
    out = []
    for m in range(n // 2 + 1):
        k = n - 2 * m
        c = math.factorial(n) / 2 ** n / (math.factorial(m) * math.factorial(k))
        out.append((k, c))
    return out


def _autograd_cart(lxyz, z, cen, omega=None):
    import torch
    X = torch.tensor(np.asarray(cen, dtype=np.float64).reshape(12), requires_grad=True)
    zt = [float(v) for v in z]

    def ss(Xv):
        A, B, Cc, D = Xv[0:3], Xv[3:6], Xv[6:9], Xv[9:12]
        p, q = zt[0] + zt[1], zt[2] + zt[3]
        P = (zt[0] * A + zt[1] * B) / p
        Q = (zt[2] * Cc + zt[3] * D) / q
        Kab = torch.exp(-zt[0] * zt[1] / p * torch.sum((A - B) ** 2))
        Kcd = torch.exp(-zt[2] * zt[3] / q * torch.sum((Cc - D) ** 2))
        R = torch.sqrt(torch.sum((P - Q) ** 2))
        a = p * q / (p + q) if omega is None else 1.0 / (1 / p + 1 / q + 1 / omega ** 2)
        return Kab * Kcd * (math.pi ** 2 / (p * q)) ** 1.5 * torch.erf(math.sqrt(a) * R) / R

    # operator: product over (centre, dir) of sum_k coef a^(-(n+k)/2) d^k/dX^k
    terms = [((), 1.0)]
    for c in range(4):
        for d in range(3):
            n = int(lxyz[c][d])
            if n == 0:
                continue
            new = []
            for (idx, w) in terms:
                for k, cf in _hermite_expansion(n):
                    new.append((idx + (3 * c + d,) * k, w * cf * zt[c] ** (-(n + k) / 2.0)))
            terms = new
    total = 0.0
    for idx, w in terms:
        f = ss(X)
        for v in idx:
            (g,) = torch.autograd.grad(f, X, create_graph=True)
            f = g[v]
        total += w * float(f)
    return total


@pytest.mark.parametrize("case", range(14))
def test_cartesian_integrals_vs_autograd(oracle_lib, case):
    """Obara-Saika/HGP integrals for Cartesian components up to f (the raised shells of the
    derivative) equal Hermite-derivative combinations of the closed-form (ss|ss), obtained
    by torch autograd (independent of the oracle's recursions)."""
    rng = np.random.default_rng(100 + case)
    comps = [
        [[1, 0, 0], [0, 0, 0], [0, 0, 0], [0, 0, 0]],
        [[0, 1, 0], [1, 0, 0], [0, 0, 0], [0, 0, 0]],
        [[0, 0, 0], [0, 0, 0], [0, 0, 1], [0, 1, 0]],
        [[2, 0, 0], [0, 0, 0], [0, 1, 0], [0, 0, 0]],
        [[1, 1, 0], [0, 0, 1], [1, 0, 0], [0, 0, 0]],
        [[0, 0, 2], [0, 1, 0], [0, 0, 1], [1, 0, 0]],
        [[3, 0, 0], [0, 0, 0], [0, 0, 0], [0, 0, 0]],
        [[1, 2, 0], [1, 0, 0], [0, 0, 0], [0, 1, 0]],
        [[0, 1, 1], [0, 1, 0], [1, 1, 0], [0, 0, 0]],
        [[1, 0, 0], [1, 0, 1], [0, 0, 0], [2, 0, 0]],
        [[0, 0, 1], [0, 0, 0], [2, 1, 0], [0, 0, 0]],
        [[1, 0, 1], [0, 2, 0], [0, 1, 0], [0, 0, 1]],
        [[2, 0, 0], [1, 0, 0], [0, 1, 1], [0, 0, 0]],
        [[0, 0, 0], [0, 1, 0], [0, 0, 0], [1, 1, 1]],
    ][case]
    z = np.exp(rng.uniform(math.log(0.3), math.log(3.0), 4))
    cen = rng.uniform(-1.2, 1.2, (4, 3))
    for op, om in ((0, None), (1, 0.3)):
        v = oracle_lib.prim_eri(np.array(comps, dtype=np.int32).reshape(12), z, cen, op,
                                om or 0.0)
        ref = _autograd_cart(comps, z, cen, om)
        assert abs(v - ref) <= 1e-10 * max(1.0, abs(ref)), (comps, op, v, ref)


# --------------------------------------------------------------- normalisation
def test_contraction_normalisation(oracle_lib, mol0):
    """x^l component self-overlap = 1 with the textbook Gaussian moment
    int x^(2l) exp(-s r^2) = (2l-1)!!/(2s)^l (pi/s)^(3/2)."""
    c = oracle_lib.norm_coefs(mol0)
    df = lambda n: float(np.prod(np.arange(n, 0, -2))) if n > 0 else 1.0
    for s in range(mol0.n_shells):
        o, k, l = mol0.shell_prim_off[s], mol0.shell_nprim[s], mol0.shell_l[s]
        z, cc = mol0.exps[o:o + k], c[o:o + k]
        S = 0.0
        for i in range(k):
            for j in range(k):
                ss = z[i] + z[j]
                S += cc[i] * cc[j] * df(2 * l - 1) / (2 * ss) ** l * (math.pi / ss) ** 1.5
        assert abs(S - 1.0) < 1e-13


def test_component_normalisation_via_far_charge(oracle_lib):
    """(mu mu|c c) R -> <mu|mu><c|c> = 1 for a tight s function c far away: every Cartesian
    component (angular factor included) is normalised to one."""
    Rf = 2000.0
    shells = [(0, 0, [3.0, 0.6], [0.4, 0.8]), (0, 1, [1.3, 0.4], [0.5, 0.6]),
              (0, 2, [0.8], [1.0]), (1, 0, [500.0], [1.0])]
    m = molecules.make([[0, 0, 0], [Rf, 0, 0]], shells)
    T = oracle_lib.eri_tensor(m, 0)
    n = m.n_bf
    for mu in range(n - 1):
        v = T[mu, mu, n - 1, n - 1] * Rf
        assert abs(v - 1.0) < 1e-6, (mu, v)


# ---------------------------------------------------------- long-range limits
def _overlap_1d(i, j, a, b, A, B):
    p = a + b
    P = (a * A + b * B) / p
    s = 0.0
    for k in range(i + 1):
        for l in range(j + 1):
            t = k + l
            if t % 2:
                continue
            mom = (float(np.prod(np.arange(t - 1, 0, -2))) if t > 1 else 1.0) / (2 * p) ** (t // 2)
            s += math.comb(i, k) * math.comb(j, l) * (P - A) ** (i - k) * (P - B) ** (j - l) * mom
    return s * math.sqrt(math.pi / p) * math.exp(-a * b / p * (A - B) ** 2)


def test_long_range_limits(oracle_lib):
    """omega -> infinity: (ab|cd)_lr -> (ab|cd); omega -> 0: (ab|cd)_lr ~ (2 omega/sqrt(pi)) S_ab S_cd."""
    rng = np.random.default_rng(9)
    for _ in range(12):
        comps = np.zeros((4, 3), dtype=np.int32)
        for c in range(4):                       # l <= 2 per function
            for _k in range(int(rng.integers(0, 3))):
                comps[c, int(rng.integers(0, 3))] += 1
        z = np.exp(rng.uniform(math.log(0.4), math.log(4.0), 4))
        cen = rng.uniform(-1, 1, (4, 3))
        full = oracle_lib.prim_eri(comps.reshape(12), z, cen, 0, 0.0)
        big = oracle_lib.prim_eri(comps.reshape(12), z, cen, 1, 1e7)
        assert abs(big - full) < 1e-9 * max(1.0, abs(full))
        om = 1e-4
        small = oracle_lib.prim_eri(comps.reshape(12), z, cen, 1, om)
        Sab = np.prod([_overlap_1d(comps[0][d], comps[1][d], z[0], z[1], cen[0][d], cen[1][d]) for d in range(3)])
        Scd = np.prod([_overlap_1d(comps[2][d], comps[3][d], z[2], z[3], cen[2][d], cen[3][d]) for d in range(3)])
        ref = 2 * om / math.sqrt(math.pi) * Sab * Scd
        assert abs(small - ref) < 1e-7 * max(abs(ref), 1e-4 * abs(Sab * Scd) * om), (small, ref)


# ------------------------------------------------------ gradient-level pins
def _fd_grad(oracle_lib, m, atoms, h=2e-3, **kw):
    fd = {}
    for a in atoms:
        for x in range(3):
            vals = []
            for hh in (h, h / 2):
                cp = m.coords.copy(); cp[a, x] += hh
                cm = m.coords.copy(); cm[a, x] -= hh
                vals.append((oracle_lib.energy(m, coords=cp, **kw) - oracle_lib.energy(m, coords=cm, **kw)) / (2 * hh))
            fd[(a, x)] = (4 * vals[1] - vals[0]) / 3
    return fd


@pytest.mark.parametrize("terms", [1, 2, 4, 7])
def test_gradient_vs_finite_difference_small(oracle_lib, terms):
    """Analytic gradient = central FD (Richardson) of the pseudo-energy with fixed densities
    (the paper's own validation method), per term of Gamma."""
    m = molecules.small_mixed()
    g = oracle_lib.grad(m, terms=terms)
    fd = _fd_grad(oracle_lib, m, range(m.n_atoms), terms=terms)
    for (a, x), v in fd.items():
        assert abs(v - g[a, x]) < 1e-8 * max(1.0, abs(g[a, x])), (terms, a, x, v, g[a, x])


def test_gradient_vs_finite_difference_config0(oracle_lib, mol0):
    g = oracle_lib.grad(mol0)
    fd = _fd_grad(oracle_lib, mol0, [0, 3], h=1e-3)
    for (a, x), v in fd.items():
        assert abs(v - g[a, x]) < 2e-8, (a, x, v, g[a, x])


def test_translational_invariance(oracle_lib, mol0):
    """sum_A dE/dA = 0: the oracle forms all four centre derivatives explicitly."""
    g = oracle_lib.grad(mol0)
    assert np.abs(g.sum(axis=0)).max() < 1e-9
    m = molecules.small_mixed()
    g = oracle_lib.grad(m)
    assert np.abs(g.sum(axis=0)).max() < 1e-12 * max(1.0, np.abs(g).max())


def test_brute_vs_fast(oracle_lib, mol0):
    """Every ordered quartet with the literal Gamma of eq gamma = unique quartets with the
    permutation-averaged Gamma and degeneracy weights."""
    g = oracle_lib.grad(mol0)
    gb = oracle_lib.grad_brute(mol0)
    assert np.abs(g - gb).max() < 1e-9
    m = molecules.small_mixed()
    for terms in (1, 2, 4):
        assert np.abs(oracle_lib.grad(m, terms=terms) - oracle_lib.grad_brute(m, terms=terms)).max() < 1e-11


def test_rotation_covariance(oracle_lib):
    """Rotating the molecule (densities in the Cartesian-component basis transformed only for
    s functions -- use an s-only basis) rotates the gradient."""
    rng = np.random.default_rng(4)
    coords = rng.uniform(-2, 2, (4, 3))
    shells = [(a, 0, [2.0, 0.5], [0.5, 0.6]) for a in range(4)] + [(a, 0, [0.3], [1.0]) for a in range(4)]
    m = molecules.make(coords, shells)
    g = oracle_lib.grad(m)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    m2 = molecules.make(coords @ Q.T, shells, dens=(m.P0, m.PD, m.R))
    g2 = oracle_lib.grad(m2)
    assert np.abs(g2 - g @ Q.T).max() < 1e-11


# ------------------------------------------------ Gamma against the MO forms
def _mo_molecule(seed=21):
    m = molecules.small_mixed(seed)
    n = m.n_bf
    rng = np.random.default_rng(seed)
    Cm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    no = 4
    Co, Cv = Cm[:, :no], Cm[:, no:]
    X = rng.standard_normal((no, n - no))
    X /= np.linalg.norm(X)
    return m, Co, Cv, X


def test_gamma_transition_and_ground_state_vs_mo_form(oracle_lib):
    """With P0 = 2 C_o C_o^T, PDelta = 0, R = C_o X C_v^T the pseudo-energy equals
      2 sum_ij (ii|jj) - sum_ij [alpha (ij|ij) + beta (ij|ij)_lr]              (closed-shell RSH)
      + sum_{ia,jb} X_ia X_jb [2(ia|jb) - alpha (ij|ab) - beta (ij|ab)_lr]     (eq dE_mo)
    evaluated from the AO integral tensors by MO transformation."""
    m, Co, Cv, X = _mo_molecule()
    n = m.n_bf
    P0 = 2 * Co @ Co.T
    R = Co @ X @ Cv.T
    Z = np.zeros((n, n))
    I = oracle_lib.eri_tensor(m, 0)
    Il = oracle_lib.eri_tensor(m, 1)
    a, b = m.alpha, m.beta

    def mo(T, C1, C2, C3, C4):
        return np.einsum("pqrs,pi,qj,rk,sl->ijkl", T, C1, C2, C3, C4, optimize=True)

    oo = mo(I, Co, Co, Co, Co); ool = mo(Il, Co, Co, Co, Co)
    e_gs = 2 * np.einsum("iijj->", oo) - a * np.einsum("ijij->", oo) - b * np.einsum("ijij->", ool)
    ovov = mo(I, Co, Cv, Co, Cv)
    oovv = mo(I, Co, Co, Cv, Cv); oovvl = mo(Il, Co, Co, Cv, Cv)
    e_x = (2 * np.einsum("ia,jb,iajb->", X, X, ovov) - a * np.einsum("ia,jb,ijab->", X, X, oovv)
           - b * np.einsum("ia,jb,ijab->", X, X, oovvl))
    e = oracle_lib.energy(m, P0=P0, PD=Z, R=R)
    assert abs(e - (e_gs + e_x)) < 1e-11 * max(1.0, abs(e)), (e, e_gs + e_x)
    # each part separately
    assert abs(oracle_lib.energy(m, P0=P0, PD=Z, R=Z) - e_gs) < 1e-11 * max(1.0, abs(e_gs))
    assert abs(oracle_lib.energy(m, P0=Z, PD=Z, R=R) - e_x) < 1e-12 * max(1.0, abs(e_x))


def test_gamma_relaxed_density_vs_fock_form(oracle_lib):
    """The PDelta part of the pseudo-energy is PDelta contracted with the two-electron part of
    the closed-shell RSH Fock matrix of P0:
      sum_{mu nu} PD_{mu nu} sum_{lam sig} P0_{lam sig} [(mu nu|lam sig)
                    - alpha/2 (mu sig|lam nu) - beta/2 (mu sig|lam nu)_lr]."""
    m, Co, Cv, X = _mo_molecule(22)
    n = m.n_bf
    P0 = 2 * Co @ Co.T
    rng = np.random.default_rng(1)
    S = rng.standard_normal((n, n)); PD = 0.1 * (S + S.T)
    Z = np.zeros((n, n))
    I = oracle_lib.eri_tensor(m, 0)
    Il = oracle_lib.eri_tensor(m, 1)
    F2 = (np.einsum("mnls,ls->mn", I, P0) - m.alpha / 2 * np.einsum("msln,ls->mn", I, P0)
          - m.beta / 2 * np.einsum("msln,ls->mn", Il, P0))
    ref = np.sum(PD * F2)
    e = oracle_lib.energy(m, P0=P0, PD=PD, R=Z) - oracle_lib.energy(m, P0=P0, PD=Z, R=Z)
    assert abs(e - ref) < 1e-11 * max(1.0, abs(ref)), (e, ref)


def test_coulomb_two_centre_s_only(oracle_lib):
    """alpha = beta = 0, R = 0, PDelta = 0: textbook Coulomb gradient 1/2 sum P P d(..|..);
    two s-only atoms -> equal and opposite forces along the bond axis, and for single primitives
    the closed form d/dR of the s-type integrals."""
    A = np.array([0.0, 0.0, 0.0]); B = np.array([0.7, -1.1, 1.6])
    za, zb = 0.9, 0.35
    m = molecules.make([A, B], [(0, 0, [za], [1.0]), (1, 0, [zb], [1.0])],
                       dens=(np.array([[1.0, 0.0], [0.0, 1.0]]), np.zeros((2, 2)), np.zeros((2, 2))))
    g = oracle_lib.grad(m, terms=1)
    u = (B - A) / np.linalg.norm(B - A)
    assert np.abs(g[0] + g[1]).max() < 1e-14
    assert np.linalg.norm(np.cross(g[1], u)) < 1e-14
    # E = 1/2 [(aa|aa) + (bb|bb) + 2 (aa|bb)]; only (aa|bb) depends on R: dE/dR = d(aa|bb)/dR
    Rr = np.linalg.norm(B - A)
    a = 1.0 / (1 / (2 * za) + 1 / (2 * zb))
    s = math.sqrt(a)
    dIdR = 2 * s / math.sqrt(math.pi) * math.exp(-a * Rr * Rr) / Rr - math.erf(s * Rr) / Rr ** 2
    assert abs(g[1] @ u - dIdR) < 1e-13
