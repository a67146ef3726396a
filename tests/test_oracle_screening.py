"""Pins of the oracle's screening (section II.E: density-multiplied Schwarz bound), checked
against what the mathematics fixes rather than against the oracle itself:

- Q_ab is the Cauchy-Schwarz factor of the ERI tensor: the largest diagonal element of
  each shell-pair block of the full integral tensor (brute force, config 0), and every
  integral is bounded by Q_ab Q_cd;
- the density factor M_abcd = bound / (Q_ab Q_cd) bounds the two-particle densities the
  quartet is contracted with: with Gamma^sym built here from the paper's literal Gamma
  (eq gamma) averaged over the 8 index permutations, every component satisfies
  |Gamma^sym| + |Gamma^lr,sym| <= (2 + alpha + beta + 1/2 + (alpha + beta)/4) M_abcd.
  A bound that drops an index pairing or one orientation of the non-symmetric R fails it;
- the screened gradient differs from the unscreened one exactly by the skipped quartets'
  contributions, and those stay within a stated multiple of the threshold.
"""
import numpy as np
import pytest

from tests import molecules


@pytest.fixture(scope="module")
def eri0(oracle_lib, mol0):
    return oracle_lib.eri_tensor(mol0)


def _shell_slices(mol):
    return [slice(int(o), int(o) + (int(l) + 1) * (int(l) + 2) // 2)
            for o, l in zip(mol.shell_ao_off, mol.shell_l)]


def _pidx(a, b):
    a, b = max(a, b), min(a, b)
    return a * (a + 1) // 2 + b


def test_schwarz_factor_is_cauchy_schwarz(oracle_lib, mol0, eri0):
    T = eri0
    sl = _shell_slices(mol0)
    ns = mol0.n_shells
    Q = oracle_lib.schwarz(mol0)
    diag = np.einsum("mnmn->mn", T)
    Qb = np.zeros(ns * (ns + 1) // 2)
    for a in range(ns):
        for b in range(a + 1):
            Qb[_pidx(a, b)] = np.sqrt(diag[sl[a], sl[b]].max())
    assert np.abs(Q - Qb).max() <= 1e-12 * Qb.max()
    # |(mu nu|lam sig)| <= Q_ab Q_cd for every component (positive-definite kernel)
    Qm = np.zeros((ns, ns))
    for a in range(ns):
        for b in range(ns):
            Qm[a, b] = Q[_pidx(a, b)]
    Qao = np.zeros((mol0.n_bf, mol0.n_bf))
    for a in range(ns):
        for b in range(ns):
            Qao[sl[a], sl[b]] = Qm[a, b]
    assert np.all(np.abs(T) <= np.multiply.outer(Qao, Qao) * (1 + 1e-12) + 1e-300)


def _gamma_sym_abs(mol):
    """|Gamma^sym| + |Gamma^lr,sym| for every AO quadruple: the literal Gamma of eq gamma
    (P read as P0, D = P0 + 2 PDelta) averaged over the 8 permutations that leave
    (mu nu|lam sig) unchanged."""
    P, D, R = mol.P0, mol.P0 + 2.0 * mol.PD, mol.R
    al, be = mol.alpha, mol.beta
    G = (2.0 * np.einsum("nm,ls->mnls", R, R) - al * np.einsum("sm,ln->mnls", R, R)
         + 0.5 * (np.einsum("mn,ls->mnls", D, P) - 0.5 * al * np.einsum("ms,ln->mnls", D, P)))
    Gl = -be * np.einsum("sm,ln->mnls", R, R) - 0.25 * be * np.einsum("ms,ln->mnls", D, P)
    perms = [(0, 1, 2, 3), (1, 0, 2, 3), (0, 1, 3, 2), (1, 0, 3, 2),
             (2, 3, 0, 1), (3, 2, 0, 1), (2, 3, 1, 0), (3, 2, 1, 0)]
    sym = lambda X: sum(X.transpose(p) for p in perms) / 8.0
    return np.abs(sym(G)) + np.abs(sym(Gl))


def _sparse_densities(mol, seed, nblk=6):
    """P0, PDelta (symmetric) and R (not symmetric) that are zero outside a few random shell
    blocks, so that each quartet's Gamma comes from few index pairings: a bound that misses
    a pairing (or one orientation of R) then meets a nonzero Gamma with M = 0."""
    rng = np.random.default_rng(seed)
    sl = _shell_slices(mol)
    n, ns = mol.n_bf, mol.n_shells

    def blocks():
        X = np.zeros((n, n))
        for _ in range(nblk):
            a, b = rng.integers(0, ns, 2)
            X[sl[a], sl[b]] = rng.standard_normal(X[sl[a], sl[b]].shape)
        return X
    S = blocks()
    P0 = S + S.T
    S = blocks()
    return P0, 0.1 * (S + S.T), blocks()


@pytest.mark.parametrize("dens", ["stated"] + [f"sparse{k}" for k in range(6)])
def test_density_factor_bounds_gamma(oracle_lib, mol0, dens):
    import copy
    mol = copy.copy(mol0)
    if dens != "stated":
        mol.P0, mol.PD, mol.R = _sparse_densities(mol0, int(dens[6:]))
    ns = mol.n_shells
    sl = _shell_slices(mol)
    Gabs = _gamma_sym_abs(mol)
    # shell-block maxima of |Gamma^sym| + |Gamma^lr,sym|
    off = np.asarray(mol.shell_ao_off, dtype=np.int64)
    B = Gabs
    for ax in range(4):
        B = np.maximum.reduceat(B, off, axis=ax)
    quart = np.array([(a, b, c, d) for a in range(ns) for b in range(a + 1)
                      for c in range(a + 1) for d in range(c + 1)
                      if _pidx(a, b) >= _pidx(c, d)], dtype=np.int32)
    bound = oracle_lib.quartet_bounds(mol, quart)
    Q = oracle_lib.schwarz(mol)
    qq = np.array([Q[_pidx(a, b)] * Q[_pidx(c, d)] for a, b, c, d in quart])
    ok = qq > 1e-200
    M = bound[ok] / qq[ok]
    blk = B[tuple(quart[ok].T)]
    al_be = mol.alpha + mol.beta
    C = 2.0 + al_be + 0.5 + 0.25 * al_be
    # every quartet with a nonzero Gamma has a nonzero density factor, within C of it
    assert np.all(M[blk > 0] > 0)
    ratio = blk[M > 0] / M[M > 0]
    assert ratio.max() <= C * (1 + 1e-12), ratio.max()
    # the bound is not loose by orders of magnitude either: some quartet comes within 10x
    assert ratio.max() >= C / 10.0
    assert len(sl) == ns


@pytest.mark.parametrize("case,tau,dg_max,mult", [("config0", 1e-10, 2e-8, 200.0),
                                                 ("small_mixed", 1e-4, 1e-3, 20.0)])
def test_screened_gradient_error(oracle_lib, mol0, case, tau, dg_max, mult):
    mol = mol0 if case == "config0" else molecules.small_mixed()
    g0 = oracle_lib.grad(mol)
    gt, st = oracle_lib.grad(mol, tau=tau, return_stats=True)
    skip, sb = oracle_lib.screen_select(mol, tau, keep=False)
    keep, kb = oracle_lib.screen_select(mol, tau, keep=True)
    assert len(skip) == st["skipped"] and len(keep) == st["quartets"]
    assert np.all(sb < tau) and np.all(kb >= tau)
    c = oracle_lib.quartet_contribs(mol, skip)
    # the screened gradient misses exactly the skipped quartets' contributions
    miss = np.zeros_like(g0)
    for k, q in enumerate(skip):
        for x in range(4):
            miss[mol.shell_atom[q[x]]] += c[k, x]
    assert np.abs((g0 - gt) - miss).max() <= 1e-13
    # and they are small: within mult * tau per component, within dg_max per atom
    assert np.abs(c).max() <= mult * tau
    assert np.abs(g0 - gt).max() <= dg_max
