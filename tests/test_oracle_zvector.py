"""Pins of the oracle's Z-vector pieces (section II.B, eqs cphf, cphf_a, sigma, zfock; no
exchange-correlation kernel):

- A of eq cphf_a, written from its molecular-orbital definition, is symmetric;
- its product with a vector b equals the AO route of eqs sigma and zfock,
  C_v^T F(C_v b C_o^T) C_o with F the oracle's Fock-type matrix of coefficients
  (4, -2 alpha, -2 beta) -- two independent constructions, so an index slip in either
  (or in the reading that eq zfock's two exchange orderings sum to 2 K(Bs)) fails it;
- the direct solve satisfies eq cphf."""
import numpy as np

from tests import molecules


def _orbitals(m, n_occ, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((m.n_bf, m.n_bf)))
    eo = np.sort(rng.uniform(-1.2, -0.3, n_occ))
    ev = np.sort(rng.uniform(0.2, 2.0, m.n_bf - n_occ))
    return Q[:, :n_occ], Q[:, n_occ:], eo, ev


def test_cphf_matrix_symmetric_and_matches_fock_route(oracle_lib):
    m = molecules.small_mixed()
    Co, Cv, eo, ev = _orbitals(m, 4, 1)
    A = oracle_lib.cphf_matrix(m, Co, Cv)
    assert np.abs(A - A.T).max() <= 1e-12 * np.abs(A).max()
    rng = np.random.default_rng(2)
    b = rng.standard_normal((Cv.shape[1], Co.shape[1]))
    F = oracle_lib.fock(m, Cv @ b @ Co.T, 4.0, -2 * m.alpha, -2 * m.beta)
    sigma = Cv.T @ F @ Co
    ref = (A @ b.reshape(-1)).reshape(b.shape)
    assert np.abs(sigma - ref).max() <= 1e-11 * np.abs(ref).max()


def test_direct_solve_satisfies_equation(oracle_lib):
    m = molecules.small_mixed()
    Co, Cv, eo, ev = _orbitals(m, 4, 3)
    L = np.random.default_rng(4).standard_normal((Cv.shape[1], Co.shape[1]))
    Z = oracle_lib.zvector(m, Co, Cv, eo, ev, L)
    A = oracle_lib.cphf_matrix(m, Co, Cv)
    d = (eo[None, :] - ev[:, None]).reshape(-1)
    lhs = d * Z.reshape(-1) - A @ Z.reshape(-1)
    assert np.abs(lhs - L.reshape(-1)).max() <= 1e-10 * np.abs(L).max()
