"""The Krylov Z-vector solve on the GPU (tdg_zvector: section II.B, eqs cphf, cphf_a,
sigma, zfock, without the exchange-correlation kernel) against the oracle's direct dense
solve of eq cphf with A written from its molecular-orbital definition.  Orbitals are seeded
orthonormal columns, energies seeded with an occupied-virtual gap, L seeded."""
import numpy as np
import pytest

from tests import molecules

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tdg():
    from paper_2407_16586_amd import tdgrad
    tdgrad.lib()
    return tdgrad


def _case(m, n_occ, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((m.n_bf, m.n_bf)))
    eo = np.sort(rng.uniform(-1.2, -0.3, n_occ))
    ev = np.sort(rng.uniform(0.2, 2.0, m.n_bf - n_occ))
    L = rng.standard_normal((m.n_bf - n_occ, n_occ))
    return Q[:, :n_occ], Q[:, n_occ:], eo, ev, L


@pytest.mark.parametrize("case", ["small_mixed", "config0", "config0_spherical"])
def test_zvector_against_direct_solve(tdg, oracle_lib, case):
    from paper_2407_16586_amd import synth
    if case == "small_mixed":
        m, no = molecules.small_mixed(), 4
    elif case == "config0":
        m, no = synth.config0(), 8
    else:
        m, no = synth.spherical_copy(synth.config0(), seed=9), 8
    Co, Cv, eo, ev, L = _case(m, no, 11)
    ref = oracle_lib.zvector(m, Co, Cv, eo, ev, L)
    for tau, relative, tol in ((0.0, False, 1e-8), (1e-12, True, 1e-7)):
        p = tdg.Plan(m, schwarz_tol=tau)
        Z, it, res = p.zvector(Co, Cv, eo, ev, L, relative=relative, tol=1e-11, max_iter=60)
        err = np.abs(Z - ref).max() / np.abs(ref).max()
        print(f"{case} tau {tau} relative {relative}: {it} products, residual {res:.1e}, rel err {err:.2e}",
              flush=True)
        assert err <= tol
        p.close()


def test_zvector_arguments(tdg):
    m = molecules.small_mixed()
    Co, Cv, eo, ev, L = _case(m, 4, 12)
    p = tdg.Plan(m, schwarz_tol=0.0)
    with pytest.raises(tdg.TdgError):
        p.zvector(Co, Cv, eo[::-1] + 3.0, ev, L)   # occupied energies above the virtual ones
