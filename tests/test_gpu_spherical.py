"""Spherical d functions (tdg_basis_t.spherical = 1) on the GPU against the oracle: the
gradient (FP64 and mixed) and the Fock-type matrix, whose densities and matrices count five
functions per d shell.  The library transforms them to its Cartesian functions on entry
(and the Fock-type matrix back on exit); the oracle does the same with its own transform,
pinned by orthonormality."""
import numpy as np
import pytest

from paper_2407_16586_amd import synth
from tests import molecules

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tdg():
    from paper_2407_16586_amd import tdgrad
    tdgrad.lib()
    return tdgrad


def _say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("case", ["small_mixed", "config0"])
def test_spherical_gradient(tdg, oracle_lib, case):
    base = molecules.small_mixed() if case == "small_mixed" else synth.config0()
    m = synth.spherical_copy(base, seed=5)
    _say(case, "spherical: n_bf", m.n_bf, "of", base.n_bf, "Cartesian")
    for tau in (0.0, 1e-10):
        ref = oracle_lib.grad(m, tau=tau)
        p = tdg.Plan(m, schwarz_tol=tau)
        assert p.n_bf == m.n_bf
        g = p.grad(m.P0, m.PD, m.R)
        err = np.abs(g - ref).max()
        _say(f"  tau {tau}: FP64 max abs error {err:.2e}")
        assert err <= 1e-9 * max(1.0, np.abs(ref).max())
    pm = tdg.Plan(m, schwarz_tol=1e-10, precision=1)
    gm = pm.grad(m.P0, m.PD, m.R)
    err = np.abs(gm - oracle_lib.grad(m, tau=1e-10)).max()
    _say(f"  mixed: max abs error {err:.2e}")
    assert err <= 1e-6


def test_spherical_fock(tdg, oracle_lib):
    m = synth.spherical_copy(molecules.small_mixed(), seed=6)
    rng = np.random.default_rng(16)
    B = rng.standard_normal((m.n_bf, m.n_bf))
    p = tdg.Plan(m, schwarz_tol=0.0)
    for cf in ((2.0, -m.alpha, -m.beta), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)):
        ref = oracle_lib.fock(m, B, *cf)
        F = p.fock(B, *cf)
        assert F.shape == ref.shape
        e = np.abs(F - ref).max() / np.abs(ref).max()
        _say("spherical Fock", cf, "rel err", e)
        assert e <= 1e-10


def test_spherical_batch_noalloc_and_update_coords(tdg, oracle_lib):
    """The other entry points share the transform: a batch of a spherical and a Cartesian
    molecule equals single calls; the allocation-free call and a geometry update of a
    spherical plan equal the oracle."""
    import torch
    ms = synth.spherical_copy(molecules.small_mixed(), seed=8)
    mc = synth.config0()
    ps, pc = tdg.Plan(ms, schwarz_tol=1e-12), tdg.Plan(mc, schwarz_tol=1e-12)
    gb = tdg.grad_batch([ps, pc], [(ms.P0, ms.PD, ms.R), (mc.P0, mc.PD, mc.R)])
    for g, p, m in zip(gb, (ps, pc), (ms, mc)):
        assert np.abs(g - p.grad(m.P0, m.PD, m.R)).max() <= 1e-12 * max(1.0, np.abs(g).max())
    dev = torch.device("cuda:0")
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    out = torch.zeros((ms.n_atoms, 3), dtype=torch.float64, device=dev)
    ps.grad_device_noalloc(t(ms.P0), t(ms.PD), t(ms.R), out)
    torch.cuda.synchronize()
    ref = oracle_lib.grad(ms, tau=1e-12)
    assert np.abs(out.cpu().numpy() - ref).max() <= 1e-9 * max(1.0, np.abs(ref).max())
    x1 = ms.coords + np.random.default_rng(3).uniform(-0.2, 0.2, ms.coords.shape)
    ps.update_coords(x1)
    g1 = ps.grad(ms.P0, ms.PD, ms.R)
    ref1 = oracle_lib.grad(ms, tau=1e-12, coords=x1)
    _say("spherical after update_coords: max abs error", np.abs(g1 - ref1).max())
    assert np.abs(g1 - ref1).max() <= 1e-9 * max(1.0, np.abs(ref1).max())
