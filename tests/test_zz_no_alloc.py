"""The allocation-free entry point (tdg_grad_jk_noalloc) against tdg_grad_jk on the same
plans and device densities: two calls in a row, the second on a smaller molecule, then a
third on the first molecule again (its task list overwrites the shared static buffer)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_noalloc_matches_grad_jk():
    import torch
    from paper_2407_16586_amd import synth, tdgrad
    tdgrad.lib()
    dev = torch.device("cuda:0")
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    cases = []
    for mol, prec in ((synth.config1(), 0), (synth.config0(), 1), (synth.config1(), 1)):
        print("no-alloc:", mol.name, "precision", prec, flush=True)
        plan = tdgrad.Plan(mol, schwarz_tol=1e-10, precision=prec)
        P0, PD, R = t(mol.P0), t(mol.PD), t(mol.R)
        ref = torch.zeros((mol.n_atoms, 3), dtype=torch.float64, device=dev)
        st_ref = plan.grad_device(P0, PD, R, ref, stats=True)   # also tunes the plan's variants
        plan.grad_device(P0, PD, R, ref)
        out = torch.full((mol.n_atoms, 3), 7.0, dtype=torch.float64, device=dev)
        st = plan.grad_device_noalloc(P0, PD, R, out, stats=True)
        torch.cuda.synchronize()
        g, r = out.cpu().numpy(), ref.cpu().numpy()
        err = np.abs(g - r).max()
        print("  quartets", st["quartets"], st_ref["quartets"], "max |noalloc - grad_jk|", err, flush=True)
        assert st["quartets"] == st_ref["quartets"]
        # the same kernels on the same tasks; only the order of the atomic additions differs
        assert err <= 1e-12 * max(1.0, np.abs(r).max())
        cases.append(plan)
    # a chunked call (task lists of at most 100,000 quartets through the static buffer)
    mol = synth.config1()
    plan = tdgrad.Plan(mol, schwarz_tol=1e-10, max_tasks=100_000)
    P0, PD, R = t(mol.P0), t(mol.PD), t(mol.R)
    ref = torch.zeros((mol.n_atoms, 3), dtype=torch.float64, device=dev)
    plan.grad_device(P0, PD, R, ref)
    out = torch.zeros_like(ref)
    st = plan.grad_device_noalloc(P0, PD, R, out, stats=True)
    torch.cuda.synchronize()
    err = np.abs(out.cpu().numpy() - ref.cpu().numpy()).max()
    print("  chunked: chunks", st["chunks"], "max |noalloc - grad_jk|", err, flush=True)
    assert st["chunks"] > 1 and err <= 1e-12 * max(1.0, np.abs(ref.cpu().numpy()).max())
    # plans the call does not serve
    det = tdgrad.Plan(synth.config0(), deterministic=True)
    m0 = synth.config0()
    o = torch.zeros((m0.n_atoms, 3), dtype=torch.float64, device=dev)
    with pytest.raises(tdgrad.TdgError) as e:
        det.grad_device_noalloc(t(m0.P0), t(m0.PD), t(m0.R), o)
    assert e.value.status == tdgrad.TDG_EUNSUPPORTED
