"""The rest of the C-ABI boundary on the GPU: geometry updates, the deterministic reduction,
the screening switch, the exact survivor set of the screening (section II.E) and
per-quartet contributions against the oracle at full system size."""
import numpy as np
import pytest

from tests import molecules

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tdg():
    from paper_2407_16586_amd import tdgrad
    tdgrad.lib()
    return tdgrad


def _say(*a):
    print(*a, flush=True)


def _key(q, ns):
    """Order-free key of unique shell quartets [n, 4] (pairs and pair order canonicalised)."""
    q = np.asarray(q, dtype=np.int64)
    a, b = np.maximum(q[:, 0], q[:, 1]), np.minimum(q[:, 0], q[:, 1])
    c, d = np.maximum(q[:, 2], q[:, 3]), np.minimum(q[:, 2], q[:, 3])
    p1, p2 = a * (a + 1) // 2 + b, c * (c + 1) // 2 + d
    npair = ns * (ns + 1) // 2
    return np.maximum(p1, p2) * npair + np.minimum(p1, p2)


# ------------------------------------------------------------------ geometry updates
def test_update_coords_matches_fresh_plan(tdg, oracle_lib, mol0):
    _say("update_coords: config0 moved to a second geometry")
    p = tdg.Plan(mol0, schwarz_tol=0.0)
    g_a = p.grad(mol0.P0, mol0.PD, mol0.R)
    rng = np.random.default_rng(7)
    x1 = mol0.coords + rng.uniform(-0.3, 0.3, mol0.coords.shape)
    p.update_coords(x1)
    g_b = p.grad(mol0.P0, mol0.PD, mol0.R)
    fresh = tdg.Plan(mol0, schwarz_tol=0.0)
    fresh.update_coords(x1)
    ref = oracle_lib.grad(mol0, coords=x1)
    _say("  moved vs oracle", np.abs(g_b - ref).max(), "moved vs first geometry", np.abs(g_b - g_a).max())
    assert np.abs(g_b - ref).max() <= 1e-8
    assert np.abs(g_b - fresh.grad(mol0.P0, mol0.PD, mol0.R)).max() <= 1e-12
    assert np.abs(g_b - g_a).max() > 1e-3
    p.update_coords(mol0.coords)   # and back
    assert np.abs(p.grad(mol0.P0, mol0.PD, mol0.R) - g_a).max() <= 1e-12
    with pytest.raises(tdg.TdgError):
        p.update_coords(np.full_like(x1, np.nan))
    assert np.abs(p.grad(mol0.P0, mol0.PD, mol0.R) - g_a).max() <= 1e-12  # unchanged on error


def test_update_coords_finite_difference(tdg, oracle_lib):
    """The GPU gradient at displaced geometries reached through update_coords equals central
    differences (Richardson) of the oracle's pseudo-energy at those geometries."""
    m = molecules.small_mixed()
    p = tdg.Plan(m, schwarz_tol=0.0)
    rng = np.random.default_rng(11)
    for trial in range(2):
        x = m.coords + rng.uniform(-0.2, 0.2, m.coords.shape)
        p.update_coords(x)
        g = p.grad(m.P0, m.PD, m.R)
        for a, k in ((trial, 0), (trial + 1, 2), (3, 1)):
            vals = []
            for h in (2e-3, 1e-3):
                xp = x.copy(); xp[a, k] += h
                xm = x.copy(); xm[a, k] -= h
                vals.append((oracle_lib.energy(m, coords=xp) - oracle_lib.energy(m, coords=xm)) / (2 * h))
            fd = (4 * vals[1] - vals[0]) / 3
            _say("  fd", trial, a, k, g[a, k], fd, abs(g[a, k] - fd))
            assert abs(g[a, k] - fd) <= 1e-8 * max(1.0, abs(fd))


# ------------------------------------------------------------------ deterministic mode
@pytest.mark.parametrize("precision", [0, 1])
def test_deterministic_repeatable(tdg, precision):
    from paper_2407_16586_amd import synth
    m = synth.config1()
    _say("deterministic: 60-atom chain, precision", precision)
    kw = dict(schwarz_tol=1e-10, precision=precision)
    p = tdg.Plan(m, deterministic=True, **kw)
    g1, st = p.grad(m.P0, m.PD, m.R, stats=True)
    g2 = p.grad(m.P0, m.PD, m.R)
    g3 = tdg.Plan(m, deterministic=True, **kw).grad(m.P0, m.PD, m.R)
    ga = tdg.Plan(m, autotune=False, **kw).grad(m.P0, m.PD, m.R)
    _say("  quartets", st["quartets"], "vs atomics", np.abs(g1 - ga).max())
    assert np.array_equal(g1, g2) and np.array_equal(g1, g3)
    assert np.abs(g1 - ga).max() <= 1e-13 * max(1.0, np.abs(ga).max())
    # chunked deterministic calls keep the same per-atom order within each chunk
    g4 = tdg.Plan(m, deterministic=True, max_tasks=1_000_000, **kw).grad(m.P0, m.PD, m.R)
    g5 = tdg.Plan(m, deterministic=True, max_tasks=1_000_000, **kw).grad(m.P0, m.PD, m.R)
    assert np.array_equal(g4, g5) and np.abs(g4 - g1).max() <= 1e-13 * max(1.0, np.abs(ga).max())


def test_deterministic_batch_matches_single(tdg):
    from paper_2407_16586_amd import synth
    mols = [synth.droplet(n, 20240716 + 500 + n) for n in (12, 20)]
    plans = [tdg.Plan(m, deterministic=True) for m in mols]
    outs = tdg.grad_batch(plans, [(m.P0, m.PD, m.R) for m in mols])
    for m, o in zip(mols, outs):
        assert np.array_equal(o, tdg.Plan(m, deterministic=True).grad(m.P0, m.PD, m.R))


def test_screening_switch(tdg, mol0):
    p = tdg.Plan(mol0, screening=1)
    with pytest.raises(tdg.TdgError) as e:
        p.grad(mol0.P0, mol0.PD, mol0.R)
    assert e.value.status == tdg.TDG_ESTATE
    with pytest.raises(tdg.TdgError):
        tdg.Plan(mol0, screening=2)
    q = tdg.Plan(mol0)                        # an attached estimator is ignored with screening=0
    est = tdg.Estimator(seed=1)
    g0, s0 = q.grad(mol0.P0, mol0.PD, mol0.R, stats=True)
    q.set_screen_model(est, 1e30, np.inf)     # would veto everything
    g1, s1 = q.grad(mol0.P0, mol0.PD, mol0.R, stats=True)
    assert s1["ml_skipped"] == 0 and s1["quartets"] == s0["quartets"]
    assert np.abs(g1 - g0).max() <= 1e-12


# ------------------------------------------------------------------ exact survivor set
TAU = 1e-10
BAND = 1e-9   # relative band around tau where FP64 (GPU) and extended-precision (oracle) bounds may disagree


@pytest.mark.parametrize("case", ["config0", "small_mixed", "chain60"])
def test_survivor_set_exact(tdg, oracle_lib, mol0, case):
    from paper_2407_16586_amd import synth
    m = {"config0": lambda: mol0, "small_mixed": lambda: molecules.small_mixed(),
         "chain60": synth.config1}[case]()
    tau = TAU if case != "small_mixed" else 1e-4
    _say("survivor set", case, "tau", tau)
    gq, n = tdg.Plan(m, schwarz_tol=tau).screen_list(m.P0, m.PD, m.R)
    assert len(gq) == n
    oq, ob = oracle_lib.screen_select(m, tau, keep=True)
    gk, ok = _key(gq, m.n_shells), _key(oq, m.n_shells)
    assert len(np.unique(gk)) == len(gk)          # no quartet twice
    only_gpu = np.setdiff1d(gk, ok)
    only_orc = np.setdiff1d(ok, gk)
    _say("  gpu", len(gk), "oracle", len(ok), "gpu only", len(only_gpu), "oracle only", len(only_orc))
    # a difference is allowed only where the oracle's bound sits within the rounding band of tau
    if len(only_orc):
        b = ob[np.isin(ok, only_orc)]
        assert np.all(np.abs(b / tau - 1.0) <= BAND), b
    if len(only_gpu):
        q = gq[np.isin(gk, only_gpu)]
        b = oracle_lib.quartet_bounds(m, q)
        assert np.all(np.abs(b / tau - 1.0) <= BAND), b
    assert len(only_gpu) + len(only_orc) <= max(2, len(ok) // 10**6)
    # the library's orientation: l_a >= l_b, l_c >= l_d, pair class of ab >= cd
    l = m.shell_l[gq]
    assert np.all(l[:, 0] >= l[:, 1]) and np.all(l[:, 2] >= l[:, 3])
    pc = lambda x, y: x * (x + 1) // 2 + y
    assert np.all(pc(l[:, 0], l[:, 1]) >= pc(l[:, 2], l[:, 3]))


def test_survivor_list_stride(tdg, mol0):
    p = tdg.Plan(mol0, schwarz_tol=TAU)
    full, n = p.screen_list(mol0.P0, mol0.PD, mol0.R)
    part, n2 = p.screen_list(mol0.P0, mol0.PD, mol0.R, stride=7)
    assert n == n2 and np.array_equal(part, full[::7])
    few, _ = p.screen_list(mol0.P0, mol0.PD, mol0.R, cap=5)
    assert np.array_equal(few, full[:5])


# ------------------------------------------------------------------ per-quartet contributions
# Per-quartet bars.  FP64: a quartet's value is a sum over up to 16^4 primitive quartets with
# mixed-sign contraction coefficients and exponents up to 5000, so its rounding is relative to
# the largest primitive terms rather than to the (possibly cancelled) sum: 1e-9 of the
# quartet's largest component, plus 1e-13 absolute.  FP32 tables (mixed route): unit roundoff
# 6e-8, amplified by the same cancellation: 3e-5 of the largest component plus 1e-9.
REL64, ABS64 = 1e-9, 1e-13
REL32, ABS32 = 3e-5, 1e-9
def _compare_quartets(tdg, oracle_lib, m, q, prec, rel, abs_tol, label):
    p = tdg.Plan(m, schwarz_tol=0.0, autotune=False)
    got = p.quartet_contribs(m.P0, m.PD, m.R, q, precision=prec)
    ref = oracle_lib.quartet_contribs(m, q)
    scale = np.abs(ref).reshape(len(q), -1).max(axis=1)
    err = np.abs(got - ref).reshape(len(q), -1).max(axis=1)
    worst = int(np.argmax(err / (rel * scale + abs_tol)))
    r = err / np.maximum(scale, 1e-300)
    _say(f"  {label}: {len(q)} quartets, worst {err[worst]:.3e} at |c|max {scale[worst]:.3e}",
         "quartet", q[worst].tolist(), "largest |c|", scale.max(),
         "relative error median/99%/max", np.percentile(r, 50), np.percentile(r, 99), r.max(),
         "largest absolute", err.max())
    assert np.all(err <= rel * scale + abs_tol)
    return got, ref


def test_quartet_contribs_config0_all_orders(tdg, oracle_lib, mol0):
    """Every surviving quartet of config 0, listed in the library's orientation and in a
    shuffled one (pairs and shells swapped): the contributions follow the listed shells."""
    p = tdg.Plan(mol0, schwarz_tol=TAU)
    q, _ = p.screen_list(mol0.P0, mol0.PD, mol0.R)
    _compare_quartets(tdg, oracle_lib, mol0, q, 0, REL64, ABS64, "config0 FP64")
    rng = np.random.default_rng(3)
    qs = q.copy()
    sw = rng.random(len(q)) < 0.5
    qs[sw] = qs[sw][:, [2, 3, 0, 1]]
    sw = rng.random(len(q)) < 0.5
    qs[sw] = qs[sw][:, [1, 0, 2, 3]]
    sw = rng.random(len(q)) < 0.5
    qs[sw] = qs[sw][:, [0, 1, 3, 2]]
    _compare_quartets(tdg, oracle_lib, mol0, qs, 0, REL64, ABS64, "config0 FP64 shuffled")
    _compare_quartets(tdg, oracle_lib, mol0, q, 1, REL32, ABS32, "config0 FP32 tables")


def test_quartet_contribs_sixteen_primitives(tdg, oracle_lib):
    """Contraction degree 16 (the library's maximum) on s, p and d shells: per quartet and in
    the full gradient."""
    rng = np.random.default_rng(16)
    ex = lambda lo, hi, n=16: list(np.sort(np.exp(rng.uniform(np.log(lo), np.log(hi), n)))[::-1])
    cf = lambda n=16: list(rng.standard_normal(n))
    coords = np.array([[0.0, 0.0, 0.0], [2.1, 0.4, -0.3], [-0.5, 1.9, 1.2]])
    # 16 primitives on an s, a p, a d and a second p shell; the other d shell has 2 (so that the
    # oracle's extended-precision d-shell quartets stay within seconds)
    shells = [(0, 0, ex(0.1, 5000), cf()), (0, 1, ex(0.1, 500), cf()), (0, 2, ex(0.2, 50), cf()),
              (1, 0, ex(0.1, 100, 3), cf(3)), (1, 2, ex(0.3, 20, 2), cf(2)), (2, 1, ex(0.1, 30), cf())]
    m = molecules.make(coords, shells, seed=16)
    ns = m.n_shells
    # every unique quartet except those on one atom (their contribution is zero)
    q = np.array([(a, b, c, d) for a in range(ns) for b in range(a + 1) for c in range(ns) for d in range(c + 1)
                  if a * (a + 1) // 2 + b >= c * (c + 1) // 2 + d
                  and len({int(m.shell_atom[x]) for x in (a, b, c, d)}) > 1], dtype=np.int32)
    got, ref_q = _compare_quartets(tdg, oracle_lib, m, q, 0, REL64, ABS64, "16 primitives FP64")
    # the listed quartets are all unique ones but those on one atom (which contribute zero), so
    # the oracle's gradient is their sum; summed here rather than recomputed by the slow oracle
    ref = np.zeros((m.n_atoms, 3))
    for k, qq in enumerate(q):
        for x in range(4):
            ref[m.shell_atom[qq[x]]] += ref_q[k, x]
    g = tdg.Plan(m, schwarz_tol=0.0).grad(m.P0, m.PD, m.R)
    _say("  16 primitives gradient", np.abs(g - ref).max())
    assert np.abs(g - ref).max() <= 1e-8


@pytest.mark.parametrize("case", ["waters133", "droplet120"])
def test_quartet_sample_at_scale(tdg, oracle_lib, case):
    """A systematic sample of the screened quartets of the 133-water cluster (3325 functions)
    and of a 120-atom droplet, each compared with the oracle quartet by quartet (FP64 and
    FP32-table kernels)."""
    from paper_2407_16586_amd import synth
    m = synth.config3() if case == "waters133" else synth.droplet(120, 20240716 + 2 + 1000 * 65)
    p = tdg.Plan(m, schwarz_tol=TAU)
    _, n = p.screen_list(m.P0, m.PD, m.R, cap=0)
    q, _ = p.screen_list(m.P0, m.PD, m.R, stride=max(1, n // 1500))
    _say(case, "n_bf", m.n_bf, "survivors", n, "sample", len(q))
    _compare_quartets(tdg, oracle_lib, m, q, 0, REL64, ABS64, case + " FP64")
    _compare_quartets(tdg, oracle_lib, m, q, 1, REL32, ABS32, case + " FP32 tables")
