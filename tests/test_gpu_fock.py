"""Parity of the Fock-type matrix (tdg_fock; section II.B, eqs G_2e and zfock, two-electron
part) with the oracle, which writes F out by its definition over every ordered shell quartet.

Tolerance: the kernels are FP64 throughout; an element sums at most a few times 10^5
quartet contributions, each exact to the Rys table's fit (about 1e-14 relative) and
FP64 rounding, against the oracle's extended-precision Obara-Saika values.  The bar is
|F - F_oracle| <= 1e-10 max|F_oracle| per element (no screening).  With screening at tau,
the skipped quartets' contributions are each below 72 tau (36 components, weight <= 2)
and the test states the measured effect next to a 1e-7 bound."""
import numpy as np
import pytest

from tests import molecules

pytestmark = pytest.mark.gpu
REL = 1e-10


@pytest.fixture(scope="module")
def tdg():
    from paper_2407_16586_amd import tdgrad
    tdgrad.lib()
    return tdgrad


def _say(*a):
    print(*a, flush=True)


def _coefs(m):
    return {"G_2e": (2.0, -m.alpha, -m.beta), "zfock": (4.0, -2 * m.alpha, -2 * m.beta),
            "J": (1.0, 0.0, 0.0), "K": (0.0, 1.0, 0.0), "K_lr": (0.0, 0.0, 1.0)}


def _err(F, ref):
    return np.abs(F - ref).max() / np.abs(ref).max()


def test_fock_small_mixed_all_terms(tdg, oracle_lib):
    """s, p and d shells on four atoms, non-symmetric B, every coefficient set."""
    m = molecules.small_mixed()
    rng = np.random.default_rng(12)
    B = rng.standard_normal((m.n_bf, m.n_bf))
    p = tdg.Plan(m, schwarz_tol=0.0)
    parts = [oracle_lib.fock(m, B, *c) for c in ((1, 0, 0), (0, 1, 0), (0, 0, 1))]
    for name, cf in _coefs(m).items():
        _say("small_mixed", name)
        ref = cf[0] * parts[0] + cf[1] * parts[1] + cf[2] * parts[2]
        F = p.fock(B, *cf)
        e = _err(F, ref)
        _say("  rel err", e)
        assert e <= REL, (name, e)
        assert np.abs(F - F.T).max() <= 1e-13 * np.abs(F).max()


@pytest.fixture(scope="module")
def config0_parts(oracle_lib, mol0):
    rng = np.random.default_rng(13)
    B = mol0.P0 + 0.2 * rng.standard_normal(mol0.P0.shape)
    return B, [oracle_lib.fock(mol0, B, *c) for c in ((1, 0, 0), (0, 1, 0), (0, 0, 1))]


def test_fock_config0(tdg, mol0, config0_parts):
    B, parts = config0_parts
    p = tdg.Plan(mol0, schwarz_tol=0.0)
    for name, cf in _coefs(mol0).items():
        _say("config0", name)
        ref = cf[0] * parts[0] + cf[1] * parts[1] + cf[2] * parts[2]
        F, st = p.fock(B, *cf, stats=True)
        e = _err(F, ref)
        _say("  rel err", e, "quartets", st["quartets"])
        assert e <= REL, (name, e)
    ns = mol0.n_shells
    npair = ns * (ns + 1) // 2
    assert st["quartets"] == npair * (npair + 1) // 2  # no screening: every unique quartet


def test_fock_config0_screened_and_device(tdg, mol0, config0_parts):
    import torch
    B, parts = config0_parts
    cf = _coefs(mol0)["G_2e"]
    ref = cf[0] * parts[0] + cf[1] * parts[1] + cf[2] * parts[2]
    p = tdg.Plan(mol0, schwarz_tol=1e-10)
    F, st = p.fock(B, *cf, stats=True)
    ns = mol0.n_shells
    npair = ns * (ns + 1) // 2
    d = np.abs(F - ref).max()
    _say("config0 tau 1e-10: quartets", st["quartets"], "of", npair * (npair + 1) // 2, "max abs diff", d)
    assert d <= 1e-7
    dev = torch.device("cuda:0")
    Bd = torch.from_numpy(B).to(dev)
    out = torch.empty_like(Bd)
    p.fock_device(Bd, out, *cf)
    torch.cuda.synchronize()
    assert np.abs(out.cpu().numpy() - F).max() <= 1e-12 * np.abs(F).max()


def test_fock_zero_and_single_element(tdg, oracle_lib):
    m = molecules.small_mixed()
    p = tdg.Plan(m, schwarz_tol=1e-12)
    cf = _coefs(m)["G_2e"]
    Z = np.zeros((m.n_bf, m.n_bf))
    F, st = p.fock(Z, *cf, stats=True)
    assert st["quartets"] == 0 and not F.any()
    E = Z.copy()
    E[3, 17] = 1.0   # one element: Bs has two halves
    ref = oracle_lib.fock(m, E, *cf)
    assert _err(p.fock(E, *cf), ref) <= REL


def test_fock_relative_screening(tdg, mol0, config0_parts):
    """A Krylov-like vector shrunk by 2^-28 (a power of two, so that every bound scales
    exactly): absolute screening at 1e-10 drops most quartets (config 0 keeps 2852 of 21092);
    relative screening (B scaled to a unit largest element, F scaled back) keeps the
    survivors of the unscaled matrix and returns its F times 2^-28."""
    B, parts = config0_parts
    cf = _coefs(mol0)["G_2e"]
    ref = cf[0] * parts[0] + cf[1] * parts[1] + cf[2] * parts[2]
    s = 2.0 ** -28
    p = tdg.Plan(mol0, schwarz_tol=1e-10)
    Bm = B / np.abs(0.5 * (B + B.T)).max()    # largest |Bs| element one
    F1, st1 = p.fock(Bm, *cf, stats=True)
    Fa, sta = p.fock(s * Bm, *cf, stats=True)
    Fr, str_ = p.fock(s * Bm, *cf, relative=True, stats=True)
    _say("relative screening: quartets", st1["quartets"], "absolute on the shrunk matrix", sta["quartets"],
         "relative", str_["quartets"])
    assert str_["quartets"] == st1["quartets"] and sta["quartets"] < st1["quartets"] // 4
    assert np.abs(Fr - s * F1).max() <= 1e-13 * s * np.abs(F1).max()
    refm = ref / np.abs(0.5 * (B + B.T)).max()
    assert np.abs(Fr / s - refm).max() <= 1e-7


def test_fock_errors(tdg):
    m = molecules.small_mixed()
    p = tdg.Plan(m, schwarz_tol=0.0)
    B = np.zeros((m.n_bf, m.n_bf))
    with pytest.raises(tdg.TdgError):
        p.fock(B, 1.0, 0.0, float("nan"))
    q = tdg.Plan(m, schwarz_tol=0.0, terms=3, omega=0.0)
    with pytest.raises(tdg.TdgError):
        q.fock(B, 1.0, 0.0, 1.0)       # long-range exchange without omega
    with pytest.raises(ValueError):
        p.fock(np.zeros((3, 3)))


def test_fock_chain60_sampled(tdg, oracle_lib):
    """The benchmark's 60-atom chain (500 functions) without screening and at tau = 1e-10:
    sampled shell-pair blocks (diagonal, one-centre, bonded and distant pairs, every
    momentum pair) against the oracle's blocks."""
    from paper_2407_16586_amd import synth
    m = synth.config1()
    rng = np.random.default_rng(14)
    B = m.P0 + 0.05 * rng.standard_normal(m.P0.shape)
    cf = _coefs(m)["G_2e"]
    ns = m.n_shells
    sl = m.shell_l
    pairs = [(0, 0)]
    for la in range(3):
        for lb in range(3):
            a = int(rng.choice(np.where(sl == la)[0]))
            same = np.where((sl == lb) & (m.shell_atom == m.shell_atom[a]))[0]
            pairs.append((a, int(same[0]) if len(same) else int(rng.choice(np.where(sl == lb)[0]))))
    pairs += [(int(rng.integers(ns)), int(rng.integers(ns))) for _ in range(6)]
    pairs = np.array(pairs, dtype=np.int32)
    _say("chain60: oracle blocks for", len(pairs), "pairs")
    blocks = oracle_lib.fock_blocks(m, B, pairs, *cf)
    scale = max(np.abs(b).max() for b in blocks)
    off = m.shell_ao_off
    nc = (sl + 1) * (sl + 2) // 2
    for tau, tol in ((0.0, REL), (1e-10, 1e-7 / scale)):
        p = tdg.Plan(m, schwarz_tol=tau)
        F, st = p.fock(B, *cf, stats=True)
        worst = max(np.abs(F[off[a]:off[a] + nc[a], off[b]:off[b] + nc[b]] - blk).max()
                    for (a, b), blk in zip(pairs, blocks)) / scale
        _say(f"  tau {tau}: quartets {st['quartets']} kernels {st['ms_kernels']:.1f} ms, rel err {worst:.2e}")
        assert worst <= tol, (tau, worst)


def test_fock_droplet120_stored_blocks(tdg):
    """The 120-atom droplet (1000 functions) of the at-scale quartet samples: eq G_2e of its
    ground-state density, unscreened (6.7e9 unique quartets) and at tau = 1e-10, against
    eight shell-pair blocks stored by tests/golden/make_golden.py from the oracle."""
    import json
    import os
    from paper_2407_16586_amd import synth
    with open(os.path.join(os.path.dirname(__file__), "golden", "droplet120_fock_p0.json")) as fh:
        gf = json.load(fh)
    m = synth.droplet(120, 20240716 + 2 + 1000 * 65)
    assert m.n_bf == gf["n_bf"]
    B = getattr(m, gf["density"])
    off, sl = m.shell_ao_off, m.shell_l
    nc = (sl + 1) * (sl + 2) // 2
    scale = max(np.abs(np.array(b)).max() for b in gf["blocks"])
    for tau, tol in ((0.0, REL), (1e-10, 1e-7 / scale)):
        p = tdg.Plan(m, schwarz_tol=tau)
        F, st = p.fock(B, *gf["coefs"], stats=True)
        worst = max(np.abs(F[off[a]:off[a] + nc[a], off[b]:off[b] + nc[b]] - np.array(blk)).max()
                    for (a, b), blk in zip(gf["pairs"], gf["blocks"])) / scale
        _say(f"droplet120 tau {tau}: quartets {st['quartets']} kernels {st['ms_kernels']:.1f} ms, rel err {worst:.2e}")
        assert worst <= tol, (tau, worst)
        p.close()
