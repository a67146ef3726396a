"""Write the oracle's gradients (and sampled Fock-type matrix blocks) for the stored parity
cases (calls only oracle/ and the seeded input generator).
Usage: python tests/golden/make_golden.py [name ...]"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2407_16586_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

CASES = {
    # 60-atom chain, 500 Cartesian functions, density-multiplied Schwarz threshold 1e-10
    "chain60_tau1e-10": dict(mol=synth.config1, tau=1e-10),
    # the same chain with def2-SVP-shaped exponent ranges and positive coefficients
    "chain60svp_tau1e-10": dict(mol=lambda: synth.config1("svp"), tau=1e-10),
    # molecule 32 of the 64-droplet batch: 61 atoms, 505 Cartesian functions
    "droplet61_tau1e-10": dict(mol=lambda: synth.config2_molecule(32), tau=1e-10),
}

FOCK_CASES = {
    # Fock-type matrix of eq G_2e, (cJ, cK, cKlr) = (2, -alpha, -beta), of the chain's relaxed
    # difference density: blocks of 10 shell pairs (seeded sample, diagonal pair included)
    "chain60_fock_pd": dict(mol=synth.config1, dens="PD", npairs=10, seed=21),
    # the same for the 120-atom droplet of the at-scale quartet samples (ground-state density),
    # eight shell pairs
    "droplet120_fock_p0": dict(mol=lambda: synth.droplet(120, 20240716 + 2 + 1000 * 65), dens="P0", npairs=8,
                               seed=22),
}


def make_fock(name):
    spec = FOCK_CASES[name]
    mol = spec["mol"]()
    B = getattr(mol, spec["dens"])
    rng = np.random.default_rng(spec["seed"])
    ns = mol.n_shells
    sl = np.asarray(mol.shell_l)
    pick = lambda l: int(rng.choice(np.where(sl == l)[0]))
    pairs = [(0, 0)] + [(pick(la), pick(lb)) for la, lb in ((1, 1), (2, 0), (2, 1), (2, 2))]
    pairs += [tuple(int(x) for x in rng.integers(0, ns, 2)) for _ in range(spec["npairs"] - len(pairs))]
    cf = (2.0, -mol.alpha, -mol.beta)
    t = time.time()
    blocks = oracle.fock_blocks(mol, B, np.array(pairs, dtype=np.int32), *cf)
    dt = time.time() - t
    out = {"case": name, "density": spec["dens"], "coefs": cf, "n_bf": mol.n_bf, "pairs": pairs,
           "blocks": [b.tolist() for b in blocks], "oracle_seconds": dt,
           "generator": "tests/golden/make_golden.py (oracle.fock_blocks, synthetic seeded inputs)"}
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f, indent=1)
    print(name, f"{dt:.1f}s", flush=True)


def make(name):
    if name in FOCK_CASES:
        return make_fock(name)
    spec = CASES[name]
    mol = spec["mol"]()
    t = time.time()
    g, st = oracle.grad(mol, tau=spec["tau"], return_stats=True)
    dt = time.time() - t
    out = {"case": name, "tau": spec["tau"], "n_atoms": mol.n_atoms, "n_bf": mol.n_bf,
           "oracle_stats": st, "oracle_seconds": dt, "grad": g.tolist(),
           "generator": "tests/golden/make_golden.py (oracle.grad, synthetic seeded inputs)"}
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f, indent=1)
    print(name, st, f"{dt:.1f}s", flush=True)


if __name__ == "__main__":
    oracle.build(force=False)
    for n in (sys.argv[1:] or list(CASES) + list(FOCK_CASES)):
        make(n)
