"""Write the oracle's gradients for the stored parity cases (calls only oracle/ and the
seeded input generator).  Usage: python tests/golden/make_golden.py [name ...]"""
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


def make(name):
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
    for n in (sys.argv[1:] or CASES):
        make(n)
