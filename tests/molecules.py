"""Hand-built small molecules for the oracle's pins (inputs only, no method arithmetic)."""
import numpy as np

from paper_2407_16586_amd.synth import Molecule, ncart


def make(coords, shells, n_occ=1, dens=None, seed=0):
    """shells: list of (atom, l, exps, coefs)."""
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    sa, sl, sn, sp, so, ex, co = [], [], [], [], [], [], []
    ao = 0
    for atom, l, e, c in shells:
        sa.append(atom); sl.append(l); sn.append(len(e)); sp.append(len(ex)); so.append(ao)
        ex.extend(e); co.extend(c); ao += ncart(l)
    i32 = lambda v: np.ascontiguousarray(v, dtype=np.int32)
    m = Molecule(name="custom", coords=coords, Z=i32(np.ones(len(coords))),
                 shell_atom=i32(sa), shell_l=i32(sl), shell_nprim=i32(sn),
                 shell_prim_off=i32(sp), shell_ao_off=i32(so),
                 exps=np.ascontiguousarray(ex, dtype=np.float64),
                 coefs=np.ascontiguousarray(co, dtype=np.float64), n_occ=n_occ)
    n = m.n_bf
    rng = np.random.default_rng(seed)
    if dens is None:
        A = rng.standard_normal((n, n))
        P0 = A @ A.T / n
        S = rng.standard_normal((n, n))
        PD = 0.05 * (S + S.T)
        R = 0.3 * rng.standard_normal((n, n))
        dens = (P0, PD, R)
    m.P0, m.PD, m.R = (np.ascontiguousarray(x, dtype=np.float64) for x in dens)
    return m


def small_mixed(seed=3):
    """1 heavy-like atom (s,s,p,d) + 2 light atoms (s,p), moderate exponents, 4 atoms total."""
    rng = np.random.default_rng(seed)
    coords = np.array([[0.0, 0.0, 0.0], [1.9, 0.3, -0.2], [-0.4, 2.1, 0.5], [0.6, -0.7, 2.2]])
    coords += rng.uniform(-0.1, 0.1, coords.shape)
    shells = [
        (0, 0, [40.0, 6.0, 1.2], [0.3, 0.5, 0.4]),
        (0, 1, [3.0, 0.7], [0.6, 0.5]),
        (0, 2, [0.9], [1.0]),
        (1, 0, [5.0, 0.8], [0.4, 0.7]),
        (1, 1, [1.1], [1.0]),
        (2, 0, [2.0], [1.0]),
        (2, 2, [0.6], [1.0]),
        (3, 1, [0.5], [1.0]),
    ]
    return make(coords, shells, seed=seed)
