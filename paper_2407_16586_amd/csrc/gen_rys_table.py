"""Generate the Rys quadrature table used by the HIP kernels (rys_table.inc).

Rys quadrature (used for every ERI class, section II.C) replaces the Boys
function by an n-point Gauss rule for the weight exp(-T u) u^(-1/2)/2 on
u in [0, 1] (u = t^2):  sum_i w_i u_i^k = F_k(T) for k < 2n.

For each n = 1..5 and each interval [2j, 2j+2) of T < 64 the roots u_i(T) and
weights w_i(T) are interpolated by degree-13 polynomials in the local
variable x = T - 2j - 1 in [-1, 1] (monomial coefficients, Horner order).
The interpolation data are exact Gauss rules computed at 50 significant
digits with mpmath: Boys moments F_0..F_{2n-1} from the confluent
hypergeometric form, the modified Chebyshev algorithm for the three-term
recurrence, and the eigen-decomposition of the Jacobi matrix (Golub-Welsch).
For T >= 64 the rule is the large-T limit: u_i = x_i^2/T, w_i = W_i/sqrt(T)
with (x_i, W_i) the positive nodes/weights of the 2n-point Gauss-Hermite rule.

The script verifies the double-precision evaluation against fresh mpmath
rules at random T and fails if the relative error exceeds 1e-13.
"""
from __future__ import annotations

import os
import sys

import mpmath as mp
import numpy as np

NMAX = 5
WIDTH = 2
TMAX = 64
DEG = 13
NINT = TMAX // WIDTH

mp.mp.dps = 50


def boys(m, T):
    T = mp.mpf(T)
    if T == 0:
        return mp.mpf(1) / (2 * m + 1)
    return mp.hyp1f1(m + mp.mpf(1) / 2, m + mp.mpf(3) / 2, -T) / (2 * m + 1)


def gauss_rule(n, T):
    """n-point Gauss rule for exp(-T u) u^(-1/2)/2 on [0,1]: (roots ascending, weights)."""
    mom = [boys(k, T) for k in range(2 * n)]
    a = [mp.mpf(0)] * n
    b = [mp.mpf(0)] * n
    prev = [mp.mpf(0)] * (2 * n)
    cur = mom[:]
    a[0] = mom[1] / mom[0]
    b[0] = mom[0]
    for k in range(1, n):
        nxt = [mp.mpf(0)] * (2 * n)
        for l in range(k, 2 * n - k):
            nxt[l] = cur[l + 1] - a[k - 1] * cur[l] - (b[k - 1] * prev[l] if k > 1 else 0)
        a[k] = nxt[k + 1] / nxt[k] - cur[k] / cur[k - 1]
        b[k] = nxt[k] / cur[k - 1]
        prev, cur = cur, nxt
    J = mp.zeros(n, n)
    for i in range(n):
        J[i, i] = a[i]
        if i + 1 < n:
            J[i, i + 1] = J[i + 1, i] = mp.sqrt(b[i + 1])
    E, Q = mp.eigsy(J)
    order = sorted(range(n), key=lambda i: E[i])
    return [E[i] for i in order], [mom[0] * Q[0, i] ** 2 for i in order]


def hermite_half(n):
    """positive nodes x_i and weights W_i of the 2n-point Gauss-Hermite rule (weight exp(-x^2)),
    numpy's nodes polished by Newton on H_2n at 50 digits, weights from the Christoffel form
    W = 2^(m-1) m! sqrt(pi) / (m^2 H_{m-1}(x)^2), m = 2n."""
    m = 2 * n
    xs, _ = np.polynomial.hermite.hermgauss(m)
    out = []
    for x0 in xs:
        if x0 <= 0:
            continue
        xr = mp.findroot(lambda t: mp.hermite(m, t), mp.mpf(float(x0)))
        wr = mp.mpf(2) ** (m - 1) * mp.factorial(m) * mp.sqrt(mp.pi) / (m ** 2 * mp.hermite(m - 1, xr) ** 2)
        out.append((xr, wr))
    out.sort()
    return [o[0] for o in out], [o[1] for o in out]


def cheb_to_monomial(c):
    """Chebyshev series coefficients -> monomial coefficients (ascending powers)."""
    D = len(c) - 1
    T = [[mp.mpf(0)] * (D + 1) for _ in range(D + 1)]
    T[0][0] = mp.mpf(1)
    if D >= 1:
        T[1][1] = mp.mpf(1)
    for k in range(2, D + 1):
        for j in range(D + 1):
            v = -T[k - 2][j]
            if j > 0:
                v += 2 * T[k - 1][j - 1]
            T[k][j] = v
    return [sum(c[k] * T[k][j] for k in range(D + 1)) for j in range(D + 1)]


def fit_interval(n, j):
    nodes = [mp.cos(mp.pi * (2 * i + 1) / (2 * (DEG + 1))) for i in range(DEG + 1)]
    rules = [gauss_rule(n, WIDTH * j + (WIDTH / 2) * (x + 1)) for x in nodes]
    out = []
    for kind in (0, 1):
        for i in range(n):
            f = [r[kind][i] for r in rules]
            c = []
            for k in range(DEG + 1):
                s = sum(f[q] * mp.cos(k * mp.acos(nodes[q])) for q in range(DEG + 1))
                c.append(s * 2 / (DEG + 1) if k else s / (DEG + 1))
            out.append(cheb_to_monomial(c))
    return out  # 2n polynomials: u_0..u_{n-1}, w_0..w_{n-1}


def eval_double(table, asym, n, T):
    if T >= TMAX:
        xs, ws = asym[n]
        return [x * x / T for x in xs], [w / np.sqrt(T) for w in ws]
    j = int(T // WIDTH)
    x = T - WIDTH * j - WIDTH / 2
    polys = table[n][j]
    vals = []
    for p in polys:
        acc = p[-1]
        for c in reversed(p[:-1]):
            acc = acc * x + c
        vals.append(acc)
    return vals[:n], vals[n:]


def main(out_path):
    table = {}
    asym = {}
    for n in range(1, NMAX + 1):
        table[n] = []
        for j in range(NINT):
            polys = fit_interval(n, j)
            table[n].append([[float(c) for c in p] for p in polys])
        xs, ws = hermite_half(n)
        asym[n] = ([float(x) for x in xs], [float(w) for w in ws])
    # verification against exact rules
    rng = np.random.default_rng(1)
    tests = list(rng.uniform(0, TMAX, 300)) + list(rng.uniform(TMAX, 4 * TMAX, 40)) + \
        [0.0, 1e-9, 2.0, 63.999, 64.0, 1e4]
    worst = 0.0
    for n in range(1, NMAX + 1):
        for T in tests:
            u, w = eval_double(table, asym, n, T)
            ue, we = gauss_rule(n, T)
            for i in range(n):
                worst = max(worst, abs(u[i] - float(ue[i])) / float(ue[i]),
                            abs(w[i] - float(we[i])) / float(we[i]))
    if worst > 1e-13:
        raise SystemExit(f"Rys table verification failed: worst relative error {worst:.3e}")
    lines = [
        "// Rys quadrature table for n = 1..5 roots; generated by gen_rys_table.py (do not edit).",
        f"// worst relative error of roots/weights at 1730 verification points: {worst:.2e}",
        f"#define RYS_NMAX {NMAX}",
        f"#define RYS_WIDTH {WIDTH}.0",
        f"#define RYS_TMAX {TMAX}.0",
        f"#define RYS_NINT {NINT}",
        f"#define RYS_NCOEF {DEG + 1}",
        "// rys_poly_n[interval][2n polynomials: u_0..u_{n-1}, w_0..w_{n-1}][coef, ascending powers of",
        "//   x = T - RYS_WIDTH*(interval + 1/2)]",
    ]
    for n in range(1, NMAX + 1):
        vals = [c for j in range(NINT) for p in table[n][j] for c in p]
        lines.append(f"__device__ const double rys_poly_{n}[{len(vals)}] = {{")
        for k in range(0, len(vals), 4):
            lines.append("  " + ", ".join(repr(v) for v in vals[k:k + 4]) + ",")
        lines.append("};")
    lines.append("// large-T limit: positive 2n-point Gauss-Hermite nodes x_i and weights W_i")
    for n in range(1, NMAX + 1):
        xs, ws = asym[n]
        lines.append(f"__device__ const double rys_herm_x_{n}[{n}] = {{{', '.join(repr(v) for v in xs)}}};")
        lines.append(f"__device__ const double rys_herm_w_{n}[{n}] = {{{', '.join(repr(v) for v in ws)}}};")
    tmp = out_path + ".tmp"
    with open(tmp, "w") as f:
        f.write("\n".join(lines) + "\n")
    os.replace(tmp, out_path)
    print(f"wrote {out_path}; worst relative error {worst:.2e}")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else
         os.path.join(os.path.dirname(os.path.abspath(__file__)), "rys_table.inc"))
