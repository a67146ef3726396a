"""Algorithmic work of the ERI-derivative evaluation, per primitive quartet of a class.

Counted for the method as formulated here (Rys quadrature, translational
invariance, contraction with the two-particle density on the fly), per Rys
root r of the n = floor((L+1)/2)+1 roots of a class (L = la+lb+lc+ld), and
doubled when the long-range root set is present:

  roots     : the rule's two degree-13 polynomials (Horner)        2*13 FMA = 52 flop
  set-up    : rho, T, recurrence coefficients, prefactor           ~30 flop (per primitive quartet, once)
  VRR       : (la+lb+2)(lc+ld+2) entries per direction, 5 flop each (two-term recurrences)
  HRR       : bra transfer sum_j (la+lb+1-j)(lc+ld+2) entries, ket transfer
              sum_l (la+1)(lb+2)(lc+ld+1-l) entries, 2 flop each, per direction
  derivative: for each of the (la+1)(lb+1)(lc+1)(ld+1) index quadruples and
              each of the 3 differentiated centres: 2 zeta X(+) - l X(-), 3 flop,
              per direction
  contract  : for each of the N = n_a n_b n_c n_d Cartesian components:
              4 products (Gamma weights of the three 2D factors) + 9 FMA = 22 flop

These are floating-point operations of the algorithm (FMA = 2), independent of
how a compiler schedules them; the roofline fraction divides them by the
FP64 vector peak.
"""
from __future__ import annotations

from .tdgrad import CLASSES


def ncart(l: int) -> int:
    return (l + 1) * (l + 2) // 2


def nroots(la, lb, lc, ld) -> int:
    return (la + lb + lc + ld + 1) // 2 + 1


def flops_per_root(la, lb, lc, ld) -> int:
    nm, mm = la + lb + 1, lc + ld + 1
    vrr = 5 * (nm + 1) * (mm + 1)
    hrr_bra = sum((nm - j) * (mm + 1) for j in range(lb + 1))
    hrr_ket = sum((la + 1) * (lb + 2) * (mm - l) for l in range(ld + 1))
    hrr = 2 * (hrr_bra + hrr_ket)
    deriv = 3 * 3 * (la + 1) * (lb + 1) * (lc + 1) * (ld + 1)
    per_dir = vrr + hrr + deriv
    n = ncart(la) * ncart(lb) * ncart(lc) * ncart(ld)
    return 52 + 3 * per_dir + 22 * n


def flops_per_prim_quartet(cls, long_range: bool = True) -> int:
    la, lb, lc, ld = cls
    sets = 2 if long_range else 1
    return 30 + sets * nroots(la, lb, lc, ld) * flops_per_root(la, lb, lc, ld)


FLOPS_PER_PRIM = {c: flops_per_prim_quartet(c) for c in CLASSES}


# ---------------------------------------------------------------------------
# Fock-type matrix (section II.B, eqs G_2e and zfock), per primitive quartet of a class,
# with n = floor(L/2) + 1 roots per kernel (no derivative) and, per root,
#   roots     : 52 flop (as above)
#   VRR/HRR   : the same recurrences for momenta (la+lb, lc+ld) per direction
#   contract  : N components, two products and one sum of the three 2D factors = 3 flop
# and per shell quartet (once, after the primitive sums): the six output blocks J_ab, J_cd,
# K_ac, K_ad, K_bc, K_bd, N multiply-adds each = 12 N flop, plus 3 N flop that weight and
# combine the full- and long-range exchange integrals.
def fock_flops_per_root(la, lb, lc, ld) -> int:
    nm, mm = la + lb, lc + ld
    vrr = 5 * (nm + 1) * (mm + 1)
    hrr_bra = sum((nm - j) * (mm + 1) for j in range(lb + 1))
    hrr_ket = sum((la + 1) * (lb + 1) * (mm - l) for l in range(ld + 1))
    per_dir = vrr + 2 * (hrr_bra + hrr_ket)
    n = ncart(la) * ncart(lb) * ncart(lc) * ncart(ld)
    return 52 + 3 * per_dir + 3 * n


def fock_flops(cls, prim_quartets: int, quartets: int, long_range: bool = True) -> int:
    la, lb, lc, ld = cls
    sets = 2 if long_range else 1
    n = ncart(la) * ncart(lb) * ncart(lc) * ncart(ld)
    per_prim = 30 + sets * ((la + lb + lc + ld) // 2 + 1) * fock_flops_per_root(la, lb, lc, ld)
    return per_prim * prim_quartets + 15 * n * quartets
