"""Error bounds for the Schur-complement estimator Delta = |z|^2 - |xi|^2 when its three
solves stop at a relative residual eps (test helper, not collected by pytest).

The estimator for one pair (Sec. 4.1 eq. stacc with eq. detschur and eq. inverseschur):
    t  = D_wb xi,          w1 = D_ww^-1 t        (white block solves, U)
    t2 = D_bw w1,          w2 = D_bb^-1 t2       (black block solves, U)
    phi = xi - P w2                              ((1 - PQ(U)) xi)
    v  = D'_wb phi,        x  = D'^-1 v          (one full solve, U')
    z  = phi - P [x]_black,                      Delta = |z|^2 - |xi|^2.
A solve that stops at relative residual eps leaves an error D^-1 r with |r| <= eps |rhs|.
To first order, Delta moves by 2 Re <z, dz>, and each residual enters dz through a
linear map whose adjoint can be applied to z; Cauchy-Schwarz then bounds each term by
(adjoint image of z) x eps |rhs|. With g5 D g5 = D^dagger (gamma5-hermiticity, which also
holds for D_bb, D_ww and gives (D_wb)^dagger = g5 D_bw g5):
    a0 = D'^-dagger [P z]_black                      full solve:  2 |a0| eps |v|
    y  = P (z - g5 D'_bw g5 a0)                      (K^dagger z restricted to range(P))
    a2 = D_bb^-dagger y                              black solves: 2 |a2| eps |t2|
    a1 = D_ww^-dagger g5 D_wb g5 a2                  white solves: 2 |a1| eps |t|
    |dDelta| <= 2 eps (|a0| |v| + |a2| |t2| + |a1| |t|) (1 + 10% for second order).
The adjoint images are computed with the library's FP64 solves (g5 conjugated; a loose
tolerance suffices, since only their norms enter) and the oracle's hops and projector.
The bound uses the actual vectors of the pair, so it is far tighter than one built from
operator norms; it is still a worst case over the direction of each residual.
"""
from __future__ import annotations

import numpy as np

from oracle import dirac


def norm(v) -> float:
    return float(np.linalg.norm(np.asarray(v).ravel()))


def adjoint_weights(psms, ctx, g, opU, opP, slot_up: int, z, tol: float = 1e-9):
    """|a0|, |a2|, |a1| of the module docstring for one pair (z = M xi)."""
    g5 = dirac.gamma5_apply
    prm = psms.default_params(tol=tol, max_iter=5000)
    u0 = g.restrict(g.project(z), g.black)
    a0 = g5(ctx.solve(slot_up, g5(u0), prm)[0])
    y = g.project(z - g5(opP.D_bw(g5(a0))))
    a2 = g5(ctx.solve_block(0, 0, g5(y), prm)[0])
    s = g5(opU.D_wb(g5(a2)))
    a1 = g5(ctx.solve_block(0, 1, g5(s), prm)[0])
    return norm(a0), norm(a2), norm(a1)


def pair_bound(eps: float, weights, rhs_norms) -> float:
    """2 eps sum_k |a_k| |rhs_k| with 10% for the second-order terms."""
    (n0, n2, n1), (v, t2, t) = weights, rhs_norms
    return 1.1 * 2.0 * eps * (n0 * v + n2 * t2 + n1 * t)
