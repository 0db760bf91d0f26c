"""Stochastic estimator of fermion-determinant ratios (Sec. 4.1 eq. stacc,
App. A.2 eq. paccstoch, App. C.1 eq. Deltaistoch).

For one Gaussian vector ``xi`` (density ``exp(-|xi|^2)``) the estimator is
``Delta = |M xi|^2 - |xi|^2`` and the filter accepts with ``min{1, e^-Delta}``.
``E_xi[e^-Delta] = det(M^dagger M)^-1``, so ``ln mean_j e^-Delta_j`` estimates
``ln det(D'^dagger D') - ln det(D^dagger D)`` for the ratio operator.

* FULL:  ``M = D(U')^-1 D(U)`` (eq. Mdef); ``xi`` is the raw noise.
* SCHUR: ``M = (1 - PQ(U'))^-1 (1 - PQ(U))`` on the range of ``P``
  (eq. detschur lets ``1 - PQ`` stand for the Schur complement); ``xi = P eta``.

With N interpolation steps (Sec. 4.3, eqs. gfparam, param, Mparam, staccN) the
determinant factorises over the intermediate fields U_0 = U, ..., U_N = U' and
the estimator sums one independent one-step term per factor.
"""
from __future__ import annotations

import numpy as np

from .schur import Operator
from .solvers import norm2


def delta_full(op_U: Operator, op_Up: Operator, eta: np.ndarray, tol=1e-14) -> float:
    y = op_Up.solve(op_U.D(eta), tol=tol)
    return norm2(y) - norm2(eta)


def delta_schur(op_U: Operator, op_Up: Operator, eta: np.ndarray, tol=1e-14) -> float:
    xi = op_U.g.project(eta)
    phi = op_U.schur_apply(xi)
    y = op_Up.schur_inverse_direct(phi, tol=tol)
    return norm2(y) - norm2(xi)


def log_ratio_estimate(deltas) -> float:
    """``ln mean_j exp(-Delta_j)`` (computed stably)."""
    d = -np.asarray(deltas, float)
    m = d.max()
    return float(m + np.log(np.mean(np.exp(d - m))))


def exact_moments(lams: np.ndarray):
    """For eigenvalues of M^dagger M: ``E[e^-Delta] = prod 1/lambda``,
    ``E[Delta] = sum (lambda - 1)``, ``Var[Delta] = sum (lambda - 1)^2`` (eq. varstoch2)."""
    lams = np.asarray(lams, float)
    return float(np.exp(-np.sum(np.log(lams)))), float(np.sum(lams - 1)), float(np.sum((lams - 1) ** 2))


def interpolated_field(U: np.ndarray, Up: np.ndarray, N: int, i: int) -> np.ndarray:
    """U_i of eq. gfparam with the gauge transformation g = 1 (no relative gauge
    fixing): ((N - i) U + i U') / N link by link, so U_0 = U and U_N = U'. The
    intermediate links are not SU(3); the operator takes their Hermitian conjugates
    for backward hops, which keeps it gamma5-Hermitian (Sec. 4.3)."""
    return ((N - i) / N) * U + (i / N) * Up


def delta_interpolated(geom, U: np.ndarray, Up: np.ndarray, kappa: float, etas, op: str = "schur",
                       tol=1e-14) -> float:
    """eq. staccN: Delta = sum_i (|M_i xi_i|^2 - |xi_i|^2) over the N = len(etas)
    factors of eq. param, M_i = D(U_{i+1})^-1 D(U_i) (eq. Mparam; with op "schur" the
    Schur complements of the two fields, as for one step), each factor with its own
    noise field etas[i]."""
    N = len(etas)
    one = delta_schur if op == "schur" else delta_full
    ops = [Operator(geom, interpolated_field(U, Up, N, i), kappa) for i in range(N + 1)]
    return float(sum(one(ops[i], ops[i + 1], etas[i], tol=tol) for i in range(N)))
