"""Stochastic estimator of fermion-determinant ratios (Sec. 4.1 eq. stacc,
App. A.2 eq. paccstoch, App. C.1 eq. Deltaistoch).

For one Gaussian vector ``xi`` (density ``exp(-|xi|^2)``) the estimator is
``Delta = |M xi|^2 - |xi|^2`` and the filter accepts with ``min{1, e^-Delta}``.
``E_xi[e^-Delta] = det(M^dagger M)^-1``, so ``ln mean_j e^-Delta_j`` estimates
``ln det(D'^dagger D') - ln det(D^dagger D)`` for the ratio operator.

* FULL:  ``M = D(U')^-1 D(U)`` (eq. Mdef); ``xi`` is the raw noise.
* SCHUR: ``M = (1 - PQ(U'))^-1 (1 - PQ(U))`` on the range of ``P``
  (eq. detschur lets ``1 - PQ`` stand for the Schur complement); ``xi = P eta``.

Only one interpolation step (N = 1) is computed here.
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
