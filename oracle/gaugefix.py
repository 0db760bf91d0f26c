"""Relative gauge fixing of a field pair (Sec. 4.2, eqs. sprodgf, relgf, choiceg; App. B,
eqs. GF:fminendform, ming, GF:Delta, GF:theta).

TEST INFRASTRUCTURE ONLY: used by the test-suite and nothing in the library.

With g1 = g2^-1 = g (eq. choiceg) the link term of eq. relgf is
    Re Tr{1 - g(x+mu) U(x,mu)^+ g(x)^+ g(x)^+ U'(x,mu) g(x+mu)}
  = Re Tr{1 - U(x,mu)^+ G(x)^+ U'(x,mu) G(x+mu)},   G = g^2,
the Landau-like form of App. B (eq. GF:fminendform): a one-sided fixing of U' to U by G,
minimised site by site against Delta(x) = W_f(x) + W_b(x) (eq. GF:Delta). Steepest
descent (eq. ming) on the current field U'_G = U'^(G^-1) (G(x)^+ U'(x,mu) G(x+mu)), where
    Delta(x) = sum_mu [U'_G(x,mu) U(x,mu)^+ + U'_G(x-mu,mu)^+ U(x-mu,mu)],
    C(x) = Delta - Delta^+ - Tr(Delta - Delta^+)/3,
    k(x) = exp(alpha/2 C(x)) on the domain,   G -> G k,
and theta(x) = -Tr C(x)^2 >= 0 (eq. GF:theta). At the end g = G^(1/2) (principal root)
gives the pair (U^g, U'^(g^-1)) of eq. matrixMgf and the end points of eq. gfparam.

Readings (the paper is ambiguous or garbled here):
* the step of eq. ming acts on G = g^2, the field that enters eq. GF:fminendform, as the
  Landau-gauge procedure it follows acts on the one field it transforms;
* the sign of the exponent is the one that lowers eq. relgf (the aim App. B states); with
  Delta as written, exp(-alpha/2 C) raises it;
* eq. GF:theta is the trace of the square of C (the trace of C vanishes), with the sign
  that makes it non-negative, and the stopping test uses its mean over the domain;
* "no convergence" is a step that raises eq. relgf: it is rejected and alpha lowered by
  0.01, down to 0.10 (App. B); a rejected step at 0.10 ends the iteration;
* the domain is the set of block-interior sites (no nearest neighbour in another block:
  local coordinates 1 .. b_mu - 2 in every direction), where the proposals change links
  (Sec. 4.2, App. B); G = g = 1 elsewhere.
The SU(3) exponential and square root are taken from eigendecompositions (library steps).
"""
from __future__ import annotations

import numpy as np

from . import lattice


def dag(A):
    return np.conj(np.swapaxes(A, -1, -2))


def interior_sites(L, b) -> np.ndarray:
    loc = lattice.coords(L) % np.asarray(b)
    return np.all((loc > 0) & (loc < np.asarray(b) - 1), axis=1)


def relgf_functional(U, Up) -> float:
    """eq. sprodgf of the pair: (1/12V) sum_{x,mu} Re Tr{1 - U(x,mu)^+ U'(x,mu)}."""
    V = U.shape[0]
    tr = np.einsum("xmij,xmij->", np.conj(U), Up)  # sum Tr(U^+ U')
    return float((12 * V - tr.real) / (12 * V))


def transform_pair(U, Up, h, L):
    """(U^h, U'^(h^-1)): U(x,mu) -> h(x) U h(x+mu)^+, U'(x,mu) -> h(x)^+ U' h(x+mu)."""
    A, B = np.empty_like(U), np.empty_like(Up)
    for mu in range(4):
        hn = h[lattice.neighbour(L, mu, +1)]
        A[:, mu] = h @ U[:, mu] @ dag(hn)
        B[:, mu] = dag(h) @ Up[:, mu] @ hn
    return A, B


def delta_and_theta(U, Up, L):
    """Delta(x) of eq. GF:Delta on the current pair, C(x), theta(x)."""
    D = np.zeros((U.shape[0], 3, 3), np.complex128)
    for mu in range(4):
        D += Up[:, mu] @ dag(U[:, mu])
        bw = lattice.neighbour(L, mu, -1)
        D += dag(Up[bw, mu]) @ U[bw, mu]
    C = D - dag(D)
    C = C - (np.trace(C, axis1=1, axis2=2) / 3.0)[:, None, None] * np.eye(3)
    theta = -np.einsum("xij,xji->x", C, C).real
    return D, C, theta


def expm_antihermitian(X):
    """exp(X) for anti-Hermitian [n, 3, 3] X from the eigenvectors of the Hermitian -iX."""
    w, v = np.linalg.eigh(-1j * X)
    return (v * np.exp(1j * w)[:, None, :]) @ dag(v)


def sqrt_su3(G):
    """Principal square root of [n, 3, 3] unitary G (eigenphases halved)."""
    w, v = np.linalg.eig(G)
    r = (v * np.exp(0.5j * np.angle(w))[:, None, :]) @ np.linalg.inv(v)
    return r


def relative_gauge_fix(U, Up, L, b, alpha=0.15, alpha_min=0.10, theta_tol=1e-3, max_iter=500):
    """Steepest descent of App. B. Returns (g, U^g, U'^(g^-1), history) with history a list
    of (eq. relgf, mean theta, alpha) before each step."""
    dom = interior_sites(L, b)
    V = U.shape[0]
    one = np.broadcast_to(np.eye(3, dtype=np.complex128), (V, 3, 3))
    G = one.copy()
    Upc = Up.copy()
    f = relgf_functional(U, Upc)
    hist = []
    it = 0
    while it < max_iter:
        _, C, theta = delta_and_theta(U, Upc, L)
        th = float(theta[dom].mean()) if dom.any() else 0.0
        hist.append((f, th, alpha))
        if th < theta_tol:
            break
        k = one.copy()
        k[dom] = expm_antihermitian(0.5 * alpha * C[dom])
        # U'_G -> U'_G^(k^-1): U'(x,mu) -> k(x)^+ U'(x,mu) k(x+mu)
        trial = np.empty_like(Upc)
        for mu in range(4):
            trial[:, mu] = dag(k) @ Upc[:, mu] @ k[lattice.neighbour(L, mu, +1)]
        fn = relgf_functional(U, trial)
        it += 1
        if fn > f:
            if alpha - 0.01 < alpha_min - 1e-12:
                break
            alpha -= 0.01
            continue
        Upc, f = trial, fn
        G = G @ k
    g = one.copy()
    g[dom] = sqrt_su3(G[dom])
    Ug, Upg = transform_pair(U, Up, g, L)
    return g, Ug, Upg, hist
