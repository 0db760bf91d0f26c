"""Recursive domain decomposition (Sec. 3, eq. ddrec; the second acceptance step of
eq. 4step): the Dirichlet operator D_B of an outer block B is itself decomposed into
sub-blocks b', det D_B = prod_{b' in B} det D_b' det Dhat_B, and its Schur complement
Dhat_B (which again has Dirichlet boundary conditions) is estimated stochastically
block by block, Delta_B = |M_B xi_B|^2 - |xi_B|^2 with M_B = Dhat_B(U')^-1 Dhat_B(U).

TEST INFRASTRUCTURE ONLY: used by the test-suite and nothing in the library.

The direct sum over outer blocks of the D_B is D with every hop across an outer-block
face removed, i.e. D of the gauge field whose links across outer faces are zero; the
sub-block decomposition, Q, P and 1 - PQ of that operator are those of schur.py with
the projector of the outer geometry (``schur.Geometry(L, b, outer=...)``). Everything is
then block-diagonal over the outer blocks, so one noise field gives one independent
estimate per outer block.
"""
from __future__ import annotations

import numpy as np

from . import lattice, schur


def cut_links(U: np.ndarray, L, outer) -> np.ndarray:
    """U with U(x, mu) = 0 for the links that leave x's outer block (x_mu mod outer_mu =
    outer_mu - 1): the gauge field whose Dirac operator is the direct sum of the D_B."""
    x = lattice.coords(L)
    out = U.copy()
    for mu in range(4):
        out[x[:, mu] % outer[mu] == outer[mu] - 1, mu] = 0
    return out


def outer_block_sums(geom: schur.Geometry, psi: np.ndarray) -> np.ndarray:
    """|psi|^2 summed over the sites of each outer block (lexicographic outer order)."""
    oid = lattice.block_id(geom.L, geom.outer)
    w = np.sum(np.abs(psi.reshape(geom.V, -1)) ** 2, axis=1)
    return np.bincount(oid, weights=w, minlength=int(oid.max()) + 1)


def delta_block_schur(op_U: schur.Operator, op_Up: schur.Operator, eta: np.ndarray, tol=1e-14) -> np.ndarray:
    """Delta_B for every outer block B (operators built on the cut fields and the outer
    geometry): z = (1 - PQ(U'))^-1 (1 - PQ(U)) xi with xi = P eta, then
    Delta_B = |z_B|^2 - |xi_B|^2 (eq. Deltaistoch per block)."""
    g = op_U.g
    xi = g.project(eta)
    phi = op_U.schur_apply(xi)
    z = op_Up.schur_inverse_direct(phi, tol=tol)
    return outer_block_sums(g, z) - outer_block_sums(g, xi)
