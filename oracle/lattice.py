"""Lattice geometry for the oracle (Sec. 3 of the paper, Fig. bgr).

Blocks are the non-overlapping boxes ``x // b``; they are coloured like a
checker board by the parity of the sum of block coordinates. Reading taken
where the paper is silent: the block containing the origin is black.

The projector ``P`` (Sec. 4.4): on a black site with exactly one nearest
neighbour outside its block, located at ``y + mu``, ``P = (1 + gamma_mu)/2``;
at ``y - mu``, ``P = (1 - gamma_mu)/2``; with two or more outside neighbours
``P = 1``; on block-interior black sites and on all white sites ``P = 0``.
This is the choice that makes ``D_wb P = D_wb`` hold with ``P^2 = P`` (both
checked by the tests) and reproduces eq. dimproj.
"""
from __future__ import annotations

import numpy as np

from .dirac import GAMMA, ONE4


def volume(L) -> int:
    return int(np.prod(L))


def coords(L) -> np.ndarray:
    g = np.meshgrid(*[np.arange(n) for n in L], indexing="ij")
    return np.stack([a.reshape(-1) for a in g], axis=1)


def site_index(L, x: np.ndarray) -> np.ndarray:
    x = np.asarray(x)
    return ((x[..., 0] * L[1] + x[..., 1]) * L[2] + x[..., 2]) * L[3] + x[..., 3]


def neighbour(L, mu: int, sign: int) -> np.ndarray:
    """Index of x + sign*mu for every site (periodic wrap)."""
    x = coords(L)
    x[:, mu] = (x[:, mu] + sign) % L[mu]
    return site_index(L, x)


def block_coords(L, b) -> np.ndarray:
    return coords(L) // np.asarray(b)


def block_id(L, b) -> np.ndarray:
    NB = np.asarray(L) // np.asarray(b)
    B = block_coords(L, b)
    return ((B[:, 0] * NB[1] + B[:, 1]) * NB[2] + B[:, 2]) * NB[3] + B[:, 3]


def is_black(L, b) -> np.ndarray:
    """Site mask of the black blocks (block coordinate sum even)."""
    return block_coords(L, b).sum(axis=1) % 2 == 0


def parity(L) -> np.ndarray:
    return coords(L).sum(axis=1) % 2


def projector_matrices(L, b, outer=None) -> np.ndarray:
    """Per-site 4x4 spin matrices of P, shape [V, 4, 4] (colour identity implied).

    With ``outer`` (recursive domain decomposition, eq. ddrec): the operator is the
    Dirichlet operator of the outer blocks ``x // outer``, so a neighbour across an outer
    face is no neighbour, and P counts only the out-of-block neighbours that stay in the
    site's outer block."""
    V = volume(L)
    bid = block_id(L, b)
    black = is_black(L, b)
    oid = block_id(L, outer) if outer is not None else np.zeros(V, int)
    out_nb = np.zeros((V, 4, 2), bool)  # [site, mu, (forward, backward)] outside own block
    for mu in range(4):
        for k, sign in enumerate((+1, -1)):
            nb = neighbour(L, mu, sign)
            out_nb[:, mu, k] = (bid[nb] != bid) & (oid[nb] == oid)
    n_out = out_nb.reshape(V, 8).sum(axis=1)
    P = np.zeros((V, 4, 4), np.complex128)
    for mu in range(4):
        one_fwd = black & (n_out == 1) & out_nb[:, mu, 0]
        one_bwd = black & (n_out == 1) & out_nb[:, mu, 1]
        P[one_fwd] = (ONE4 + GAMMA[mu]) / 2
        P[one_bwd] = (ONE4 - GAMMA[mu]) / 2
    P[black & (n_out >= 2)] = ONE4
    return P


def apply_projector(Pm: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """``(P psi)(x) = P(x) psi(x)``; psi [V, 4, 3]."""
    return np.matmul(Pm, psi)


def dim_projector_closed_form(L, b) -> int:
    """eq. dimproj: 6 prod(L/l) (sum_nu V_b / l_nu - 4 sum_nu (l_nu - 1))."""
    L = np.asarray(L)
    l = np.asarray(b)
    Vb = int(np.prod(l))
    return int(6 * np.prod(L // l) * (sum(Vb // int(x) for x in l) - 4 * int(np.sum(l - 1))))
