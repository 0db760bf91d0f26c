"""The hierarchy of acceptance steps for one level of recursive domain decomposition
(Sec. 2, eq. hierarchy; Sec. 3, eq. 4step; App. A.2, eq. paccstoch; App. C, eqs. Si,
DeltaSi).

TEST INFRASTRUCTURE ONLY: used by the test-suite and nothing in the library.

A proposal U -> U' that changes links inside the smallest blocks b' only goes through
    1) the block filter: every b' separately, Delta_1 = beta_1 dS1_b',
       dS1_b' = -2 (ln|det D_b'(U')| - ln|det D_b'(U)|) (exact, blockdet.py);
    2) the block-Schur filter: every outer block B separately, on the field U1 that holds
       U' in the blocks b' accepted at step 1 and U elsewhere,
       Delta_2 = dS2_B + beta_2 sum_{b' in B} dS1(U1 vs U),
       dS2_B = |M_B xi_B|^2 - |xi_B|^2 with one noise field (recursive.py);
    3) the global filter on U2 (U1 in the outer blocks accepted at step 2, U elsewhere),
       Delta_3 = dS3 + beta_3 sum_{b'} dS1(U2 vs U), dS3 the Schur estimator of the outer
       blocks' decomposition with one noise field (estimator.py);
each accepted when u < exp(-Delta) for its own uniform u in [0, 1) (min{1, e^-Delta}, one
Delta per decision, eq. paccstoch). The parameters beta_i multiply the exactly computed
block-determinant action S^(1) at each step (App. C, eq. Si); the stochastic terms take
none (App. C), and the beta_i of S^(1) sum to its target coefficient 1. The proposal
step 0) and the gauge-action parts of App. C are the caller's.
"""
from __future__ import annotations

import numpy as np

from . import blockdet, estimator, lattice, recursive, schur


def link_blocks(L, b):
    """[V, 4] lexicographic block index of each link's block, -1 for links that leave
    their block (the link from x to x + mu)."""
    bid = lattice.block_id(L, b)
    out = np.empty((bid.size, 4), int)
    for mu in range(4):
        nb = lattice.neighbour(L, mu, +1)
        out[:, mu] = np.where(bid[nb] == bid, bid, -1)
    return out


def merge(U, Up, L, b, accept):
    """U' on the links inside the blocks with accept[k] (k lexicographic), U elsewhere."""
    lb = link_blocks(L, b)
    take = (lb >= 0) & np.asarray(accept, bool)[np.maximum(lb, 0)]
    out = U.copy()
    out[take] = Up[take]
    return out


def filter_step(U, Up, kappa, L, b_small, b_outer, u1, u2, u3, eta2, eta3, beta=(1.0, 0.0, 0.0)):
    """One pass of the three filters. Returns a dict with the exponents, decisions and the
    field after each step (U3 is the new state)."""
    lb = link_blocks(L, b_small)
    if np.any(np.abs(U[lb < 0] - Up[lb < 0]) > 0):
        raise ValueError("the proposal changes links between the smallest blocks")
    dS1 = blockdet.block_filter_delta(U, Up, kappa, L, b_small)
    d1 = beta[0] * dS1
    a1 = np.asarray(u1) < np.exp(-d1)
    U1 = merge(U, Up, L, b_small, a1)
    # step 2 on the outer blocks' Dirichlet operators
    g2 = schur.Geometry(L, b_small, outer=b_outer)
    op_U = schur.Operator(g2, recursive.cut_links(U, L, b_outer), kappa)
    op_1 = schur.Operator(g2, recursive.cut_links(U1, L, b_outer), kappa)
    dS2 = recursive.delta_block_schur(op_U, op_1, eta2)
    small_in_outer = _small_to_outer(L, b_small, b_outer)
    acc1_dS1 = np.where(a1, dS1, 0.0)
    d2 = dS2 + beta[1] * np.bincount(small_in_outer, weights=acc1_dS1, minlength=dS2.size)
    a2 = np.asarray(u2) < np.exp(-d2)
    U2 = merge(U, U1, L, b_outer, a2)
    # step 3: the global Schur complement of the outer blocks
    g3 = schur.Geometry(L, b_outer)
    dS3 = estimator.delta_schur(schur.Operator(g3, U, kappa), schur.Operator(g3, U2, kappa), eta3)
    d3 = dS3 + beta[2] * float(np.sum(acc1_dS1 * a2[small_in_outer]))
    a3 = bool(u3 < np.exp(-d3))
    return {"dS1": dS1, "delta1": d1, "accept1": a1, "U1": U1, "dS2": dS2, "delta2": d2, "accept2": a2, "U2": U2,
            "dS3": dS3, "delta3": d3, "accept3": a3, "U3": U2 if a3 else U}


def _small_to_outer(L, b_small, b_outer) -> np.ndarray:
    """Lexicographic outer block of each lexicographic small block."""
    NB = np.asarray(L) // np.asarray(b_small)
    NO = np.asarray(L) // np.asarray(b_outer)
    B = np.stack(np.meshgrid(*[np.arange(n) for n in NB], indexing="ij"), -1).reshape(-1, 4)
    O = B * np.asarray(b_small) // np.asarray(b_outer)
    return ((O[:, 0] * NO[1] + O[:, 1]) * NO[2] + O[:, 2]) * NO[3] + O[:, 3]
