"""Exact block determinants for the block filter (Sec. 3: eq. ddfactor and the first
acceptance step of eq. 4step; the paper computes the determinants of blocks of up to
about 6^4 points exactly by LU).

TEST INFRASTRUCTURE ONLY: used by the test-suite and nothing in the library.

The block operator ``D_b`` is the principal sub-matrix of ``D`` on the sites of block
``b``: hops that leave the block are dropped (Dirichlet boundary conditions, Sec. 3).
Its log-determinant is taken by dense LU (numpy ``slogdet``, LAPACK getrf) of that
sub-matrix, written out as the definition, with no even-odd reduction.

``det D_b`` is real, because ``gamma_5 D_b gamma_5 = D_b^dagger`` (the block restriction
keeps gamma5-hermiticity), so its phase is 0 or pi.
"""
from __future__ import annotations

import numpy as np

from . import dirac, lattice


def block_logdets(U: np.ndarray, kappa: float, L, b, antiperiodic: bool = True) -> np.ndarray:
    """``ln det D_b`` (complex, imaginary part in (-pi, pi]) for every block, in
    lexicographic block order (block coordinate ``x // b``, direction 3 fastest)."""
    D = dirac.dirac_matrix(U, kappa, L, antiperiodic).tocsr()
    bid = lattice.block_id(L, b)
    nblk = int(np.prod(np.asarray(L) // np.asarray(b)))
    out = np.empty(nblk, np.complex128)
    for k in range(nblk):
        s = np.nonzero(bid == k)[0]
        d = (12 * s[:, None] + np.arange(12)[None, :]).reshape(-1)
        sign, logabs = np.linalg.slogdet(D[d][:, d].toarray())
        out[k] = logabs + 1j * np.angle(sign)
    return out


def block_filter_delta(U: np.ndarray, Up: np.ndarray, kappa: float, L, b, antiperiodic: bool = True) -> np.ndarray:
    """Exponent of the block filter per block (first step of eq. 4step, accepted with
    min{1, e^-Delta}): ``Delta_b = -ln[det(D_b'^+ D_b') / det(D_b^+ D_b)]
    = -2 (ln|det D_b(U')| - ln|det D_b(U)|)``."""
    a = block_logdets(U, kappa, L, b, antiperiodic).real
    c = block_logdets(Up, kappa, L, b, antiperiodic).real
    return -2.0 * (c - a)
