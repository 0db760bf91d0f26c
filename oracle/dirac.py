"""The Wilson-Dirac operator (eq. Dw, Sec. 5 of the paper), FP64.

Normalisation: ``D = 2 kappa (D_w + m_0) = 1 - kappa H`` with
``kappa = 1 / (2 m_0 + 8)`` and

    H psi(x) = sum_mu [ U(x,mu) (1 - gamma_mu) psi(x + mu)
                        + U(x - mu, mu)^dagger (1 + gamma_mu) psi(x - mu) ].

The rescaling by ``2 kappa`` cancels in every determinant ratio and in the
Schur complement. Fermions are periodic in space and antiperiodic in time
(Sec. 6): a hop across the time boundary picks up a factor -1.

Gamma matrices (the paper does not fix a basis; reading taken): the chiral
basis ``gamma_0 = [[0, -1], [-1, 0]]``, ``gamma_k = [[0, -i s_k], [i s_k, 0]]``
(``s_k`` Pauli matrices), so that ``gamma_5 = gamma_0 gamma_1 gamma_2 gamma_3
= diag(1, 1, -1, -1)``.

Field layout: spinor ``psi[V, 4, 3]``, links ``U[V, 4, 3, 3]``, site index
lexicographic with direction 0 (time) slowest.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

_S1 = np.array([[0, 1], [1, 0]], np.complex128)
_S2 = np.array([[0, -1j], [1j, 0]], np.complex128)
_S3 = np.array([[1, 0], [0, -1]], np.complex128)
_Z2 = np.zeros((2, 2), np.complex128)
_I2 = np.eye(2, dtype=np.complex128)

GAMMA = np.array(
    [np.block([[_Z2, -_I2], [-_I2, _Z2]])]
    + [np.block([[_Z2, -1j * s], [1j * s, _Z2]]) for s in (_S1, _S2, _S3)]
)
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
ONE4 = np.eye(4, dtype=np.complex128)


def kappa_from_mass(m0: float) -> float:
    return 1.0 / (2.0 * m0 + 8.0)


def _grid(L, a: np.ndarray, tail) -> np.ndarray:
    return a.reshape(tuple(L) + tail)


def hopping(U: np.ndarray, psi: np.ndarray, L, antiperiodic: bool = True) -> np.ndarray:
    """``H psi`` (the sum over the 8 nearest-neighbour hops)."""
    P = _grid(L, psi, (4, 3))
    Ug = _grid(L, U, (4, 3, 3))
    out = np.zeros_like(P)
    for mu in range(4):
        Umu = Ug[..., mu, :, :]
        fwd = np.roll(P, -1, axis=mu)          # psi(x + mu)
        bwd = np.roll(P, 1, axis=mu)           # psi(x - mu)
        if antiperiodic and mu == 0:
            fwd[-1] = -fwd[-1]
            bwd[0] = -bwd[0]
        Ub = np.roll(Umu, 1, axis=mu)          # U(x - mu, mu)
        # colour: U acts on the last index; spin matrix on the spin index
        f = np.matmul(ONE4 - GAMMA[mu], fwd)
        out += np.matmul(f, np.swapaxes(Umu, -1, -2))
        g = np.matmul(ONE4 + GAMMA[mu], bwd)
        out += np.matmul(g, Ub.conj())
    return out.reshape(psi.shape)


def apply_D(U: np.ndarray, psi: np.ndarray, kappa: float, L, antiperiodic: bool = True) -> np.ndarray:
    """``D psi = psi - kappa H psi``."""
    return psi - kappa * hopping(U, psi, L, antiperiodic)


def apply_Dw_plus_m0(U, psi, kappa, L, antiperiodic=True):
    """``(D_w + m_0) psi`` in the paper's normalisation: ``D psi / (2 kappa)``."""
    return apply_D(U, psi, kappa, L, antiperiodic) / (2.0 * kappa)


def dirac_matrix(U: np.ndarray, kappa: float, L, antiperiodic: bool = True) -> sp.csr_matrix:
    """Sparse ``12V x 12V`` matrix of ``D``; dof index ``12 x + 3 spin + colour``."""
    from .lattice import coords, site_index

    V = int(np.prod(L))
    x = coords(L)
    rows, cols, vals = [np.arange(12 * V)], [np.arange(12 * V)], [np.ones(12 * V, np.complex128)]
    sidx = np.arange(4)[:, None] * 3 + np.arange(3)[None, :]  # (spin, colour) -> 3s + c
    for mu in range(4):
        for sign in (+1, -1):
            y = x.copy()
            y[:, mu] = (y[:, mu] + sign) % L[mu]
            yi = site_index(L, y)
            crosses = (x[:, mu] + sign < 0) | (x[:, mu] + sign >= L[mu])
            bc = np.where(crosses & antiperiodic & (mu == 0), -1.0, 1.0)
            if sign > 0:
                S = ONE4 - GAMMA[mu]
                C = U[:, mu]                        # U(x, mu)
            else:
                S = ONE4 + GAMMA[mu]
                C = np.conj(np.swapaxes(U[yi, mu], -1, -2))  # U(x - mu, mu)^dagger
            # entry[(x,s,a),(y,t,b)] = -kappa * bc * S[s,t] * C[x][a,b]
            blk = -kappa * bc[:, None, None, None, None] * S[None, :, None, :, None] * C[:, None, :, None, :]
            r = 12 * np.arange(V)[:, None, None, None, None] + sidx[None, :, :, None, None]
            c = 12 * yi[:, None, None, None, None] + sidx[None, None, None, :, :]
            r, c = np.broadcast_arrays(r, c)
            nz = blk != 0
            rows.append(r[nz])
            cols.append(c[nz])
            vals.append(blk[nz])
    M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(12 * V, 12 * V))
    return M.tocsr()


def gamma5_apply(psi: np.ndarray) -> np.ndarray:
    return np.matmul(GAMMA5, psi)


def gauge_transform_links(U: np.ndarray, g: np.ndarray, L) -> np.ndarray:
    """``U^g(x, mu) = g(x) U(x, mu) g(x + mu)^dagger`` (Sec. 4.2)."""
    from .lattice import neighbour

    out = np.empty_like(U)
    for mu in range(4):
        gn = g[neighbour(L, mu, +1)]
        out[:, mu] = g @ U[:, mu] @ np.conj(np.swapaxes(gn, -1, -2))
    return out


def gauge_transform_spinor(psi: np.ndarray, g: np.ndarray) -> np.ndarray:
    """``(G psi)(x) = g(x) psi(x)`` (colour rotation)."""
    return np.matmul(psi, np.swapaxes(g, -1, -2))


def free_field_momentum_operator(p: np.ndarray, kappa: float) -> np.ndarray:
    """Momentum-space free operator ``D(p) = 1 - 2 kappa sum cos p + 2 i kappa sum gamma sin p``.

    Derived from eq. Dw with ``U = 1`` acting on ``exp(i p x) u``."""
    return (1 - 2 * kappa * np.sum(np.cos(p))) * ONE4 + 2j * kappa * np.einsum("m,mst->st", np.sin(p), GAMMA)


def free_field_logdet(L, kappa: float, antiperiodic: bool = True) -> float:
    """``ln |det D|`` for ``U = 1``: ``6 sum_p ln[(1 - 2k sum cos p)^2 + 4k^2 sum sin^2 p]``
    over the allowed momenta (``p_0 = (2n+1) pi / L_0`` if antiperiodic)."""
    grids = []
    for mu, n in enumerate(L):
        k = np.arange(n)
        grids.append((2 * k + (1 if (antiperiodic and mu == 0) else 0)) * np.pi / n)
    P = np.meshgrid(*grids, indexing="ij")
    a = 1 - 2 * kappa * sum(np.cos(q) for q in P)
    s2 = 4 * kappa**2 * sum(np.sin(q) ** 2 for q in P)
    return float(6 * np.sum(np.log(a**2 + s2)))
