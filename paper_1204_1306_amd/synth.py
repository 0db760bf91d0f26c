"""Seeded synthetic inputs: gauge fields, block-local proposals and Gaussian noise.

This module only draws inputs. It holds none of the method's arithmetic (no
Dirac operator, no projector, no block operator), so that both the CPU
oracle and the HIP path can consume exactly the same arrays.

Conventions shared with every consumer (boundary layout):

* lattice sizes ``L = (L0, L1, L2, L3)``, direction 0 is time;
* site index ``((x0*L1 + x1)*L2 + x2)*L3 + x3``;
* gauge field ``U[V, 4, 3, 3]`` complex128, ``U[x, mu]`` is the link from
  ``x`` to ``x + mu``;
* spinor fields ``psi[V, 4, 3]`` (spin, colour) complex128.

Link recipe. ``U = exp(i eps H)`` with ``H = sum_a h_a lambda_a / 2``,
``h_a ~ N(0, 1)`` (unit-Gaussian su(3) coordinates in the Gell-Mann
normalisation ``Tr T_a T_b = delta_ab / 2``), exponentiated by a Hermitian
eigendecomposition, then re-unitarised (Gram-Schmidt on rows 0 and 1, row 2
is the complex conjugate of their cross product). Random numbers are drawn
site by site in lexicographic order, then direction, then the 8 coordinates.

Proposal recipe. A proposal ``U'`` changes only links inside blocks: either
the links that have both endpoints in one block and at most one endpoint on
its boundary (the active links of the domain-decomposed update, Sec. 3 of
the paper), or, where that set is empty (blocks of extent 2), every link with
both endpoints in one block. A changed link becomes
``reunitarise(exp(i eps' H') U)`` with ``H'`` drawn as above. ``eps'`` is
either one number or drawn per block from a uniform range, first, in block
lexicographic order.

Noise recipe. Complex Gaussian with density ``exp(-|eta|^2)`` per complex
component, i.e. real and imaginary parts ``N(0, 1/2)`` (the pseudofermion
measure of App. A.2 of the paper).
"""
from __future__ import annotations

import numpy as np

_GELL_MANN = np.zeros((8, 3, 3), dtype=np.complex128)
_GELL_MANN[0][0, 1] = _GELL_MANN[0][1, 0] = 1
_GELL_MANN[1][0, 1], _GELL_MANN[1][1, 0] = -1j, 1j
_GELL_MANN[2][0, 0], _GELL_MANN[2][1, 1] = 1, -1
_GELL_MANN[3][0, 2] = _GELL_MANN[3][2, 0] = 1
_GELL_MANN[4][0, 2], _GELL_MANN[4][2, 0] = -1j, 1j
_GELL_MANN[5][1, 2] = _GELL_MANN[5][2, 1] = 1
_GELL_MANN[6][1, 2], _GELL_MANN[6][2, 1] = -1j, 1j
_GELL_MANN[7] = np.diag([1, 1, -2]) / np.sqrt(3)


def lattice_volume(L) -> int:
    return int(np.prod(L))


def reunitarise(M: np.ndarray) -> np.ndarray:
    """Project ``[..., 3, 3]`` matrices onto SU(3): Gram-Schmidt rows 0, 1;
    row 2 = conj(row0 x row1)."""
    r0 = M[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = M[..., 1, :]
    r1 = r1 - np.sum(r0.conj() * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.cross(r0, r1).conj()
    return np.stack([r0, r1, r2], axis=-2)


def _expi_hermitian(H: np.ndarray, eps: float | np.ndarray) -> np.ndarray:
    w, v = np.linalg.eigh(H)
    ph = np.exp(1j * np.asarray(eps)[..., None] * w)
    return (v * ph[..., None, :]) @ np.swapaxes(v.conj(), -1, -2)


def random_su3(rng: np.random.Generator, n: int, eps) -> np.ndarray:
    """``n`` matrices ``reunitarise(exp(i eps H))``; ``eps`` scalar or [n]."""
    h = rng.standard_normal((n, 8))
    H = np.einsum("na,aij->nij", h, _GELL_MANN) / 2.0
    return reunitarise(_expi_hermitian(H, np.broadcast_to(np.asarray(eps, float), (n,))))


def gauge_field(L, eps: float, seed: int) -> np.ndarray:
    """Seeded SU(3) gauge field ``U[V, 4, 3, 3]``."""
    V = lattice_volume(L)
    rng = np.random.default_rng(seed)
    return random_su3(rng, V * 4, eps).reshape(V, 4, 3, 3)


def unit_gauge_field(L) -> np.ndarray:
    V = lattice_volume(L)
    U = np.zeros((V, 4, 3, 3), np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1
    return U


def coords(L) -> np.ndarray:
    """``[V, 4]`` integer coordinates in the site order."""
    g = np.meshgrid(*[np.arange(n) for n in L], indexing="ij")
    return np.stack([a.reshape(-1) for a in g], axis=1)


def intra_block_link_sets(L, b):
    """Boolean masks ``[V, 4]``: (active, intra). ``intra``: both link endpoints
    in one block. ``active``: intra and at most one endpoint on the block's
    boundary (a site is on the boundary when one of its nearest neighbours
    lies in another block)."""
    L = np.asarray(L)
    b = np.asarray(b)
    x = coords(L)
    loc = x % b
    on_bnd = np.any((loc == 0) | (loc == b - 1), axis=1)  # [V]
    V = x.shape[0]
    active = np.zeros((V, 4), bool)
    intra = np.zeros((V, 4), bool)
    for mu in range(4):
        y = x.copy()
        y[:, mu] = (y[:, mu] + 1) % L[mu]
        same = np.all(x // b == y // b, axis=1)
        yi = ((y[:, 0] * L[1] + y[:, 1]) * L[2] + y[:, 2]) * L[3] + y[:, 3]
        intra[:, mu] = same
        active[:, mu] = same & ~(on_bnd & on_bnd[yi])
    return active, intra


def block_index(L, b) -> np.ndarray:
    """Lexicographic block index of each site (block coordinate x // b)."""
    L = np.asarray(L)
    b = np.asarray(b)
    B = coords(L) // b
    NB = L // b
    return ((B[:, 0] * NB[1] + B[:, 1]) * NB[2] + B[:, 2]) * NB[3] + B[:, 3]


def proposal(U: np.ndarray, L, b, eps_prime, seed: int) -> np.ndarray:
    """Block-local proposal ``U'`` (see module docstring).

    ``eps_prime`` is a float, or a pair ``(lo, hi)`` for one uniform draw per
    block (drawn first, in block lexicographic order)."""
    rng = np.random.default_rng(seed)
    L = np.asarray(L)
    b = np.asarray(b)
    nblk = int(np.prod(L // b))
    if isinstance(eps_prime, (tuple, list)):
        eps_b = rng.uniform(eps_prime[0], eps_prime[1], size=nblk)
    else:
        eps_b = np.full(nblk, float(eps_prime))
    active, intra = intra_block_link_sets(L, b)
    sel = active if active.any() else intra
    site, mu = np.nonzero(sel)
    eps_link = eps_b[block_index(L, b)[site]]
    R = random_su3(rng, site.size, eps_link)
    Up = U.copy()
    Up[site, mu] = reunitarise(R @ U[site, mu])
    return Up


def gaussian_noise(L, n: int, seed: int) -> np.ndarray:
    """``n`` complex Gaussian spinor fields ``[n, V, 4, 3]``, Re/Im ~ N(0, 1/2)."""
    V = lattice_volume(L)
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n, V, 4, 3, 2))
    return (z[..., 0] + 1j * z[..., 1]) / np.sqrt(2.0)


def gauge_transform(rng_seed: int, V: int, eps: float = 1.0) -> np.ndarray:
    """Random SU(3) gauge transformation ``g[V, 3, 3]`` (input for covariance tests)."""
    return random_su3(np.random.default_rng(rng_seed), V, eps)


# Workloads of the paper's shapes (lattice, blocks, kappa, link spread, proposal
# spread, numbers of proposals and noise vectors, seeds).
WORKLOADS = {
    "4x4x4x4": dict(L=(4, 4, 4, 4), b=(2, 2, 2, 2), kappa=0.12, eps=0.5, eps_prime=0.05,
        nprop=1, nnoise=4, seed_U=1001, seed_Up=1101, seed_noise=1501, tol=1e-12),
    "8x8x8x8": dict(L=(8, 8, 8, 8), b=(4, 4, 4, 4), kappa=0.15, eps=0.6, eps_prime=0.05,
        nprop=1, nnoise=16, seed_U=2001, seed_Up=2101, seed_noise=2501, tol=1e-10),
    "16x16x16x16-batched": dict(L=(16, 16, 16, 16), b=(4, 4, 4, 4), kappa=0.155, eps=0.6, eps_prime=(0.02, 0.1),
        nprop=8, nnoise=64, seed_U=3001, seed_Up=3101, seed_noise=3501, tol=1e-10),
    "16x16x16x16-network": dict(L=(16, 16, 16, 16), b=(4, 4, 4, 4), kappa=0.157, eps=0.6, eps_prime=(0.02, 0.1),
        nprop=1, nnoise=8, seed_U=4999, seed_Up=4899, seed_noise=4501, tol=1e-10),
    "32x32x32x32": dict(L=(32, 32, 32, 32), b=(8, 8, 8, 8), kappa=0.1575, eps=0.6, eps_prime=(0.02, 0.1),
        nprop=4, nnoise=32, seed_U=5001, seed_Up=5101, seed_noise=5501, tol=1e-10,
        sap_b=(4, 4, 4, 4)),
}


def workload_inputs(name: str, nprop: int | None = None, nnoise: int | None = None):
    """Gauge field, proposals and raw noise for a named workload."""
    w = dict(WORKLOADS[name])
    nprop = w["nprop"] if nprop is None else nprop
    nnoise = w["nnoise"] if nnoise is None else nnoise
    U = gauge_field(w["L"], w["eps"], w["seed_U"])
    Ups = [proposal(U, w["L"], w["b"], w["eps_prime"], w["seed_Up"] + p) for p in range(nprop)]
    eta = gaussian_noise(w["L"], nnoise, w["seed_noise"])
    return w, U, Ups, eta
