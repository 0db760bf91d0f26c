"""Block operators and the Schur complement (Sec. 3 eq. domdec / ddfactor,
Sec. 4.4 eqs. detschur, inverseschur, dimproj).

In the block-major site order (black blocks first) the operator splits as
``D = [[D_bb, D_bw], [D_wb, D_ww]]``. Every piece is an exact sub-matrix of the
one operator ``D``: ``D_bb = D[black, black]`` (which is block diagonal with
the Dirichlet block operators ``D_b``, because two black blocks are never
nearest neighbours), ``D_wb = D[white, black]`` and so on. Here each piece is
written as "restrict the input, apply D, restrict the output".

``Q = D_bb^-1 D_bw D_ww^-1 D_wb`` acts on the black sites, the Schur complement
is ``1 - Q``, and its action on the range of ``P`` is ``1 - PQ``.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import dirac, lattice
from .solvers import DenseLU, cgne


class Geometry:
    """Blocks ``b`` of the Schur complement; with ``outer``, the projector of the
    Dirichlet operator of the outer blocks (recursive decomposition, eq. ddrec), whose
    links across outer faces the caller removes (``recursive.cut_links``)."""

    def __init__(self, L, b, antiperiodic: bool = True, outer=None):
        self.L = tuple(int(v) for v in L)
        self.b = tuple(int(v) for v in b)
        self.outer = tuple(int(v) for v in outer) if outer is not None else None
        self.antiperiodic = antiperiodic
        self.V = lattice.volume(self.L)
        self.black = lattice.is_black(self.L, self.b)
        self.white = ~self.black
        self.block = lattice.block_id(self.L, self.b)
        self.Pm = lattice.projector_matrices(self.L, self.b, self.outer)

    def dofs(self, site_mask: np.ndarray) -> np.ndarray:
        """Flat dof indices (12 x + 3 s + c) of the sites in the mask."""
        s = np.nonzero(site_mask)[0]
        return (12 * s[:, None] + np.arange(12)[None, :]).reshape(-1)

    def restrict(self, psi: np.ndarray, site_mask: np.ndarray) -> np.ndarray:
        out = np.zeros_like(psi)
        out[site_mask] = psi[site_mask]
        return out

    def project(self, psi: np.ndarray) -> np.ndarray:
        return lattice.apply_projector(self.Pm, psi)


class Operator:
    """``D(U)`` with its block decomposition; solves by LU where affordable."""

    def __init__(self, geom: Geometry, U: np.ndarray, kappa: float, direct: bool | None = None):
        self.g = geom
        self.U = U
        self.kappa = kappa
        # dense LU of the whole operator up to 3072 unknowns, of each block up to 3072
        self.direct = (12 * geom.V <= 3072) if direct is None else direct
        self.direct_blocks = 12 * int(np.prod(geom.b)) <= 3072
        self._mat = None
        self._lu = {}

    # --- the operator and its pieces -------------------------------------
    def D(self, psi):
        return dirac.apply_D(self.U, psi, self.kappa, self.g.L, self.g.antiperiodic)

    def Ddag(self, psi):
        # gamma_5 D gamma_5 = D^dagger (gamma_5-hermiticity, checked by the tests)
        return dirac.gamma5_apply(self.D(dirac.gamma5_apply(psi)))

    def piece(self, out_mask, in_mask, psi):
        """``D[out, in]`` applied to psi (zero outside ``out``)."""
        return self.g.restrict(self.D(self.g.restrict(psi, in_mask)), out_mask)

    def D_bb(self, psi):
        return self.piece(self.g.black, self.g.black, psi)

    def D_ww(self, psi):
        return self.piece(self.g.white, self.g.white, psi)

    def D_bw(self, psi):
        return self.piece(self.g.black, self.g.white, psi)

    def D_wb(self, psi):
        return self.piece(self.g.white, self.g.black, psi)

    # --- matrices and factorisations --------------------------------------
    def matrix(self) -> sp.csr_matrix:
        if self._mat is None:
            self._mat = dirac.dirac_matrix(self.U, self.kappa, self.g.L, self.g.antiperiodic)
        return self._mat

    def sub_matrix(self, out_mask, in_mask):
        return self.matrix()[self.g.dofs(out_mask)][:, self.g.dofs(in_mask)]

    def _factor(self, key):
        if key not in self._lu:
            if key == "full":
                self._lu[key] = DenseLU(self.matrix().toarray())
            else:
                # one dense LU per block: D_bb is block diagonal
                self._lu[key] = {int(k): DenseLU(self.sub_matrix(self.g.block == k, self.g.block == k).toarray())
                                 for k in np.unique(self.g.block[self.g.black if key == "black" else self.g.white])}
        return self._lu[key]

    def solve(self, b, tol=1e-14):
        """``D^-1 b`` on the full lattice."""
        if self.direct:
            return self._factor("full").solve(b)
        x, _, _ = cgne(self.D, self.Ddag, b, tol=tol)
        return x

    def solve_colour(self, b, colour: str, tol=1e-14):
        """``D_bb^-1 b`` (colour 'black') or ``D_ww^-1 b`` ('white'); b supported on that colour."""
        mask = self.g.black if colour == "black" else self.g.white
        if self.direct_blocks:
            out = np.zeros_like(b)
            for k, lu in self._factor(colour).items():
                d = self.g.dofs(self.g.block == k)
                out.reshape(-1)[d] = lu.solve(b.reshape(-1)[d])
            return out
        A = (lambda v: self.piece(mask, mask, v))
        Adag = (lambda v: self.g.restrict(self.Ddag(self.g.restrict(v, mask)), mask))
        x, _, _ = cgne(A, Adag, self.g.restrict(b, mask), tol=tol)
        return x

    # --- Schur complement ---------------------------------------------------
    def Q(self, xi):
        """``Q xi = D_bb^-1 D_bw D_ww^-1 D_wb xi`` (xi on black sites)."""
        t = self.D_wb(xi)
        t = self.solve_colour(t, "white")
        t = self.D_bw(t)
        return self.solve_colour(t, "black")

    def schur_apply(self, xi):
        """``(1 - P Q) xi``."""
        return xi - self.g.project(self.Q(xi))

    def schur_complement_apply(self, xi):
        """``(1 - Q) xi`` on the black sites (the Schur complement D-hat of eq. ddfactor)."""
        return self.g.restrict(xi, self.g.black) - self.Q(xi)

    def schur_inverse_direct(self, phi, tol=1e-14):
        """Solve ``(1 - P Q) y = phi`` on the range of P with GMRES (no use of eq. inverseschur)."""
        sel = self.g.dofs(self.g.black)
        n = sel.size

        def mv(v):
            f = np.zeros(12 * self.g.V, np.complex128)
            f[sel] = v
            f = f.reshape(self.g.V, 4, 3)
            return self.schur_apply(f).reshape(-1)[sel]

        A = spla.LinearOperator((n, n), matvec=mv, dtype=np.complex128)
        rhs = phi.reshape(-1)[sel]
        y, info = spla.gmres(A, rhs, rtol=tol, atol=0.0, restart=200, maxiter=50)
        if info != 0:
            raise RuntimeError(f"GMRES did not converge (info={info})")
        out = np.zeros(12 * self.g.V, np.complex128)
        out[sel] = y
        return out.reshape(phi.shape)

    def schur_inverse_formula(self, phi, tol=1e-14):
        """eq. inverseschur: ``(1 - PQ)^-1 phi = phi - P [D^-1 (0 + D_wb phi)]_black``."""
        v = self.D_wb(phi)
        x = self.solve(v, tol=tol)
        return phi - self.g.project(self.g.restrict(x, self.g.black))


def dim_projector(geom: Geometry) -> int:
    """Rank of P counted from its per-site matrices."""
    return int(round(np.sum(np.trace(geom.Pm, axis1=1, axis2=2).real))) * 3
