"""Pins of the oracle's recursive domain decomposition (Sec. 3, eq. ddrec; eq. 4step
step 2): the cut field's operator is exactly the direct sum of the outer blocks'
Dirichlet operators taken from the uncut D; the determinant of each outer block factorises
over its sub-blocks and its Schur complement (dense LU on both sides); the outer-geometry
projector keeps P^2 = P and D_wb P = D_wb for the cut operator and gives
det(1 - Q_B) = det(1 - P Q_B); the per-block estimator is the quadratic form of
M_B^dagger M_B - 1 with M_B built densely."""
import numpy as np
import pytest

from oracle import blockdet, dirac, lattice, recursive, schur
from oracle.solvers import dense_logdet
from paper_1204_1306_amd import synth

# outer blocks shorter than the lattice in every direction (so no wrap-around hop lies
# inside one), each holding an even number of sub-blocks per direction
L, B, OUTER, KAPPA = (8, 4, 4, 4), (2, 1, 1, 1), (4, 2, 2, 2), 0.14


def _setup(seed=701):
    U = synth.gauge_field(L, 0.6, seed)
    return U, recursive.cut_links(U, L, OUTER)


def _dofs(mask):
    s = np.nonzero(mask)[0]
    return (12 * s[:, None] + np.arange(12)[None, :]).reshape(-1)


def test_cut_field_is_the_direct_sum_of_outer_block_operators():
    U, Uc = _setup()
    D = dirac.dirac_matrix(U, KAPPA, L).toarray()
    Dc = dirac.dirac_matrix(Uc, KAPPA, L).toarray()
    oid = lattice.block_id(L, OUTER)
    for a in np.unique(oid):
        da = _dofs(oid == a)
        for c in np.unique(oid):
            dc = _dofs(oid == c)
            if a == c:
                assert np.array_equal(Dc[np.ix_(da, dc)], D[np.ix_(da, dc)])
            else:
                assert not np.any(Dc[np.ix_(da, dc)])


def _dhat_blocks(Uc, g):
    A = dirac.dirac_matrix(Uc, KAPPA, L).toarray()
    Bd, Wd = g.dofs(g.black), g.dofs(g.white)
    Q = np.linalg.solve(A[np.ix_(Bd, Bd)], A[np.ix_(Bd, Wd)] @ np.linalg.solve(A[np.ix_(Wd, Wd)], A[np.ix_(Wd, Bd)]))
    return A, Bd, Q


def test_outer_block_determinant_factorises():
    """ln det D_B = sum_{b' in B} ln det D_b' + ln det Dhat_B (eq. ddrec), per outer block B,
    with D_B taken from the uncut operator and Dhat_B from the cut one."""
    U, Uc = _setup()
    g = schur.Geometry(L, B, outer=OUTER)
    D = dirac.dirac_matrix(U, KAPPA, L).toarray()
    _, Bd, Q = _dhat_blocks(Uc, g)
    oid = lattice.block_id(L, OUTER)
    sub = blockdet.block_logdets(U, KAPPA, L, B)
    sub_of = lattice.block_id(L, B)
    black_sites = np.nonzero(g.black)[0]
    for a in np.unique(oid):
        lhs = dense_logdet(D[np.ix_(_dofs(oid == a), _dofs(oid == a))]).real
        rows = np.isin(np.repeat(black_sites, 12), np.nonzero(oid == a)[0])
        dhat = np.eye(rows.sum()) - Q[np.ix_(rows, rows)]
        assert not np.any(Q[np.ix_(rows, ~rows)])  # Q is block-diagonal over outer blocks
        subs = sub[np.unique(sub_of[oid == a])].real.sum()
        assert lhs == pytest.approx(subs + dense_logdet(dhat).real, abs=1e-9)


def test_outer_projector_properties():
    U, Uc = _setup()
    g = schur.Geometry(L, B, outer=OUTER)
    g0 = schur.Geometry(L, B)
    Pm = g.Pm
    assert np.allclose(Pm @ Pm, Pm)
    # range(P_outer) lies in range(P): fewer sites count as block boundaries
    assert np.allclose(g0.Pm @ Pm, Pm)
    assert lattice.dim_projector_closed_form(L, B) > schur.dim_projector(g)
    opc = schur.Operator(g, Uc, KAPPA)
    for e in synth.gaussian_noise(L, 2, 702):
        assert np.abs(opc.D_wb(e) - opc.D_wb(g.project(e))).max() < 1e-13


def test_projected_schur_determinant_per_outer_block():
    """det(1 - Q) = det(1 - P Q) on the black sites of each outer block (eq. detschur)."""
    _, Uc = _setup(703)
    g = schur.Geometry(L, B, outer=OUTER)
    _, Bd, Q = _dhat_blocks(Uc, g)
    P = np.zeros((Bd.size, Bd.size), complex)
    black_sites = np.nonzero(g.black)[0]
    for k, s in enumerate(black_sites):
        P[12 * k:12 * k + 12, 12 * k:12 * k + 12] = np.kron(g.Pm[s], np.eye(3))
    oid = lattice.block_id(L, OUTER)
    for a in np.unique(oid):
        rows = np.isin(np.repeat(black_sites, 12), np.nonzero(oid == a)[0])
        Qa, Pa = Q[np.ix_(rows, rows)], P[np.ix_(rows, rows)]
        n = rows.sum()
        assert dense_logdet(np.eye(n) - Qa).real == pytest.approx(dense_logdet(np.eye(n) - Pa @ Qa).real, abs=1e-10)


def test_block_schur_estimator_is_the_quadratic_form():
    """Delta_B = xi_B^dagger (M_B^dagger M_B - 1) xi_B with M_B = (1 - P Q_B(U'))^-1 (1 - P Q_B(U))
    on range(P) of block B, built densely; the sum over B is the whole-lattice estimator of
    the cut operators."""
    U, Uc = _setup(704)
    Up = synth.proposal(U, L, B, 0.1, 705)
    Upc = recursive.cut_links(Up, L, OUTER)
    g = schur.Geometry(L, B, outer=OUTER)
    opU, opP = schur.Operator(g, Uc, KAPPA), schur.Operator(g, Upc, KAPPA)
    _, Bd, Q = _dhat_blocks(Uc, g)
    _, _, Qp = _dhat_blocks(Upc, g)
    black_sites = np.nonzero(g.black)[0]
    P = np.zeros((Bd.size, Bd.size), complex)
    for k, s in enumerate(black_sites):
        P[12 * k:12 * k + 12, 12 * k:12 * k + 12] = np.kron(g.Pm[s], np.eye(3))
    I = np.eye(Bd.size)
    M = np.linalg.solve(I - P @ Qp, I - P @ Q)
    oid = lattice.block_id(L, OUTER)
    for eta in synth.gaussian_noise(L, 2, 706):
        d = recursive.delta_block_schur(opU, opP, eta)
        xi = g.project(eta).reshape(-1)[Bd]
        y = M @ xi
        for a in np.unique(oid):
            rows = np.isin(np.repeat(black_sites, 12), np.nonzero(oid == a)[0])
            q = np.vdot(y[rows], y[rows]).real - np.vdot(xi[rows], xi[rows]).real
            assert d[a] == pytest.approx(q, rel=1e-9, abs=1e-9)
        assert np.isclose(d.sum(), np.vdot(y, y).real - np.vdot(xi, xi).real, rtol=1e-9, atol=1e-9)
