"""Pins of the oracle's exact block determinants (Sec. 3, eq. ddfactor, eq. 4step step 1)
against facts fixed by the mathematics: another algorithm (the product of eigenvalues),
blocks whose determinant is 1 for any links, gauge invariance, realness from
gamma5-hermiticity, the even-odd reduction inside a block, and the factorisation
det D = prod_b det D_b det Dhat."""
import numpy as np
import pytest

from oracle import blockdet, dirac, lattice, schur
from oracle.solvers import dense_logdet
from paper_1204_1306_amd import synth


def _block_matrix(U, kappa, L, b, k):
    D = dirac.dirac_matrix(U, kappa, L).tocsr()
    s = np.nonzero(lattice.block_id(L, b) == k)[0]
    d = (12 * s[:, None] + np.arange(12)[None, :]).reshape(-1)
    return D[d][:, d].toarray(), s


def _wrap(z):
    return np.angle(np.exp(1j * z))


def test_block_logdet_equals_sum_of_log_eigenvalues():
    """LU (slogdet) against the eigenvalues (QR iterations) of the same 192-dim block."""
    L, b = (4, 4, 4, 4), (2, 2, 2, 2)
    U = synth.gauge_field(L, 0.6, 501)
    ld = blockdet.block_logdets(U, 0.14, L, b)
    for k in (0, 5, 13):
        A, _ = _block_matrix(U, 0.14, L, b, k)
        lam = np.linalg.eigvals(A)
        ref = np.sum(np.log(lam))
        assert ld[k].real == pytest.approx(ref.real, abs=1e-10)
        assert abs(_wrap(ld[k].imag - ref.imag)) < 1e-8


@pytest.mark.parametrize("L,b", [((8, 4, 4, 4), (4, 1, 1, 1)), ((4, 4, 4, 8), (1, 1, 1, 4)),
                                 ((4, 4, 4, 4), (1, 2, 1, 1))])
def test_chain_blocks_have_unit_determinant(L, b):
    """A block that extends in one direction only (shorter than the lattice, so it holds no
    wrap-around hop) is an open chain whose hops go forward on the spin space of
    (1 - gamma_mu)/2 and backward on that of (1 + gamma_mu)/2: in that spin basis the
    matrix is triangular with unit diagonal, so det D_b = 1 for any links."""
    U = synth.gauge_field(L, 0.9, 502)
    ld = blockdet.block_logdets(U, 0.2, L, b)
    assert np.abs(ld).max() < 1e-12


def test_block_determinants_gauge_invariant():
    L, b = (4, 4, 4, 4), (2, 2, 2, 2)
    U = synth.gauge_field(L, 0.6, 503)
    g = synth.gauge_transform(504, int(np.prod(L)))
    a = blockdet.block_logdets(U, 0.13, L, b)
    c = blockdet.block_logdets(dirac.gauge_transform_links(U, g, L), 0.13, L, b)
    assert np.abs(a.real - c.real).max() < 1e-10
    assert np.abs(_wrap(a.imag - c.imag)).max() < 1e-8


def test_block_determinants_are_real():
    """gamma5 D_b gamma5 = D_b^dagger, so det D_b is real: phase 0 or pi."""
    L, b = (4, 4, 4, 4), (2, 2, 2, 2)
    U = synth.gauge_field(L, 0.8, 505)
    ph = blockdet.block_logdets(U, 0.16, L, b).imag
    assert np.all(np.minimum(np.abs(_wrap(ph)), np.abs(_wrap(ph - np.pi))) < 1e-9)


def test_even_odd_reduction_inside_a_block():
    """With the sites of a block ordered even then odd, D_b = [[1, A_eo], [A_oe, 1]], so
    det D_b = det(1 - A_eo A_oe) (eq. ddfactor with blocks of one site, inside the block):
    the form the GPU factorises."""
    L, b = (8, 4, 4, 4), (4, 2, 2, 2)
    U = synth.gauge_field(L, 0.6, 506)
    ld = blockdet.block_logdets(U, 0.15, L, b)
    par = lattice.parity(L)
    for k in (0, 3):
        A, s = _block_matrix(U, 0.15, L, b, k)
        ev = np.repeat(par[s] == 0, 12)
        Aee, Aoo = A[np.ix_(ev, ev)], A[np.ix_(~ev, ~ev)]
        assert np.abs(Aee - np.eye(Aee.shape[0])).max() == 0
        assert np.abs(Aoo - np.eye(Aoo.shape[0])).max() == 0
        red = np.eye(Aee.shape[0]) - A[np.ix_(ev, ~ev)] @ A[np.ix_(~ev, ev)]
        ref = dense_logdet(red)
        assert ld[k].real == pytest.approx(ref.real, abs=1e-10)


def test_factorisation_with_the_block_determinants():
    """ln det D = sum_b ln det D_b + ln det Dhat (eq. ddfactor), Dhat dense on the black sites."""
    L, b = (4, 4, 4, 4), (2, 2, 2, 2)
    U = synth.gauge_field(L, 0.6, 507)
    kappa = 0.14
    g = schur.Geometry(L, b)
    A = dirac.dirac_matrix(U, kappa, L).toarray()
    Bd, Wd = g.dofs(g.black), g.dofs(g.white)
    dhat = np.eye(Bd.size) - np.linalg.solve(A[np.ix_(Bd, Bd)], A[np.ix_(Bd, Wd)] @ np.linalg.solve(A[np.ix_(Wd, Wd)],
                                                                                                A[np.ix_(Wd, Bd)]))
    lhs = dense_logdet(A).real
    rhs = blockdet.block_logdets(U, kappa, L, b).real.sum() + dense_logdet(dhat).real
    assert lhs == pytest.approx(rhs, abs=1e-9)


def test_block_filter_delta():
    """Delta_b = -2 (ln|det D_b(U')| - ln|det D_b(U)|): zero on blocks the proposal leaves
    alone, and the full-lattice exponent splits into the block part plus the Schur part."""
    L, b = (4, 4, 4, 4), (2, 2, 2, 2)
    kappa = 0.13
    U = synth.gauge_field(L, 0.6, 508)
    Up = U.copy()
    bid = lattice.block_id(L, b)
    rng = np.random.default_rng(509)
    for k in (2, 9):  # change intra-block links of two blocks only
        s = np.nonzero(bid == k)[0][:3]
        Up[s, 3] = synth.random_su3(rng, len(s), 0.3) @ U[s, 3]
    d = blockdet.block_filter_delta(U, Up, kappa, L, b)
    others = np.setdiff1d(np.arange(d.size), [2, 9])
    assert np.abs(d[others]).max() < 1e-12
    assert np.abs(d[[2, 9]]).min() > 1e-4
