"""Pins of the oracle's relative gauge fixing (Sec. 4.2, eqs. relgf, choiceg; App. B):
a proposal that is a pure gauge transformation g0 of U on the domain is undone exactly
(g^2 = g0, eq. relgf reaches zero, and every interpolated field of eq. gfparam coincides,
so the interpolated estimator vanishes for any noise); on a generic proposal eq. relgf
falls at every accepted step, theta falls below the stopping value, g stays in SU(3) and
is 1 off the domain; and the variance of the interpolated estimator (dense eigenvalues)
falls when the proposal carries a gauge rotation."""
import numpy as np
import pytest

from oracle import dirac, estimator, gaugefix, schur
from paper_1204_1306_amd import synth

L, B = (8, 4, 4, 4), (4, 4, 4, 4)


def _pure_gauge_pair(seed, eps_g=0.3):
    U = synth.gauge_field(L, 0.6, seed)
    dom = gaugefix.interior_sites(L, B)
    g0 = np.broadcast_to(np.eye(3, dtype=complex), (U.shape[0], 3, 3)).copy()
    g0[dom] = synth.random_su3(np.random.default_rng(seed + 1), int(dom.sum()), eps_g)
    return U, dirac.gauge_transform_links(U, g0, L), g0, dom


def test_pure_gauge_proposal_is_undone():
    U, Up, g0, dom = _pure_gauge_pair(901)
    f0 = gaugefix.relgf_functional(U, Up)
    g, Ug, Upg, hist = gaugefix.relative_gauge_fix(U, Up, L, B, theta_tol=1e-20, max_iter=400)
    f1 = gaugefix.relgf_functional(Ug, Upg)
    assert f0 > 1e-3 and f1 < 1e-12
    assert np.abs(g @ g - g0).max() < 1e-6
    assert np.abs(Ug - Upg).max() < 1e-6
    # all interpolated fields coincide: the estimator with N factors vanishes
    g_ = schur.Geometry(L, (2, 2, 2, 2))
    etas = synth.gaussian_noise(L, 2, 902)
    d = estimator.delta_interpolated(g_, Ug, Upg, 0.13, etas, op="full", tol=1e-13)
    d1 = estimator.delta_interpolated(g_, U, Up, 0.13, etas, op="full", tol=1e-13)
    assert abs(d) < 1e-5 < abs(d1)


def test_descent_on_a_generic_proposal():
    U = synth.gauge_field(L, 0.6, 903)
    Up = synth.proposal(U, L, B, 0.3, 904)
    g, Ug, Upg, hist = gaugefix.relative_gauge_fix(U, Up, L, B, max_iter=500)
    f = [h[0] for h in hist]
    assert all(b <= a + 1e-15 for a, b in zip(f, f[1:]))
    assert hist[-1][1] < 1e-3 and hist[0][1] > 1e-3
    dom = gaugefix.interior_sites(L, B)
    assert np.abs(g[~dom] - np.eye(3)).max() == 0
    assert np.abs(g @ gaugefix.dag(g) - np.eye(3)).max() < 1e-12
    assert np.abs(np.linalg.det(g) - 1).max() < 1e-12
    # the fields are the transforms of the inputs by g and g^-1
    assert np.abs(Ug - dirac.gauge_transform_links(U, g, L)).max() < 1e-12
    assert np.abs(Upg - dirac.gauge_transform_links(Up, gaugefix.dag(g), L)).max() < 1e-12


def test_interpolated_variance_falls():
    """N = 2 factors of the full-operator ratio on a 4^4 lattice with one 4^4 block (16
    domain sites): the stochastic variance sum_i sum_k (lambda_k - 1)^2 of eq. varstoch2
    per factor, from dense eigenvalues, with and without the gauge fixing, for a proposal
    that rotates the domain sites by a gauge transformation and perturbs a few links."""
    L4, B4 = (4, 4, 4, 4), (4, 4, 4, 4)
    U = synth.gauge_field(L4, 0.5, 905)
    dom = gaugefix.interior_sites(L4, B4)
    g0 = np.broadcast_to(np.eye(3, dtype=complex), (U.shape[0], 3, 3)).copy()
    g0[dom] = synth.random_su3(np.random.default_rng(906), int(dom.sum()), 0.4)
    Up = synth.proposal(dirac.gauge_transform_links(U, g0, L4), L4, (2, 2, 2, 2), 0.05, 907)
    _, Ug, Upg, _ = gaugefix.relative_gauge_fix(U, Up, L4, B4, max_iter=500)

    def var(A, Bf, N=2):
        tot = 0.0
        for i in range(N):
            Ui = estimator.interpolated_field(A, Bf, N, i)
            Uj = estimator.interpolated_field(A, Bf, N, i + 1)
            M = np.linalg.solve(dirac.dirac_matrix(Uj, 0.12, L4).toarray(), dirac.dirac_matrix(Ui, 0.12, L4).toarray())
            tot += estimator.exact_moments(np.linalg.eigvalsh(M.conj().T @ M))[2]
        return tot

    v1, vg = var(U, Up), var(Ug, Upg)
    assert vg < 0.5 * v1
