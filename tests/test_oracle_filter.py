"""Pins of the oracle's filter hierarchy (Sec. 2, eq. 4step, App. A.2, App. C):
* the reverse transition with the noise M xi has exponent -Delta (M -> M^-1, the property
  detailed balance rests on, Sec. 4.2 / App. A.2);
* the stochastic acceptance averaged over the noise is at most the exact one,
  E[min(1, e^-Delta)] <= min(1, det(M^+ M)^-1) (Sec. 4.1), by Monte Carlo on dense M;
* decisions follow u < e^-Delta, a proposal equal to U is accepted at every step, a
  rejected step leaves U, and the blocks that were not accepted keep their links;
* a proposal that changes links between the smallest blocks is refused."""
import numpy as np
import pytest

from oracle import blockdet, dirac, estimator, filter as filt, schur
from paper_1204_1306_amd import synth

L, BS, BO, KAPPA = (8, 4, 4, 4), (2, 2, 2, 2), (4, 4, 4, 4), 0.13


def test_reverse_transition_has_the_opposite_exponent():
    L4, b = (4, 4, 4, 4), (2, 2, 2, 2)
    U = synth.gauge_field(L4, 0.5, 1101)
    Up = synth.proposal(U, L4, b, 0.1, 1102)
    g = schur.Geometry(L4, b)
    opU, opP = schur.Operator(g, U, 0.12), schur.Operator(g, Up, 0.12)
    eta = g.project(synth.gaussian_noise(L4, 1, 1103)[0])
    d = estimator.delta_schur(opU, opP, eta)
    Meta = opP.schur_inverse_direct(opU.schur_apply(eta))
    d_rev = estimator.delta_schur(opP, opU, Meta)
    assert d_rev == pytest.approx(-d, abs=1e-10)


def test_stochastic_acceptance_bounded_by_exact():
    L2 = (2, 2, 2, 2)
    U = synth.gauge_field(L2, 0.5, 1104)
    Up = synth.proposal(U, L2, (2, 2, 2, 2), 0.15, 1105)
    M = np.linalg.solve(dirac.dirac_matrix(Up, 0.12, L2).toarray(), dirac.dirac_matrix(U, 0.12, L2).toarray())
    lam = np.linalg.eigvalsh(M.conj().T @ M)
    exact = min(1.0, float(np.exp(-np.sum(np.log(lam)))))
    n = 20000
    eta = synth.gaussian_noise(L2, n, 1106).reshape(n, -1)
    d = np.sum(np.abs(eta @ M.T) ** 2, axis=1) - np.sum(np.abs(eta) ** 2, axis=1)
    stoch = np.minimum(1.0, np.exp(-d))
    se = stoch.std() / np.sqrt(n)
    # Jensen: min(1, .) is concave and E[e^-Delta] = det(M^+ M)^-1; the gap is many se here
    assert stoch.mean() + 5 * se < exact


def _pair(seed):
    U = synth.gauge_field(L, 0.6, seed)
    Up = synth.proposal(U, L, BS, 0.2, seed + 1)
    return U, Up


def test_decisions_and_merges():
    U, Up = _pair(1110)
    rng = np.random.default_rng(1112)
    nsmall = int(np.prod(np.asarray(L) // np.asarray(BS)))
    nouter = int(np.prod(np.asarray(L) // np.asarray(BO)))
    u1, u2, u3 = rng.uniform(size=nsmall), rng.uniform(size=nouter), 0.3
    eta2, eta3 = synth.gaussian_noise(L, 2, 1113)
    r = filt.filter_step(U, Up, KAPPA, L, BS, BO, u1, u2, u3, eta2, eta3)
    assert np.array_equal(r["accept1"], u1 < np.exp(-r["delta1"]))
    assert np.array_equal(r["accept2"], u2 < np.exp(-r["delta2"]))
    assert r["accept3"] == (u3 < np.exp(-r["delta3"]))
    assert 0 < r["accept1"].sum() < nsmall  # the seeds give a mix
    # exact step: the exponent is the block-determinant ratio
    assert np.allclose(r["dS1"], blockdet.block_filter_delta(U, Up, KAPPA, L, BS))
    # links of blocks not accepted keep U; accepted ones take U'
    lb = filt.link_blocks(L, BS)
    for k in range(nsmall):
        m = lb == k
        ref = Up if r["accept1"][k] else U
        assert np.array_equal(r["U1"][m], ref[m])
    # a proposal equal to U passes every step
    same = filt.filter_step(U, U, KAPPA, L, BS, BO, u1, u2, 0.999, eta2, eta3)
    assert same["accept1"].all() and same["accept2"].all() and same["accept3"]
    assert np.abs(same["delta2"]).max() < 1e-9 and abs(same["delta3"]) < 1e-9
    # a rejected last step leaves U
    rej = filt.filter_step(U, Up, KAPPA, L, BS, BO, u1, u2, 1.0 - 1e-16, eta2, eta3)
    if not rej["accept3"]:
        assert np.array_equal(rej["U3"], U)


def test_beta_moves_the_block_term_between_steps():
    U, Up = _pair(1120)
    nsmall = int(np.prod(np.asarray(L) // np.asarray(BS)))
    nouter = int(np.prod(np.asarray(L) // np.asarray(BO)))
    zeros1, zeros2 = np.zeros(nsmall), np.zeros(nouter)
    eta2, eta3 = synth.gaussian_noise(L, 2, 1121)
    r = filt.filter_step(U, Up, KAPPA, L, BS, BO, zeros1, zeros2, 0.0, eta2, eta3, beta=(0.5, 0.25, 0.25))
    assert np.allclose(r["delta1"], 0.5 * r["dS1"])
    # u = 0 accepts everything, so U1 = U' and step 2 sees the block term of all sub-blocks
    per_outer = filt._small_to_outer(L, BS, BO)
    assert np.allclose(r["delta2"] - r["dS2"], 0.25 * np.bincount(per_outer, weights=r["dS1"]))
    assert r["delta3"] - r["dS3"] == pytest.approx(0.25 * r["dS1"].sum())


def test_proposal_across_blocks_is_refused():
    U, Up = _pair(1130)
    bad = Up.copy()
    lb = filt.link_blocks(L, BS)
    x = np.argwhere(lb < 0)[0]
    bad[x[0], x[1]] = synth.random_su3(np.random.default_rng(1131), 1, 0.2)[0] @ U[x[0], x[1]]
    with pytest.raises(ValueError):
        filt.filter_step(U, bad, KAPPA, L, BS, BO, np.zeros(64), np.zeros(8), 0.0, *synth.gaussian_noise(L, 2, 1))
