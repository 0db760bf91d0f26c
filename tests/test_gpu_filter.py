"""GPU parity of the filter hierarchy of one recursion level (Sec. 2 eq. hierarchy,
Sec. 3 eq. 4step, App. A.2 eq. paccstoch, App. C) against the oracle's: the same
proposal, uniforms and noise give the same decisions at every step and the exponents
within 1e-8 (exact block term: 1e-9; stochastic steps: solves to 1e-12); the state it
leaves is the oracle's; beta moves the exact block term between the steps; a proposal
that changes links between the smallest blocks is refused."""
import sys

import numpy as np
import pytest

from oracle import filter as filt
from paper_1204_1306_amd import synth

pytestmark = pytest.mark.gpu

L, BS, BO, KAPPA = (8, 8, 8, 8), (2, 2, 2, 2), (4, 4, 4, 4), 0.15


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def psms():
    from paper_1204_1306_amd import psms as m

    m.load_library()
    return m


@pytest.mark.parametrize("beta", [(1.0, 0.0, 0.0), (0.6, 0.3, 0.1)])
def test_filter_step_matches_oracle(psms, beta):
    say(f"case filter hierarchy 8^4, blocks 2^4 in 4^4, beta {beta}")
    U = synth.gauge_field(L, 0.6, 1201)
    Up = synth.proposal(U, L, BS, 0.15, 1202)
    nsmall = int(np.prod(np.asarray(L) // np.asarray(BS)))
    nouter = int(np.prod(np.asarray(L) // np.asarray(BO)))
    u = np.random.default_rng(1203).uniform(size=nsmall + nouter + 1)
    eta = synth.gaussian_noise(L, 2, 1204)
    inner = psms.Context(L, BS, KAPPA, outer_b=BO)
    outer = psms.Context(L, BO, KAPPA)
    for c in (inner, outer):
        c.gauge_load(0, U)
        c.gauge_load(1, Up)
    solve = psms.default_params(tol=1e-12, max_iter=5000)
    r = psms.filter_step(inner, outer, 0, 1, u, eta, beta=beta, solve=solve, slot_out=5)
    ref = filt.filter_step(U, Up, KAPPA, L, BS, BO, u[:nsmall], u[nsmall:nsmall + nouter], u[-1], eta[0], eta[1],
                           beta=beta)
    say(f"  accepted: step 1 {r['accept1'].sum()}/{nsmall}, step 2 {r['accept2'].sum()}/{nouter}, step 3 "
        f"{r['accept3']}; Delta3 {r['delta3']:.10f} oracle {ref['delta3']:.10f}")
    e1 = np.abs(r["delta1"] - ref["delta1"]).max()
    e2 = np.abs(r["delta2"] - ref["delta2"]).max()
    e3 = abs(r["delta3"] - ref["delta3"])
    say(f"  |dDelta| step 1 {e1:.2e}, step 2 {e2:.2e}, step 3 {e3:.2e}")
    assert e1 < 1e-9 and e2 < 1e-8 and e3 < 1e-8
    # decisions: identical unless a threshold lies within the exponents' error of u
    m1 = np.abs(np.exp(-ref["delta1"]) - u[:nsmall]) > 1e-8
    m2 = np.abs(np.exp(-ref["delta2"]) - u[nsmall:nsmall + nouter]) > 1e-7
    assert np.array_equal(r["accept1"][m1], ref["accept1"][m1]) and m1.sum() > nsmall - 2
    assert np.array_equal(r["accept2"][m2], ref["accept2"][m2]) and m2.sum() > nouter - 2
    assert r["accept3"] == ref["accept3"]
    assert 0 < r["accept1"].sum() < nsmall
    # the state left in slot 5 is the oracle's
    psi = synth.gaussian_noise(L, 1, 1205)
    outer.gauge_load(6, ref["U3"])
    assert np.abs(outer.apply_dw(5, psi) - outer.apply_dw(6, psi)).max() < 1e-14
    inner.close()
    outer.close()


def test_filter_step_refuses_nonlocal_proposals(psms):
    U = synth.gauge_field(L, 0.6, 1211)
    Up = U.copy()
    lb = filt.link_blocks(L, BS)
    x = np.argwhere(lb < 0)[0]
    Up[x[0], x[1]] = synth.random_su3(np.random.default_rng(1213), 1, 0.2)[0] @ U[x[0], x[1]]
    inner = psms.Context(L, BS, KAPPA, outer_b=BO)
    outer = psms.Context(L, BO, KAPPA)
    for c in (inner, outer):
        c.gauge_load(0, U)
        c.gauge_load(1, Up)
    n = int(np.prod(np.asarray(L) // np.asarray(BS))) + int(np.prod(np.asarray(L) // np.asarray(BO))) + 1
    with pytest.raises(psms.PsmsError) as e:
        psms.filter_step(inner, outer, 0, 1, np.zeros(n), synth.gaussian_noise(L, 2, 1214))
    assert e.value.status == -1
    inner.close()
    outer.close()
