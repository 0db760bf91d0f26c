"""GPU parity of the relative gauge fixing (Sec. 4.2, App. B) and of the gauge-fixed
interpolated estimator (Sec. 4.3, eqs. gfparam, staccN) against the oracle:
* a pure-gauge proposal U' = U^g0 (g0 on the block-interior sites) is undone: g^2 = g0,
  eq. relgf reaches zero and the two fixed fields coincide;
* on a generic proposal, twelve steps of the descent give the oracle's g to 1e-10 (both
  FP64, the same accept/reject decisions), and the default stopping rule the oracle's g;
* the interpolated estimator (N = 2 and 3) on the fixed pair matches the oracle's on the
  oracle's fixed pair within 1e-8 (solves to 1e-12 / 1e-14), for SCHUR and FULL."""
import sys

import numpy as np
import pytest

from oracle import dirac, estimator, gaugefix, schur
from paper_1204_1306_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def psms():
    from paper_1204_1306_amd import psms as m

    m.load_library()
    return m


def test_pure_gauge_proposal_is_undone(psms):
    L, b = (8, 8, 8, 8), (4, 4, 4, 4)
    say("case gauge fixing: pure-gauge proposal 8^4")
    U = synth.gauge_field(L, 0.6, 1001)
    dom = gaugefix.interior_sites(L, b)
    g0 = np.broadcast_to(np.eye(3, dtype=complex), (U.shape[0], 3, 3)).copy()
    g0[dom] = synth.random_su3(np.random.default_rng(1002), int(dom.sum()), 0.3)
    Up = dirac.gauge_transform_links(U, g0, L)
    ctx = psms.Context(L, b, 0.15)
    ctx.gauge_load(0, U)
    ctx.gauge_load(1, Up)
    g, st = ctx.relative_gauge_fix(0, 1, 2, 3, want_g=True, theta_tol=1e-20, max_iter=400)
    say(f"  stats {st}; |g^2 - g0| = {np.abs(g @ g - g0).max():.2e}")
    assert st["functional_start"] > 1e-3 and st["functional_end"] < 1e-12
    assert np.abs(g @ g - g0).max() < 1e-6
    psi = synth.gaussian_noise(L, 1, 1003)
    assert np.abs(ctx.apply_dw(2, psi) - ctx.apply_dw(3, psi)).max() < 1e-6
    ctx.close()


def test_descent_matches_oracle(psms):
    L, b = (8, 8, 8, 8), (4, 4, 4, 4)
    U = synth.gauge_field(L, 0.6, 1011)
    Up = synth.proposal(U, L, b, 0.3, 1012)
    ctx = psms.Context(L, b, 0.15)
    ctx.gauge_load(0, U)
    ctx.gauge_load(1, Up)
    for kw in (dict(max_iter=12, theta_tol=0.0), dict()):
        say(f"case gauge fixing against the oracle {kw}")
        g, st = ctx.relative_gauge_fix(0, 1, 2, 3, want_g=True, **kw)
        gr, Ugr, Upgr, hist = gaugefix.relative_gauge_fix(U, Up, L, b, **kw)
        err = np.abs(g - gr).max()
        say(f"  gpu {st}; oracle {len(hist)} checks, final {hist[-1]}; |g - g_oracle| = {err:.2e}")
        assert err < 1e-10
        assert st["functional_end"] == pytest.approx(gaugefix.relgf_functional(Ugr, Upgr), abs=1e-13)
    ctx.close()


@pytest.mark.parametrize("op", ["schur", "full"])
def test_gauge_fixed_interpolated_estimator(psms, op):
    w, U, Ups, _ = synth.workload_inputs("8x8x8x8", nprop=1)
    L, b, kappa = w["L"], w["b"], w["kappa"]
    Up = Ups[0]
    _, Ug, Upg, _ = gaugefix.relative_gauge_fix(U, Up, L, b)
    ctx = psms.Context(L, b, kappa)
    ctx.gauge_load(0, U)
    ctx.gauge_load(1, Up)
    _, st = ctx.relative_gauge_fix(0, 1, 2, 3)
    say(f"case gauge-fixed interpolation ({op}); fix {st}")
    g = schur.Geometry(L, b)
    for N in (2, 3):
        eta = synth.gaussian_noise(L, N * 2, 1021 + N)
        d, sd = ctx.logdet_ratio(psms.OP_SCHUR if op == "schur" else psms.OP_FULL, 2, [3], eta,
                                 psms.default_params(tol=1e-12, max_iter=5000), n_interp=N)
        for j in range(2):
            ref = estimator.delta_interpolated(g, Ug, Upg, kappa, [eta[i * 2 + j] for i in range(N)], op=op)
            err = abs(d[0, j] - ref)
            say(f"  N={N} j={j}: gpu {d[0, j]:.12f} oracle {ref:.12f} |diff| {err:.2e} (bound 1e-8)")
            assert err < 1e-8
    ctx.close()
