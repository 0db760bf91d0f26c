"""GPU parity of the recursive domain decomposition (Sec. 3, eq. ddrec; the block-Schur
filter, step 2 of eq. 4step) against the oracle: a context with outer (Dirichlet) blocks
applies D with the hops across outer faces removed and the projector of that operator
(both against the oracle to rounding), and psms_logdet_ratio_blocks gives one Delta per
outer block, each within 1e-8 absolute of the oracle's (solves to 1e-12 / 1e-14); their
sum is the Schur estimator of the same context."""
import sys

import numpy as np
import pytest

from oracle import dirac, recursive, schur
from paper_1204_1306_amd import synth

pytestmark = pytest.mark.gpu

L, B, OUTER, KAPPA = (8, 8, 8, 8), (2, 2, 2, 2), (4, 4, 4, 4), 0.15


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def psms():
    from paper_1204_1306_amd import psms as m

    m.load_library()
    return m


def test_outer_block_operator_and_projector(psms):
    say("case outer-block operator 8^4, sub-blocks 2^4, outer blocks 4^4")
    U = synth.gauge_field(L, 0.6, 801)
    Uc = recursive.cut_links(U, L, OUTER)
    psi = synth.gaussian_noise(L, 2, 802)
    ctx = psms.Context(L, B, KAPPA, outer_b=OUTER)
    ctx.gauge_load(0, U)
    out = ctx.apply_dw(0, psi)
    g = schur.Geometry(L, B, outer=OUTER)
    for k in range(2):
        ref = dirac.apply_D(Uc, psi[k], KAPPA, L)
        err = np.linalg.norm(out[k] - ref) / np.linalg.norm(ref)
        say(f"  D_w (cut) field {k}: {err:.2e}")
        assert err < 1e-13
        assert np.abs(ctx.apply_proj(psi[k]) - g.project(psi[k])).max() < 1e-15
    # mixed precision keeps the cut (a zero link is exact in the 12-real form)
    mx = ctx.apply_dw(0, psi, psms.MIXED)
    err = np.linalg.norm(mx[0] - dirac.apply_D(Uc, psi[0], KAPPA, L)) / np.linalg.norm(psi[0])
    say(f"  mixed: {err:.2e}")
    assert err < 2e-6
    ctx.close()


@pytest.mark.parametrize("prec", ["f64", "mixed"])
def test_block_schur_deltas_against_oracle(psms, prec):
    say(f"case per-outer-block Delta ({prec})")
    U = synth.gauge_field(L, 0.6, 811)
    Up = synth.proposal(U, L, OUTER, 0.1, 812)
    eta = synth.gaussian_noise(L, 2, 813)
    ctx = psms.Context(L, B, KAPPA, outer_b=OUTER)
    ctx.gauge_load(0, U)
    ctx.gauge_load(1, Up)
    kw = {} if prec == "f64" else dict(prec=psms.MIXED)
    prm = psms.default_params(tol=1e-12, max_iter=5000, **kw)
    d, st = ctx.logdet_ratio_blocks(0, [1], eta, prm)
    say(f"  stats {st}; shape {d.shape}")
    assert d.shape == (1, 2, 16) and st["converged"] == 1
    g = schur.Geometry(L, B, outer=OUTER)
    opU = schur.Operator(g, recursive.cut_links(U, L, OUTER), KAPPA)
    opP = schur.Operator(g, recursive.cut_links(Up, L, OUTER), KAPPA)
    for j in range(2):
        ref = recursive.delta_block_schur(opU, opP, eta[j])
        err = np.abs(d[0, j] - ref).max()
        say(f"  j={j}: Delta_B in [{ref.min():.4f}, {ref.max():.4f}], max |gpu - oracle| = {err:.2e} (bound 1e-8)")
        assert err < 1e-8
    # the sum over outer blocks is the Schur estimator of the same (cut) operators
    tot, _ = ctx.logdet_ratio(psms.OP_SCHUR, 0, [1], eta, prm)
    assert np.abs(d.sum(axis=2) - tot).max() < 2e-8
    ctx.close()
