"""GPU checks at the full workload sizes, in the launch configurations the
benchmark uses (all noise vectors and proposals of a workload in one call).

The oracle cannot compute every Delta at 16^4 or 32^4 in seconds, so:
* at 8^4 the oracle computes a sample of the Deltas outright;
* at 16^4 and 32^4, for a sample of (proposal, noise) pairs, Delta is rebuilt
  from single GPU sub-solves (D_ww^-1, D_bb^-1, the full solve of the Schur
  inverse) each of which the oracle certifies through its own operator (true
  residual <= tolerance), and the oracle composes the rest (hops, projector,
  norms). The batched Deltas must agree with that within the error bound that
  the solve tolerance implies (|dDelta| <~ 2 |xi|^2 * cond * tol);
* every batched Delta is compared between the BF16/FP32-inner and the FP64
  solver (same bound), and the true residual the library reports must meet the
  tolerance.
"""
import sys

import numpy as np
import pytest

import bench
from oracle import schur
from paper_1204_1306_amd import synth

pytestmark = pytest.mark.gpu

COND = 50.0  # generous condition-number allowance in the Delta bound


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def resid(apply, x, b):
    return float(np.linalg.norm((b - apply(x)).ravel()) / np.linalg.norm(b.ravel()))


@pytest.fixture(scope="module")
def psms():
    from paper_1204_1306_amd import psms as m

    m.load_library()
    return m


def _load(psms, w, U, Ups):
    ctx = psms.Context(w["L"], w["b"], w["kappa"], sap_b=w.get("sap_b"))
    ctx.gauge_load(0, U)
    for p, Up in enumerate(Ups):
        ctx.gauge_load(1 + p, Up)
    return ctx


def _certified_delta(psms, ctx, w, U, Up, slot_up, eta, tol):
    """Delta = |(1-PQ')^-1 (1-PQ) xi|^2 - |xi|^2 from GPU sub-solves, each certified
    by the oracle's operator; the oracle applies hops, P and norms."""
    g = schur.Geometry(w["L"], w["b"])
    opU = schur.Operator(g, U, w["kappa"], direct=False)
    opP = schur.Operator(g, Up, w["kappa"], direct=False)
    prm = psms.default_params(tol=tol, max_iter=5000)
    xi = g.project(eta)
    t = opU.D_wb(xi)
    w1, _ = ctx.solve_block(0, 1, t, prm)  # D_ww^-1
    r1 = resid(opU.D_ww, w1, t)
    t2 = opU.D_bw(w1)
    w2, _ = ctx.solve_block(0, 0, t2, prm)  # D_bb^-1
    r2 = resid(opU.D_bb, w2, t2)
    y = xi - g.project(w2)
    v = opP.D_wb(y)
    x, _ = ctx.solve(slot_up, v, prm)  # eq. inverseschur: one full solve with U'
    r3 = resid(opP.D, x, v)
    z = y - g.project(g.restrict(x, g.black))
    say(f"  certified sub-solves: residuals {r1:.2e} {r2:.2e} {r3:.2e}")
    assert max(r1, r2, r3) <= tol * 1.01
    return float(np.vdot(z, z).real - np.vdot(xi, xi).real), float(np.vdot(xi, xi).real)


def test_8x4_bench_configuration_against_oracle(psms):
    """8^4, 4^4 blocks, kappa 0.15, 16 noise vectors in one call, in the benchmark's
    mixed and plain modes; the oracle computes Delta for 3 of the 16 noise vectors."""
    w, U, Ups, eta = synth.workload_inputs("8x8x8x8")
    ctx = _load(psms, w, U, Ups)
    ctx.autotune(0, None)
    d_mx, s_mx = ctx.logdet_ratio(psms.OP_SCHUR, 0, [1], eta, bench.mode_params(psms, "mixed", w["tol"], "8x8x8x8"))
    d_64, s_64 = ctx.logdet_ratio(psms.OP_SCHUR, 0, [1], eta, bench.mode_params(psms, "plain", w["tol"], "8x8x8x8"))
    say(" mixed", s_mx, "plain", s_64)
    assert s_mx["converged"] and s_64["converged"]
    assert s_mx["true_rel_residual"] <= w["tol"] and s_64["true_rel_residual"] <= w["tol"]
    g = schur.Geometry(w["L"], w["b"])
    xi2 = np.array([np.vdot(g.project(e), g.project(e)).real for e in eta])
    bound = 2 * xi2 * w["tol"] * COND
    assert np.all(np.abs(d_mx[0] - d_64[0]) < bound)
    opU = schur.Operator(g, U, w["kappa"])
    opP = schur.Operator(g, Ups[0], w["kappa"])
    from oracle import estimator

    for j in (0, 7, 15):
        ref = estimator.delta_schur(opU, opP, eta[j])
        say(f"  j={j}: gpu mixed {d_mx[0, j]:.12f} plain {d_64[0, j]:.12f} oracle {ref:.12f} bound {bound[j]:.1e}")
        assert abs(d_mx[0, j] - ref) < bound[j]
        assert abs(d_64[0, j] - ref) < bound[j]


def test_16x4_full_batch(psms):
    """16^4, 4^4 blocks, kappa 0.155, 8 proposals (eps' per block in [0.02, 0.1]) x 64
    noise: the whole batch with BF16 inner storage and with plain FP64; two sampled
    pairs rebuilt from oracle-certified sub-solves."""
    w, U, Ups, eta = synth.workload_inputs("16x16x16x16-batched")
    ctx = _load(psms, w, U, Ups)
    ctx.autotune(0, None)
    slots = list(range(1, 1 + len(Ups)))
    fast = bench.mode_params(psms, "mixed_bf16", w["tol"])
    fast.rhs_chunk = 128
    plain = bench.mode_params(psms, "plain", w["tol"])
    plain.rhs_chunk = 128
    d_bf, s_bf = ctx.logdet_ratio(psms.OP_SCHUR, 0, slots, eta, fast)
    say(" bf16", s_bf)
    d_64, s_64 = ctx.logdet_ratio(psms.OP_SCHUR, 0, slots, eta, plain)
    say(" f64", s_64)
    assert d_bf.shape == (8, 64) and np.all(np.isfinite(d_bf))
    assert s_bf["converged"] and s_64["converged"]
    assert s_bf["true_rel_residual"] <= w["tol"] and s_64["true_rel_residual"] <= w["tol"]
    g = schur.Geometry(w["L"], w["b"])
    xi2 = np.array([np.vdot(g.project(e), g.project(e)).real for e in eta])
    bound = 2 * xi2[None, :] * w["tol"] * COND
    worst = float(np.max(np.abs(d_bf - d_64) / bound))
    say(f"  max |d_bf16 - d_f64| / bound = {worst:.3f}; Delta range [{d_64.min():.3f}, {d_64.max():.3f}]")
    assert worst < 1.0
    for p, j in ((0, 5), (7, 63)):
        ref, x2 = _certified_delta(psms, ctx, w, U, Ups[p], 1 + p, eta[j], w["tol"])
        b = 2 * x2 * w["tol"] * COND
        say(f"  (p={p}, j={j}): batched bf16 {d_bf[p, j]:.10f} f64 {d_64[p, j]:.10f} certified {ref:.10f} bound {b:.1e}")
        assert abs(d_bf[p, j] - ref) < b and abs(d_64[p, j] - ref) < b


@pytest.mark.slow
@pytest.mark.timeout(600)
def test_32x4_one_proposal_batch(psms):
    """32^4, 8^4 Schur blocks (4^4 Schwarz blocks), kappa 0.1575, one proposal x 32 noise
    (one chunk of the full 4 x 32 workload): BF16-inner vs FP64 on every Delta, and one
    pair rebuilt from oracle-certified sub-solves."""
    w, U, Ups, eta = synth.workload_inputs("32x32x32x32", nprop=1)
    ctx = _load(psms, w, U, Ups)
    ctx.autotune(0, None)
    fast = bench.mode_params(psms, "mixed_bf16", w["tol"])
    fast.rhs_chunk = 16
    plain = bench.mode_params(psms, "plain", w["tol"])
    plain.rhs_chunk = 16
    d_bf, s_bf = ctx.logdet_ratio(psms.OP_SCHUR, 0, [1], eta, fast)
    say(" bf16", s_bf)
    d_64, s_64 = ctx.logdet_ratio(psms.OP_SCHUR, 0, [1], eta, plain)
    say(" f64", s_64)
    assert s_bf["converged"] and s_64["converged"]
    assert s_bf["true_rel_residual"] <= w["tol"] and s_64["true_rel_residual"] <= w["tol"]
    g = schur.Geometry(w["L"], w["b"])
    xi2 = np.array([np.vdot(g.project(e), g.project(e)).real for e in eta])
    bound = 2 * xi2 * w["tol"] * COND
    say(f"  max |d_bf16 - d_f64| / bound = {float(np.max(np.abs(d_bf[0] - d_64[0]) / bound)):.3f}")
    assert np.all(np.abs(d_bf[0] - d_64[0]) < bound)
    ref, x2 = _certified_delta(psms, ctx, w, U, Ups[0], 1, eta[3], w["tol"])
    b = 2 * x2 * w["tol"] * COND
    say(f"  (p=0, j=3): bf16 {d_bf[0, 3]:.10f} f64 {d_64[0, 3]:.10f} certified {ref:.10f} bound {b:.1e}")
    assert abs(d_bf[0, 3] - ref) < b and abs(d_64[0, 3] - ref) < b


def test_16x4_network_full_size(psms):
    """16^4 at kappa 0.157 with the 1->8->8->8->1 network: the forward pass in both
    channel-mixing forms (FP32 vector units, bf16 matrix cores) against the FP64
    network oracle on the whole lattice, then flexible GCR right-preconditioned by
    that network (Schwarz fallback allowed) meeting the FP64 true residual that the
    oracle's operator computes."""
    from oracle import dirac
    from oracle import network as net

    w, U, _, _ = synth.workload_inputs("16x16x16x16-network", nprop=0, nnoise=0)
    L, kappa = w["L"], w["kappa"]
    chans = (1, 8, 8, 8, 1)
    rng = np.random.default_rng(4601)
    ws = [0.15 * (rng.standard_normal((9, co, ci, 4, 4)) + 1j * rng.standard_normal((9, co, ci, 4, 4)))
          for ci, co in zip(chans[:-1], chans[1:])]
    flat = np.concatenate([x.ravel() for x in ws])
    r = synth.gaussian_noise(L, 2, 4602)
    say("case 16^4 network forward, oracle on the CPU")
    ref, _ = net.forward(U, ws, r[0], L)
    ctx = psms.Context(L, w["b"], kappa)
    ctx.gauge_load(0, U)
    ctx.net_init(chans)
    ctx.net_set_weights(flat)
    for mfma, tol in ((0, 2e-5), (1, 3e-2)):
        ctx.set_tuning("net_mfma", mfma)
        out = ctx.net_apply(0, r)
        err = float(np.linalg.norm((out[0] - ref).ravel()) / np.linalg.norm(ref.ravel()))
        say(f" mfma {mfma}: relative error {err:.2e}")
        assert err < tol
    say("case 16^4 network-preconditioned solve")
    x, st = ctx.solve(0, r, psms.default_params(pc=psms.PC_NET, tol=w["tol"], prec=psms.MIXED))
    say(" stats", st)
    assert st["converged"] == 1
    for k in range(r.shape[0]):
        res = r[k] - dirac.apply_D(U, x[k], kappa, L)
        assert np.linalg.norm(res) / np.linalg.norm(r[k]) <= 1.01 * w["tol"]
    ctx.close()
