"""GPU tests through the C-ABI of what the mathematics fixes for any input, of run-to-run
determinism, of the statistics of the batched estimator, of the low-precision stencil
operands element by element, and of the error paths.

* gamma5-hermiticity of D (Sec. 4.3 relies on it; eq. Dw): <phi, g5 D psi> = <g5 D phi, psi>;
* gauge covariance D(U^g) G psi = G D(U) psi (Sec. 4.2);
* invariance of 1 - PQ under gauge transformations supported on block-interior sites
  (Sec. 4.4, last paragraph);
* bitwise equality of two identical estimator calls (deterministic reductions);
* the batched estimator's sample moments against the exact ones from the dense spectrum
  of M^dagger M (eqs. stacc, varstoch2);
* the stencil with BF16 / FP32 operands against the oracle applied to the same rounded
  input, every stencil form;
* ENOTCONV, ENAN, the network fallback, and a gauge field holding NaN.
"""
import sys

import numpy as np
import pytest

from oracle import dirac, lattice, schur
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


def g5(psi):
    out = psi.copy()
    out[..., 2:, :] *= -1  # chiral basis: gamma5 = diag(1, 1, -1, -1)
    return out


def test_gamma5_hermiticity_through_the_abi(psms):
    L, b, kappa = (8, 8, 8, 8), (4, 4, 4, 4), 0.15
    say("case gamma5-hermiticity 8^4")
    ctx = psms.Context(L, b, kappa)
    ctx.gauge_load(0, synth.gauge_field(L, 0.6, 301))
    phi, psi = synth.gaussian_noise(L, 2, 302)
    Dpsi, Dphi = ctx.apply_dw(0, np.stack([psi, phi]))
    lhs = np.vdot(phi, g5(Dpsi))
    rhs = np.vdot(g5(Dphi), psi)
    scale = np.linalg.norm(phi) * np.linalg.norm(Dpsi)
    say(f"  <phi, g5 D psi> = {lhs:.12e}, <g5 D phi, psi> = {rhs:.12e}, |diff|/scale = {abs(lhs - rhs) / scale:.2e}")
    assert abs(lhs - rhs) <= 1e-13 * scale
    ctx.close()


def test_gauge_covariance_through_the_abi(psms):
    L, b, kappa = (8, 8, 8, 8), (4, 4, 4, 4), 0.15
    say("case gauge covariance 8^4")
    U = synth.gauge_field(L, 0.6, 311)
    gt = synth.gauge_transform(312, int(np.prod(L)))
    Ug = dirac.gauge_transform_links(U, gt, L)
    psi = synth.gaussian_noise(L, 1, 313)[0]
    ctx = psms.Context(L, b, kappa)
    ctx.gauge_load(0, U)
    ctx.gauge_load(1, Ug)
    lhs = ctx.apply_dw(1, dirac.gauge_transform_spinor(psi, gt))
    rhs = dirac.gauge_transform_spinor(ctx.apply_dw(0, psi), gt)
    err = np.linalg.norm(lhs - rhs) / np.linalg.norm(rhs)
    say(f"  |D(U^g) G psi - G D(U) psi| / |.| = {err:.2e}")
    assert err <= 1e-13
    # mixed precision too (FP32 links and spinors): covariant up to FP32 rounding
    lhs = ctx.apply_dw(1, dirac.gauge_transform_spinor(psi, gt), psms.MIXED)
    rhs = dirac.gauge_transform_spinor(ctx.apply_dw(0, psi, psms.MIXED), gt)
    err = np.linalg.norm(lhs - rhs) / np.linalg.norm(rhs)
    say(f"  mixed: {err:.2e}")
    assert err <= 2e-6
    ctx.close()


def test_schur_invariant_under_block_interior_gauge_transformations(psms):
    L, b, kappa = (8, 8, 8, 8), (4, 4, 4, 4), 0.15
    say("case 1 - PQ under interior gauge transformations 8^4")
    g = schur.Geometry(L, b)
    U = synth.gauge_field(L, 0.6, 321)
    gt = synth.gauge_transform(322, g.V)
    loc = lattice.coords(L) % np.asarray(b)
    interior = np.all((loc > 0) & (loc < np.asarray(b) - 1), axis=1)
    gt[~interior] = np.eye(3)
    Ug = dirac.gauge_transform_links(U, gt, L)
    xi = g.project(synth.gaussian_noise(L, 2, 323))
    ctx = psms.Context(L, b, kappa)
    ctx.gauge_load(0, U)
    ctx.gauge_load(1, Ug)
    prm = psms.default_params(tol=1e-13, max_iter=5000)
    a, sa = ctx.apply_schur(0, xi, prm)
    c, sc = ctx.apply_schur(1, xi, prm)
    err = np.linalg.norm(a - c) / np.linalg.norm(a)
    say(f"  relative difference {err:.2e} (block solves to 1e-13)")
    assert err <= 1e-11
    # the transformation is not trivial: the operator itself changes
    eta = synth.gaussian_noise(L, 1, 324)[0]
    assert np.abs(ctx.apply_dw(0, eta) - ctx.apply_dw(1, eta)).max() > 1e-3
    ctx.close()


@pytest.mark.parametrize("mode", ["plain", "mixed", "mixed_bf16"])
def test_estimator_bitwise_deterministic(psms, mode):
    import bench

    say(f"case bitwise determinism 8^4 {mode}")
    w, U, Ups, eta = synth.workload_inputs("8x8x8x8")
    ctx = psms.Context(w["L"], w["b"], w["kappa"])
    ctx.gauge_load(0, U)
    ctx.gauge_load(1, Ups[0])
    prm = bench.mode_params(psms, mode, w["tol"], "8x8x8x8")
    d1, s1 = ctx.logdet_ratio(psms.OP_SCHUR, 0, [1], eta, prm)
    d2, s2 = ctx.logdet_ratio(psms.OP_SCHUR, 0, [1], eta, prm)
    say(f"  stats {s1['inner_iters']} / {s2['inner_iters']} iterations")
    assert np.array_equal(d1, d2)
    assert s1["inner_iters"] == s2["inner_iters"]
    ctx.close()


def test_batched_estimator_moments_against_dense_spectrum(psms):
    """4^4 lattice, 2^4 blocks, kappa 0.12 (every black site is a block-boundary site, so P
    is the identity on the black sites): 4096 noise fields in one batched Schur estimate.
    The sample mean of e^-Delta must match det(M^dagger M)^-1, the sample mean of Delta
    must match sum (lambda - 1) and the sample variance sum (lambda - 1)^2, with
    M = Dhat(U')^-1 Dhat(U) built densely by the oracle, each within 5 standard errors."""
    w, U, Ups, _ = synth.workload_inputs("4x4x4x4", nnoise=0)
    L, b, kappa = w["L"], w["b"], w["kappa"]
    g = schur.Geometry(L, b)
    Bd, Wd = g.dofs(g.black), g.dofs(g.white)

    def dhat(UU):
        A = dirac.dirac_matrix(UU, kappa, L).toarray()
        return np.eye(Bd.size) - np.linalg.solve(A[np.ix_(Bd, Bd)],
                                                 A[np.ix_(Bd, Wd)] @ np.linalg.solve(A[np.ix_(Wd, Wd)], A[np.ix_(Wd, Bd)]))

    M = np.linalg.solve(dhat(Ups[0]), dhat(U))
    lam = np.linalg.eigvalsh(M.conj().T @ M)
    say(f"case batched moments 4^4: lambda in [{lam.min():.4f}, {lam.max():.4f}]")
    assert lam.min() > 0.5  # the variance of e^-Delta is finite (Sec. 4.1)
    e_exp = float(np.exp(-np.sum(np.log(lam))))
    e_mean, e_var = float(np.sum(lam - 1)), float(np.sum((lam - 1) ** 2))
    n = 4096
    eta = synth.gaussian_noise(L, n, 1601)
    ctx = psms.Context(L, b, kappa)
    ctx.gauge_load(0, U)
    ctx.gauge_load(1, Ups[0])
    d, st = ctx.logdet_ratio(psms.OP_SCHUR, 0, [1], eta, psms.default_params(tol=1e-12, max_iter=5000, rhs_chunk=1024))
    d = d[0]
    assert st["converged"] == 1
    x = np.exp(-d)
    se_x = x.std() / np.sqrt(n)
    se_m = d.std() / np.sqrt(n)
    m4 = np.mean((d - d.mean()) ** 4)
    se_v = np.sqrt(max(m4 - d.var() ** 2, 0.0) / n)
    say(f"  mean e^-Delta {x.mean():.6f} vs det^-1 {e_exp:.6f} (se {se_x:.1e}); mean Delta {d.mean():.5f} vs "
        f"{e_mean:.5f} (se {se_m:.1e}); var Delta {d.var():.5f} vs {e_var:.5f} (se {se_v:.1e})")
    assert abs(x.mean() - e_exp) < 5 * se_x
    assert abs(d.mean() - e_mean) < 5 * se_m
    assert abs(d.var() - e_var) < 5 * se_v
    # and the library's log-ratio estimate is ln of that sample mean
    assert psms.log_ratio_estimate(d[None])[0] == pytest.approx(np.log(x.mean()), rel=1e-10)
    ctx.close()


def _round_bf16(a):
    """FP64 -> FP32 -> BF16 round-to-nearest-even (the library's packing path), as FP64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def _round_c(psi, fn):
    r = psi.view(np.float64)
    return fn(r).view(np.complex128).reshape(psi.shape)


@pytest.mark.parametrize("variant", range(9))
def test_low_precision_stencil_every_form(psms, variant):
    """psms_apply_dw_lowp against the oracle's D applied (in FP64) to the input rounded
    as the library rounds it. Bounds, per complex component i of each field:
    * the FP32 arithmetic (12-real links rebuilt in FP32, 8 hops of projected spinors) is
      within e_acc = 2e-5 max|in| of the exact result (about 100 roundings of 2^-24);
    * a BF16 output adds at most 2^-8 |out_i| (round-to-nearest-even keeps 8 bits).
    A wrong neighbour, sign or spin projector gives O(1) errors; a lost BF16 rounding
    mode or a truncation instead of rounding gives up to 2^-7."""
    L, b, kappa = (8, 8, 8, 8), (4, 4, 4, 4), 0.15
    U = synth.gauge_field(L, 0.6, 331)
    psi = synth.gaussian_noise(L, 2, 332)
    ctx = psms.Context(L, b, kappa)
    ctx.gauge_load(0, U)
    ctx.set_tuning("dslash_variant_bf16", variant)
    ctx.set_tuning("dslash_variant_f32", variant)
    for sin, sout, rnd in ((psms.SPINOR_BF16, psms.SPINOR_BF16, _round_bf16),
                           (psms.SPINOR_BF16, psms.SPINOR_F32, _round_bf16),
                           (psms.SPINOR_F32, psms.SPINOR_F32, lambda a: a.astype(np.float32).astype(np.float64))):
        say(f"case lowp stencil form {variant} in {sin} out {sout}")
        out = ctx.apply_dw_lowp(0, psi, sin, sout)
        worst = 0.0
        for k in range(psi.shape[0]):
            xin = _round_c(psi[k], rnd)
            ref = dirac.apply_D(U, xin, kappa, L)
            e_acc = 2e-5 * np.abs(xin).max()
            bound = e_acc + (2.0 ** -8 * np.abs(ref) + e_acc if sout == psms.SPINOR_BF16 else 0.0)
            err = np.abs(out[k] - ref)
            worst = max(worst, float((err / bound).max()))
        say(f"  max error / bound = {worst:.3f}")
        assert worst <= 1.0
    with pytest.raises(psms.PsmsError):
        ctx.apply_dw_lowp(0, psi, psms.SPINOR_F32, psms.SPINOR_BF16)
    ctx.close()


def test_error_paths(psms):
    L, b, kappa = (8, 8, 8, 8), (4, 4, 4, 4), 0.15
    U = synth.gauge_field(L, 0.6, 341)
    bvec = synth.gaussian_noise(L, 2, 342)
    ctx = psms.Context(L, b, kappa)
    ctx.gauge_load(0, U)
    say("case ENOTCONV: max_iter 1")
    for prec in (psms.F64, psms.MIXED):
        x, st = ctx.solve(0, bvec, psms.default_params(tol=1e-12, max_iter=1, prec=prec), check=False)
        assert st["converged"] == 0 and st["inner_iters"] >= 1
        assert np.all(np.isfinite(x))
        with pytest.raises(psms.PsmsError) as e:
            ctx.solve(0, bvec, psms.default_params(tol=1e-12, max_iter=1, prec=prec))
        assert e.value.status == -4
        say(f"  prec {prec}: {st}")
    say("case ENAN: NaN in the right-hand side")
    bad = bvec.copy()
    bad[1, 17, 2, 1] = np.nan
    for prec in (psms.F64, psms.MIXED):
        with pytest.raises(psms.PsmsError) as e:
            ctx.solve(0, bad, psms.default_params(prec=prec))
        assert e.value.status == -6
    say("case network fallback: untrained network, restart 2")
    ctx.net_init((1, 4, 1), seed=3, scale=0.05)
    x, st = ctx.solve(0, bvec, psms.default_params(pc=psms.PC_NET, restart=2, tol=1e-10, max_iter=4000))
    say(f"  {st}")
    assert st["used_fallback"] == 1 and st["converged"] == 1
    for k in range(2):
        res = bvec[k] - dirac.apply_D(U, x[k], kappa, L)
        assert np.linalg.norm(res) / np.linalg.norm(bvec[k]) <= 1.01e-10
    say("case gauge field with NaN")
    Ubad = U.copy()
    Ubad[5, 2, 1, 1] = np.nan
    with pytest.raises(psms.PsmsError) as e:
        ctx.gauge_load(3, Ubad)
    assert e.value.status == -1
    with pytest.raises(psms.PsmsError):
        ctx.apply_dw(3, bvec)  # the slot was left unloaded
    ctx.close()
