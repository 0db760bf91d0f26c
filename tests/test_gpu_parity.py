"""GPU parity: the HIP path (through the C-ABI) against the FP64 CPU oracle on the
same seeded inputs. Sizes span several blocks and both colours; tolerances are
stated per test."""
import sys

import numpy as np
import pytest

from oracle import dirac, estimator, lattice, schur
from paper_1204_1306_amd import synth

pytestmark = pytest.mark.gpu

# the last shape has 384 sites per parity: a ragged tail for 256-site tiles
GEOMS = [((4, 4, 4, 4), (2, 2, 2, 2)), ((8, 8, 8, 8), (4, 4, 4, 4)), ((8, 4, 4, 8), (4, 2, 2, 2)),
         ((12, 4, 4, 4), (2, 2, 2, 2))]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


@pytest.fixture(scope="module")
def psms():
    from paper_1204_1306_amd import psms as m

    m.load_library()
    return m


def make_ctx(psms, L, b, kappa):
    return psms.Context(L, b, kappa)


@pytest.mark.parametrize("L,b", GEOMS)
def test_dw_f64_matches_oracle(psms, L, b):
    say("case dw_f64", L, b)
    kappa = 0.137
    U = synth.gauge_field(L, 0.6, 11)
    psi = synth.gaussian_noise(L, 3, 12)
    ctx = make_ctx(psms, L, b, kappa)
    ctx.gauge_load(0, U)
    out = ctx.apply_dw(0, psi)
    for r in range(3):
        ref = dirac.apply_D(U, psi[r], kappa, L)
        assert rel(out[r], ref) < 1e-13


@pytest.mark.parametrize("L,b", [((8, 8, 8, 8), (4, 4, 4, 4)), ((8, 4, 4, 8), (4, 2, 2, 2)),
                                 ((16, 16, 16, 16), (8, 8, 8, 8)), ((8, 16, 16, 16), (4, 8, 8, 8)),
                                 ((12, 4, 4, 4), (2, 2, 2, 2))])
def test_dw_every_stencil_form(psms, L, b):
    """Every full-lattice stencil form the autotuner can pick (variants 0..8, one right-hand
    side per thread, three right-hand sides per launch), FP64 against the oracle to 1e-13
    and FP32 links/spinors to 2e-6."""
    kappa = 0.137
    U = synth.gauge_field(L, 0.6, 13)
    psi = synth.gaussian_noise(L, 3, 14)
    ref = [dirac.apply_D(U, psi[r], kappa, L) for r in range(3)]
    ctx = make_ctx(psms, L, b, kappa)
    ctx.gauge_load(0, U)
    ctx.set_tuning("nr_f64", 1)
    ctx.set_tuning("nr_low", 1)
    for v in range(9):
        say("case stencil form", v, L)
        ctx.set_tuning("dslash_variant_f64", v)
        ctx.set_tuning("dslash_variant_f32", v)
        out = ctx.apply_dw(0, psi)
        out32 = ctx.apply_dw(0, psi, prec=psms.MIXED)
        for r in range(3):
            assert rel(out[r], ref[r]) < 1e-13
            assert rel(out32[r], ref[r]) < 2e-6


def test_dw_periodic_time(psms):
    L, b = (4, 4, 4, 4), (2, 2, 2, 2)
    U = synth.gauge_field(L, 0.6, 13)
    psi = synth.gaussian_noise(L, 1, 14)[0]
    ctx = psms.Context(L, b, 0.12, antiperiodic=False)
    ctx.gauge_load(0, U)
    assert rel(ctx.apply_dw(0, psi), dirac.apply_D(U, psi, 0.12, L, antiperiodic=False)) < 1e-13


def test_dw_free_field_plane_wave(psms):
    """GPU D on exp(ipx) u equals exp(ipx) D(p) u (closed form, not the oracle)."""
    L, b = (8, 4, 4, 8), (4, 2, 2, 2)
    kappa = 0.125
    ctx = make_ctx(psms, L, b, kappa)
    ctx.gauge_load(0, synth.unit_gauge_field(L))
    p = np.array([3 * np.pi / 8, 2 * np.pi / 4, 0.0, 6 * np.pi / 8])
    u = np.arange(12).reshape(4, 3) * (0.3 + 0.1j) + 1
    x = lattice.coords(L)
    ph = np.exp(1j * (x @ p))
    psi = ph[:, None, None] * u[None]
    out = ctx.apply_dw(0, psi)
    ref = ph[:, None, None] * (dirac.free_field_momentum_operator(p, kappa) @ u)[None]
    assert rel(out, ref) < 1e-13


def test_dw_mixed_precision(psms):
    L, b = (8, 8, 8, 8), (4, 4, 4, 4)
    kappa = 0.15
    U = synth.gauge_field(L, 0.6, 15)
    psi = synth.gaussian_noise(L, 2, 16)
    ctx = make_ctx(psms, L, b, kappa)
    ctx.gauge_load(0, U)
    out = ctx.apply_dw(0, psi, prec=psms.MIXED)
    for r in range(2):
        # FP32 storage of links and spinors: relative error a few units of 2^-24 per term
        assert rel(out[r], dirac.apply_D(U, psi[r], kappa, L)) < 2e-6


def test_non_su3_links_in_both_precisions(psms):
    """Links scaled off SU(3): the load reports it, FP64 is exact, and mixed precision runs
    on FP32 18-real links (a 12-real rebuild would be off by the scale) within FP32
    rounding; the network, which takes 12-real links only, refuses the slot."""
    L, b = (4, 4, 4, 4), (2, 2, 2, 2)
    U = 0.9 * synth.gauge_field(L, 0.6, 17)
    ctx = make_ctx(psms, L, b, 0.12)
    assert ctx.gauge_load(0, U, allow_non_su3=True) is False
    psi = synth.gaussian_noise(L, 1, 18)[0]
    ref = dirac.apply_D(U, psi, 0.12, L)
    assert rel(ctx.apply_dw(0, psi), ref) < 1e-13
    assert rel(ctx.apply_dw(0, psi, prec=psms.MIXED), ref) < 2e-6
    ctx.net_init((1, 1))
    with pytest.raises(psms.PsmsError):
        ctx.net_apply(0, psi)


@pytest.mark.parametrize("L,b", GEOMS)
def test_block_pieces_and_projector(psms, L, b):
    say("case blocks", L, b)
    kappa = 0.14
    U = synth.gauge_field(L, 0.6, 21)
    psi = synth.gaussian_noise(L, 1, 22)[0]
    g = schur.Geometry(L, b)
    op = schur.Operator(g, U, kappa)
    ctx = make_ctx(psms, L, b, kappa)
    ctx.gauge_load(0, U)
    assert rel(ctx.apply_block(0, 0, psi), op.D_bb(psi)) < 1e-13
    assert rel(ctx.apply_block(0, 1, psi), op.D_ww(psi)) < 1e-13
    assert rel(ctx.apply_hop_bw(0, 0, psi), op.D_wb(psi)) < 1e-13
    assert rel(ctx.apply_hop_bw(0, 1, psi), op.D_bw(psi)) < 1e-13
    assert rel(ctx.apply_proj(psi), g.project(psi)) < 1e-15


def test_dhat_even_odd(psms):
    L, b = (4, 4, 4, 8), (2, 2, 2, 2)
    kappa = 0.13
    U = synth.gauge_field(L, 0.6, 31)
    psi = synth.gaussian_noise(L, 1, 32)[0]
    even = lattice.parity(L) == 0
    pe = psi.copy()
    pe[~even] = 0
    H = lambda v: dirac.hopping(U, v, L)
    t = H(pe)
    t[even] = 0
    ref = pe - kappa**2 * H(t)
    ref[~even] = 0
    ctx = make_ctx(psms, L, b, kappa)
    ctx.gauge_load(0, U)
    assert rel(ctx.apply_dhat_ee(0, psi), ref) < 1e-13


@pytest.mark.parametrize("eo,lanes", [(0, 0), (1, 2), (3, 2), (1, 4), (3, 4)])
@pytest.mark.parametrize("prec", ["f64", "mixed_f32", "mixed_bf16"])
def test_solve_parity(psms, prec, eo, lanes):
    """Full solves with Schwarz blocks solved by plain or even-odd minimal residual (links
    staged in LDS or read from L2, 2 or 4 lanes per site): FP64 true residual <= 1e-10
    through the oracle's operator."""
    L, b = (8, 8, 8, 8), (4, 4, 4, 4)
    kappa = 0.15
    say("case solve", prec, "eo", eo, "lanes", lanes)
    U = synth.gauge_field(L, 0.6, 2001)
    bvec = synth.gaussian_noise(L, 2, 41)
    ctx = make_ctx(psms, L, b, kappa)
    ctx.gauge_load(0, U)
    ctx.set_tuning("block_eo", eo)
    ctx.set_tuning("block_eo_lanes", lanes)
    kw = dict(tol=1e-10)
    if prec != "f64":
        kw.update(prec=psms.MIXED, inner_storage=psms.SPINOR_BF16 if prec == "mixed_bf16" else psms.SPINOR_F32)
    x, st = ctx.solve(0, bvec, psms.default_params(**kw))
    say(" stats", st)
    assert st["converged"] == 1
    for r in range(2):
        res = bvec[r] - dirac.apply_D(U, x[r], kappa, L)
        assert np.linalg.norm(res) / np.linalg.norm(bvec[r]) <= 1e-10 * 1.01


@pytest.mark.parametrize("link16", [0, 1, 2])
def test_solve_schwarz_link_storage(psms, link16):
    """Mixed-precision solves whose Schwarz sweeps stage their links in LDS as FP32 (0),
    as FP16 12-real links (1) or as whole FP16 links with the fields exchanged between
    lanes in FP16 (2): the flexible solver meets the FP64 true residual either way, so the
    rounding inside the preconditioner never reaches the answer."""
    L, b = (8, 8, 8, 8), (4, 4, 4, 4)
    kappa = 0.155
    U = synth.gauge_field(L, 0.6, 2002)
    bvec = synth.gaussian_noise(L, 2, 43)
    ctx = make_ctx(psms, L, b, kappa)
    ctx.gauge_load(0, U)
    ctx.set_tuning("sap_link16", link16)
    ctx.set_tuning("block_eo_lanes", 2)  # the two-lane form, which stages the links
    for st_ in (psms.SPINOR_F32, psms.SPINOR_BF16):
        say("case solve, Schwarz LDS form", link16, "storage", st_)
        x, st = ctx.solve(0, bvec, psms.default_params(tol=1e-10, prec=psms.MIXED, inner_storage=st_))
        say(" stats", st)
        assert st["converged"] == 1
        for r in range(2):
            res = bvec[r] - dirac.apply_D(U, x[r], kappa, L)
            assert np.linalg.norm(res) / np.linalg.norm(bvec[r]) <= 1e-10 * 1.01


def test_schwarz_sweep_forms_apply_the_same_preconditioner(psms):
    """The Schwarz sweep's LDS forms against the FP32 form on the same input. A solve cut
    off at max_iter = 1 (three inner iterations with the lagged convergence check, true
    residual about 6e-4) depends on the preconditioner through every Krylov vector: the
    forms must reach the same residual (within 10%) and the same solution (measured: about
    1e-5 relative; bound 2e-2). A wrong sign, neighbour or spin projector in a hop makes the
    preconditioner worse, which raises that residual and moves the solution by far more.
    Converged, each form meets the FP64 true residual in about the same number of
    iterations."""
    L, b = (8, 8, 8, 8), (4, 4, 4, 4)
    kappa = 0.155
    U = synth.gauge_field(L, 0.6, 2003)
    bvec = synth.gaussian_noise(L, 2, 44)
    ctx = make_ctx(psms, L, b, kappa)
    ctx.gauge_load(0, U)
    ctx.set_tuning("block_eo_lanes", 2)  # the two-lane form, which stages the links
    one, iters, res1 = {}, {}, {}
    for form in (0, 1, 2):
        ctx.set_tuning("sap_link16", form)
        prm = psms.default_params(tol=1e-12, max_iter=1, prec=psms.MIXED, inner_storage=psms.SPINOR_F32)
        one[form], st1 = ctx.solve(0, bvec, prm, check=False)
        res1[form] = st1["true_rel_residual"]
        say(f"  form {form}: solve cut off at max_iter 1: {st1}")
        x, st = ctx.solve(0, bvec, psms.default_params(tol=1e-10, prec=psms.MIXED, inner_storage=psms.SPINOR_F32))
        iters[form] = st["inner_iters"]
        for r in range(2):
            res = bvec[r] - dirac.apply_D(U, x[r], kappa, L)
            assert np.linalg.norm(res) / np.linalg.norm(bvec[r]) <= 1e-10 * 1.01
    for form in (1, 2):
        d = rel(one[form], one[0])
        say(f"  Schwarz form {form} against FP32: cut-off solution differs by {d:.2e}, residual "
            f"{res1[form]:.3e} against {res1[0]:.3e}; iterations {iters[form]} against {iters[0]}")
        assert d < 2e-2
        assert abs(res1[form] - res1[0]) <= 0.1 * res1[0]
        assert abs(iters[form] - iters[0]) <= max(2, iters[0] // 10)


def test_schwarz_sweep_fp16_form_on_other_block_shapes(psms):
    """The FP16 form of the Schwarz sweep on 256-site blocks that are not 4^4 (8 x 4 x 4 x 2):
    it then takes the face update site by site and stages every forward link of the block.
    The mixed solve meets the FP64 true residual in about the iterations of the FP32 form."""
    L, b = (16, 8, 8, 8), (8, 4, 4, 2)
    kappa = 0.15
    U = synth.gauge_field(L, 0.6, 2004)
    bvec = synth.gaussian_noise(L, 2, 45)
    ctx = make_ctx(psms, L, b, kappa)
    ctx.gauge_load(0, U)
    ctx.set_tuning("block_eo_lanes", 2)
    iters = {}
    for form in (0, 2):
        ctx.set_tuning("sap_link16", form)
        x, st = ctx.solve(0, bvec, psms.default_params(tol=1e-10, prec=psms.MIXED, inner_storage=psms.SPINOR_F32))
        say(f"  blocks {b}, Schwarz form {form}: {st}")
        assert st["converged"] == 1
        iters[form] = st["inner_iters"]
        for r in range(2):
            res = bvec[r] - dirac.apply_D(U, x[r], kappa, L)
            assert np.linalg.norm(res) / np.linalg.norm(bvec[r]) <= 1e-10 * 1.01
    assert abs(iters[2] - iters[0]) <= max(2, iters[0] // 10)


def test_solve_small_against_lu(psms):
    L, b = (4, 4, 4, 4), (2, 2, 2, 2)
    kappa = 0.12
    U = synth.gauge_field(L, 0.5, 1001)
    g = schur.Geometry(L, b)
    op = schur.Operator(g, U, kappa)
    bvec = synth.gaussian_noise(L, 1, 42)[0]
    ctx = make_ctx(psms, L, b, kappa)
    ctx.gauge_load(0, U)
    for pc in (psms.PC_SAP, psms.PC_NONE):
        x, st = ctx.solve(0, bvec, psms.default_params(tol=1e-12, pc=pc))
        assert rel(x, op.solve(bvec)) < 1e-10


@pytest.mark.parametrize("eo,lanes", [(0, 0), (1, 2), (1, 4)])
@pytest.mark.parametrize("colour", [0, 1])
def test_block_solve_parity(psms, colour, eo, lanes):
    """D_bb^-1 / D_ww^-1 (Dirichlet blocks of 256 sites, 16 blocks): plain and even-odd
    preconditioned minimal residual (2 or 4 lanes per site) to 1e-12 against the
    oracle's per-block dense LU."""
    L, b = (8, 8, 8, 8), (4, 4, 4, 4)
    kappa = 0.15
    say("case block", colour, "eo", eo, "lanes", lanes)
    U = synth.gauge_field(L, 0.6, 51)
    g = schur.Geometry(L, b)
    op = schur.Operator(g, U, kappa)
    bvec = synth.gaussian_noise(L, 1, 52)[0]
    ctx = make_ctx(psms, L, b, kappa)
    ctx.gauge_load(0, U)
    ctx.set_tuning("block_eo", eo)
    ctx.set_tuning("block_eo_lanes", lanes)
    x, st = ctx.solve_block(0, colour, bvec, psms.default_params(tol=1e-12, max_iter=5000))
    say(" block stats", st)
    mask = g.black if colour == 0 else g.white
    ref = op.solve_colour(g.restrict(bvec, mask), "black" if colour == 0 else "white")
    assert rel(x, ref) < 1e-10


@pytest.mark.parametrize("mixed", [0, 1])
@pytest.mark.parametrize("eo", [0, 1])
@pytest.mark.parametrize("L,b", [((8, 8, 8, 16), (4, 4, 4, 8)), ((4, 4, 4, 4), (2, 2, 2, 2))])
def test_block_solve_global_memory_parity(psms, L, b, eo, mixed):
    """Block inverses on blocks that are not LDS-resident (512- and 16-site blocks, the
    global-memory solver): plain or even-odd minimal residual, in FP64 or with FP32 inner
    solves and FP64 defect correction, to 1e-11 against the oracle's block solves."""
    kappa = 0.13
    say("case block global", L, b, "eo", eo, "mixed", mixed)
    U = synth.gauge_field(L, 0.6, 57)
    g = schur.Geometry(L, b)
    op = schur.Operator(g, U, kappa)
    bvec = synth.gaussian_noise(L, 2, 58)
    ctx = make_ctx(psms, L, b, kappa)
    ctx.gauge_load(0, U)
    ctx.set_tuning("block_eo", eo)
    prm = psms.default_params(tol=1e-11, max_iter=20000, prec=psms.MIXED if mixed else psms.F64)
    for colour in (0, 1):
        x, st = ctx.solve_block(0, colour, bvec, prm)
        say(" block stats", colour, st)
        mask = g.black if colour == 0 else g.white
        for k in range(2):
            ref = op.solve_colour(g.restrict(bvec[k], mask), "black" if colour == 0 else "white")
            assert rel(x[k], ref) < 1e-9


def test_schur_apply_and_inverse(psms):
    L, b = (8, 8, 8, 8), (4, 4, 4, 4)
    kappa = 0.15
    U = synth.gauge_field(L, 0.6, 61)
    g = schur.Geometry(L, b)
    op = schur.Operator(g, U, kappa)
    xi = g.project(synth.gaussian_noise(L, 1, 62)[0])
    ctx = make_ctx(psms, L, b, kappa)
    ctx.gauge_load(0, U)
    prm = psms.default_params(tol=1e-12, max_iter=5000)
    out, _ = ctx.apply_schur(0, xi, prm)
    assert rel(out, op.schur_apply(xi)) < 1e-10
    y, st = ctx.apply_schur_inv(0, xi, psms.default_params(tol=1e-12))
    assert rel(y, op.schur_inverse_direct(xi, tol=1e-13)) < 1e-9


def _oracle_deltas(w, U, Ups, eta, kind):
    g = schur.Geometry(w["L"], w["b"])
    opU = schur.Operator(g, U, w["kappa"])
    out = np.zeros((len(Ups), eta.shape[0]))
    for p, Up in enumerate(Ups):
        opP = schur.Operator(g, Up, w["kappa"])
        for j in range(eta.shape[0]):
            f = estimator.delta_schur if kind == "schur" else estimator.delta_full
            out[p, j] = f(opU, opP, eta[j])
    return out


def test_logdet_ratio_small_workload(psms):
    """4^4 lattice, 2^4 blocks, kappa 0.12, 4 noise vectors, solves to 1e-12:
    same-noise Delta within 1e-8 absolute of the oracle."""
    w, U, Ups, eta = synth.workload_inputs("4x4x4x4")
    ctx = make_ctx(psms, w["L"], w["b"], w["kappa"])
    ctx.gauge_load(0, U)
    ctx.gauge_load(1, Ups[0])
    prm = psms.default_params(tol=1e-12, max_iter=5000)
    for op, kind in ((psms.OP_SCHUR, "schur"), (psms.OP_FULL, "full")):
        d, st = ctx.logdet_ratio(op, 0, [1], eta, prm)
        ref = _oracle_deltas(w, U, Ups, eta, kind)
        say(" delta", kind, d.ravel(), ref.ravel(), st)
        assert np.abs(d - ref).max() < 1e-8
        # the log-ratio estimate from these Deltas against the oracle's from its own
        lhat = psms.log_ratio_estimate(d)
        assert abs(lhat[0] - estimator.log_ratio_estimate(ref[0])) < 1e-8


def test_logdet_ratio_interpolated(psms):
    """Gauge-field interpolation (Sec. 4.3, eqs. gfparam, Mparam, staccN) with N = 3 on the
    4^4 workload, two proposals: same-noise Delta (sum over the three factors, each with its
    own noise group) within 1e-8 absolute of the oracle, SCHUR and FULL, in FP64 and in mixed
    precision (the intermediate fields are not SU(3): their inner solves use FP32 18-real
    links inside FP64 defect correction), and the two slots the call borrows are free again
    afterwards."""
    w, U, Ups, _ = synth.workload_inputs("4x4x4x4", nprop=2)
    N, nn = 3, 2
    eta = synth.gaussian_noise(w["L"], N * nn, 4711)
    ctx = make_ctx(psms, w["L"], w["b"], w["kappa"])
    ctx.gauge_load(0, U)
    ctx.gauge_load(1, Ups[0])
    ctx.gauge_load(2, Ups[1])
    prm = psms.default_params(tol=1e-12, max_iter=5000)
    g = schur.Geometry(w["L"], w["b"])
    prm_mixed = psms.default_params(tol=1e-12, max_iter=5000, prec=psms.MIXED)
    for op, kind in ((psms.OP_SCHUR, "schur"), (psms.OP_FULL, "full")):
        refs = {(p, j): estimator.delta_interpolated(g, U, Ups[p], w["kappa"], [eta[i * nn + j] for i in range(N)],
                                                     op=kind) for p in range(2) for j in range(nn)}
        for name, pr in (("f64", prm), ("mixed", prm_mixed)):
            say("case interpolated", kind, name, "N", N)
            d, st = ctx.logdet_ratio(op, 0, [1, 2], eta, pr, n_interp=N)
            assert d.shape == (2, nn)
            assert st["true_rel_residual"] <= 1.01e-12
            for p in range(2):
                for j in range(nn):
                    say(f"  p {p} j {j}: {d[p, j]:.12f} oracle {refs[p, j]:.12f}")
                    assert abs(d[p, j] - refs[p, j]) < 1e-8
    ctx.gauge_load(62, U)  # a borrowed slot, loadable again
    ctx.gauge_load(63, U)


def test_logdet_ratio_interpolated_split_schwarz_blocks(psms):
    """The interpolated estimator (N = 2) in a context whose Schwarz blocks (2^4) differ from
    its domain blocks (4^4), so the intermediate fields are formed in both link layouts:
    the same Deltas as the unsplit context, in FP64 and in mixed precision (whose FP32
    18-real links of the intermediate fields then exist in both layouts). All solve to
    1e-12, where each Delta is within 1e-8 of the exact value (the 8^4 estimator tests
    against the oracle), so any two agree to 2e-8."""
    w, U, Ups, _ = synth.workload_inputs("8x8x8x8", nprop=1)
    N, nn = 2, 2
    eta = synth.gaussian_noise(w["L"], N * nn, 4801)
    out = []
    for prec in (psms.F64, psms.MIXED):
        prm = psms.default_params(tol=1e-12, max_iter=5000, prec=prec)
        for sap_b in (None, (2, 2, 2, 2)):
            say("case interpolated, Schwarz blocks", sap_b, "prec", prec)
            ctx = psms.Context(w["L"], w["b"], w["kappa"], sap_b=sap_b)
            ctx.gauge_load(0, U)
            ctx.gauge_load(1, Ups[0])
            d, st = ctx.logdet_ratio(psms.OP_SCHUR, 0, [1], eta, prm, n_interp=N)
            say("  delta", d.ravel(), st)
            assert st["converged"] == 1
            out.append(d)
            ctx.close()
    diff = max(float(np.abs(o - out[0]).max()) for o in out[1:])
    say(f"  max |case - unsplit FP64| = {diff:.2e} (bound 2e-8)")
    assert diff < 2e-8


def test_dw_mixed_on_links_that_are_not_su3(psms):
    """A field between U and U' (eq. gfparam with N = 2) is not SU(3): psms_gauge_load
    reports PSMS_ENOTSU3, and the mixed-precision stencil then runs on FP32 copies of all
    18 reals of each link. Against the oracle's D on the same field: FP32 operands within
    2e-6 relative (as for SU(3) links), BF16 input with FP32 output within the bound of
    a BF16 input (2^-8 relative per component, 8e-3 on the field). A second load of
    another field into the slot replaces its FP32 copies. The network (12-real links only)
    and psms_apply_dw_noalloc in MIXED (which may not allocate the copies) refuse it."""
    w, U, Ups, _ = synth.workload_inputs("8x8x8x8", nprop=2)
    L = w["L"]
    psi = synth.gaussian_noise(L, 2, 4901)
    ctx = make_ctx(psms, L, w["b"], w["kappa"])
    for k, Up in enumerate(Ups):
        Um = 0.5 * (U + Up)
        say("case mixed stencil, interpolated field", k)
        assert ctx.gauge_load(0, Um, allow_non_su3=True) is False
        out = ctx.apply_dw(0, psi, prec=psms.MIXED)
        for r in range(2):
            ref = dirac.apply_D(Um, psi[r], w["kappa"], L)
            e = rel(out[r], ref)
            say(f"  FP32 18-real links: rel {e:.2e}")
            assert e < 2e-6
        lp = ctx.apply_dw_lowp(0, psi, psms.SPINOR_BF16, psms.SPINOR_F32)
        e = rel(lp[0], dirac.apply_D(Um, psi[0], w["kappa"], L))
        say(f"  BF16 input, FP32 output: rel {e:.2e}")
        assert e < 8e-3
    ctx.net_init((1, 2, 1))
    with pytest.raises(psms.PsmsError):
        ctx.net_apply(0, psi)
    import torch

    dpsi = torch.from_numpy(psi).to("cuda:0")
    dout = torch.empty_like(dpsi)
    assert ctx.apply_dw_noalloc(0, dpsi, dout, prec=psms.MIXED, check=False) == -5  # PSMS_ENOTSU3
    assert ctx.apply_dw_noalloc(0, dpsi, dout, prec=psms.F64, check=False) == 0
    ctx.close()


def test_logdet_ratio_mixed_vs_f64_8x4(psms):
    """8^4 lattice, 4^4 blocks, kappa 0.15: FP64, mixed precision (FP32 and BF16 inner
    storage) and FP32 block passes, all solving to 1e-12, against the oracle (1e-14) on the
    same noise: same-noise Delta within 1e-8 absolute (the stated tolerance)."""
    w, U, Ups, eta = synth.workload_inputs("8x8x8x8", nnoise=4)
    ctx = make_ctx(psms, w["L"], w["b"], w["kappa"])
    ctx.gauge_load(0, U)
    ctx.gauge_load(1, Ups[0])
    ref = _oracle_deltas(w, U, Ups, eta[:2], "schur")
    say(" ref", ref.ravel())
    runs = {"f64": dict(), "mixed": dict(prec=psms.MIXED),
            "bf16": dict(prec=psms.MIXED, inner_storage=psms.SPINOR_BF16, inner_tol=1e-2, restart=32)}
    out = {}
    for name, kw in runs.items():
        d, st = ctx.logdet_ratio(psms.OP_SCHUR, 0, [1], eta, psms.default_params(tol=1e-12, max_iter=5000, **kw))
        err = float(np.abs(d[0, :2] - ref[0]).max())
        say(f" {name}: {d.ravel()} {st}; max |gpu - oracle| = {err:.2e} (bound 1e-8)")
        assert st["converged"] == 1 and err < 1e-8
        out[name] = d
    assert np.abs(out["f64"] - out["mixed"]).max() < 2e-8
    assert np.abs(out["f64"] - out["bf16"]).max() < 2e-8
    # the block inverses to tolerance as FP32 passes inside FP64 defect correction
    ctx.set_tuning("block_tol_prec", 1)
    dp, sp = ctx.logdet_ratio(psms.OP_SCHUR, 0, [1], eta, psms.default_params(tol=1e-12, max_iter=5000,
                                                                              prec=psms.MIXED))
    ctx.set_tuning("block_tol_prec", 0)
    err = float(np.abs(dp[0, :2] - ref[0]).max())
    say(f" dp32 {dp.ravel()} {sp}; max |gpu - oracle| = {err:.2e}")
    assert sp["converged"] == 1 and err < 1e-8
    assert np.abs(dp - out["f64"]).max() < 2e-8


def test_split_schwarz_blocks_same_results(psms):
    """Schwarz blocks smaller than the domain blocks (solver in a second block layout):
    the solve and the Schur estimator agree with the oracle and with the unsplit context."""
    w, U, Ups, eta = synth.workload_inputs("8x8x8x8", nnoise=2)
    ctx = psms.Context(w["L"], w["b"], w["kappa"], sap_b=(2, 2, 2, 2))
    ctx.gauge_load(0, U)
    ctx.gauge_load(1, Ups[0])
    bvec = synth.gaussian_noise(w["L"], 1, 141)[0]
    x, st = ctx.solve(0, bvec, psms.default_params(tol=1e-11, prec=psms.MIXED))
    res = bvec - dirac.apply_D(U, x, w["kappa"], w["L"])
    assert np.linalg.norm(res) / np.linalg.norm(bvec) <= 1.01e-11
    d_split, _ = ctx.logdet_ratio(psms.OP_SCHUR, 0, [1], eta, psms.default_params(tol=1e-12, max_iter=5000))
    ref = _oracle_deltas(w, U, Ups, eta, "schur")
    err = float(np.abs(d_split[0] - ref[0]).max())
    say(" split", d_split.ravel(), "oracle", ref.ravel(), f"max diff {err:.2e} (bound 1e-8)")
    assert err < 1e-8
