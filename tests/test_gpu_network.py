"""GPU parity of the learned preconditioner against the FP64 network oracle:
forward, loss and Wirtinger gradients, the Wilson-weight layer against D, a short
training run on the GPU, checkpoint round trip, and flexible GCR with the network
as right preconditioner (exact to the FP64 residual)."""
import os
import sys

import numpy as np
import pytest

from oracle import dirac
from oracle import network as net
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


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def flat(ws):
    return np.concatenate([w.ravel() for w in ws])


def unflat(v, chans):
    out, o = [], 0
    for cin, cout in zip(chans[:-1], chans[1:]):
        n = 9 * cout * cin * 16
        out.append(v[o:o + n].reshape(9, cout, cin, 4, 4))
        o += n
    return out


def rand_weights(seed, chans, scale=0.15):
    rng = np.random.default_rng(seed)
    return [scale * (rng.standard_normal((9, co, ci, 4, 4)) + 1j * rng.standard_normal((9, co, ci, 4, 4)))
            for ci, co in zip(chans[:-1], chans[1:])]


# FP32 vector-unit mixing: FP32 weights, activations and links; matrix-core mixing:
# bf16 inputs to the MFMA (8-bit mantissa) with FP32 accumulation
TOL = {0: 2e-5, 1: 3e-2}


@pytest.mark.parametrize("mfma", [0, 1])
@pytest.mark.parametrize("chans", [(1, 1), (1, 3, 2, 1), (1, 8, 8, 8, 1)])
def test_net_forward_parity(psms, chans, mfma):
    say("case net forward", chans, "mfma", mfma)
    L, b = (4, 4, 4, 8), (2, 2, 2, 2)
    U = synth.gauge_field(L, 0.6, 101)
    r = synth.gaussian_noise(L, 2, 102)
    ctx = psms.Context(L, b, 0.13)
    ctx.set_tuning("net_mfma", mfma)
    ctx.gauge_load(0, U)
    ctx.net_init(chans)
    ws = rand_weights(103, chans)
    ctx.net_set_weights(flat(ws))
    out = ctx.net_apply(0, r)
    for k in range(2):
        ref, _ = net.forward(U, ws, r[k], L)
        assert rel(out[k], ref) < TOL[mfma]


@pytest.mark.parametrize("mfma", [0, 1])
def test_net_wilson_layer_is_dirac(psms, mfma):
    L, b = (8, 4, 4, 8), (4, 2, 2, 2)
    U = synth.gauge_field(L, 0.6, 111)
    r = synth.gaussian_noise(L, 1, 112)[0]
    W = np.zeros((9, 1, 1, 4, 4), complex)
    W[0, 0, 0] = np.eye(4)
    for mu in range(4):
        W[1 + 2 * mu, 0, 0] = -0.14 * (np.eye(4) - dirac.GAMMA[mu])
        W[2 + 2 * mu, 0, 0] = -0.14 * (np.eye(4) + dirac.GAMMA[mu])
    ctx = psms.Context(L, b, 0.14)
    ctx.set_tuning("net_mfma", mfma)
    ctx.gauge_load(0, U)
    ctx.net_init((1, 1))
    ctx.net_set_weights(W.ravel())
    assert rel(ctx.net_apply(0, r), dirac.apply_D(U, r, 0.14, L)) < (2e-6 if mfma == 0 else 1e-2)


@pytest.mark.parametrize("mfma", [0, 1])
def test_net_loss_and_gradient_parity(psms, mfma):
    chans = (1, 2, 3, 2, 1)
    L, b = (4, 4, 4, 4), (2, 2, 2, 2)
    U = synth.gauge_field(L, 0.6, 121)
    rs = synth.gaussian_noise(L, 3, 122)
    es = synth.gaussian_noise(L, 3, 123)
    ws = rand_weights(124, chans, scale=0.3)
    ctx = psms.Context(L, b, 0.13)
    ctx.set_tuning("net_mfma", mfma)
    ctx.gauge_load(0, U)
    ctx.net_init(chans)
    ctx.net_set_weights(flat(ws))
    loss, g = ctx.net_loss_grad(0, rs, es)
    ref_loss, ref_g = net.backward(U, ws, list(rs), list(es), L)
    say(" loss", loss, ref_loss, "grad rel err", rel(g, flat(ref_g)))
    assert loss == pytest.approx(ref_loss, rel=1e-5 if mfma == 0 else 3e-2)
    assert rel(g, flat(ref_g)) < (1e-4 if mfma == 0 else 5e-2)


def test_net_large_launch_agrees_with_small_launch(psms):
    """The matrix-core layer on a launch of 4096 workgroups (16^4, four fields: the shape
    of the training and preconditioning passes) against two fields (2048 workgroups).
    Every field takes the same MFMA steps in the same order, so the forward results agree
    to FP32 rounding (1e-6), the loss and its gradient over four pairs equal the sums over
    two + two pairs (the gradient's site reduction is split differently: 1e-5), and the
    large launch's forward matches the FP64 oracle within the bf16 tolerance."""
    chans = (1, 8, 8, 8, 1)
    L, b = (16, 16, 16, 16), (4, 4, 4, 4)
    U = synth.gauge_field(L, 0.6, 4999)
    r = synth.gaussian_noise(L, 4, 4702)
    e = synth.gaussian_noise(L, 4, 4703)
    ws = rand_weights(4701, chans)
    ctx = psms.Context(L, b, 0.157)
    ctx.set_tuning("net_mfma", 1)
    ctx.gauge_load(0, U)
    ctx.net_init(chans)
    ctx.net_set_weights(flat(ws))
    say("case net large launch: forward")
    out4 = ctx.net_apply(0, r)
    out2 = ctx.net_apply(0, r[:2])
    d = rel(out4[:2], out2)
    say(f"  |N4 - N2| / |N2| = {d:.2e}")
    assert d < 1e-6
    ref, _ = net.forward(U, ws, r[3], L)
    err = rel(out4[3], ref)
    say(f"  large launch against the FP64 oracle: {err:.2e} (bound {TOL[1]})")
    assert err < TOL[1]
    say("case net large launch: loss and gradient")
    l4, g4 = ctx.net_loss_grad(0, r, e)
    la, ga = ctx.net_loss_grad(0, r[:2], e[:2])
    lb, gb = ctx.net_loss_grad(0, r[2:], e[2:])
    say(f"  loss {l4} vs {la + lb}; gradient {rel(g4, ga + gb):.2e}")
    assert l4 == pytest.approx(la + lb, rel=1e-6)
    assert rel(g4, ga + gb) < 1e-5
    ctx.close()


def test_net_training_reduces_loss_and_checkpoints(psms, tmp_path):
    L, b = (8, 8, 8, 8), (4, 4, 4, 4)
    kappa = 0.15
    ctx = psms.Context(L, b, kappa)
    for s in range(2):
        ctx.gauge_load(s, synth.gauge_field(L, 0.6, 4000 + s))
    ctx.net_init((1, 4, 4, 1), seed=3, scale=0.05)
    st = ctx.net_train([0, 1], npairs=64, batch=8, epochs=3, chunk=32, lr=3e-3, solve_tol=1e-6,
                       ckpt_path=str(tmp_path / "net.bin"))
    say(" train", st)
    assert st["final_loss"] < 0.8 * st["first_loss"]
    w = ctx.net_get_weights()
    ctx2 = psms.Context(L, b, kappa)
    ctx2.gauge_load(0, synth.gauge_field(L, 0.6, 4000))
    ctx2.net_load(str(tmp_path / "net.bin"))
    assert np.array_equal(ctx2.net_get_weights(), w)


@pytest.mark.parametrize("prec", ["f64", "mixed"])
def test_gcr_with_network_preconditioner_is_exact(psms, prec):
    L, b = (8, 8, 8, 8), (4, 4, 4, 4)
    kappa = 0.15
    U = synth.gauge_field(L, 0.6, 2001)
    bvec = synth.gaussian_noise(L, 2, 131)
    ctx = psms.Context(L, b, kappa)
    ctx.gauge_load(0, U)
    ctx.net_init((1, 4, 4, 1), seed=5, scale=0.05)
    kw = dict(tol=1e-10, pc=psms.PC_NET, restart=32, max_iter=3000)
    if prec == "mixed":
        kw["prec"] = psms.MIXED
    x, st = ctx.solve(0, bvec, psms.default_params(**kw))
    say(" stats", st)
    assert st["converged"] == 1
    for k in range(2):
        res = bvec[k] - dirac.apply_D(U, x[k], kappa, L)
        assert np.linalg.norm(res) / np.linalg.norm(bvec[k]) <= 1.01e-10


def test_trained_network_gains_over_untrained_and_no_preconditioner(psms):
    """What training buys: on a held-out configuration at near-critical kappa, flexible
    GCR right-preconditioned by the network trained on the GPU (residual/correction pairs
    from the plain solver on four other seeded configurations) needs at most half the
    iterations of the same network untrained and fewer than no preconditioner, and every
    solve meets the FP64 true-residual tolerance (the network never changes the answer)."""
    L, b = (8, 8, 8, 8), (4, 4, 4, 4)
    kappa = 0.157
    ctx = psms.Context(L, b, kappa)
    for s in range(4):
        ctx.gauge_load(10 + s, synth.gauge_field(L, 0.6, 4000 + s))
    U = synth.gauge_field(L, 0.6, 4999)
    ctx.gauge_load(0, U)
    bvec = synth.gaussian_noise(L, 4, 141)
    base = dict(tol=1e-10, restart=32, max_iter=4000, net_fallback=0)

    def run(pc):
        x, st = ctx.solve(0, bvec, psms.default_params(pc=pc, **base))
        assert st["converged"] == 1 and st["used_fallback"] == 0
        for k in range(bvec.shape[0]):
            res = bvec[k] - dirac.apply_D(U, x[k], kappa, L)
            assert np.linalg.norm(res) / np.linalg.norm(bvec[k]) <= 1.01e-10
        return st["inner_iters"]

    import time

    t0 = time.perf_counter()
    n_sap = run(psms.PC_SAP)
    t_sap = time.perf_counter() - t0
    n_none = run(psms.PC_NONE)
    ctx.net_init((1, 8, 8, 8, 1), seed=7, scale=0.05)
    n_untrained = run(psms.PC_NET)
    tr = ctx.net_train([10, 11, 12, 13], npairs=512, batch=8, epochs=2, chunk=64, lr=2e-3, solve_tol=1e-6)
    t0 = time.perf_counter()
    n_trained = run(psms.PC_NET)
    t_net = time.perf_counter() - t0
    say(f" iterations: none {n_none}, untrained network {n_untrained}, trained network {n_trained} ({t_net:.3f} s), "
        f"Schwarz {n_sap} ({t_sap:.3f} s); train {tr}")
    assert tr["final_loss"] < 0.5 * tr["first_loss"]
    assert n_trained <= 0.5 * n_untrained
    assert n_trained < n_none
    # against the method without the network (Schwarz-preconditioned GCR) the trained
    # network loses: it reaches 4 sites, a Schwarz block solve couples a whole block
    if not (n_trained < n_sap and t_net < t_sap):
        pytest.xfail(f"trained network {n_trained} iterations / {t_net:.3f} s against Schwarz {n_sap} / "
                     f"{t_sap:.3f} s")
