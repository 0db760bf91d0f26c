"""How close the near-critical 16^4 workload sits to the critical hopping parameter,
through the library's D_w.

D = 1 - kappa H (eq. Dw) gets an eigenvalue of vanishing real part at kappa_c =
1 / max Re spec(H). Here H v = (v - D v) / kappa is applied through psms_apply_dw
(FP64) and the eigenvalues of largest real part come from a Krylov-Schur iteration
(Stewart's restarted Arnoldi: expand to m vectors, order the Schur form of the
projected matrix by real part, keep the leading half) on the device.

Pins: the free field, where max Re spec(H) = 6 + 2 cos(pi / L_0) with antiperiodic time
(the CPU test pins the same closed form on the oracle), and, for every reported value,
the eigenpair residual |H v - lambda v| <= tol |lambda| |v| recomputed through the
library on the returned Ritz vector.
"""
import sys
import time

import numpy as np
import pytest
from krylov_schur import krylov_schur_top_re

from paper_1204_1306_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def measure(psms, L, U, kappa, tol, max_mv):
    import torch

    dev = torch.device("cuda:0")
    V = synth.lattice_volume(L)
    ctx = psms.Context(L, (4, 4, 4, 4), kappa, stream=torch.cuda.current_stream().cuda_stream)
    ctx.gauge_load(0, torch.from_numpy(U).to(dev))

    def hop(v):
        return (v - ctx.apply_dw(0, v.view(V, 4, 3)).view(-1)) / kappa

    t0 = time.perf_counter()
    lam, vec, nmv = krylov_schur_top_re(hop, V * 12, dev, tol=tol, max_mv=max_mv)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    r = torch.linalg.vector_norm(hop(vec) - lam * vec).item() / torch.linalg.vector_norm(vec).item()
    ctx.close()
    return lam, r, nmv, dt


@pytest.fixture(scope="module")
def psms():
    from paper_1204_1306_amd import psms as m

    m.load_library()
    return m


def test_free_field_edge_through_the_library(psms):
    L = (16, 8, 8, 8)
    say(f"case free field {L}")
    lam, r, nmv, dt = measure(psms, L, synth.unit_gauge_field(L), 0.12, 1e-10, 4000)
    want = 6.0 + 2.0 * np.cos(np.pi / L[0])
    say(f"  max Re spec(H) = {lam.real:.12f} (closed form {want:.12f}), residual {r:.1e}, {nmv} products, {dt:.1f} s")
    assert abs(lam.real - want) <= 1e-9
    assert r <= 1e-8 * abs(lam)


def test_kappa_c_of_the_near_critical_workload(psms):
    workload = "16x16x16x16-network"
    w = synth.WORKLOADS[workload]
    say(f"case kappa_c {workload} (seed {w['seed_U']})")
    U = synth.gauge_field(w["L"], w["eps"], w["seed_U"])
    tol = 1e-5
    lam, r, nmv, dt = measure(psms, w["L"], U, w["kappa"], tol, 12000)
    kc = 1.0 / lam.real
    say(f"  max Re spec(H) = {lam.real:.6f} (Im {lam.imag:+.3e}), residual {r:.1e}, {nmv} products, {dt:.1f} s: "
        f"kappa_c = {kc:.5f}; kappa = {w['kappa']} is {w['kappa'] / kc:.4f} of it, "
        f"min Re spec(D) = {1 - w['kappa'] * lam.real:.4f}")
    assert r <= 10 * tol * abs(lam)
    assert w["kappa"] < kc
