"""GPU edge cases of the estimator path: zero fields, more proposals than one launch
addresses, ragged right-hand-side chunks; the autotuner's cache file. Oracle comparisons on the 4^4 workload,
whose Deltas the oracle computes exactly by dense LU."""
import sys

import numpy as np
import pytest

from oracle import dirac, estimator, schur
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


def test_zero_right_hand_side_and_zero_noise(psms):
    """A zero right-hand side next to nonzero ones solves to exactly zero while the others
    converge; a zero noise vector gives Delta = 0 exactly (xi = 0)."""
    w, U, Ups, eta = synth.workload_inputs("8x8x8x8", nnoise=3)
    ctx = psms.Context(w["L"], w["b"], w["kappa"])
    ctx.gauge_load(0, U)
    ctx.gauge_load(1, Ups[0])
    b = eta.copy()
    b[1] = 0
    for prec in (psms.F64, psms.MIXED):
        x, st = ctx.solve(0, b, psms.default_params(tol=1e-10, prec=prec))
        say(" solve", prec, st)
        assert st["converged"] == 1
        assert np.all(x[1] == 0)
        for k in (0, 2):
            res = b[k] - dirac.apply_D(U, x[k], w["kappa"], w["L"])
            assert np.linalg.norm(res) / np.linalg.norm(b[k]) <= 1.01e-10
        d, st = ctx.logdet_ratio(psms.OP_SCHUR, 0, [1], b, psms.default_params(tol=1e-10, prec=prec))
        say(" delta", d, st)
        assert d[0, 1] == 0.0
        assert np.all(np.isfinite(d))


def test_more_proposals_than_one_launch_addresses(psms):
    """17 proposals (one launch addresses at most 16 gauge fields) x 2 noise vectors on the
    4^4 workload: every Delta against the oracle's exact value to 1e-8."""
    w, U, _, eta = synth.workload_inputs("4x4x4x4", nnoise=2)
    Ups = [synth.proposal(U, w["L"], w["b"], w["eps_prime"], 7000 + p) for p in range(17)]
    ctx = psms.Context(w["L"], w["b"], w["kappa"])
    ctx.gauge_load(0, U)
    for p, Up in enumerate(Ups):
        ctx.gauge_load(1 + p, Up)
    d, st = ctx.logdet_ratio(psms.OP_SCHUR, 0, list(range(1, 18)), eta, psms.default_params(tol=1e-12, max_iter=5000))
    say(" stats", st)
    assert d.shape == (17, 2)
    g = schur.Geometry(w["L"], w["b"])
    opU = schur.Operator(g, U, w["kappa"])
    for p in (0, 8, 15, 16):
        opP = schur.Operator(g, Ups[p], w["kappa"])
        for j in range(2):
            ref = estimator.delta_schur(opU, opP, eta[j])
            assert abs(d[p, j] - ref) < 1e-8, (p, j, d[p, j], ref)


def test_ragged_right_hand_side_chunks(psms):
    """Noise vectors solved in chunks that do not divide their number (5 vectors, 2 per
    chunk) give the Deltas of the unchunked solve: both solve to 1e-12, where each Delta is
    within 1e-8 of the exact value at this size, so they agree to 2e-8."""
    w, U, Ups, eta = synth.workload_inputs("8x8x8x8", nnoise=5)
    ctx = psms.Context(w["L"], w["b"], w["kappa"])
    ctx.gauge_load(0, U)
    ctx.gauge_load(1, Ups[0])
    full, _ = ctx.logdet_ratio(psms.OP_SCHUR, 0, [1], eta, psms.default_params(tol=1e-12, max_iter=5000))
    prm = psms.default_params(tol=1e-12, max_iter=5000)
    prm.rhs_chunk = 2
    chunked, st = ctx.logdet_ratio(psms.OP_SCHUR, 0, [1], eta, prm)
    diff = float(np.abs(full[0] - chunked[0]).max())
    say(" full", full, "chunked", chunked, st, f"max diff {diff:.2e} (bound 2e-8)")
    assert diff < 2e-8


def test_autotune_cache_round_trip(psms, tmp_path):
    """psms_autotune with a cache file: a timed run appends one entry for this device and
    geometry; a second context on the same geometry then takes the last entry for that key
    (here one edited to values the timing would not all pick) without timing, and the
    operator still matches the oracle under those values."""
    import json
    import time

    w, U, _, _ = synth.workload_inputs("8x8x8x8", nprop=0, nnoise=0)
    path = str(tmp_path / "tune.jsonl")
    ctx = psms.Context(w["L"], w["b"], w["kappa"])
    ctx.gauge_load(0, U)
    first = ctx.autotune(0, path)
    ctx.close()
    lines = open(path).read().splitlines()
    assert len(lines) == 1
    entry = json.loads(lines[0])
    for k in psms.Context.TUNING_KEYS:
        assert entry[k] == first[k], k
    edited = dict(entry, dslash_variant_f64=3, nr_low=4)
    with open(path, "a") as f:
        f.write(json.dumps(edited) + "\n")
    ctx = psms.Context(w["L"], w["b"], w["kappa"])
    ctx.gauge_load(0, U)
    t0 = time.perf_counter()
    got = ctx.autotune(0, path)
    dt = time.perf_counter() - t0
    say(" cached tuning", got, f"in {dt * 1e3:.1f} ms")
    assert got["dslash_variant_f64"] == 3 and got["nr_low"] == 4
    assert len(open(path).read().splitlines()) == 2  # read, nothing appended
    psi = synth.gaussian_noise(w["L"], 2, 77)
    out = ctx.apply_dw(0, psi)
    for k in range(2):
        ref = dirac.apply_D(U, psi[k], w["kappa"], w["L"])
        assert np.linalg.norm(out[k] - ref) / np.linalg.norm(ref) < 1e-13
    ctx.close()
