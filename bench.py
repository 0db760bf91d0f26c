"""Benchmark of the stochastic determinant-ratio estimator on one MI355X.

A step is one pass of the whole hot path over one batch of synthetic input: for
every proposal U'_p and Gaussian noise vector eta_j of the workload,
Delta_pj = |M xi_j|^2 - |xi_j|^2 with M the Schur-complement ratio operator:
projector, Dirichlet block solves with U, inter-block hops, one full-lattice solve
with U' per pair (flexible GCR, Schwarz preconditioner, FP64 true residual to the
workload's tolerance), FP64 accumulation. Gauge fields and noise are resident in
HBM before the timed region.

The default workload is the largest one: the 32^4 lattice with 8^4 Schur blocks
(4^4 Schwarz blocks), kappa 0.1575, 4 proposals x 32 noise vectors in one call,
tolerance 1e-10. The value is its seconds per estimate with BF16 Krylov storage,
FP32 inner solves and FP64 defect correction, all blocks, noise vectors and
proposals batched per launch. Beside it: the same batch fully in FP64, the learned
preconditioner on the same workload, D_w at 32^4, the batched 16^4 workload, the
network, the interpolation leg, and the CPU oracle. Prints one JSON line; progress
goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "D_w GB/s vs HBM peak; s per det-ratio estimate, learned/mixed vs plain FP64"
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X published FP32 vector rate
HOP_FLOPS = 168  # one Wilson hop of one site: projection 12, two SU(3) products 132, reconstruction 24


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Schwarz cycles x block iterations where the measured best differs from the library
# default (4 x 6, best for mixed at 8^4 and for both modes at 16^4): plain FP64 at 8^4
# prefers 5 x 6. At 32^4 (s per step of 4 proposals x 32 noise fields): BF16-mixed 4 x 6
# 3.71, 5 x 6 3.64, 5 x 8 3.58, 6 x 6 3.58, 6 x 8 3.68, 7 x 6 3.75; plain FP64 4 x 6 13.6,
# 6 x 6 13.1, 5 x 8 12.4.
SAP_TUNED = {("8x8x8x8", "plain"): (5, 6), ("32x32x32x32", "mixed_bf16"): (6, 6), ("32x32x32x32", "plain"): (5, 8)}


def mode_params(psms, mode: str, tol: float, workload: str | None = None):
    kw = {}
    if (workload, mode) in SAP_TUNED:
        kw["sap_cycles"], kw["block_iters"] = SAP_TUNED[(workload, mode)]
    if mode == "plain":
        return psms.default_params(tol=tol, prec=psms.F64, pc=psms.PC_SAP, **kw)
    if mode == "mixed":
        return psms.default_params(tol=tol, prec=psms.MIXED, pc=psms.PC_SAP, inner_storage=psms.SPINOR_F32,
                                   inner_tol=1e-6, **kw)
    if mode == "mixed_bf16":
        return psms.default_params(tol=tol, prec=psms.MIXED, pc=psms.PC_SAP, inner_storage=psms.SPINOR_BF16,
                                   inner_tol=1e-2, restart=32, **kw)
    if mode == "learned":
        return psms.default_params(tol=tol, prec=psms.MIXED, pc=psms.PC_NET, inner_storage=psms.SPINOR_F32,
                                   inner_tol=1e-4, restart=32, max_iter=4000)
    raise ValueError(mode)


def setup(workload: str, nprop=None, nnoise=None, inputs=None):
    import torch

    from paper_1204_1306_amd import psms, synth

    w, U, Ups, eta = inputs if inputs is not None else synth.workload_inputs(workload, nprop=nprop, nnoise=nnoise)
    stream = torch.cuda.current_stream().cuda_stream
    ctx = psms.Context(w["L"], w["b"], w["kappa"], stream=stream, sap_b=w.get("sap_b"))
    dev = torch.device("cuda:0")
    ctx.gauge_load(0, torch.from_numpy(U).to(dev))
    for p, Up in enumerate(Ups):
        ctx.gauge_load(1 + p, torch.from_numpy(Up).to(dev))
    noise = torch.from_numpy(eta).to(dev)
    delta = torch.empty((len(Ups), eta.shape[0]), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    return psms, ctx, w, noise, delta, len(Ups)


FAMILIES = ("dslash", "dslash_part", "block_mr", "block_solve", "blas", "net")

# HBM bytes per launch of a kernel family, from two rocprofv3 counter passes over this
# benchmark (FETCH_SIZE, then WRITE_SIZE; the summaries are in profiles/), each scaled
# by the factor that makes the counter read the known byte count of the plain copy
# kernel of the same run (copy_ceiling). Keyed by (family, workload, mode). A figure
# holds only for the kernel source it was taken on: `sha256` is that of the file
# holding the kernel, and a changed file turns the figure into null.
TRAFFIC = {
    # even-odd block kernel on 4^4 blocks, BF16 fields, kappa times the whole links staged in
    # LDS as FP16, FP16 hop arithmetic; 4 proposals x 8 right-hand sides per launch, averaged
    # over the sweeps of 6 Schwarz cycles
    ("block_mr", "32x32x32x32", "mixed_bf16"): {"bytes_per_launch": 6382000000, "source": "kernels_block.hip",
                                           "sha256": "97ef50bee5a396358c791e3fe589bf81cfc90be1cc65a2949c777f6906e129a5"},
    # full-lattice FP64 stencil at 32^4 on 4^4 blocks, one right-hand side, form 8
    ("dslash_f64_v8", "32x32x32x32/4x4x4x4", "dw"): {"bytes_per_launch": 1893000000, "source": "kernels_dirac.hip",
                                             "sha256": "c083afed6e527de12ae2a837c75e252447a736494b865db2b63ba0e8503ac78d"},
}


def block_sweep_flops(L, b, nprop: int, nrhs: int, cycles: int, block_iters: int) -> float:
    """Algorithmic flops of one Schwarz sweep launch (the even-odd minimal-residual block
    solver over the blocks of one colour), averaged over the 2 * cycles sweeps of a
    Schwarz application. Per site and right-hand side: ceil(block_iters / 2) even-odd
    iterations, each applying the in-block hops of every site once (n_in hops of 168
    flops) plus about 192 flops of inner products and updates; the right-hand side and the
    final odd solve apply the in-block hops of half the sites each; the face update applies
    the n_out hops that leave the block (all sweeps but the first)."""
    n_out = sum(2.0 / bm for bm in b)
    n_in = 8.0 - n_out
    n = (block_iters + 1) // 2
    face = (2 * cycles - 1) / (2 * cycles)
    per_site = HOP_FLOPS * n_in * (n + 1) + 192.0 * n + HOP_FLOPS * n_out * face
    sites = 1
    for v in L:
        sites *= v
    return sites / 2 * nprop * nrhs * per_site


def traffic_for(family: str, workload: str, mode: str):
    import hashlib

    t = TRAFFIC.get((family, workload, mode))
    if not t:
        return None
    path = os.path.join(ROOT, "paper_1204_1306_amd", "csrc", t["source"])
    try:
        with open(path, "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != t["sha256"]:
                return None
    except OSError:
        return None
    return t["bytes_per_launch"]


def run_steps(psms, ctx, noise, delta, nprop, params, steps, warmup, profile=False, profile_steps=None):
    """Times `steps` unprofiled steps; with `profile`, then runs `profile_steps` (default
    `steps`) more steps with per-family kernel timing (the event bookkeeping is kept out of
    the timed region, where it would add to every launch of a latency-bound step)."""
    import torch

    slots = list(range(1, 1 + nprop))
    for _ in range(warmup):
        ctx.logdet_ratio(psms.OP_SCHUR, 0, slots, noise, params, delta=delta)
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, st = ctx.logdet_ratio(psms.OP_SCHUR, 0, slots, noise, params, delta=delta)
        stats.append(st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    d = delta.cpu().numpy().copy()
    fam = {}
    if profile:
        ctx.profile(True)
        for _ in range(steps if profile_steps is None else profile_steps):
            ctx.logdet_ratio(psms.OP_SCHUR, 0, slots, noise, params, delta=delta)
        torch.cuda.synchronize()
        fam = {f: ctx.profile_read(f) for f in FAMILIES}
        ctx.profile(False)
    return dt, stats, fam, d


def dw_bandwidth(psms, L, b, kappa, U=None, reps=20, nrhs_list=(1, 4, 8)):
    """Full-lattice D_w launches on device-resident fields, HIP events on the library's
    stream, on an L lattice (32^4: its working set exceeds the 256 MB Infinity Cache)
    laid out in blocks b (the 4^4 Schwarz layout of the 32^4 solver). Operands: FP64;
    FP32 12-real links with FP32 spinors; the same links with BF16 spinors (the
    operands of the BF16 inner solves); each for 1, 4 and 8 right-hand sides (the
    links are read once per launch in the algorithmic bytes). Every stencil form is
    timed on each shape and the fastest is reported with its form number (the
    autotuner's pick for the solvers, which must serve several shapes at once, is
    reported beside it)."""
    import torch

    from paper_1204_1306_amd import synth

    dev = torch.device("cuda:0")
    ctx = psms.Context(L, b, kappa, stream=torch.cuda.current_stream().cuda_stream)
    ctx.gauge_load(0, torch.from_numpy(U if U is not None else synth.gauge_field(L, 0.6, 5001)).to(dev))
    tune = ctx.autotune(0, None)
    out = {"lattice": "x".join(map(str, L)), "blocks": "x".join(map(str, b)), "tuning": tune}
    forms = (("f64", "dslash_variant_f64", lambda x: ctx.apply_dw(0, x, psms.F64)),
             ("mixed", "dslash_variant_f32", lambda x: ctx.apply_dw(0, x, psms.MIXED)),
             ("bf16", "dslash_variant_bf16", lambda x: ctx.apply_dw_lowp(0, x, psms.SPINOR_BF16, psms.SPINOR_BF16)))
    ctx.set_tuning("nr_f64", 1)
    ctx.set_tuning("nr_low", 1)
    for n in nrhs_list:
        psi = torch.from_numpy(synth.gaussian_noise(L, n, 7)).to(dev)
        for name, key, fn in forms:
            best = None
            for v in range(9):
                ctx.set_tuning(key, v)
                fn(psi)
                torch.cuda.synchronize()
                ctx.profile(True)
                for _ in range(reps):
                    fn(psi)
                torch.cuda.synchronize()
                r = ctx.profile_read("dslash")
                ctx.profile(False)
                cur = {"gbs": r["bytes"] / (r["ms"] * 1e-3) / 1e9, "us_per_launch": 1e3 * r["ms"] / r["launches"],
                       "bytes_per_launch": r["bytes"] / r["launches"], "form": v}
                if best is None or cur["us_per_launch"] < best["us_per_launch"]:
                    best = cur
            ctx.set_tuning(key, tune[key])
            out[name if n == 1 else f"{name}_n{n}"] = best
        del psi
        torch.cuda.empty_cache()
    ctx.close()
    return out


def copy_ceiling(mib=512, reps=10):
    """A plain device copy of known size (an elementwise kernel reading and writing
    `mib` MiB each way): the achievable HBM rate on this GPU, and the kernel against
    which the HBM byte counters of a profiled run are calibrated."""
    import torch

    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        torch.mul(src, 1.0, out=dst)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 2 * n * 4
    del src, dst
    return {"bytes_per_launch": nbytes, "us_per_launch": round(1e3 * ms, 2), "gbs": round(nbytes / (ms * 1e-3) / 1e9, 1)}


def learned_leg(psms, ctx, w, noise, nprop, nnoise, steps, npairs, train_lattice=(16, 16, 16, 16)):
    """The learned preconditioner on the workload's geometry. The network (1-8-8-8-1
    channels) is trained on the GPU on seeded configurations of the near-critical 16^4
    lattice (kappa 0.157, links exp(i 0.6 H), seeds 4000 + k), outside the timed region;
    its weights act on any lattice, so they are loaded into the workload's context. Then
    the estimator is timed with the network as right preconditioner of the mixed-precision
    solver on the first `nprop` proposals x `nnoise` noise fields of the workload."""
    import torch

    from paper_1204_1306_amd import synth

    dev = torch.device("cuda:0")
    tctx = psms.Context(train_lattice, (4, 4, 4, 4), 0.157, stream=torch.cuda.current_stream().cuda_stream)
    train_slots = []
    for k in range(4):
        tctx.gauge_load(k, torch.from_numpy(synth.gauge_field(train_lattice, 0.6, 4000 + k)).to(dev))
        train_slots.append(k)
    chans = (1, 8, 8, 8, 1)
    tctx.net_init(chans, seed=7, scale=0.05)
    t0 = time.perf_counter()
    tr = tctx.net_train(train_slots, npairs=npairs, batch=8, epochs=2, chunk=64, lr=2e-3, solve_tol=1e-6)
    t_train = time.perf_counter() - t0
    weights = tctx.net_get_weights()
    tctx.close()
    ctx.net_init(chans)
    ctx.net_set_weights(weights)
    prm = mode_params(psms, "learned", w["tol"])
    sub = noise[:nnoise]
    delta = torch.empty((nprop, nnoise), dtype=torch.float64, device=dev)
    dt, st, fam, d = run_steps(psms, ctx, sub, delta, nprop, prm, steps, 0, profile=True, profile_steps=1)
    return {"s_per_estimate": dt / steps / (nprop * nnoise), "estimates_per_step": nprop * nnoise,
            "train_lattice": "x".join(map(str, train_lattice)), "train_seconds": t_train, "train": tr,
            "solver": st[-1], "net_ms_per_step": fam["net"]["ms"]}, d


def net_leg(psms, L=(16, 16, 16, 16), nrhs=8, reps=10):
    """Applications of the gauge-covariant network (1-8-8-8-1 channels, the learned
    preconditioner's shape) to nrhs fields on an L lattice (the near-critical 16^4
    workload's size), timed on the library's stream. Algorithmic flops count the
    complex spin mixing (9 transports x C_in x C_out complex 4x4 spin matrices on 3
    colours, 8 flops per complex multiply-add) and the parallel transports (8
    directions x C_in fields x 4 spins x a 3x3 complex matrix-vector product); the
    matrix cores execute the mixing as a real GEMM of twice the mixing flops."""
    import torch

    from paper_1204_1306_amd import synth

    dev = torch.device("cuda:0")
    ctx = psms.Context(L, tuple(max(2, v // 4) for v in L), 0.157, stream=torch.cuda.current_stream().cuda_stream)
    ctx.gauge_load(0, torch.from_numpy(synth.gauge_field(L, 0.6, 4999)).to(dev))
    chans = (1, 8, 8, 8, 1)
    ctx.net_init(chans, seed=7, scale=0.05)
    psi = torch.from_numpy(synth.gaussian_noise(L, nrhs, 11)).to(dev)
    out = {"lattice": "x".join(map(str, L)), "nrhs": nrhs, "channels": list(chans)}
    V = int(np.prod(L))
    mix = sum(9 * ci * co * 48 * 8 for ci, co in zip(chans[:-1], chans[1:]))
    transport = sum(8 * ci * 4 * 9 * 8 for ci in chans[:-1])
    for name, flag in (("mfma_bf16", 1), ("valu_fp32", 0)):
        ctx.set_tuning("net_mfma", flag)
        ctx.net_apply(0, psi)
        torch.cuda.synchronize()
        ctx.profile(True)
        for _ in range(reps):
            ctx.net_apply(0, psi)
        torch.cuda.synchronize()
        r = ctx.profile_read("net")
        ctx.profile(False)
        ms = r["ms"] / reps
        out[name] = {"ms_per_apply": round(ms, 3),
                     "algorithmic_tflops": round(nrhs * V * (mix + transport) / (ms * 1e-3) / 1e12, 2),
                     "mixing_gemm_tflops": round(nrhs * V * 2 * mix / (ms * 1e-3) / 1e12, 2)}
    ctx.close()
    return out


def batched_leg(psms, workload: str, steps: int, rhs_chunk: int):
    """The batched workload (all proposals x noise vectors of it in one call), with
    BF16 Krylov storage and FP32 inner solves against plain FP64, same tolerance."""
    import torch

    _, ctx, w, noise, delta, nprop = setup(workload)
    tune = ctx.autotune(0, None)
    nest = nprop * noise.shape[0]
    out = {"workload": workload, "estimates_per_step": nest, "rhs_chunk": rhs_chunk,
           "tuning": {k: tune[k] for k in ("dslash_variant_f64", "dslash_variant_f32", "dslash_variant_bf16", "nr_f64",
                                            "nr_low")}}
    d = {}
    for mode in ("mixed_bf16", "plain"):
        prm = mode_params(psms, mode, w["tol"], workload)
        prm.rhs_chunk = rhs_chunk
        dt, st, _, d[mode] = run_steps(psms, ctx, noise, delta, nprop, prm, steps, 1)
        out[mode] = {"s_per_estimate": dt / steps / nest, "ms_per_step": 1e3 * dt / steps, "solver": st[-1]}
        log(f"batched {workload} {mode}: {1e3 * dt / steps:.1f} ms/step")
    out["speedup_vs_plain_f64"] = out["plain"]["s_per_estimate"] / out["mixed_bf16"]["s_per_estimate"]
    out["max_abs_delta_diff"] = float(np.abs(d["mixed_bf16"] - d["plain"]).max())
    ctx.close()
    del noise, delta
    torch.cuda.empty_cache()
    return out


def interpolation_leg(psms, ctx, w, nprop, steps: int, ns=(1, 2, 4)):
    """The estimator with gauge-field interpolation (N factors, FP64), without and with
    the relative gauge fixing of the pair (App. B, default parameters; g on the
    block-interior sites): seconds per estimate and the spread of Delta over the noise
    fields, which the method reduces about as 1/sqrt(N). Each factor draws its own seeded
    noise; both variants see the same noise. Then the unfixed pair in mixed precision
    (FP32 inner solves; the intermediate fields, not SU(3), on FP32 18-real links), with
    the largest difference of its Deltas from the FP64 ones."""
    import torch

    from paper_1204_1306_amd import synth

    prm = mode_params(psms, "plain", w["tol"])
    nn = w["nnoise"]
    out = {}
    t0 = time.perf_counter()
    g_fix = {}
    for p in range(nprop):
        _, g_fix[p] = ctx.relative_gauge_fix(0, 1 + p, 40 + 2 * p, 41 + 2 * p)
    torch.cuda.synchronize()
    out["gauge_fix_seconds"] = time.perf_counter() - t0
    out["gauge_fix"] = g_fix[0]
    mixed = mode_params(psms, "mixed", w["tol"])
    d_f64 = {}
    for variant in ("", "fixed_", "mixed_"):
        fixed = variant == "fixed_"
        pv = mixed if variant == "mixed_" else prm
        for n in ns:
            eta = torch.from_numpy(synth.gaussian_noise(w["L"], n * nn, 9100 + n)).to("cuda")
            delta = torch.empty((1, nn), dtype=torch.float64, device="cuda")
            ds, dt_all, it = [], 0.0, 0
            for p in range(nprop):
                a, b = (40 + 2 * p, 41 + 2 * p) if fixed else (0, 1 + p)
                ctx.logdet_ratio(psms.OP_SCHUR, a, [b], eta, pv, delta=delta, n_interp=n)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(steps):
                    _, st = ctx.logdet_ratio(psms.OP_SCHUR, a, [b], eta, pv, delta=delta, n_interp=n)
                torch.cuda.synchronize()
                dt_all += (time.perf_counter() - t0) / steps
                it += st["inner_iters"]
                ds.append(delta.cpu().numpy()[0])
            d = np.concatenate(ds)
            out[f"{variant}n{n}"] = {"s_per_estimate": dt_all / (nprop * nn), "ms_per_step": 1e3 * dt_all,
                                     "delta_std": float(d.std()), "delta_mean": float(d.mean()), "inner_iters": it}
            if variant == "":
                d_f64[n] = d
            elif variant == "mixed_":
                out[f"{variant}n{n}"]["max_abs_delta_diff_vs_f64"] = float(np.abs(d - d_f64[n]).max())
    return out


def cpu_baseline(workload: str, inputs, budget_s: float = 25.0):
    """The CPU oracle (numpy, FP64) on a bounded sample of the workload.

    * One matrix-free application of D on the whole lattice, timed: the oracle's D_w rate.
    * The full-lattice solve of one Schur estimate (proposal 0, noise 0): the oracle's CG
      on the normal equations for D(U') x = D_wb xi, run for `budget_s` seconds; the
      iterations still needed for the workload's tolerance are extrapolated from the
      residual decay of the last half of the iterations run, and the per-estimate time is
      (iterations run + still needed) x the measured time per iteration. The Dirichlet
      block solves that form (1 - PQ(U)) xi are left out, so the figure is a lower bound
      on the oracle's seconds per estimate."""
    from oracle import dirac, schur
    from oracle.solvers import norm2

    w, U, Ups, eta = inputs
    g = schur.Geometry(w["L"], w["b"])
    opP = schur.Operator(g, Ups[0], w["kappa"], direct=False)
    t0 = time.perf_counter()
    dirac.apply_D(U, eta[0], w["kappa"], w["L"])
    t_dw = time.perf_counter() - t0
    xi = g.project(eta[0])
    v = opP.D_wb(xi)
    bn = np.sqrt(norm2(v))
    x = np.zeros_like(v)
    r = v.copy()
    z = opP.Ddag(r)
    p = z.copy()
    zz = norm2(z)
    it, hist = 0, []
    t1 = time.perf_counter()
    while time.perf_counter() - t1 < budget_s and it < 5000 and (not hist or hist[-1] > w["tol"]):
        q = opP.D(p)
        a = zz / norm2(q)
        x += a * p
        r -= a * q
        it += 1
        hist.append(np.sqrt(norm2(r)) / bn)
        z = opP.Ddag(r)
        zn = norm2(z)
        p = z + (zn / zz) * p
        zz = zn
    t_cg = time.perf_counter() - t1
    per_it = t_cg / max(it, 1)
    h = np.array(hist)
    k0 = len(h) // 2
    rate = (np.log(h[-1]) - np.log(h[k0])) / max(len(h) - 1 - k0, 1)
    need = it if h[-1] <= w["tol"] else it + (np.log(w["tol"]) - np.log(h[-1])) / min(rate, -1e-12)
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count()
    threads = os.environ.get("OMP_NUM_THREADS")
    V = int(np.prod(w["L"]))
    return {"value": float(per_it * need), "unit": "s/estimate",
            "cores": int(threads) if threads and threads.isdigit() else cores, "kind": "oracle",
            "dw_seconds": t_dw, "dw_gbs": V * 960 / t_dw / 1e9,
            "sample": (f"{workload}: one oracle D_w application on the whole lattice in {t_dw:.2f} s; the full solve of "
                       f"one Schur estimate (proposal 0, noise 0) by CG on the normal equations, {it} iterations in "
                       f"{t_cg:.1f} s reaching {h[-1]:.2e}"
                       + ("" if h[-1] <= w["tol"] else f", extrapolated to {need:.0f} iterations for {w['tol']:g} from "
                          f"the residual decay of its last {len(h) - k0} iterations")
                       + "; block solves not included (lower bound)")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="32x32x32x32")
    ap.add_argument("--mode", default="mixed_bf16")
    ap.add_argument("--rhs-chunk", type=int, default=32, help="right-hand sides per solver launch (memory)")
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--plain-warmup", type=int, default=1, help="untimed plain steps first (buffers, first launches)")
    ap.add_argument("--plain-rhs-chunk", type=int, default=16, help="FP64 Krylov bases are 4x larger than BF16")
    ap.add_argument("--nprop", type=int, default=None)
    ap.add_argument("--nnoise", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--learned-pairs", type=int, default=512)
    ap.add_argument("--learned-estimates", default="1x8", help="proposals x noise of the learned leg")
    ap.add_argument("--cpu-budget", type=float, default=25.0)
    ap.add_argument("--dw-blocks", default="4,4,4,4")
    ap.add_argument("--batched-workload", default="16x16x16x16-batched", help="'none' skips the batched leg")
    ap.add_argument("--no-net-leg", action="store_true")
    ap.add_argument("--no-interp-leg", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=1)
    ap.add_argument("--batched-rhs-chunk", type=int, default=128)
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the library has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only (WORLD_SIZE > 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1204_1306_amd import synth

    t_setup = time.perf_counter()
    inputs = synth.workload_inputs(args.workload, nprop=args.nprop, nnoise=args.nnoise)
    psms, ctx, w, noise, delta, nprop = setup(args.workload, inputs=inputs)
    nnoise = noise.shape[0]
    nest = nprop * nnoise
    tune = ctx.autotune(0, None)
    log(f"workload {args.workload}: L={w['L']} b={w['b']} kappa={w['kappa']} {nprop} proposals x {nnoise} noise; "
        f"setup {time.perf_counter() - t_setup:.1f} s; tuning {tune}")

    fast = mode_params(psms, args.mode, w["tol"], args.workload)
    fast.rhs_chunk = args.rhs_chunk
    dt, stats, fam, d_fast = run_steps(psms, ctx, noise, delta, nprop, fast, args.steps, args.warmup, profile=True,
                                       profile_steps=1)
    ms_per_step = 1e3 * dt / args.steps
    log(f"{args.mode}: {ms_per_step:.2f} ms/step, solver {stats[-1]}")
    log("  kernel families (ms over one profiled step):", {f: round(v["ms"], 2) for f, v in fam.items()})

    learned = None
    d_learned = None
    if not args.no_learned:
        try:
            lp, ln = (int(v) for v in args.learned_estimates.split("x"))
            learned, d_learned = learned_leg(psms, ctx, w, noise, min(lp, nprop), min(ln, nnoise), 1,
                                             args.learned_pairs)
            log(f"learned: {learned}")
        except Exception as e:  # reported, not hidden
            learned = {"error": repr(e)}
    ctx.close()
    torch.cuda.empty_cache()

    # plain FP64 on the same batch, in a fresh context (its Krylov basis is FP64);
    # --plain-steps 0 skips it (profiling runs of the headline step alone)
    plain = mode_params(psms, "plain", w["tol"], args.workload)
    plain.rhs_chunk = args.plain_rhs_chunk
    s_plain, stp, d_plain = None, [None], None
    if args.plain_steps > 0:
        _, ctxp, _, _, _, _ = setup(args.workload, inputs=(w, inputs[1], inputs[2], inputs[3][:0]))
        for k, v in tune.items():
            ctxp.set_tuning(k, v)
        dtp, stp, _, d_plain = run_steps(psms, ctxp, noise, delta, nprop, plain, args.plain_steps, args.plain_warmup)
        s_plain = dtp / args.plain_steps / nest
        log(f"plain f64: {1e3 * dtp / args.plain_steps:.2f} ms/step, solver {stp[-1]}")
        if learned and d_learned is not None and "error" not in learned:
            learned["max_abs_delta_diff_vs_plain"] = float(np.abs(d_learned - d_plain[:d_learned.shape[0],
                                                                                       :d_learned.shape[1]]).max())
        ctxp.close()
    del noise, delta
    torch.cuda.empty_cache()

    copy = copy_ceiling()
    log(f"copy: {copy}")
    dwb = tuple(int(v) for v in args.dw_blocks.split(","))
    dw = dw_bandwidth(psms, w["L"], dwb, w["kappa"], U=inputs[1])
    log(f"D_w: {dw}")

    batched = None
    if args.batched_workload != "none":
        try:
            batched = batched_leg(psms, args.batched_workload, args.batched_steps, args.batched_rhs_chunk)
        except Exception as e:  # reported, not hidden
            batched = {"error": repr(e)}

    interp = None
    if not args.no_interp_leg:
        try:
            _, ictx, iw, _, _, inprop = setup("8x8x8x8")
            interp = interpolation_leg(psms, ictx, iw, inprop, 2)
            ictx.close()
            log(f"interpolation: {interp}")
        except Exception as e:  # reported, not hidden
            interp = {"error": repr(e)}

    net = None
    if not args.no_net_leg:
        try:
            net = net_leg(psms)
            log(f"network: {net}")
        except Exception as e:  # reported, not hidden
            net = {"error": repr(e)}

    # roofline of the dominant kernel family (by time) among those with a bytes model
    cand = [f for f in fam if fam[f]["launches"] > 0 and fam[f]["bytes"] > 0]
    dom = max(cand, key=lambda f: fam[f]["ms"])
    ach = fam[dom]["bytes"] / (fam[dom]["ms"] * 1e-3) / 1e9
    total_ms = sum(v["ms"] for v in fam.values())
    roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic_for(dom, args.workload, args.mode), "kernel": dom,
            "us_per_launch": round(1e3 * fam[dom]["ms"] / fam[dom]["launches"], 2),
            "bytes_per_launch": fam[dom]["bytes"] / fam[dom]["launches"],
            "time_share": round(fam[dom]["ms"] / max(total_ms, 1e-9), 3),
            "family_ms": {f: round(v["ms"], 2) for f, v in fam.items()}}
    if dom == "block_mr":
        # the same launches against the FP32 vector peak (the sweeps' arithmetic intensity
        # sits near the ridge: both figures are given)
        sb = w.get("sap_b") or w["b"]
        pch = min(nprop, 16)  # proposals per solver launch (the library's limit)
        flops = block_sweep_flops(w["L"], sb, pch, max(1, fast.rhs_chunk // pch), fast.sap_cycles, fast.block_iters)
        tfl = flops / (1e-3 * fam[dom]["ms"] / fam[dom]["launches"]) / 1e12
        roof["alu"] = {"flops_per_launch": flops, "achieved_tflops": round(tfl, 2),
                       "peak_tflops": FP32_VECTOR_PEAK_TFLOPS, "frac": round(tfl / FP32_VECTOR_PEAK_TFLOPS, 4),
                       "flop_per_byte": round(flops / roof["bytes_per_launch"], 2)}

    cpu = None
    if not args.no_cpu_baseline:
        try:
            cpu = cpu_baseline(args.workload, inputs, args.cpu_budget)
        except Exception as e:  # the baseline is context; report why it is missing
            cpu = {"value": None, "error": repr(e)}

    value = dt / args.steps / nest
    dtype = {"mixed": "f32+f64", "mixed_bf16": "bf16+f32+f64", "plain": "f64", "learned": "f32+f64"}[args.mode]
    dw_keys = [k for k, v in dw.items() if isinstance(v, dict) and "gbs" in v]
    line = {
        "metric": METRIC, "value": value, "unit": "s/estimate", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": (f"{'x'.join(map(str, w['L']))} lattice, {'x'.join(map(str, w['b']))} "
                                f"Schur blocks, kappa {w['kappa']}, links exp(i {w['eps']} H), {nprop} proposal(s) x "
                                f"{nnoise} noise in one call, Schur-complement ratio, relative residual {w['tol']:g}"),
                   "mode": args.mode, "estimates_per_step": nest, "rhs_chunk": args.rhs_chunk,
                   "schwarz_blocks": "x".join(map(str, w.get("sap_b") or w["b"])),
                   "schwarz": {"cycles": fast.sap_cycles, "block_iters": fast.block_iters,
                               "plain_cycles": plain.sap_cycles, "plain_block_iters": plain.block_iters}},
        "plain_f64_s_per_estimate": s_plain,
        "plain_f64_rhs_chunk": args.plain_rhs_chunk,
        "speedup_vs_plain_f64": s_plain / value if s_plain else None,
        "max_abs_delta_diff_vs_plain": float(np.abs(d_fast - d_plain).max()) if d_plain is not None else None,
        # ln mean_j exp(-Delta_pj) per proposal, from the same noise in both modes
        "log_ratio_estimate": {"fast": [round(float(v), 8) for v in psms.log_ratio_estimate(d_fast)],
                               "plain": ([round(float(v), 8) for v in psms.log_ratio_estimate(d_plain)]
                                         if d_plain is not None else None)},
        "learned": learned,
        "batched": batched,
        "interpolation": interp,
        "network": net,
        "dw_lattice": dw["lattice"],
        "dw_blocks": dw["blocks"],
        "dw_tuning": dw["tuning"],
        "dw_gbs": {k: round(dw[k]["gbs"], 1) for k in dw_keys},
        "dw_us_per_launch": {k: round(dw[k]["us_per_launch"], 2) for k in dw_keys},
        "dw_form": {k: dw[k]["form"] for k in dw_keys},
        "dw_frac_of_hbm_peak": {k: round(dw[k]["gbs"] / HBM_PEAK_GBS, 4) for k in dw_keys},
        "dw_traffic_bytes_per_launch": {"f64": traffic_for(f"dslash_f64_v{dw['f64']['form']}",
                                                          f"{dw['lattice']}/{dw['blocks']}", "dw")},
        "copy_ceiling": copy,
        "solver": {"fast": stats[-1], "plain": stp[-1]},
        "tuning": tune,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
