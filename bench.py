"""Benchmark of the stochastic determinant-ratio estimator on one MI355X.

A step is one pass of the whole hot path over one batch of synthetic input: for
every proposal U'_p and Gaussian noise vector eta_j of the workload,
Delta_pj = |M xi_j|^2 - |xi_j|^2 with M the Schur-complement ratio operator:
projector, Dirichlet block solves with U, inter-block hops, one full-lattice solve
with U' per pair (flexible GCR, Schwarz preconditioner, FP64 true residual to the
workload's tolerance), FP64 accumulation. Gauge fields and noise are resident in
HBM before the timed region.

The default workload is the 8^4 lattice with 4^4 blocks, kappa 0.15, 16 noise
vectors, tolerance 1e-10, timed once with FP32 inner solves and FP64 defect
correction (the value) and once fully in FP64 (plain). Prints one JSON line;
progress goes to stderr.
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Schwarz cycles x block iterations where the measured best differs from the library
# default (4 x 6, best for mixed at 8^4 and for both modes at 16^4 and 32^4): plain
# FP64 at 8^4 prefers 5 x 6.
SAP_TUNED = {("8x8x8x8", "plain"): (5, 6)}


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


def setup(workload: str, nprop=None, nnoise=None):
    import torch

    from paper_1204_1306_amd import psms, synth

    w, U, Ups, eta = synth.workload_inputs(workload, nprop=nprop, nnoise=nnoise)
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
    # even-odd FP32 block kernel, four lanes per site, links staged in LDS; 8 blocks x 16
    # right-hand sides, Schwarz sweeps (4 cycles x 6 block iterations, averaged over launches)
    ("block_mr", "8x8x8x8", "mixed"): {"bytes_per_launch": 27262906, "source": "kernels_block.hip",
                                  "sha256": "3d1ecb116bacd732d136ac32d3a26135b09d40adacb7f9b296ca9c1871b2326e"},
    # full-lattice FP64 stencil at 32^4 on 4x4x8x16 blocks, four lanes per site (variant 6)
    # and split form (variant 1); keyed by lattice/block shape
    ("dslash_f64_v6", "32x32x32x32/4x4x8x16", "dw"): {"bytes_per_launch": 1351452507, "source": "kernels_dirac.hip",
                                              "sha256": "972445184e6d1e397207f9b942531f8af75d7f6d8ce2c60c172ca9605582bc3b"},
    ("dslash_f64_v1", "32x32x32x32/4x4x8x16", "dw"): {"bytes_per_launch": 1322265086, "source": "kernels_dirac.hip",
                                              "sha256": "972445184e6d1e397207f9b942531f8af75d7f6d8ce2c60c172ca9605582bc3b"},
}


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


def run_steps(psms, ctx, noise, delta, nprop, params, steps, warmup, profile=False):
    """Times `steps` unprofiled steps; with `profile`, then runs the same number of steps
    again with per-family kernel timing (the event bookkeeping is kept out of the timed
    region, where it would add to every launch of a latency-bound step)."""
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
        for _ in range(steps):
            ctx.logdet_ratio(psms.OP_SCHUR, 0, slots, noise, params, delta=delta)
        torch.cuda.synchronize()
        fam = {f: ctx.profile_read(f) for f in FAMILIES}
        ctx.profile(False)
    return dt, stats, fam, d


def dw_blocks(L, spec: str = "auto"):
    """Block layout of the D_w leg. The operator does not depend on it; the layout sets
    which sites a workgroup tile and its concurrent neighbours touch. "auto" takes blocks
    of L/8, L/8, L/4, L/2 (4x4x8x16 at 32^4: long along the fastest direction, measured
    best among the shapes tried), else an explicit "b0,b1,b2,b3"."""
    if spec != "auto":
        return tuple(int(v) for v in spec.split(","))
    b = (L[0] // 8, L[1] // 8, L[2] // 4, L[3] // 2)
    ok = all(x >= 2 and x % 2 == 0 and l % x == 0 and (l // x) % 2 == 0 for x, l in zip(b, L))
    return b if ok else tuple(max(2, v // 4) for v in L)


def dw_bandwidth(psms, L, b, kappa, reps=20):
    """Full-lattice D_w launches on device-resident fields (FP64 and mixed), HIP events on
    the library's stream, on an L lattice (32^4 by default: its working set exceeds the
    256 MB Infinity Cache)."""
    import torch

    from paper_1204_1306_amd import synth

    dev = torch.device("cuda:0")
    ctx = psms.Context(L, b, kappa, stream=torch.cuda.current_stream().cuda_stream)
    ctx.gauge_load(0, torch.from_numpy(synth.gauge_field(L, 0.6, 5001)).to(dev))
    tune = ctx.autotune(0, None)
    psi = torch.from_numpy(synth.gaussian_noise(L, 1, 7)).to(dev)
    out = {"lattice": "x".join(map(str, L)), "blocks": "x".join(map(str, b)), "tuning": tune}
    for name, prec in (("f64", psms.F64), ("mixed", psms.MIXED)):
        ctx.apply_dw(0, psi, prec)
        torch.cuda.synchronize()
        ctx.profile(True)
        for _ in range(reps):
            ctx.apply_dw(0, psi, prec)
        torch.cuda.synchronize()
        r = ctx.profile_read("dslash")
        ctx.profile(False)
        out[name] = {"gbs": r["bytes"] / (r["ms"] * 1e-3) / 1e9, "us_per_launch": 1e3 * r["ms"] / r["launches"],
                     "bytes_per_launch": r["bytes"] / r["launches"]}
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


def learned_leg(psms, ctx, w, noise, delta, nprop, steps, npairs):
    """Train the gauge-covariant network on seeded configurations of the workload's
    geometry (outside the timed region), then time the estimator with it as the right
    preconditioner of the mixed-precision solver."""
    import torch

    from paper_1204_1306_amd import synth

    dev = torch.device("cuda:0")
    train_slots = []
    for k in range(4):
        ctx.gauge_load(40 + k, torch.from_numpy(synth.gauge_field(w["L"], w["eps"], 9000 + k)).to(dev))
        train_slots.append(40 + k)
    ctx.net_init((1, 8, 8, 8, 1), seed=7, scale=0.05)
    t0 = time.perf_counter()
    tr = ctx.net_train(train_slots, npairs=npairs, batch=8, epochs=2, chunk=64, lr=2e-3, solve_tol=1e-6)
    t_train = time.perf_counter() - t0
    prm = mode_params(psms, "learned", w["tol"])
    dt, st, fam, d = run_steps(psms, ctx, noise, delta, nprop, prm, steps, 1, profile=True)
    return {"s_per_estimate": dt / steps / (nprop * noise.shape[0]), "train_seconds": t_train, "train": tr,
            "solver": st[-1], "net_ms_per_step": fam["net"]["ms"] / steps}, d


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
    """The estimator with gauge-field interpolation (N factors, FP64): seconds per
    estimate and the spread of Delta over the noise fields, which the method reduces
    about as 1/sqrt(N). Each factor draws its own seeded noise."""
    import torch

    from paper_1204_1306_amd import synth

    prm = mode_params(psms, "plain", w["tol"])
    slots = list(range(1, 1 + nprop))
    nn = w["nnoise"]
    out = {}
    for n in ns:
        eta = torch.from_numpy(synth.gaussian_noise(w["L"], n * nn, 9100 + n)).to("cuda")
        delta = torch.empty((nprop, nn), dtype=torch.float64, device="cuda")
        ctx.logdet_ratio(psms.OP_SCHUR, 0, slots, eta, prm, delta=delta, n_interp=n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, st = ctx.logdet_ratio(psms.OP_SCHUR, 0, slots, eta, prm, delta=delta, n_interp=n)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        d = delta.cpu().numpy()
        out[f"n{n}"] = {"s_per_estimate": dt / (nprop * nn), "ms_per_step": 1e3 * dt,
                        "delta_std": float(d.std()), "delta_mean": float(d.mean()),
                        "inner_iters": st["inner_iters"]}
    return out


def cpu_baseline(workload: str, budget_s: float = 20.0):
    """The CPU oracle on a bounded sample of the workload: one Schur estimate (one
    proposal, one noise vector). The Dirichlet block solves are timed on two blocks per
    colour (dense LU) and scaled to all blocks; the full solve is CG on the normal
    equations, run until the workload tolerance or the time budget, and scaled to the
    tolerance from the observed residual decay when the budget ends first."""
    from oracle import schur
    from oracle.solvers import norm2
    from paper_1204_1306_amd import synth

    w, U, Ups, eta = synth.workload_inputs(workload, nprop=1, nnoise=1)
    g = schur.Geometry(w["L"], w["b"])
    opU = schur.Operator(g, U, w["kappa"], direct=False)
    opP = schur.Operator(g, Ups[0], w["kappa"], direct=False)
    xi = g.project(eta[0])
    nsample = min(2, g.V // int(np.prod(w["b"])) // 2)
    t0 = time.perf_counter()
    for mask in (g.black, g.white):
        for k in np.unique(g.block[mask])[:nsample]:
            m = g.block == k
            lu = schur.DenseLU(opU.sub_matrix(m, m).toarray())
            lu.solve(xi.reshape(-1)[g.dofs(m)])
    t_blk = (time.perf_counter() - t0) / (2 * nsample)
    nblk = g.V // int(np.prod(w["b"]))
    t_schur = t_blk * nblk
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
    return {"value": float(t_schur + per_it * need), "unit": "s/estimate",
            "cores": int(threads) if threads and threads.isdigit() else cores, "kind": "oracle",
            "sample": (f"one {workload} Schur estimate (1 proposal x 1 noise): block solves by dense LU timed on "
                       f"{nsample} blocks per colour ({t_blk:.3f} s each) x {nblk} blocks = {t_schur:.2f} s; full solve "
                       f"by CG on the normal equations, {it} iterations in {t_cg:.1f} s reaching {h[-1]:.1e}"
                       + ("" if h[-1] <= w["tol"] else f", scaled to {need:.0f} iterations for {w['tol']:g}"))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="8x8x8x8")
    ap.add_argument("--mode", default="mixed")
    ap.add_argument("--plain-steps", type=int, default=10)
    ap.add_argument("--nprop", type=int, default=None)
    ap.add_argument("--nnoise", type=int, default=None)
    ap.add_argument("--rhs-chunk", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--learned-pairs", type=int, default=512)
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--dw-lattice", default="32,32,32,32")
    ap.add_argument("--dw-blocks", default="auto")
    ap.add_argument("--batched-workload", default="16x16x16x16-batched", help="'none' skips the batched leg")
    ap.add_argument("--no-net-leg", action="store_true")
    ap.add_argument("--no-interp-leg", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=2)
    ap.add_argument("--batched-rhs-chunk", type=int, default=128)
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only (WORLD_SIZE > 1).", file=sys.stderr)
        sys.exit(2)

    psms, ctx, w, noise, delta, nprop = setup(args.workload, args.nprop, args.nnoise)
    nnoise = noise.shape[0]
    nest = nprop * nnoise
    tune = ctx.autotune(0, None)
    log(f"workload {args.workload}: L={w['L']} b={w['b']} kappa={w['kappa']} {nprop} proposals x {nnoise} noise; "
        f"tuning {tune}")

    fast = mode_params(psms, args.mode, w["tol"], args.workload)
    fast.rhs_chunk = args.rhs_chunk
    dt, stats, fam, d_fast = run_steps(psms, ctx, noise, delta, nprop, fast, args.steps, args.warmup, profile=True)
    ms_per_step = 1e3 * dt / args.steps
    log(f"{args.mode}: {ms_per_step:.2f} ms/step, solver {stats[-1]}")
    log("  kernel families (ms over the timed steps):", {f: round(v["ms"], 2) for f, v in fam.items()})

    plain = mode_params(psms, "plain", w["tol"], args.workload)
    plain.rhs_chunk = args.rhs_chunk
    dtp, stp, _, d_plain = run_steps(psms, ctx, noise, delta, nprop, plain, args.plain_steps, 1)
    s_plain = dtp / args.plain_steps / nest
    log(f"plain f64: {1e3 * dtp / args.plain_steps:.2f} ms/step, solver {stp[-1]}")

    # the same mixed step with the noise and Delta in (pageable) host memory: the library
    # stages the noise over PCIe and returns Delta to the host in every call
    host_buffers = None
    try:
        noise_h = noise.cpu().numpy()
        delta_h = np.empty((nprop, nest // nprop), np.float64)
        slots = list(range(1, 1 + nprop))
        ctx.logdet_ratio(psms.OP_SCHUR, 0, slots, noise_h, fast, delta=delta_h)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.logdet_ratio(psms.OP_SCHUR, 0, slots, noise_h, fast, delta=delta_h)
        dth = time.perf_counter() - t0
        host_buffers = {"s_per_estimate": dth / args.steps / nest, "ms_per_step": 1e3 * dth / args.steps,
                        "max_abs_delta_diff": float(np.abs(delta_h - d_fast).max())}
        log(f"host buffers: {host_buffers}")
    except Exception as e:  # reported, not hidden
        host_buffers = {"error": repr(e)}

    interp = None
    if not args.no_interp_leg:
        try:
            interp = interpolation_leg(psms, ctx, w, nprop, max(1, args.plain_steps // 2))
            log(f"interpolation: {interp}")
        except Exception as e:  # reported, not hidden
            interp = {"error": repr(e)}

    learned = None
    if not args.no_learned:
        try:
            learned, d_learned = learned_leg(psms, ctx, w, noise, delta, nprop, max(1, args.plain_steps // 2),
                                             args.learned_pairs)
            learned["max_abs_delta_diff_vs_plain"] = float(np.abs(d_learned - d_plain).max())
            log(f"learned: {learned}")
        except Exception as e:  # reported, not hidden
            learned = {"error": repr(e)}

    batched = None
    if args.batched_workload != "none":
        try:
            batched = batched_leg(psms, args.batched_workload, args.batched_steps, args.batched_rhs_chunk)
        except Exception as e:  # reported, not hidden
            batched = {"error": repr(e)}

    net = None
    if not args.no_net_leg:
        try:
            net = net_leg(psms)
            log(f"network: {net}")
        except Exception as e:  # reported, not hidden
            net = {"error": repr(e)}

    copy = copy_ceiling()
    log(f"copy: {copy}")
    dwL = tuple(int(v) for v in args.dw_lattice.split(","))
    dw = dw_bandwidth(psms, dwL, dw_blocks(dwL, args.dw_blocks), w["kappa"])
    log(f"D_w: {dw}")

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

    cpu = None
    if not args.no_cpu_baseline:
        try:
            cpu = cpu_baseline(args.workload, args.cpu_budget)
        except Exception as e:  # the baseline is context; report why it is missing
            cpu = {"value": None, "error": repr(e)}

    value = dt / args.steps / nest
    dtype = {"mixed": "f32+f64", "mixed_bf16": "bf16+f32+f64", "plain": "f64", "learned": "f32+f64"}[args.mode]
    line = {
        "metric": METRIC, "value": value, "unit": "s/estimate", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": (f"{'x'.join(map(str, w['L']))} lattice, {'x'.join(map(str, w['b']))} "
                                f"blocks, kappa {w['kappa']}, links exp(i {w['eps']} H), {nprop} proposal(s) x {nnoise} "
                                f"noise, Schur-complement ratio, relative residual {w['tol']:g}"),
                   "mode": args.mode, "estimates_per_step": nest,
                   "schwarz": {"cycles": fast.sap_cycles, "block_iters": fast.block_iters,
                               "plain_cycles": plain.sap_cycles, "plain_block_iters": plain.block_iters}},
        "plain_f64_s_per_estimate": s_plain,
        "speedup_vs_plain_f64": s_plain / value,
        "max_abs_delta_diff_vs_plain": float(np.abs(d_fast - d_plain).max()),
        # PCIe-inclusive: the same step with the noise and Delta in pageable host memory
        "host_buffers": host_buffers,
        # gauge-field interpolation with N factors (FP64): cost and spread of Delta
        "interpolation": interp,
        # ln mean_j exp(-Delta_pj) per proposal, from the same noise in both modes
        "log_ratio_estimate": {"fast": [round(float(v), 10) for v in psms.log_ratio_estimate(d_fast)],
                               "plain": [round(float(v), 10) for v in psms.log_ratio_estimate(d_plain)]},
        "learned": learned,
        "batched": batched,
        "network": net,
        "dw_lattice": dw["lattice"],
        "dw_blocks": dw["blocks"],
        "dw_tuning": dw["tuning"],
        "dw_gbs": {k: round(v["gbs"], 1) for k, v in dw.items() if isinstance(v, dict) and "gbs" in v},
        "dw_us_per_launch": {k: round(v["us_per_launch"], 2) for k, v in dw.items() if isinstance(v, dict) and "gbs" in v},
        "dw_frac_of_hbm_peak": {k: round(v["gbs"] / HBM_PEAK_GBS, 4) for k, v in dw.items()
                                if isinstance(v, dict) and "gbs" in v},
        "dw_traffic_bytes_per_launch": {"f64": traffic_for(f"dslash_f64_v{dw['tuning']['dslash_variant_f64']}",
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
