"""Train the gauge-covariant network preconditioner on the GPU and compare it with
Schwarz-preconditioned flexible GCR on a held-out configuration.

    python -m paper_1204_1306_amd.train_network [--lattice 16,16,16,16] [--kappa 0.157]
        [--configs 32] [--pairs 20000] [--chunk 512] [--out net.bin]

Training data are residual/correction pairs (r, e = D^-1 r) that the library's
mixed-precision Schwarz-GCR solver produces on seeded configurations (links
exp(i 0.6 H), seeds 4000 .. 4000 + configs - 1), generated and consumed chunk by
chunk; the held-out configuration has seed 4999. Prints one JSON line with the
training statistics and, on the held-out configuration, the iterations and seconds
of flexible GCR to relative residual 1e-10 with no preconditioner, with the network,
and with Schwarz, each checked by its FP64 true residual.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--lattice", default="16,16,16,16")
    ap.add_argument("--blocks", default="4,4,4,4")
    ap.add_argument("--kappa", type=float, default=0.157)
    ap.add_argument("--configs", type=int, default=32)
    ap.add_argument("--pairs", type=int, default=20000)
    ap.add_argument("--chunk", type=int, default=512)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--epochs", type=int, default=1)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--nrhs", type=int, default=8, help="right-hand sides of the held-out comparison")
    ap.add_argument("--out", default=None, help="checkpoint file of the trained network")
    args = ap.parse_args()

    import torch

    from paper_1204_1306_amd import psms, synth

    L = tuple(int(v) for v in args.lattice.split(","))
    b = tuple(int(v) for v in args.blocks.split(","))
    dev = torch.device("cuda:0")
    ctx = psms.Context(L, b, args.kappa, stream=torch.cuda.current_stream().cuda_stream)
    t0 = time.perf_counter()
    for k in range(args.configs):
        ctx.gauge_load(k, torch.from_numpy(synth.gauge_field(L, 0.6, 4000 + k)).to(dev))
        print(f"config {k} loaded", file=sys.stderr, flush=True)
    held = 63
    ctx.gauge_load(held, torch.from_numpy(synth.gauge_field(L, 0.6, 4999)).to(dev))
    t_load = time.perf_counter() - t0
    ctx.autotune(held, None)
    chans = (1, 8, 8, 8, 1)
    ctx.net_init(chans, seed=7, scale=0.05)
    t0 = time.perf_counter()
    tr = ctx.net_train(list(range(args.configs)), npairs=args.pairs, batch=args.batch, epochs=args.epochs,
                       chunk=args.chunk, lr=args.lr, solve_tol=1e-6,
                       ckpt_path=args.out)
    t_train = time.perf_counter() - t0
    print(f"trained: {tr}", file=sys.stderr, flush=True)

    bvec = torch.from_numpy(synth.gaussian_noise(L, args.nrhs, 4998)).to(dev)
    res = {}
    for name, pc in (("none", psms.PC_NONE), ("network", psms.PC_NET), ("schwarz", psms.PC_SAP)):
        prm = psms.default_params(tol=1e-10, pc=pc, restart=32, max_iter=8000, net_fallback=0)
        ctx.solve(held, bvec, prm)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st = ctx.solve(held, bvec, prm)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[name] = {"iterations": st["inner_iters"], "seconds": dt, "true_rel_residual": st["true_rel_residual"],
                     "converged": st["converged"]}
        print(f"{name}: {res[name]}", file=sys.stderr, flush=True)
    print(json.dumps({"lattice": "x".join(map(str, L)), "kappa": args.kappa, "configs": args.configs,
                      "pairs": args.pairs, "chunk": args.chunk, "channels": list(chans), "load_seconds": t_load,
                      "train_seconds": t_train, "train": tr, "held_out_seed": 4999, "nrhs": args.nrhs,
                      "held_out": res}), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
