"""Benchmark: full LBE time steps (fluid + ions + Poisson + charge) per second
on the parallel-plate electro-osmosis slab, 64 x 64 x 130 lattice sites.

Prints ONE JSON line (rank 0, one GPU):
  metric "MLUPS per full LBE step (fluid+ions+Poisson)" = lattice sites x
  steps / wall seconds / 1e6, counting every site, with the inputs resident
  in HBM; a roofline object for the kernel that takes the most GPU time, and
  the FP64 oracle timed on the host cores on a bounded sample of the same
  workload.
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

import paper_1907_04732_amd as lbe  # noqa: E402
import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0

# Algorithmic HBM bytes per lattice site for one launch of each kernel
# (FP64 form).  fluid: 19 populations in + out, 2 species in, phi, 3 velocity
# components out, the node's flag word.  ions: 2 species in + out, phi, 3
# velocity components in, Poisson source out, flag word.  sor (one colour
# launch, per lattice site): the launch must read phi at every node of the
# other three colours (6 B per site), read and write its own quarter (4 B),
# read the source (2 B) and flag word (1 B) of its quarter.  resid: phi,
# source and flag word once.
BYTES_PER_SITE_F64 = {"fluid": 19 * 16 + 16 + 8 + 24 + 4, "ions": 32 + 8 + 24 + 8 + 4,
                      "sor": 13, "resid": 20, "charge": 0, "totals": 0, "observe": 0,
                      "sor32": 0, "correct": 0}


def make_context(w: W.Workload, precision: int, solver: int, check_every: int):
    p = lbe.make_params(w.shape, w.z, w.D, w.lB, tau=w.tau, rho0=w.rho0, Eapp=w.Eapp,
                        omega=w.omega, tol=w.tol, max_iter=1_000_000, check_every=check_every,
                        precision=precision, poisson=solver)
    return lbe.Lbe(p, w.node_type, w.phi_s, w.n_init, w.n_ref)


def sync():
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.synchronize()
    except Exception:
        pass


def cpu_baseline(w_full: W.Workload, seconds=20.0):
    """The FP64 oracle on a lateral 16 x 16 crop of the same slab (same
    column physics, Poisson tolerance and SOR settings), timed over whole
    steps after its initial solve; returned as MLUPS."""
    import oracle
    crop = W.eo_slab(noise=True, nx=16, ny=16, nfluid=w_full.shape[2] - 2)
    p = oracle.make_params(crop.shape, crop.z, crop.D, crop.lB, crop.tau, crop.rho0, crop.Eapp,
                           crop.omega, crop.tol, 1_000_000, 4)
    o = oracle.Oracle(p, crop.node_type, crop.phi_s, crop.n_init, crop.n_ref)
    n = crop.node_type.size
    steps, t0 = 0, time.perf_counter()
    while True:
        o.step(1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= 200:
            break
    return dict(value=n * steps / el / 1e6, unit="MLUPS", cores=1, kind="oracle",
                sample=f"16x16x{crop.shape[2]} lateral crop of the slab, {steps} steps after the "
                       f"initial solve, tol {crop.tol:g}, single-threaded C oracle")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--form", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--solver", choices=["sor", "mg"], default="sor")
    ap.add_argument("--check-every", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the LBE step is not sharded across GPUs in this "
              "build (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    precision = lbe.FP64 if args.form == "fp64" else lbe.FP32_MIXED
    solver = lbe.SOR4 if args.solver == "sor" else lbe.MG
    w = W.eo_slab(noise=True)
    N = w.node_type.size
    nfluid = int((w.node_type == 0).sum())
    print(f"bench: {w.name}, {N} sites, form {args.form}, solver {args.solver}", file=sys.stderr,
          flush=True)
    g = make_context(w, precision, solver, args.check_every)
    g.step(args.warmup)
    tot0 = g.totals()
    sync()
    t0 = time.perf_counter()
    g.step(args.steps)
    sync()
    el = time.perf_counter() - t0
    tot1 = g.totals()
    sweeps = (tot1["poisson_total"] - tot0["poisson_total"]) / args.steps
    mlups = N * args.steps / el / 1e6
    print(f"bench: {args.steps} steps in {el:.3f} s, {mlups:.2f} MLUPS, {sweeps:.1f} sweeps/step",
          file=sys.stderr, flush=True)

    # second timed window with per-launch HIP events on the library's stream
    g.profile(True)
    g.step(args.steps)
    kt = g.kernel_times()
    g.profile(False)
    bytes_tab = BYTES_PER_SITE_F64
    dom = max(kt, key=lambda k: kt[k][0])
    ms, cnt = kt[dom]
    avg_s = ms / 1e3 / max(cnt, 1)
    per_launch_bytes = bytes_tab.get(dom, 0) * N
    achieved = per_launch_bytes / avg_s / 1e9 if avg_s > 0 else 0.0
    for k, (kms, kc) in sorted(kt.items(), key=lambda kv: -kv[1][0]):
        if kc:
            print(f"bench: kernel {k:8s} {kms:9.3f} ms total, {kc:7d} launches, "
                  f"{kms / kc * 1e3:8.2f} us avg", file=sys.stderr, flush=True)

    out = {
        "metric": "MLUPS per full LBE step (fluid+ions+Poisson)",
        "value": round(mlups, 3),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == lbe.FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": w.name, "sites": N, "fluid_sites": nfluid,
                   "form": args.form, "poisson": args.solver, "omega": w.omega, "tol": w.tol,
                   "debye": w.extra["debye"], "Eapp": list(w.Eapp),
                   "sweeps_per_step": round(sweeps, 2),
                   "fluid_mlups": round(nfluid * args.steps / el / 1e6, 3)},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "bytes_per_launch": per_launch_bytes,
                     "avg_launch_us": round(avg_s * 1e6, 3), "traffic": None},
    }
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
