"""Benchmark: full LBE time steps (fluid + ions + Poisson + electrode charge)
per second on the parallel-plate electro-osmosis slab, 64 x 64 x 130 lattice
sites (128 fluid planes, Debye length 8, +-0.1 kT/e, E_x = 1e-3), Poisson
solved to ||R||_inf <= 1e-10 every step.

Prints ONE JSON line.  `value` is the headline form (FP32-mixed storage and
collision, multigrid Poisson correction inside FP64 defect correction); the
FP64 form with multigrid and the FP64 form with the paper's SOR solver are
measured in the same run under "forms".  MLUPS = lattice sites x steps / wall
seconds / 1e6 over the timed steps, inputs resident in HBM.  A second window
of the same length brackets every launch with HIP events on the library's
stream to give per-kernel average durations and the cells each launch
covers; the roofline object is for the kernel kind with the largest total
time, with measured traffic from the rocprofv3 summary in profiles/ when the
kernel sources are unchanged since it was taken.  "shapes" repeats the
measurement on the coaxial (1.64 M sites) and porous-electrode (7.08 M
sites) lattices.  "adjoint" times the reverse mode on the porous electrode
(a checkpointed FP32-mixed record and one gradient of the electrode charge).
cpu_baseline times the FP64 oracle.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import paper_1907_04732_amd as lbe  # noqa: E402
import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0


def bytes_per_cell(kind: str, form: str, K: int, extrap: bool = False):
    """Algorithmic HBM bytes per cell of the grid level a launch works on
    (lattice sites for the finest level), or None where no byte model applies
    (the one-work-group coarse-level kernel, the electrode-charge gather).

    fluid: 19 populations in + out, K concentrations in, K partially
      updated concentrations out, phi (FP64), velocity out, flag word.
      ions (advection pass): K concentrations, K partial updates in, K new
      concentrations out, velocity in, Poisson source (FP64) out, flag word;
      with the extrapolated warm start also phi and the two previous
      potentials in + out, without it phi in and its kept copy out (the
      state a failed step goes back to).  One colour of a four-colour SOR
      sweep reads phi (or the correction) at every site, and reads the
      source, reads the flag word and writes the value of its own quarter.
      Jacobi sweep (the multigrid smoother): correction in and out,
      right-hand side, flag word.  Restriction, per fine cell: correction,
      residual and flag word in; per coarse cell (1/8): flag word in, rhs and
      zeroed correction out.  Prolongation, per fine cell: correction in and
      out, flag word; per coarse cell: correction and flag word.  Outer
      residual: phi, source, flag word in; correction rhs and zeroed
      correction out (multigrid).  correct: phi in + out, correction, flag
      word.
      Reverse mode: adj_moments reads the 19 stored populations and writes
      rho and m; adj_fluid reads phi, the K concentrations, rho and m, the 19
      population adjoints and K concentration adjoints of t+1, and writes 19
      population adjoints, the force adjoint and u; adj_ions reads phi, K
      concentrations, u, force adjoint, K concentration adjoints and writes K
      adjoints and the Poisson-adjoint source; adj_fold reads lambda and K
      concentrations, updates K adjoints and the summed lambda, writes the
      warm start.
    """
    f64 = form == "fp64"
    pop = 8 if f64 else 4     # population / concentration storage
    vel = 8 if f64 else 4     # velocity storage
    cor = 8 if f64 else 4     # Poisson correction storage (multigrid)
    table = {
        "fluid": 19 * pop * 2 + 2 * K * pop + 8 + 3 * vel + 4,
        "ions": 3 * K * pop + 3 * vel + 8 + 4 + (48 if extrap else 16),
        "sor": 8 + (8 + 8 + 4) / 4,
        "sor32": 4 + (4 + 4 + 4) / 4,
        "mg_smooth0": 3 * cor + 4,
        # the finest level's last sweep of a cycle also adds e to phi
        "mg_smooth0_phi": 3 * cor + 4 + 16,
        "mg_smooth": 3 * cor + 4,
        "mg_restrict": 2 * cor + 4 + (4 + 2 * cor) / 8,
        "mg_prolong": 2 * cor + 4 + (cor + 4) / 8,
        "resid": 8 + 8 + 4,
        "mg_resid": 8 + 8 + 4 + 2 * cor,
        "correct": 16 + cor + 4,
        "fcg_beta": cor + 8 + 4,
        "fcg_dir": cor + 16 + 4,
        "fcg_apply": 8 + 8 + 8 + 4,
        "fcg_update": 8 + 8 + 16 + 16 + 2 * cor + 4,
        # reverse mode: FP64 adjoint fields, concentrations in the form's storage
        "adj_moments": 19 * pop + 32 + 4,
        "adj_fluid": 8 + K * pop + 32 + 2 * 19 * 8 + 8 * K + 24 + 24 + 4,
        "adj_ions": 8 + K * pop + 24 + 24 + 2 * 8 * K + 8 + 4,
        "adj_fold": 8 + K * pop + 2 * 8 * K + 16 + 8 + 4,
    }
    return table.get(kind)


def sources_hash():
    """Hash of the kernel sources (file names and contents under csrc/)."""
    import hashlib
    d = os.path.join(ROOT, "paper_1907_04732_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h", ".cpp")):
            h.update(f.encode())
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload: str):
    """Measured bytes per launch, {(form, kind): fetch + write}, from the
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary in profiles/, or {} when there
    is none or the kernel sources have changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"step_traffic_{workload}.txt")
    if not os.path.exists(path):
        return {}
    rows, src = {}, None
    with open(path) as fh:
        for line in fh:
            t = line.split()
            if len(t) == 5 and t[0] == "traffic":
                rows[(t[1], t[2])] = float(t[3]) + float(t[4])
            elif len(t) == 2 and t[0] == "sources":
                src = t[1]
    return rows if src == sources_hash() else {}


_torch = None


def init_device():
    """Bring the device up through torch before the library touches it (torch
    does not attach to a device the HIP runtime has already initialised in
    this process); torch.cuda.synchronize() then waits for every stream on
    the device, the library's own included."""
    global _torch
    import torch
    torch.cuda.init()
    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a GPU visible to torch")
    torch.zeros(1, device="cuda")
    torch.cuda.synchronize()
    _torch = torch


def sync():
    _torch.cuda.synchronize()


def step_params(w, form: str, solver: str = "mg", check_every: int = 8, krylov=False,
                light=False):
    """The launch configuration the benchmark times on workload w.
    Multigrid forms start each solve from the quadratic extrapolation of the
    last three potentials; the SOR form keeps the paper's warm start from
    phi(t).  light: one Jacobi sweep each way on every level, V(1,1): with the
    extrapolated start a step needs little reduction, and on plates, whose
    electrodes the coarse levels represent exactly, the lighter cycle needs no
    more cycles per step; curved electrodes keep V(2,2) with Krylov
    acceleration, where the V(1,1) cycle needs 1.3-2x the iterations."""
    precision = lbe.FP64 if form == "fp64" else lbe.FP32_MIXED
    poisson = lbe.SOR4 if solver == "sor" else lbe.MG
    flags = lbe.EXTRAPOLATE if solver == "mg" else 0
    if krylov and solver == "mg":
        flags |= lbe.KRYLOV
    return lbe.make_params(w.shape, w.z, w.D, w.lB, tau=w.tau, rho0=getattr(w, "rho0", 1.0),
                           Eapp=getattr(w, "Eapp", (0.0, 0.0, 0.0)),
                           omega=getattr(w, "omega", 1.8), tol=getattr(w, "tol", 1e-10),
                           max_iter=1_000_000, check_every=check_every, precision=precision,
                           poisson=poisson, flags=flags, mg_nu1=1 if light else 2,
                           mg_nu2=1 if light else 2, mg_nu1_coarse=1 if light else 0,
                           mg_nu2_coarse=1 if light else 0)


def run_form(w: W.Workload, form: str, solver: str, steps: int, warmup: int, check_every: int,
             traffic=None, krylov=False, light=False):
    p = step_params(w, form, solver, check_every, krylov, light)
    flags = p.flags
    t_init = time.perf_counter()
    if isinstance(w, W.Batch):
        g = lbe.Lbe(p, w.node_type, w.phi_s, w.n_init, w.n_ref.reshape(-1), system=w.system,
                    nsys=len(w.L))
    else:
        g = lbe.Lbe(p, w.node_type, w.phi_s, w.n_init, w.n_ref)
    print(f"bench: {form}/{solver}: context ready in {time.perf_counter() - t_init:.2f} s",
          file=sys.stderr, flush=True)
    N = w.node_type.size
    nfluid = int((w.node_type == 0).sum())
    ffrac = nfluid / N
    g.step(warmup)
    tot0 = g.totals()
    sync()
    t0 = time.perf_counter()
    g.step(steps)
    sync()
    el = time.perf_counter() - t0
    tot1 = g.totals()
    iters = (tot1["poisson_total"] - tot0["poisson_total"]) / steps
    mlups = N * steps / el / 1e6
    print(f"bench: {form}/{solver}: {steps} steps in {el:.4f} s, {mlups:.2f} MLUPS, "
          f"{iters:.2f} {'sweeps' if solver == 'sor' else 'cycles'}/step", file=sys.stderr,
          flush=True)

    # second window: HIP events around every launch, on the library's stream
    g.profile(True)
    g.step(steps)
    kt = g.kernel_times()
    g.profile(False)
    g.close()
    kernels = {}
    for k, (ms, cnt, cells) in sorted(kt.items(), key=lambda kv: -kv[1][0]):
        if not cnt:
            continue
        avg = ms / 1e3 / cnt
        b = bytes_per_cell(k, form, len(w.z), extrap=bool(flags & lbe.EXTRAPOLATE))
        row = {"total_ms": round(ms, 4), "launches": cnt, "avg_us": round(avg * 1e6, 3),
               "cells_per_launch": int(round(cells / cnt))}
        if b is not None:
            # solid cells only read their flag word
            per_launch = (ffrac * b + (1.0 - ffrac) * 4) * cells / cnt
            row["bytes_per_launch"] = int(round(per_launch))
            row["achieved_GBs"] = round(per_launch / avg / 1e9, 1)
            row["frac"] = round(per_launch / avg / 1e9 / HBM_PEAK_GBS, 4)
        t = (traffic or {}).get((f"{form}-{solver}", k))
        if t is not None:
            row["traffic_bytes_per_launch"] = int(t)
        kernels[k] = row
        print(f"bench:   {k:12s} {ms:9.3f} ms, {cnt:6d} launches, {avg * 1e6:8.2f} us avg"
              + (f", {row['achieved_GBs']:8.1f} GB/s" if b is not None else ""),
              file=sys.stderr, flush=True)
    # roofline object: the kernel kind with the largest total time
    dom = next(iter(kernels))
    d = kernels[dom]
    roof = {"bound": "hbm", "kernel": dom, "achieved": d.get("achieved_GBs"), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": d.get("frac"), "bytes_per_launch": d.get("bytes_per_launch"),
            "avg_launch_us": d["avg_us"], "traffic": d.get("traffic_bytes_per_launch")}
    return {"mlups": round(mlups, 3), "ms_per_step": round(el / steps * 1e3, 4),
            "fluid_mlups": round(nfluid * steps / el / 1e6, 3),
            "poisson_iters_per_step": round(iters, 3), "roofline": roof, "kernels": kernels}


def cpu_baseline(w_full: W.Workload, seconds=20.0):
    """The FP64 oracle on a lateral 16 x 16 crop of the same slab (same
    column physics, Poisson tolerance and SOR settings), timed over whole
    steps after its initial solve; MLUPS counts the crop's sites."""
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
    return dict(value=round(n * steps / el / 1e6, 5), unit="MLUPS", cores=1, kind="oracle",
                sample=f"16x16x{crop.shape[2]} lateral crop of the slab, {steps} steps after the "
                       f"initial solve, tol {crop.tol:g}, SOR omega {crop.omega}, "
                       "single-threaded C oracle")


def copy_calibration(nbytes=1 << 28, reps=5):
    """A plain device copy of known size (torch), for scaling the hardware
    FETCH_SIZE / WRITE_SIZE counters in a profiling run."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"bench: copy calibration {reps} x {nbytes} bytes", file=sys.stderr, flush=True)


FORMS = {"fp32-mg": ("fp32", "mg"), "fp64-mg": ("fp64", "mg"), "fp64-sor": ("fp64", "sor"),
         "fp32-sor": ("fp32", "sor")}

# Larger lattices whose working sets exceed the 256 MB last-level cache, so
# that the fluid and ion kernels stream from HBM: the coaxial capacitor
# (1.64 M sites) and the porous electrode (7.08 M sites); and the parameter
# sweep of 96 independent 8x8xL plate systems (L 16..256, Debye length 2..16,
# voltage 0.01..0.2) packed in one lattice (0.94 M sites).
SHAPES = {"coaxial_160x160x64": lambda: W.coaxial(noise=True),
          "porous_electrode_192^3": lambda: W.porous_electrode(noise=True),
          "batched_96_slabs": lambda: W.batch_slabs(noise=True)}


def run_shapes(names, forms, steps, warmup, check_every):
    out = {}
    for name in names:
        w = SHAPES[name]()
        nfluid = int((w.node_type == 0).sum())
        print(f"bench: {w.name}, {w.node_type.size} sites, {nfluid} fluid", file=sys.stderr,
              flush=True)
        res = {}
        for f in forms:
            form, solver = FORMS[f]
            r = run_form(w, form, solver, steps, warmup, check_every, krylov=True)
            keep = {k: r["kernels"][k] for k in ("fluid", "ions") if k in r["kernels"]}
            res[f] = {"mlups": r["mlups"], "ms_per_step": r["ms_per_step"],
                      "poisson_iters_per_step": r["poisson_iters_per_step"],
                      "roofline": r["roofline"], "step_kernels": keep}
        out[w.name] = {"sites": int(w.node_type.size), "fluid_sites": nfluid, "steps": steps,
                       "poisson": "multigrid-preconditioned flexible CG", "forms": res}
    return out


def run_adjoint(w: W.Workload, form: str, steps: int, every: int, check_every: int):
    """Reverse mode on workload w: lbe_record of `steps` steps with a
    checkpoint every `every`, then one lbe_adjoint (gradient of electrode 1's
    charge with respect to every node potential, l_B and the initial state),
    which recomputes each segment and runs one reverse step plus one adjoint
    Poisson solve per step.  MLUPS count lattice sites x steps.  A second
    lbe_adjoint call with HIP events around every launch gives the kernel
    averages."""
    precision = lbe.FP64 if form == "fp64" else lbe.FP32_MIXED
    p = lbe.make_params(w.shape, w.z, w.D, w.lB, tau=w.tau, rho0=w.rho0, Eapp=w.Eapp,
                        omega=w.omega, tol=w.tol, max_iter=1_000_000, check_every=check_every,
                        precision=precision, poisson=lbe.MG, flags=lbe.EXTRAPOLATE | lbe.KRYLOV)
    g = lbe.Lbe(p, w.node_type, w.phi_s, w.n_init, w.n_ref)
    N = w.node_type.size
    ffrac = float((w.node_type == 0).sum()) / N
    qbar = [1.0] + [0.0] * (g.ne - 1)
    sync()
    t0 = time.perf_counter()
    g.record(steps, every)
    sync()
    t_rec = time.perf_counter() - t0
    t0 = time.perf_counter()
    grad = g.adjoint(qbar)
    sync()
    t_adj = time.perf_counter() - t0
    dv = float(grad["phi_s"][w.node_type == 1].sum())
    print(f"bench: adjoint {form}: record {steps} steps in {t_rec:.3f} s, reverse sweep in "
          f"{t_adj:.3f} s, dQ1/dV1 = {dv:.6e}", file=sys.stderr, flush=True)
    g.profile(True)
    g.adjoint(qbar)
    kt = g.kernel_times()
    g.profile(False)
    g.close()
    kernels = {}
    for k, (ms, cnt, cells) in sorted(kt.items(), key=lambda kv: -kv[1][0]):
        if not cnt:
            continue
        avg = ms / 1e3 / cnt
        row = {"total_ms": round(ms, 4), "launches": cnt, "avg_us": round(avg * 1e6, 3)}
        b = bytes_per_cell(k, form, len(w.z), extrap=True)
        if b is not None:
            per_launch = (ffrac * b + (1.0 - ffrac) * 4) * cells / cnt
            row["bytes_per_launch"] = int(round(per_launch))
            row["achieved_GBs"] = round(per_launch / avg / 1e9, 1)
            row["frac"] = round(per_launch / avg / 1e9 / HBM_PEAK_GBS, 4)
        kernels[k] = row
        print(f"bench:   {k:12s} {ms:9.3f} ms, {cnt:6d} launches, {avg * 1e6:8.2f} us avg"
              + (f", {row['achieved_GBs']:8.1f} GB/s" if b is not None else ""),
              file=sys.stderr, flush=True)
    adj = [k for k in kernels if k.startswith("adj_") and "frac" in kernels[k]]
    dom = adj[0] if adj else None
    roof = None
    if dom:
        d = kernels[dom]
        roof = {"bound": "hbm", "kernel": dom, "achieved": d["achieved_GBs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": d["frac"], "bytes_per_launch": d["bytes_per_launch"],
                "avg_launch_us": d["avg_us"], "traffic": None}
    return {"workload": w.name, "form": form, "steps": steps, "checkpoint_every": every,
            "objective": "charge of electrode 1 at the last step",
            "record_mlups": round(N * steps / t_rec / 1e6, 3),
            "reverse_mlups": round(N * steps / t_adj / 1e6, 3),
            "gradient_mlups": round(N * steps / (t_rec + t_adj) / 1e6, 3),
            "dQ1_dV1": dv, "roofline": roof, "kernels": kernels}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--forms", default="fp32-mg,fp64-mg,fp64-sor",
                    help="comma list of " + ",".join(FORMS) + "; the first is the headline")
    ap.add_argument("--check-every", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--shapes", default=",".join(SHAPES),
                    help="comma list of larger lattices measured beside the headline (empty: none)")
    ap.add_argument("--shape-forms", default="fp32-mg,fp64-mg")
    ap.add_argument("--shape-steps", type=int, default=200)
    ap.add_argument("--adjoint-forms", default="fp32-mg",
                    help="forms of the reverse-mode measurement on the porous electrode "
                         "(empty: none)")
    ap.add_argument("--adjoint-steps", type=int, default=400)
    ap.add_argument("--adjoint-every", type=int, default=200)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the LBE step is not sharded across GPUs in this "
              "build (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    init_device()
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    w = W.eo_slab(noise=True)
    N = w.node_type.size
    print(f"bench: {w.name}, {N} sites", file=sys.stderr, flush=True)
    if args.copy_calibration:
        copy_calibration()
    traffic = load_traffic(w.name)
    res = {}
    for name in forms:
        form, solver = FORMS[name]
        # SOR needs hundreds of sweeps per step: time fewer steps
        steps = args.steps if solver == "mg" else max(2, args.steps // 10)
        res[name] = run_form(w, form, solver, steps, args.warmup if solver == "mg" else 2,
                             args.check_every, traffic, light=True)
    head = res[forms[0]]
    hform, hsolver = FORMS[forms[0]]
    out = {
        # value: the headline form's MLUPS; the FP64 form is in "forms", the
        # fraction of the HBM peak in "roofline"
        "metric": "MLUPS per full LBE step (fluid+ions+Poisson), FP64 vs FP32-mixed, % HBM peak",
        "value": head["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps if hsolver == "mg" else max(2, args.steps // 10),
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if hform == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": w.name, "sites": N, "fluid_sites": int((w.node_type == 0).sum()),
                   "form": forms[0], "tol": w.tol, "debye": w.extra["debye"],
                   "Eapp": list(w.Eapp), "omega": w.omega,
                   "poisson": ("geometric multigrid (Jacobi V(1,1) on every level), FP64 "
                               "defect correction, warm start extrapolated quadratically in "
                               "time" if hsolver == "mg" else
                               "four-colour SOR"),
                   "poisson_iters_per_step": head["poisson_iters_per_step"],
                   "fluid_mlups": head["fluid_mlups"]},
        "roofline": head["roofline"],
        "forms": {k: {kk: v[kk] for kk in ("mlups", "ms_per_step", "poisson_iters_per_step",
                                            "roofline")} for k, v in res.items()},
        "kernels": head["kernels"],
    }
    shapes = [x.strip() for x in args.shapes.split(",") if x.strip()]
    if shapes:
        out["shapes"] = run_shapes(shapes, [f.strip() for f in args.shape_forms.split(",")],
                                   args.shape_steps, args.warmup, args.check_every)
    aforms = [f.strip() for f in args.adjoint_forms.split(",") if f.strip()]
    if aforms:
        wp = W.porous_electrode(noise=True)
        out["adjoint"] = {f: run_adjoint(wp, FORMS[f][0], args.adjoint_steps, args.adjoint_every,
                                         args.check_every) for f in aforms}
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
