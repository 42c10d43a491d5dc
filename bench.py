"""Benchmark: full LBE time steps (fluid + ions + Poisson + electrode charge)
per second on the largest configuration, the 192^3 porous electrode
(7.08 M lattice sites: a seeded packing of spheres at +0.05 kT/e facing a
counter-electrode at -0.05, Debye length 4), Poisson solved to
||R||_inf <= 1e-10 every step.

Prints ONE JSON line.  `value` is the headline form (FP32-mixed storage and
collision, multigrid Poisson correction inside FP64 defect correction,
Krylov-accelerated); the FP64 form is measured in the same run under
"forms".  MLUPS = lattice sites x steps / wall seconds / 1e6 over the timed
steps, every input resident in HBM.  The timed window starts from a running
state: the context is first advanced --start-step steps (untimed), then
--warmup steps, then --steps timed steps, so that the window sees the
solver load of a running simulation rather than its first steps, where the
extrapolated warm start has no history yet.  A second window of the same
length brackets every launch with HIP events on the library's stream to give
per-kernel average durations and the cells each launch covers: `roofline`
is for the kernel kind with the largest total time, `roofline_step_passes`
for the two passes of the LB and ion update together; measured traffic
comes from the rocprofv3 summary in profiles/ while the sources still hash to
the build it was taken on.  "shapes" repeats the measurement on the
electro-osmosis slab (with the paper's SOR solver as well), the coaxial cell
and the 96-system batch, whose multigrid forms also carry "graph_chunks":
steps replayed from captured 16-step graphs with a fixed number of solver
units per step (lbe_step_chunk; CHUNK_UNITS) between two windows stepped
one by one; "adjoint" times
the reverse mode on the porous electrode (a checkpointed FP32-mixed record and one gradient of the
electrode charge).  cpu_baseline times the FP64 oracle on a lateral column
of the same porous electrode, single-threaded and on all host cores.

`python bench.py --summarize-rocprof DIR --workload NAME` (no GPU) turns the
CSV output of the rocprofv3 runs listed in profiles/ into their summaries.
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


def bytes_per_cell(kind: str, form: str, K: int, extrap: bool = False, krylov: bool = False):
    """Algorithmic HBM bytes per cell of the grid level a launch works on
    (lattice sites for the finest level), or None where no byte model applies
    (the one-work-group coarse-level kernel, the electrode-charge gather).

    fluid: 19 populations in + out, K concentrations in, K increments out,
      phi (FP64), velocity out, flag word.
      ions (advection pass): K concentrations, K increments in, K new
      concentrations out (the mixed form also reads and writes the K low
      words of its concentration pairs), velocity in, Poisson source (FP64)
      out, flag word;
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
      correction out (multigrid), and the FP64 residual out under Krylov
      acceleration.  correct: phi in + out, correction, flag
      word.  Krylov iteration: fcg_apply gathers the V-cycle's output z
      and reads q', p' and r, writing A z; fcg_update reads z, A z, p', q',
      phi and r and writes p, q, phi, r and the next cycle's rhs and start
      (the directions p, q are held in the correction's precision).
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
        "ions": 3 * K * pop + (0 if f64 else 2 * K * 4) + 3 * vel + 8 + 4
                + (48 if extrap else 16),
        "sor": 8 + (8 + 8 + 4) / 4,
        "sor32": 4 + (4 + 4 + 4) / 4,
        "mg_smooth0": 3 * cor + 4,
        # the finest level's last sweep of a cycle also adds e to phi
        "mg_smooth0_phi": 3 * cor + 4 + 16,
        "mg_smooth": 3 * cor + 4,
        "mg_restrict": 2 * cor + 4 + (4 + 2 * cor) / 8,
        "mg_prolong": 2 * cor + 4 + (cor + 4) / 8,
        "resid": 8 + 8 + 4,
        # with Krylov acceleration the check also keeps the FP64 residual
        "mg_resid": 8 + 8 + 4 + 2 * cor + (8 if krylov else 0),
        "correct": 16 + cor + 4,
        # Krylov: A z and four sums (z, q', p', r in; A z out); then p, q,
        # phi, r updated (z, A z, p', q', phi, r in; p, q, phi, r, the
        # correction's rhs and start out)
        "fcg_apply": 3 * cor + 8 + 4 + 8,
        "fcg_update": 7 * cor + 8 + 16 + 16 + 4,
        # reverse mode: FP64 adjoint fields, concentrations in the form's storage
        "adj_moments": 19 * pop + 32 + 4,
        "adj_fluid": 8 + K * pop + 32 + 2 * 19 * 8 + 8 * K + 24 + 24 + 4,
        "adj_ions": 8 + K * pop + 24 + 24 + 2 * 8 * K + 8 + 4,
        "adj_fold": 8 + K * pop + 2 * 8 * K + 16 + 8 + 4,
    }
    return table.get(kind)


def sources_hash():
    """Hash of the library's sources (lbe_build_id of a library built from them)."""
    from paper_1907_04732_amd.build import source_hash
    return source_hash()


def load_traffic(workload: str):
    """Measured bytes per launch, {(form, kind): fetch + write}, from the
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary in profiles/, or {} when there
    is none or the library's sources have changed since it was taken."""
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
                nu=(2, 2, 0, 0)):
    """The launch configuration the benchmark times on workload w.
    Multigrid forms start each solve from the quadratic extrapolation of the
    last three potentials; the SOR form keeps the paper's warm start from
    phi(t).  nu = (pre, post) Jacobi sweeps on the finest level and (pre,
    post) on the coarser ones (0, 0: the finest level's); krylov: each
    V-cycle preconditions flexible CG."""
    precision = lbe.FP64 if form == "fp64" else lbe.FP32_MIXED
    poisson = lbe.SOR4 if solver == "sor" else lbe.MG
    flags = lbe.EXTRAPOLATE if solver == "mg" else 0
    if krylov and solver == "mg":
        flags |= lbe.KRYLOV
    return lbe.make_params(w.shape, w.z, w.D, w.lB, tau=w.tau, rho0=getattr(w, "rho0", 1.0),
                           Eapp=getattr(w, "Eapp", (0.0, 0.0, 0.0)),
                           omega=getattr(w, "omega", 1.8), tol=getattr(w, "tol", 1e-10),
                           max_iter=1_000_000, check_every=check_every, precision=precision,
                           poisson=poisson, flags=flags, mg_nu1=nu[0], mg_nu2=nu[1],
                           mg_nu1_coarse=nu[2], mg_nu2_coarse=nu[3])


def make_context(w, p):
    if isinstance(w, W.Batch):
        return lbe.Lbe(p, w.node_type, w.phi_s, w.n_init, w.n_ref.reshape(-1), system=w.system,
                       nsys=len(w.L))
    return lbe.Lbe(p, w.node_type, w.phi_s, w.n_init, w.n_ref)


def roofline_of(kernels, kinds, label):
    """HBM roofline of one kernel kind, or of several kinds taken together
    (algorithmic bytes over their summed event time)."""
    rows = [kernels[k] for k in kinds if k in kernels]
    if not rows or any("bytes_per_launch" not in r for r in rows):
        return {"bound": "hbm", "kernel": label, "achieved": None, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": None, "traffic": None}
    secs = sum(r["total_ms"] for r in rows) / 1e3
    launches = rows[0]["launches"]
    alg = sum(r["bytes_per_launch"] * r["launches"] for r in rows)
    have = all("traffic_bytes_per_launch" in r for r in rows)
    traffic = (sum(r["traffic_bytes_per_launch"] * r["launches"] for r in rows) / launches
               if have else None)
    ach = alg / secs / 1e9
    return {"bound": "hbm", "kernel": label, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
            "bytes_per_launch": int(round(alg / launches)),
            "avg_launch_us": round(secs / launches * 1e6, 3),
            "traffic": None if traffic is None else int(round(traffic))}


def time_window(g, steps, chunk_units=0):
    """Wall time of `steps` steps from the context's current state: one by
    one (lbe_step), or replayed from captured graphs with `chunk_units`
    solver units per step (lbe_step_chunk).  Returns (seconds, first step,
    Poisson iterations per step, error text or None)."""
    tot0 = g.totals()
    sync()
    t0 = time.perf_counter()
    err = None
    try:
        if chunk_units:
            g.step_chunk(steps, chunk_units)
        else:
            g.step(steps)
    except lbe.LbeError as e:  # a replayed solve short of the tolerance
        err = str(e)
    sync()
    el = time.perf_counter() - t0
    tot1 = g.totals()
    done = tot1["step"] - tot0["step"]
    return el, int(tot0["step"]), (tot1["poisson_total"] - tot0["poisson_total"]) / max(done, 1), err


def run_form(w, form: str, solver: str, steps: int, warmup: int, start_step: int,
             check_every: int, traffic=None, krylov=False, nu=(2, 2, 0, 0), chunk_units=()):
    p = step_params(w, form, solver, check_every, krylov, nu)
    flags = p.flags
    t_init = time.perf_counter()
    g = make_context(w, p)
    blk_a, blk_b, nt = g.pass_blocks()
    launch = {"pass_a": "lds_tiles" if blk_a == 1 else f"block_{blk_a}",
              "pass_b": "lds_tiles" if blk_b == 1 else f"block_{blk_b}",
              "nontemporal_streams": {"pass_a": bool(nt & 1), "pass_b": bool(nt & 2)}}
    print(f"bench: {w.name} {form}/{solver}: context ready in "
          f"{time.perf_counter() - t_init:.2f} s, step passes {launch}", file=sys.stderr,
          flush=True)
    N = w.node_type.size
    nfluid = int((w.node_type == 0).sum())
    ffrac = nfluid / N
    g.step(start_step + warmup)
    tot0 = g.totals()
    sync()
    t0 = time.perf_counter()
    g.step(steps)
    sync()
    el = time.perf_counter() - t0
    tot1 = g.totals()
    iters = (tot1["poisson_total"] - tot0["poisson_total"]) / steps
    mlups = N * steps / el / 1e6
    print(f"bench: {w.name} {form}/{solver}: steps {tot0['step']}..{tot1['step']} in "
          f"{el:.4f} s, {mlups:.2f} MLUPS, {iters:.2f} "
          f"{'sweeps' if solver == 'sor' else 'iterations'}/step", file=sys.stderr, flush=True)

    # graph-replayed steps (a whole number of 16-step graphs) with a fixed
    # number of solver units per step, bracketed by windows of the same
    # length stepped one by one
    chunks = {}
    if chunk_units:
        csteps = 16 * max(1, (steps + 15) // 16)
        runs = [0] + [u for u in chunk_units] + [0]
        for i, u in enumerate(runs):
            el2, first, it2, err = time_window(g, csteps, u)
            key = f"units_{u}" if u else ("steps_before" if i == 0 else "steps_after")
            chunks[key] = {"mlups": round(N * csteps / el2 / 1e6, 3),
                           "ms_per_step": round(el2 / csteps * 1e3, 4), "first_step": first,
                           "poisson_iters_per_step": round(it2, 3), "steps": csteps}
            if err:
                chunks[key]["error"] = err
            print(f"bench: {w.name} {form}/{solver}: "
                  f"{'graphs, ' + str(u) + ' units/step' if u else 'one by one'}: "
                  f"steps {first}..{first + csteps} in {el2:.4f} s, "
                  f"{N * csteps / el2 / 1e6:.2f} MLUPS, {it2:.2f} iterations/step"
                  + (f" ({err})" if err else ""), file=sys.stderr, flush=True)

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
        b = bytes_per_cell(k, form, len(w.z), extrap=bool(flags & lbe.EXTRAPOLATE),
                           krylov=bool(flags & lbe.KRYLOV))
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
        print(f"bench:   {k:14s} {ms:9.3f} ms, {cnt:6d} launches, {avg * 1e6:8.2f} us avg"
              + (f", {row['achieved_GBs']:8.1f} GB/s" if b is not None else ""),
              file=sys.stderr, flush=True)
    dom = next(iter(kernels))
    return {"mlups": round(mlups, 3), "ms_per_step": round(el / steps * 1e3, 4),
            "launch": launch,
            "fluid_mlups": round(nfluid * steps / el / 1e6, 3),
            "first_step": int(tot0["step"]),
            "poisson_iters_per_step": round(iters, 3),
            "roofline": roofline_of(kernels, [dom], dom),
            "roofline_step_passes": roofline_of(kernels, ["fluid", "ions"], "fluid+ions"),
            "kernels": kernels, **({"graph_chunks": chunks} if chunks else {})}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_threads():
    """Host cores this process may use (the scheduler's affinity mask, capped
    by OMP_NUM_THREADS when that is set)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def cpu_baseline(seconds=15.0, nxy=32):
    """The FP64 oracle on a 32 x 32 x 192 lateral column of the porous
    electrode (every z: spheres, gap and counter-electrode), in its own
    solver settings (SOR, omega 1.8, tol 1e-10), timed over whole steps after
    its initial solve: once single-threaded and once with its OpenMP build on
    every host core this process may use.  MLUPS counts the column's sites."""
    import oracle
    col = W.porous_column(nxy=nxy)
    n = col.node_type.size
    legs = {}
    for threads in (1, cpu_threads()):
        if threads in legs:
            continue
        p = oracle.make_params(col.shape, col.z, col.D, col.lB, col.tau, col.rho0, col.Eapp,
                               col.omega, col.tol, 1_000_000, 4)
        o = oracle.Oracle(p, col.node_type, col.phi_s, col.n_init, col.n_ref,
                          threads=None if threads == 1 else threads)
        steps, t0 = 0, time.perf_counter()
        while True:
            o.step(1)
            steps += 1
            el = time.perf_counter() - t0
            if el >= seconds or steps >= 200:
                break
        legs[threads] = (n * steps / el / 1e6, steps, el, o.threads)
        print(f"bench: oracle on {col.name}, {o.threads} thread(s): {steps} steps in {el:.1f} s, "
              f"{legs[threads][0]:.4f} MLUPS", file=sys.stderr, flush=True)
    best = max(legs)
    v, steps, el, used = legs[best]
    v1, steps1, el1, _ = legs[1]
    return dict(value=round(v, 5), unit="MLUPS", cores=used, kind="oracle",
                cpu=cpu_model(),
                sample=f"{col.name}: a {nxy}x{nxy} lateral column of the porous electrode, "
                       f"{steps} whole steps after the initial solve, SOR omega {col.omega}, "
                       f"tol {col.tol:g}, FP64 C oracle on {used} OpenMP threads "
                       "(the GPU solves Poisson by multigrid instead)",
                single_thread={"value": round(v1, 5), "unit": "MLUPS", "cores": 1,
                               "steps": steps1, "seconds": round(el1, 2)})


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

# Workloads: builder and multigrid cycle, chosen by timing the cycles on the
# same GPU from a running state (steps 1000-1200).  The slab's electrodes are
# represented exactly on every level: V(1,1) everywhere.  The porous
# electrode's spheres are not: V(1,2) with two Jacobi sweeps before and three
# after on the coarse levels, as the preconditioner of flexible CG (plain
# cycles diverge there).  The coaxial cell: V(1,1) with two sweeps each way
# on the coarse levels, under flexible CG.  The 96-system batch: V(1,1), two
# sweeps each way on the coarse levels, with Krylov acceleration.
WORKLOADS = {
    "porous_electrode_192^3": (lambda: W.porous_electrode(noise=True),
                               dict(krylov=True, nu=(1, 2, 2, 3))),
    "eo_slab_64x64x130": (lambda: W.eo_slab(noise=True), dict(nu=(1, 1, 1, 1))),
    "coaxial_160x160x64": (lambda: W.coaxial(noise=True), dict(krylov=True, nu=(1, 1, 2, 2))),
    "batched_96_slabs_8x8": (lambda: W.batch_slabs(noise=True),
                             dict(krylov=True, nu=(1, 1, 2, 2))),
}

# workloads also timed with their steps replayed from captured graphs, at
# these fixed numbers of solver units per step
CHUNK_UNITS = {"eo_slab_64x64x130": (1, 2), "coaxial_160x160x64": (2, 3),
               "batched_96_slabs_8x8": (2, 3)}


def run_workload(name, forms, steps, warmup, start_step, check_every, traffic=None):
    build, settings = WORKLOADS[name]
    w = build()
    nfluid = int((w.node_type == 0).sum())
    print(f"bench: {w.name}, {w.node_type.size} sites, {nfluid} fluid", file=sys.stderr,
          flush=True)
    res = {}
    for f in forms:
        form, solver = FORMS[f]
        if solver == "sor":
            # hundreds of sweeps per step: fewer steps, from the start
            res[f] = run_form(w, form, solver, max(2, steps // 10), 2, 0, check_every, traffic)
        else:
            res[f] = run_form(w, form, solver, steps, warmup, start_step, check_every, traffic,
                              chunk_units=CHUNK_UNITS.get(name, ()), **settings)
    return w, nfluid, res


def poisson_text(settings):
    n1, n2, c1, c2 = settings.get("nu", (2, 2, 0, 0))
    if not (c1 or c2):
        c1, c2 = n1, n2
    cyc = f"Jacobi V({n1},{n2}) on the finest level, V({c1},{c2}) on the coarser ones"
    kry = ", each V-cycle preconditioning flexible CG" if settings.get("krylov") else ""
    return (f"geometric multigrid ({cyc}){kry}, FP64 defect correction, warm start "
            "extrapolated quadratically in time")


def run_adjoint(w, form: str, steps: int, every: int, check_every: int, profile_steps: int):
    """Reverse mode on workload w: lbe_record of `steps` steps with a
    checkpoint every `every`, then one lbe_adjoint (gradient of electrode 1's
    charge with respect to every node potential, l_B and the initial state),
    which recomputes each segment and runs one reverse step plus one adjoint
    Poisson solve per step.  MLUPS count lattice sites x steps.  The kernel
    averages come from a shorter record (profile_steps) whose lbe_adjoint
    call runs with HIP events around every launch."""
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
    print(f"bench: adjoint {form}: record {steps} steps in {t_rec:.3f} s", file=sys.stderr,
          flush=True)
    t0 = time.perf_counter()
    grad = g.adjoint(qbar)
    sync()
    t_adj = time.perf_counter() - t0
    dv = float(grad["phi_s"][w.node_type == 1].sum())
    print(f"bench: adjoint {form}: reverse sweep in {t_adj:.3f} s, dQ1/dV1 = {dv:.6e}",
          file=sys.stderr, flush=True)
    del grad
    g.record(profile_steps, min(every, profile_steps))
    g.profile(True)
    g.adjoint(qbar, phi_s=False, lB=False, n=False, f=False)
    kt = g.kernel_times()
    g.profile(False)
    g.close()
    kernels = {}
    for k, (ms, cnt, cells) in sorted(kt.items(), key=lambda kv: -kv[1][0]):
        if not cnt:
            continue
        avg = ms / 1e3 / cnt
        row = {"total_ms": round(ms, 4), "launches": cnt, "avg_us": round(avg * 1e6, 3)}
        b = bytes_per_cell(k, form, len(w.z), extrap=True, krylov=True)
        if b is not None:
            per_launch = (ffrac * b + (1.0 - ffrac) * 4) * cells / cnt
            row["bytes_per_launch"] = int(round(per_launch))
            row["achieved_GBs"] = round(per_launch / avg / 1e9, 1)
            row["frac"] = round(per_launch / avg / 1e9 / HBM_PEAK_GBS, 4)
        kernels[k] = row
        print(f"bench:   {k:14s} {ms:9.3f} ms, {cnt:6d} launches, {avg * 1e6:8.2f} us avg"
              + (f", {row['achieved_GBs']:8.1f} GB/s" if b is not None else ""),
              file=sys.stderr, flush=True)
    adj = [k for k in kernels if k.startswith("adj_") and "frac" in kernels[k]]
    roof = roofline_of(kernels, [adj[0]], adj[0]) if adj else None
    return {"workload": w.name, "form": form, "steps": steps, "checkpoint_every": every,
            "objective": "charge of electrode 1 at the last step",
            "record_mlups": round(N * steps / t_rec / 1e6, 3),
            "reverse_mlups": round(N * steps / t_adj / 1e6, 3),
            "gradient_mlups": round(N * steps / (t_rec + t_adj) / 1e6, 3),
            "record_s": round(t_rec, 3), "reverse_s": round(t_adj, 3),
            "dQ1_dV1": dv, "kernel_profile_steps": profile_steps, "roofline": roof,
            "kernels": kernels}


# ---- rocprofv3 summaries ------------------------------------------------------

def _csv_rows(root, suffix):
    import csv
    import glob
    rows = []
    for path in sorted(glob.glob(os.path.join(root, "**", f"*{suffix}"), recursive=True)):
        with open(path, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def _col(row, *names):
    low = {k.lower(): v for k, v in row.items() if k}
    for n in names:
        if n.lower() in low:
            return low[n.lower()]
    raise KeyError(f"none of {names} in {sorted(low)}")


def _grid(row):
    """Work-items of a dispatch (the product of the grid sizes)."""
    try:
        return int(_col(row, "Grid_Size"))
    except KeyError:
        g = 1
        for a in ("X", "Y", "Z"):
            g *= int(_col(row, f"Grid_Size_{a}"))
        return g


RING_ZRUN = 8  # planes per tile run of the plane-ring kernels (the library's default)

# (pattern in the kernel name, bench kind); a one-block second stage joins
# the kind of the launch before it
KIND_OF = [("k_fluid_", "fluid"), ("k_ions_", "ions"), ("k_outer_resid", "mg_resid"),
           ("k_jacobi", "jacobi"), ("k_restrict", "mg_restrict"), ("k_prolong", "mg_prolong"),
           ("k_mg_small", "mg_small"), ("k_fcg_az", "fcg_apply"), ("k_fcg_update", "fcg_update"),
           ("k_charge", "charge"),
           ("k_totals", "totals"), ("k_momentum", "momentum"), ("k_observe", "observe"),
           ("k_smooth", "mg_smooth"), ("k_coarse", "mg_coarse"), ("k_correct", "correct"),
           ("k_sor", "sor"), ("k_resid", "resid")]
SECOND_STAGE = ("k_final_resid", "k_fcg_coef", "k_final_charge", "k_final_sum",
                "k_final_max")


def _kernel_base(name):
    """A kernel's demangled name without its parameter list."""
    name = name.strip()
    if not name.endswith(")"):
        return name
    depth = 0
    for i in range(len(name) - 1, -1, -1):
        if name[i] == ")":
            depth += 1
        elif name[i] == "(":
            depth -= 1
            if depth == 0:
                return name[:i]
    return name


def _classify(name, grid, nsites, prev_form=None):
    """(form, kind) of one dispatch from its kernel name, or None; a kernel
    whose name carries no precision takes the form of the dispatch before
    it (prev_form)."""
    base = _kernel_base(name)
    form = prev_form
    if "float" in base or "_f32" in base:
        form = "fp32-mg"
    elif "double" in base or "_f64" in base:
        form = "fp64-mg"
    for pat, kind in KIND_OF:
        if pat in base:
            if kind == "jacobi":
                # a plane-ring launch has one work-item per cell of a plane
                # of each tile's run of RING_ZRUN planes
                cells = grid * RING_ZRUN if "_ring" in base else grid
                if cells < nsites:
                    kind = "mg_smooth"
                else:
                    kind = "mg_smooth0_phi" if "true" in base else "mg_smooth0"
            return form, kind
    return None


def summarize_rocprof(root, workload, window=(22, 10)):
    """Summaries of the kernel-trace run (root/trace) and the two counter runs
    (root/fetch, root/write) of one workload, as text."""
    build, _ = WORKLOADS[workload]
    nsites = build().node_type.size
    out = [f"# LBE step kernels, {workload}: rocprofv3 summaries", ""]
    stats = _csv_rows(os.path.join(root, "trace"), "kernel_stats.csv")
    if stats:
        out.append("kernel trace statistics (all dispatches of the run):")
        out.append(f"{'kernel':56s} {'calls':>7s} {'total_ms':>10s} {'avg_us':>9s} "
                   f"{'min_us':>8s} {'max_us':>8s}")
        for r in sorted(stats, key=lambda r: -float(_col(r, "TotalDurationNs"))):
            nm = _kernel_base(_col(r, "Name")).replace("void ", "").replace(
                "lbe::(anonymous namespace)::", "")
            out.append(f"{nm[:56]:56s} {int(_col(r, 'Calls')):7d} "
                       f"{float(_col(r, 'TotalDurationNs')) / 1e6:10.3f} "
                       f"{float(_col(r, 'AverageNs')) / 1e3:9.2f} "
                       f"{float(_col(r, 'MinNs')) / 1e3:8.2f} {float(_col(r, 'MaxNs')) / 1e3:8.2f}")
        out.append("")
    trace = _csv_rows(os.path.join(root, "trace"), "kernel_trace.csv")
    if trace:
        # the step passes and the finest-level solver kernels by form and kind,
        # over dispatches that did work (longer than 3 us: a launch of a
        # converged solve returns at once)
        agg = {}
        prev_form = None
        trace.sort(key=lambda r: int(_col(r, "Start_Timestamp")))
        for r in trace:
            name = _col(r, "Kernel_Name")
            cls = _classify(name, _grid(r), nsites, prev_form)
            dur = (int(_col(r, "End_Timestamp")) - int(_col(r, "Start_Timestamp"))) / 1e3
            if cls is not None:
                prev_form = cls[0]
            if cls is None or cls[0] is None or dur < 3.0:
                continue
            a = agg.setdefault(cls, [0, 0.0])
            a[0] += 1
            a[1] += dur
        # GPU occupancy of the timed steps: per form, the pass-A launches
        # after the launch-shape trials mark the steps; over the timed window
        # the union of kernel intervals against the wall span
        skip, count = window
        out.append(f"GPU busy fraction over the timed window (steps {skip}..{skip + count} "
                   "after the launch-shape trials, pass-A launch to pass-A launch):")
        for form_tag in ("_f32", "_f64"):
            # the context's timing runs every pass-A candidate before the
            # first pass-B launch, so the steps' pass-A launches follow it
            fb = [int(r["Start_Timestamp"]) for r in trace
                  if "k_ions" + form_tag in r["Kernel_Name"]]
            if not fb:
                continue
            fl = [r for r in trace if "k_fluid" + form_tag in r["Kernel_Name"]
                  and int(r["Start_Timestamp"]) > fb[0]]
            if len(fl) < skip + count + 1:
                continue
            t0 = int(fl[skip]["Start_Timestamp"])
            t1 = int(fl[skip + count]["Start_Timestamp"])
            busy, last = 0, t0
            for r in trace:
                a, b = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
                if b <= t0 or a >= t1:
                    continue
                a, b = max(a, last), min(b, t1)
                if b > a:
                    busy += b - a
                    last = b
            out.append(f"  {'fp32' if form_tag == '_f32' else 'fp64'}: {(t1 - t0) / 1e3 / count:.1f} "
                       f"us per step, GPU busy {100.0 * busy / (t1 - t0):.1f}%")
        out.append("")
        out.append("first-stage kernels by form and kind (dispatches longer than 3 us):")
        out.append(f"{'form':8s} {'kind':16s} {'launches':>8s} {'avg_us':>9s}")
        for (form, kind), (n, t) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
            out.append(f"{form:8s} {kind:16s} {n:8d} {t / n:9.2f}")
        out.append("")
    per = {}
    factors = {}
    for counter, sub in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
        rows = _csv_rows(os.path.join(root, sub), "counter_collection.csv")
        if not rows:
            continue
        rows.sort(key=lambda r: int(_col(r, "Dispatch_Id", "Correlation_Id")))
        # calibration: the plain 256 MiB device copy (the first kernels of
        # the run, named after copy)
        cal = [float(_col(r, "Counter_Value")) for r in rows
               if "copy" in _col(r, "Kernel_Name").lower()
               and _col(r, "Counter_Name") == counter]
        if not cal:
            raise SystemExit(f"no calibration copy in the {counter} run")
        kib = max(cal)
        factors[counter] = (1 << 28) / (kib * 1024.0)
        last = None
        prev_form = None
        for r in rows:
            if _col(r, "Counter_Name") != counter:
                continue
            name = _col(r, "Kernel_Name")
            val = float(_col(r, "Counter_Value")) * 1024.0 * factors[counter]
            base = _kernel_base(name)
            if any(s in base for s in SECOND_STAGE) and last is not None:
                per[last][counter][-1] += val
                continue
            cls = _classify(name, _grid(r), nsites, prev_form)
            if cls is not None:
                prev_form = cls[0]
            if cls is None or cls[0] is None:
                last = None
                continue
            d = per.setdefault(cls, {"FETCH_SIZE": [], "WRITE_SIZE": []})
            d[counter].append(val)
            last = cls
    if per:
        out.append("HBM-side traffic per launch (FETCH_SIZE and WRITE_SIZE, one rocprofv3 pass "
                   "each, scaled by the")
        out.append("counters' reading of a plain 256 MiB device copy in the same run: factors "
                   + ", ".join(f"{k} {v:.4f}" for k, v in factors.items()) + ");")
        out.append("mean over launches that moved more than 4 KiB (a launch of a converged "
                   "solve returns at once);")
        out.append("a kind's launch includes its one-block second stage.  MB = 1e6 bytes.")
        out.append("")
        out.append(f"{'form':8s} {'kind':16s} {'launches':>8s} {'fetch_MB':>9s} {'write_MB':>9s}")
        mach = []
        for (form, kind), d in sorted(per.items()):
            f = [v for v in d["FETCH_SIZE"] if v > 4096]
            w_ = [v for v in d["WRITE_SIZE"] if v > 4096]
            if not f or not w_:
                continue
            fm, wm = sum(f) / len(f), sum(w_) / len(w_)
            out.append(f"{form:8s} {kind:16s} {len(f):8d} {fm / 1e6:9.3f} {wm / 1e6:9.3f}")
            mach.append(f"traffic {form} {kind} {int(round(fm))} {int(round(wm))}")
        out.append("")
        out.append("machine-readable (bytes per launch; read by bench.py while the library's "
                   "sources hash to the value below):")
        out.append("")
        out.extend(mach)
        out.append(f"sources {sources_hash()}")
    return "\n".join(out) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--start-step", type=int, default=1000,
                    help="untimed steps before the warm-up: the timed window starts from a "
                         "running state (the configured runs are 4000-50000 steps long)")
    ap.add_argument("--workload", default="porous_electrode_192^3", choices=list(WORKLOADS))
    ap.add_argument("--forms", default="fp32-mg,fp64-mg",
                    help="comma list of " + ",".join(FORMS) + "; the first is the headline")
    ap.add_argument("--check-every", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--shapes", default="eo_slab_64x64x130,coaxial_160x160x64,batched_96_slabs_8x8",
                    help="comma list of other workloads measured beside the headline (empty: none)")
    ap.add_argument("--shape-forms", default="fp32-mg,fp64-mg")
    ap.add_argument("--shape-steps", type=int, default=200)
    ap.add_argument("--adjoint-forms", default="fp32-mg",
                    help="forms of the reverse-mode measurement on the porous electrode "
                         "(empty: none)")
    ap.add_argument("--adjoint-steps", type=int, default=4000)
    ap.add_argument("--adjoint-every", type=int, default=200)
    ap.add_argument("--adjoint-profile-steps", type=int, default=400)
    ap.add_argument("--summarize-rocprof", metavar="DIR",
                    help="print the summary of the rocprofv3 CSV output under DIR (trace/, "
                         "fetch/, write/) for --workload and exit (no GPU); --start-step, "
                         "--warmup and --steps name the profiled run's timed window")
    args = ap.parse_args()
    if args.summarize_rocprof:
        sys.stdout.write(summarize_rocprof(args.summarize_rocprof, args.workload,
                                           (args.start_step + args.warmup, args.steps)))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the LBE step has no multi-GPU sharding "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    init_device()
    if args.copy_calibration:
        copy_calibration()
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    w, nfluid, res = run_workload(args.workload, forms, args.steps, args.warmup,
                                  args.start_step, args.check_every, load_traffic(args.workload))
    head = res[forms[0]]
    hform, hsolver = FORMS[forms[0]]
    settings = WORKLOADS[args.workload][1]
    out = {
        # value: the headline form's MLUPS; the FP64 form is in "forms", the
        # fraction of the HBM peak in "roofline" (dominant kernel) and
        # "roofline_step_passes" (LB + ion passes)
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
        "config": {"workload": w.name, "sites": int(w.node_type.size), "fluid_sites": nfluid,
                   "form": forms[0], "tol": getattr(w, "tol", 1e-10),
                   "debye": getattr(w, "extra", {}).get("debye"),
                   "Eapp": list(getattr(w, "Eapp", (0.0, 0.0, 0.0))),
                   "timed_steps_from": head["first_step"],
                   "poisson": (poisson_text(settings) if hsolver == "mg" else
                               "four-colour SOR"),
                   "poisson_iters_per_step": head["poisson_iters_per_step"],
                   "fluid_mlups": head["fluid_mlups"]},
        "roofline": head["roofline"],
        "roofline_step_passes": head["roofline_step_passes"],
        "forms": {k: {kk: v[kk] for kk in ("mlups", "ms_per_step", "poisson_iters_per_step",
                                            "launch", "roofline", "roofline_step_passes")}
                  for k, v in res.items()},
        "kernels": head["kernels"],
    }
    shapes = [x.strip() for x in args.shapes.split(",") if x.strip()]
    sforms = [f.strip() for f in args.shape_forms.split(",") if f.strip()]
    if shapes:
        out["shapes"] = {}
        for name in shapes:
            fl = sforms + (["fp64-sor"] if name.startswith("eo_slab") else [])
            ws, nf, r = run_workload(name, fl, args.shape_steps, args.warmup, args.start_step,
                                     args.check_every, load_traffic(name))
            out["shapes"][ws.name] = {
                "sites": int(ws.node_type.size), "fluid_sites": nf,
                "steps": args.shape_steps, "poisson": poisson_text(WORKLOADS[name][1]),
                "forms": {k: {kk: v[kk] for kk in ("mlups", "ms_per_step", "first_step",
                                                    "poisson_iters_per_step", "launch",
                                                    "roofline", "roofline_step_passes",
                                                    "graph_chunks") if kk in v}
                          for k, v in r.items()}}
    aforms = [f.strip() for f in args.adjoint_forms.split(",") if f.strip()]
    if aforms:
        wp = W.porous_electrode(noise=True)
        out["adjoint"] = {f: run_adjoint(wp, FORMS[f][0], args.adjoint_steps, args.adjoint_every,
                                         args.check_every, args.adjoint_profile_steps)
                          for f in aforms}
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
