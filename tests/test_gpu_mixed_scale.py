"""The FP32-mixed form at the benchmark's own solver settings and at the
configurations' full size and length.

1. Against the FP64 oracle, element by element, on lattices large enough that
   the finest multigrid level and the one below it run in the global
   kernels (more than 2048 cells on each; the coarser levels go to the
   one-work-group kernel): a 16 x 16 x 130 lateral crop of the
   electro-osmosis slab, a 40 x 40 x 16 coaxial cell and a 32^3 crop of the
   porous electrode, each with the multigrid cycle, Krylov setting and
   quadratic warm start bench.py uses for the workload it comes from, at tol
   1e-10: exactly the launch configuration bench.py times.  The
   oracle runs its SOR (four colours, diagonal-normalised, omega 1.95: only
   the iterates depend on omega, not the fixed point) to 1e-12 on many
   threads (its OpenMP build is bit for bit the single-threaded one).
2. Against the FP64 form on the GPU (itself within 1e-12 of the oracle on
   the parity cases) at full size for the configured number of steps: the
   64 x 64 x 130 electro-osmosis slab (50000), the 160 x 160 x 64 coaxial
   cell (30000), the 192^3 porous electrode (4000) and the 96-system batch
   (one 10000-step chunk, replayed from captured graphs), each in its benchmark
   configuration.

Bars: potential within 1e-5 of the electrode voltage
difference; electrode charge Q(t) over the whole history and capacitance
Q(T)/dV within 1e-5 of |Q|; velocity within 1e-4 of its largest magnitude,
and the electro-osmotic flux (total momentum along the applied field)
within 1e-4 of the flux of |u|.
Concentrations are reported normalised by their largest departure from the
bulk value (bar 1e-3, as for the small parity cases).  The FP64 solve stops
at 1e-10 too, so part of each difference is the solver's own tolerance
(|A^-1| tol <= L^2/8 x 1e-10 on the potential: 2e-7 at L = 128).
"""
import os

import numpy as np
import pytest

import bench
import oracle
import paper_1907_04732_amd as lbe
import workloads as W

pytestmark = pytest.mark.gpu

PHI_BAR, Q_BAR, U_BAR, N_BAR = 1e-5, 1e-5, 1e-4, 1e-3
THREADS = int(os.environ.get("OMP_NUM_THREADS", "8"))


def errors(t, nref, phi_s, a, b, qa, qb):
    """Normalised maximum differences of run a against reference b."""
    fl = t == 0
    dv = phi_s[~fl].max() - phi_s[~fl].min()
    dn = np.abs(b["n"][:, fl] - np.asarray(nref).reshape(-1, 1)[: b["n"].shape[0]]).max()
    umax = np.abs(b["u"][:, fl]).max()
    return dict(
        phi=float(np.abs(a["phi"] - b["phi"]).max() / dv),
        q=float(np.abs(qa - qb).max() / np.abs(qb).max()),
        C=float((np.abs(qa[-1] - qb[-1]) / np.abs(qb[-1])).max()),
        u=float(np.abs(a["u"][:, fl] - b["u"][:, fl]).max() / umax),
        n=float(np.abs(a["n"][:, fl] - b["n"][:, fl]).max() / dn),
        umax=float(umax))


def check(errs):
    assert errs["phi"] <= PHI_BAR, errs
    assert errs["q"] <= Q_BAR and errs["C"] <= Q_BAR, errs
    assert errs["u"] <= U_BAR, errs
    assert errs["n"] <= N_BAR, errs


# the solver settings bench.py uses for the workload each crop comes from
SETTINGS = {k: v[1] for k, v in bench.WORKLOADS.items()}
CROPS = {
    "eo_slab_16x16x130": lambda: (W.eo_slab(noise=True, nx=16, ny=16),
                                  SETTINGS["eo_slab_64x64x130"], 200),
    "coaxial_40x40x16": lambda: (W.coaxial(noise=True, nx=40, ny=40, nz=16, R1=4.0, R2=18.0),
                                 SETTINGS["coaxial_160x160x64"], 200),
    "porous_crop_32^3": lambda: (W.porous_crop(n=32), SETTINGS["porous_electrode_192^3"], 120),
}


@pytest.mark.parametrize("name", list(CROPS))
def test_mixed_at_bench_settings_matches_oracle(name):
    w, settings, steps = CROPS[name]()
    g = lbe.Lbe(bench.step_params(w, "fp32", **settings), w.node_type, w.phi_s, w.n_init,
                w.n_ref)
    assert g.totals()["step"] == 0
    o = oracle.Oracle(oracle.make_params(w.shape, w.z, w.D, w.lB, w.tau, w.rho0, w.Eapp, 1.95,
                                         1e-12, 10**6, 4), w.node_type, w.phi_s, w.n_init,
                      w.n_ref, threads=THREADS)
    g.step(steps)
    o.step(steps)
    errs = errors(w.node_type, w.n_ref, w.phi_s, g.fields(f=False), o.fields(), g.qhist(),
                  o.qhist())
    print(name, steps, "steps, mixed at bench settings vs oracle:",
          {k: f"{v:.2e}" for k, v in errs.items()}, "cycles", g.totals()["poisson_total"])
    check(errs)


# the configured run lengths: 50000 steps of the slab, 30000 of the coaxial
# cell, 4000 of the porous electrode
FULL = {
    "eo_slab_64x64x130": lambda: (W.eo_slab(noise=True), SETTINGS["eo_slab_64x64x130"], 50000),
    "coaxial_160x160x64": lambda: (W.coaxial(noise=True), SETTINGS["coaxial_160x160x64"], 30000),
    "porous_electrode_192^3": lambda: (W.porous_electrode(noise=True),
                                       SETTINGS["porous_electrode_192^3"], 4000),
}


@pytest.mark.parametrize("name", list(FULL))
def test_mixed_matches_fp64_at_full_size(name):
    """Full size, the configured number of steps.  Also the conservation of
    each ion species and of the fluid mass over the run, in both forms.  The
    link fluxes are antisymmetric bit for bit, so each species count moves
    only by the rounding of the nodes' own updates: in FP64 not at all within
    1e-13; in the mixed form, whose concentrations are FP32 pairs, within
    1e-9.  The fluid mass takes the rounding of each node's collision: in
    FP64 below one ulp of the total per step; the mixed form stores its
    population deviations in single FP32 words (1e-9)."""
    w, settings, steps = FULL[name]()
    runs = {}
    for form in ("fp32", "fp64"):
        g = lbe.Lbe(bench.step_params(w, form, **settings), w.node_type, w.phi_s, w.n_init,
                    w.n_ref)
        t0 = g.totals()
        g.step(steps)
        t1 = g.totals()
        runs[form] = (g.fields(f=False), g.qhist(), t1)
        g.close()
        dn = [t1["nk"][k] / t0["nk"][k] - 1 for k in range(len(w.z))]
        dm = t1["mass"] / t0["mass"] - 1
        print(name, form, f"{steps} steps: relative drift of the ion counts "
                          f"{', '.join(f'{v:.2e}' for v in dn)}, of the fluid mass {dm:.2e}")
        if form == "fp64":
            assert max(abs(v) for v in dn) <= 1e-13
            assert abs(dm) <= steps * np.finfo(np.float64).eps
        else:
            assert max(abs(v) for v in dn) <= 1e-9 and abs(dm) <= 1e-9
    (fa, qa, ta), (fb, qb, tb) = runs["fp32"], runs["fp64"]
    errs = errors(w.node_type, w.n_ref, w.phi_s, fa, fb, qa, qb)
    if any(w.Eapp):
        # the electro-osmotic flux along the applied field (the total
        # momentum), against the flux of |u|: on the slab the profile is odd
        # about the mid-plane (Eq. 20) and its net flux nearly cancels
        ax = int(np.argmax(np.abs(w.Eapp)))
        scale = np.abs(fb["u"][ax][w.node_type == 0]).sum()
        errs["eo_flux"] = abs(ta["momentum"][ax] - tb["momentum"][ax]) / scale
    print(name, steps, "steps, mixed vs FP64 on the GPU:",
          {k: f"{v:.2e}" for k, v in errs.items()})
    check(errs)
    assert errs.get("eo_flux", 0.0) <= U_BAR


def test_batch_capacitance_mixed_matches_fp64():
    """The 96-system batch (8 x 8 x L, L 16..256, Debye length 2..16, voltage
    0.01..0.2) in its benchmark configuration for one configured chunk of
    10000 steps, the mixed form replayed from captured 16-step graphs
    (lbe_step_chunk, 16 solver units per step): every system's charge
    history and capacitance Q(T)/V against the FP64 form, and the potential
    of every system against its own voltage.  The replayed chunk gives the
    same bits as the mixed form stepped one by one."""
    w = W.batch_slabs(noise=True)
    runs = {}
    for form, graphs in (("fp32", True), ("fp32", False), ("fp64", False)):
        p = bench.step_params(w, form, **SETTINGS["batched_96_slabs_8x8"])
        g = lbe.Lbe(p, w.node_type, w.phi_s, w.n_init, w.n_ref.reshape(-1), system=w.system,
                    nsys=len(w.L))
        print("batch", form, "graphs" if graphs else "one by one", flush=True)
        t0 = g.totals()
        if graphs:
            g.step_chunk(10000, units=16)
        else:
            g.step(10000)
        t1 = g.totals()
        runs[form, graphs] = (g.fields(f=False)["phi"], g.qhist())
        g.close()
        dn = [t1["nk"][k] / t0["nk"][k] - 1 for k in range(len(w.z))]
        print("batch", form, "relative drift of the ion counts",
              ", ".join(f"{v:.2e}" for v in dn))
        assert max(abs(v) for v in dn) <= (1e-13 if form == "fp64" else 1e-9)
    assert np.array_equal(runs["fp32", True][0], runs["fp32", False][0])
    assert np.array_equal(runs["fp32", True][1], runs["fp32", False][1])
    (pa, qa), (pb, qb) = runs["fp32", True], runs["fp64", False]
    nsys = len(w.L)
    # electrodes 2s+1 and 2s+2 belong to system s
    qa3, qb3 = qa.reshape(len(qa), nsys, 2), qb.reshape(len(qb), nsys, 2)
    e_q = np.abs(qa3 - qb3).max(axis=(0, 2)) / np.abs(qb3).max(axis=(0, 2))
    e_c = np.abs(qa3[-1] - qb3[-1]).max(axis=1) / np.abs(qb3[-1]).max(axis=1)
    e_phi = np.array([np.abs(pa - pb)[w.system == s].max() for s in range(nsys)]) / w.V
    print("batch: worst system Q(t)", e_q.max(), "capacitance", e_c.max(), "phi/V", e_phi.max())
    assert e_q.max() <= Q_BAR and e_c.max() <= Q_BAR and e_phi.max() <= PHI_BAR
