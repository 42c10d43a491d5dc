"""FP32-mixed form (FP32 deviation storage and collision, FP32 Poisson
correction inside FP64 defect correction) against the FP64 oracle.

Bars: potential within 1e-5 of the electrode voltage scale,
electrode charge within 1e-5 of its magnitude, electro-osmotic velocity within
1e-4 of its peak.  Concentrations are reported normalised by the largest
departure from the bulk value.
"""
import numpy as np
import pytest

import gpu_cases as G
import oracle
import oracle_pins as P
import paper_1907_04732_amd as lbe
import theory as T
import workloads as W
from test_gpu_parity import residual_numpy

pytestmark = pytest.mark.gpu


def mixed_pair(name, solver, tol=1e-12):
    kw, shape, t, ps, n0, nref, nsteps, _ = G.case(name)
    o = oracle.Oracle(oracle.make_params(shape, **kw, tol=tol, max_iter=10**6, check_every=4), t,
                      ps, n0, nref)
    g = lbe.Lbe(lbe.make_params(shape, **kw, tol=tol, max_iter=100000, check_every=4,
                                precision=lbe.FP32_MIXED, poisson=solver), t, ps, n0, nref)
    return o, g, nsteps, t, nref


@pytest.mark.parametrize("solver", [lbe.SOR4, lbe.MG])
@pytest.mark.parametrize("name", ["slab_4x4x34", "coax_16x16x4", "slab_1x1x34"])
def test_mixed_matches_oracle(name, solver):
    o, g, nsteps, t, nref = mixed_pair(name, solver)
    steps = 200
    o.step(steps)
    g.step(steps)
    fo, fg = o.fields(), g.fields()
    vscale = 0.1
    fl = t == 0
    dn = np.abs(fo["n"][:, fl] - np.asarray(nref)[:, None]).max()
    e_phi = np.abs(fg["phi"] - fo["phi"]).max() / vscale
    e_q = np.abs(g.qhist() - o.qhist()).max() / np.abs(o.qhist()).max()
    e_n = np.abs(fg["n"] - fo["n"]).max() / dn
    _, w = lbe.velocities()
    dev = np.abs(fo["f"][:, fl] - w[:, None]).max()  # departure from rest (rho0 = 1)
    e_f = np.abs(fg["f"][:, fl] - fo["f"][:, fl]).max() / dev
    print(name, solver, f"phi {e_phi:.2e} q {e_q:.2e} n/dn {e_n:.2e} f {e_f:.2e}")
    assert e_phi <= 1e-5 and e_q <= 1e-5
    assert e_n <= 1e-3 and e_f <= 1e-3


def test_mixed_charging_curve():
    """Q(t) of the 4x4x34 capacitor over 3000 steps (a third of the way to
    steady state): FP32-mixed within 1e-5 of the FP64 oracle's Q."""
    o, g, _, t, _ = mixed_pair("slab_4x4x34", lbe.MG, tol=1e-11)
    o.step(3000)
    g.step(3000)
    qo, qg = o.qhist(), g.qhist()
    err = np.abs(qg - qo).max() / np.abs(qo).max()
    print("Q(t) rel err", err)
    assert err <= 1e-5


def test_mixed_eo_velocity():
    """Steady electro-osmotic profile of the 32-plane slab (Eq. 20 setting,
    lambda_D = 4, E_x = 1e-3): FP32-mixed within 1e-4 of the FP64 oracle's
    peak velocity, and within 3% of the closed form."""
    o, shape, t = P.run_slab(steps=14000, E=(1e-3, 0, 0), nxy=2, tol=1e-11)
    rs = W.salt_for_debye(4.0, P.LB)
    shape, t, ps = W.slab(2, 2, 32, 1, 0.05, -0.05)
    g = lbe.Lbe(lbe.make_params(shape, (1, -1), (0.05, 0.05), P.LB, Eapp=(1e-3, 0, 0), omega=1.8,
                                tol=1e-11, max_iter=1000, precision=lbe.FP32_MIXED,
                                poisson=lbe.MG), t, ps, None, (rs, rs))
    g.step(14000)
    uo = o.fields()["u"][0][t == 0]
    ug = g.fields(f=False)["u"][0][t == 0]
    err = np.abs(ug - uo).max() / np.abs(uo).max()
    z = np.arange(32) + 0.5 - 16
    th = T.eo_slab_velocity(z, 32, 0.25, 0.05, -0.05, 1e-3, P.LB, 1.0)
    err_th = np.abs(ug.reshape(32, 4)[:, 0] - th).max() / np.abs(th).max()
    print("u rel err", err, "vs closed form", err_th)
    assert err <= 1e-4
    assert err_th <= 0.03


def test_mixed_full_slab_properties():
    """64x64x130 in the mixed form with multigrid at tol 1e-10: residual of
    the FP64 potential, conservation of ions and mass."""
    w = W.eo_slab(noise=True)
    p = lbe.make_params(w.shape, w.z, w.D, w.lB, tau=w.tau, Eapp=w.Eapp, omega=w.omega,
                        tol=1e-10, max_iter=100, precision=lbe.FP32_MIXED, poisson=lbe.MG)
    g = lbe.Lbe(p, w.node_type, w.phi_s, w.n_init, w.n_ref)
    t0 = g.totals()
    g.step(20)
    t1 = g.totals()
    print("cycles", t1["poisson_iters"], "mass drift", t1["mass"] / t0["mass"] - 1,
          "N drift", [t1["nk"][k] / t0["nk"][k] - 1 for k in range(2)])
    assert abs(t1["mass"] / t0["mass"] - 1) < 1e-9
    for k in range(2):
        assert abs(t1["nk"][k] / t0["nk"][k] - 1) < 1e-9
    fg = g.fields(f=False)
    R = residual_numpy(w.shape, w.node_type, fg["phi"], fg["n"], w.z, w.lB)
    # the library's residual uses the FP64 source accumulated from the FP32
    # deviations; recomputing it from the returned n adds ~1e-15 rounding
    assert np.abs(R).max() <= 1.05e-10


@pytest.mark.parametrize("precision", [lbe.FP32_MIXED, lbe.FP64])
def test_benchmark_configuration_properties(precision):
    """The 64x64x130 slab in the launch configuration the benchmark times
    (both forms, Jacobi V(1,1) on every level, quadratic warm start, tol
    1e-10), past the warm-up: every step's solve meets the tolerance in the
    FP64 residual recomputed from the returned fields, ions and mass are
    conserved, and Gauss's law closes (sum of electrode charges = -ionic
    charge, to the solve's tolerance)."""
    w = W.eo_slab(noise=True)
    p = lbe.make_params(w.shape, w.z, w.D, w.lB, tau=w.tau, Eapp=w.Eapp, omega=w.omega,
                        tol=1e-10, max_iter=1_000_000, check_every=8,
                        precision=precision, poisson=lbe.MG, flags=lbe.EXTRAPOLATE,
                        mg_nu1=1, mg_nu2=1, mg_nu1_coarse=1, mg_nu2_coarse=1)
    g = lbe.Lbe(p, w.node_type, w.phi_s, w.n_init, w.n_ref)
    t0 = g.totals()
    g.step(40)
    t1 = g.totals()
    assert t1["step"] == 40 and t1["poisson_resid"] <= 1e-10
    assert abs(t1["mass"] / t0["mass"] - 1) < 1e-9
    for k in range(2):
        assert abs(t1["nk"][k] / t0["nk"][k] - 1) < 1e-9
    fg = g.fields(f=False)
    R = residual_numpy(w.shape, w.node_type, fg["phi"], fg["n"], w.z, w.lB)
    assert np.abs(R).max() <= 1.05e-10
    q = g.qhist()
    assert q.shape == (41, 2)
    # Gauss: Q_1 + Q_2 = -Q_ion up to eps * (sum of |R| over fluid nodes)
    eps = T.permittivity(w.lB)
    bound = eps * np.abs(R).sum() + 1e-12 * np.abs(q[-1]).max()
    assert abs(q[-1].sum() + t1["q_ion"]) <= bound
