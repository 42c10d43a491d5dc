"""The GPU library beyond the paper's main scheme, against the oracle and
closed forms: the first-order Dirichlet scheme the paper contrasts with
(Sec. II C, Fig. 1; LBE_NAIVE_DIRICHLET), electrode potentials changed during
a run (lbe_set_electrode_potential; Sec. I and IV name time-dependent and
non-linear voltages as applications), and the non-linear steady state."""
import math

import numpy as np
import pytest

import gpu_cases as G
import oracle
import paper_1907_04732_amd as lbe
import theory as T
import workloads as W
from test_gpu_parity import TOL, compare, rel

pytestmark = pytest.mark.gpu

LB = 0.4


def naive_pair(name, **over):
    kw, shape, t, ps, n0, nref, nsteps, sweeps = G.case(name)
    kw = dict(kw)
    kw["flags"] = kw.get("flags", 0) | lbe.NAIVE_DIRICHLET
    pk = dict(tol=0.0, max_iter=sweeps, check_every=4)
    pk.update(over)
    o = oracle.Oracle(oracle.make_params(shape, **kw, **pk), t, ps, n0, nref)
    return o, kw, pk, shape, t, ps, n0, nref, nsteps


@pytest.mark.parametrize("name", ["slab_4x4x34", "coax_16x16x4", "random_6x10x14_k3"])
def test_naive_scheme_step_parity(name):
    """FP64 SOR with the first-order scheme: same sweeps, same colour order,
    <= 1e-12 relative on phi, n, f, u and the charge history."""
    o, kw, pk, shape, t, ps, n0, nref, nsteps = naive_pair(name)
    g = lbe.Lbe(lbe.make_params(shape, **kw, **pk), t, ps, n0, nref)
    compare(o, g, t)
    o.step(nsteps)
    g.step(nsteps)
    compare(o, g, t)


@pytest.mark.parametrize("name", ["slab_4x4x34", "coax_16x16x4"])
def test_naive_scheme_multigrid_fixed_point(name):
    """Multigrid with the first-order scheme (wall factor 1 on every level, zero
    correction on solid coarse cells) reaches the oracle's SOR fixed point:
    at tol = 1e-14 within the |A^-1| tol bound (2e-11 of the voltage)."""
    o, kw, pk, shape, t, ps, n0, nref, nsteps = naive_pair(name, tol=1e-14, max_iter=10**6,
                                                            check_every=1)
    g = lbe.Lbe(lbe.make_params(shape, **kw, tol=1e-14, max_iter=200, poisson=lbe.MG), t, ps, n0,
                nref)
    o.step(nsteps)
    g.step(nsteps)
    fo, fg = o.fields(), g.fields()
    assert rel(fg["phi"], fo["phi"], 0.1) <= 2e-11
    assert rel(fg["n"], fo["n"]) <= 2e-11
    assert rel(g.qhist(), o.qhist()) <= 2e-11


def _schedule(name, set_every, rounds, **over):
    kw, shape, t, ps, n0, nref, nsteps, sweeps = G.case(name)
    pk = dict(tol=0.0, max_iter=sweeps, check_every=4)
    pk.update(over.pop("pk", {}))
    o = oracle.Oracle(oracle.make_params(shape, **kw, **pk), t, ps, n0, nref)
    g = lbe.Lbe(lbe.make_params(shape, **kw, **pk, **over), t, ps, n0, nref)
    for k in range(rounds):
        o.step(set_every)
        g.step(set_every)
        # a voltage ramp with a sign change of one electrode's potential
        new = np.where(t > 0, ps * (1.0 + 0.5 * (k + 1)) * (-1.0) ** k + 0.01 * t, 0.0)
        o.set_electrode_potential(new)
        g.set_electrode_potential(new)
    return o, g, t


@pytest.mark.parametrize("name", ["slab_4x4x34", "random_6x10x14_k3"])
def test_electrode_potential_schedule_parity(name):
    """Potentials changed every 5 steps (ramp and sign flips): the GPU follows
    the oracle to <= 1e-12 in every field and in the whole charge history
    (one row per step, the set call replacing the current row)."""
    o, g, t = _schedule(name, 5, 4)
    compare(o, g, t)
    assert g.qhist().shape == o.qhist().shape


@pytest.mark.parametrize("precision,tol", [(lbe.FP64, 1e-10), (lbe.FP32_MIXED, 1e-5)])
def test_electrode_potential_schedule_multigrid(precision, tol):
    """The same schedule with multigrid (and the mixed form) against the oracle
    at a solver tolerance of 1e-13: within the forms' bounds."""
    o, g, t = _schedule("slab_4x4x34", 5, 4,
                        pk=dict(tol=1e-13, max_iter=10**6, check_every=1),
                        poisson=lbe.MG, precision=precision)
    fo, fg = o.fields(), g.fields(f=False)
    assert rel(fg["phi"], fo["phi"], 0.2) <= tol
    assert rel(g.qhist(), o.qhist()) <= tol


def _steady(nf, V, debye, D, steps, flags=0, precision=lbe.FP64, nxy=2, z=(1, -1)):
    zz = np.asarray(z, float)
    ratio = 1.0 / np.abs(zz)
    rs = ratio / (4 * math.pi * LB * debye * debye * float((zz * zz * ratio).sum()))
    shape, t, ps = W.slab(nxy, nxy, nf, 1, V, -V)
    p = lbe.make_params(shape, z, D, LB, tol=1e-12, max_iter=500, poisson=lbe.MG,
                        precision=precision, flags=flags | lbe.EXTRAPOLATE)
    g = lbe.Lbe(p, t, ps, None, tuple(rs))
    g.step(steps)
    return g, shape, rs


@pytest.mark.parametrize("precision,ptol,ntol", [(lbe.FP64, 1e-8, 1e-7), (lbe.FP32_MIXED, 1e-5, 1e-5)])
def test_nonlinear_steady_state_gpu(precision, ptol, ntol):
    """dV = 1 kT/e across a 32-plane slab (lambda_D = 4): the steady state is
    the Boltzmann distribution in the discrete non-linear Poisson-Boltzmann
    potential (Newton solution, theory.nonlinear_pb_slab)."""
    nf, V = 32, 0.5
    g, shape, rs = _steady(nf, V, 4.0, (0.2, 0.2), 8000, precision=precision)
    f = g.fields(f=False)
    phi = f["phi"].reshape(shape[2], -1)[1:nf + 1].mean(axis=1)
    n = f["n"].reshape(2, shape[2], -1)[:, 1:nf + 1].mean(axis=2)
    phi_th, n_th = T.nonlinear_pb_slab(nf, (1, -1), rs * nf, LB, V, -V)
    assert np.abs(phi - phi_th).max() <= ptol * V, np.abs(phi - phi_th).max()
    assert np.abs(n / n_th - 1).max() <= ntol, np.abs(n / n_th - 1).max()
    q = g.electrode_charge()[0] / (shape[0] * shape[1])
    q_th = -T.permittivity(LB) * 2.0 * (phi_th[0] - V)
    assert abs(q / q_th - 1) <= ntol


def test_first_order_scheme_loses_an_order():
    """Fig. 4b and Sec. II C: the steady-state capacitance error against
    Debye-Hueckel (finite-gap form, gap L = number of fluid planes) falls as
    (dx/lambda_D)^2 with the mid-link scheme and only as dx/lambda_D with
    the potential held on the solid nodes.  lambda_D = 2, 4, 8 lattice
    spacings at L / lambda_D = 8, voltage 0.01 kT/e (linear regime)."""
    D, V = 0.25, 0.005
    slopes = {}
    for name, flags in (("mid-link", 0), ("naive", lbe.NAIVE_DIRICHLET)):
        errs, hs = [], []
        for debye in (2.0, 4.0, 8.0):
            nf = int(8 * debye)
            steps = int(15.0 / T.charging_rate_slab(debye, float(nf), D)) + 200
            g, shape, rs = _steady(nf, V, debye, (D, D), steps, flags=flags)
            q = g.qhist()[:, 0] / (shape[0] * shape[1])
            drift = abs(q[-1] - q[-100]) / abs(q[-1])
            assert drift < 1e-6, (name, debye, drift)
            C = q[-1] / (2 * V)
            err = abs(C / T.dh_slab_capacitance(LB, debye, float(nf)) - 1)
            errs.append(err)
            hs.append(1.0 / debye)
            print(name, debye, f"{err:.3e}")
        slopes[name] = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    print(slopes)
    assert 1.7 <= slopes["mid-link"] <= 2.3
    assert 0.8 <= slopes["naive"] <= 1.2
