"""Reverse mode of the GPU library (lbe_record / lbe_adjoint and the
torch.autograd wrapper) against the complex-step tangent oracle, central
differences of the GPU forward step, Gauss's-law invariants and the
differential capacitance of the non-linear steady state.

Tolerance of the oracle comparison: both sides are FP64 derivatives of the
same discrete map.  They differ only through the Poisson solves, which the
GPU stops at ||R||_inf <= tol (1e-13 here) while the oracle solves exactly;
with ||A^-1|| of order L^2 / 6 ~ 10 on these lattices each solve moves phi
by ~1e-12, i.e. ~1e-11 relative on a charge of order 0.1-1.  2e-9 relative
to the largest derivative leaves that margin for rounding over the steps.
"""
import numpy as np
import pytest

import gpu_cases as G
import paper_1907_04732_amd as lbe
import theory as T
import workloads as W
from oracle import tangent as TG

pytestmark = pytest.mark.gpu

RTOL = 2e-9


def _lbe(shape, t, ps, n0, f0, kw, flags, extra_flags=0, **over):
    pk = dict(tol=1e-13, max_iter=200000, check_every=2, omega=1.7)
    pk.update(over)
    pk["flags"] = flags | lbe.ALLOW_FLOATING | extra_flags
    p = lbe.make_params(shape, **kw, **pk)
    return lbe.Lbe(p, t, ps, n_init=n0, f_init=f0)


def _tangent(case, steps, **d):
    shape, t, ps, n0, f0, kw, flags = case
    tp = dict(kw)
    tp["wall"] = 1.0 if flags & lbe.NAIVE_DIRICHLET else 2.0
    q, dq, _ = TG.charge_tangent(shape, tp, t, ps, n0, f0, steps, **d)
    return q, dq


SOLVERS = {
    "sor": dict(poisson=lbe.SOR4),
    "mg": dict(poisson=lbe.MG, max_iter=400),
    "mg_krylov_extrap": dict(poisson=lbe.MG, max_iter=400,
                             extra_flags=lbe.KRYLOV | lbe.EXTRAPOLATE),
}


@pytest.mark.parametrize("solver", list(SOLVERS))
@pytest.mark.parametrize("kind", ["k2_field", "k3_naive"])
def test_adjoint_matches_tangent_oracle(kind, solver):
    """Every gradient, tested along the directions the oracle differentiates:
    each electrode's voltage, l_B, a random solid-node potential field, random
    initial concentrations and populations; for the weights of every
    electrode in turn.  12 steps in segments of 5 (a ragged last segment)."""
    case = G.adjoint_case(kind)
    shape, t, ps, n0, f0, kw, flags = case
    steps = 12
    g = _lbe(*case, **SOLVERS[solver])
    g.record(steps, every=5)
    q_gpu = g.qhist()[-1]
    rng = np.random.default_rng(31)
    fluid = t == 0
    dirs = {
        "lB": dict(dlB=1.0),
        "phi_s": dict(dphi_s=rng.standard_normal(t.size) * (~fluid)),
        "n0": dict(dn=1e-3 * rng.standard_normal(n0.shape) * fluid),
        "f0": dict(df=1e-2 * rng.standard_normal(f0.shape) * fluid),
    }
    for e in range(1, g.ne + 1):
        dirs[f"V{e}"] = dict(dphi_s=(t == e).astype(float))
    tangents = {}
    for name, d in dirs.items():
        q, dq = _tangent(case, steps, **d)
        tangents[name] = dq
    assert np.abs(q_gpu - q).max() < 1e-11 * np.abs(q).max()
    for e in range(g.ne):
        qbar = np.zeros(g.ne)
        qbar[e] = 1.0
        gr = g.adjoint(qbar)
        got = {
            "lB": gr["lB"],
            "phi_s": gr["phi_s"] @ dirs["phi_s"]["dphi_s"],
            "n0": (gr["n"] * dirs["n0"]["dn"]).sum(),
            "f0": (gr["f"] * dirs["f0"]["df"]).sum(),
        }
        for k in range(1, g.ne + 1):
            got[f"V{k}"] = gr["phi_s"][t == k].sum()
        scale = max(abs(tangents[n][e]) for n in tangents)
        for name in tangents:
            assert abs(got[name] - tangents[name][e]) <= RTOL * scale, (e, name, got[name],
                                                                       tangents[name][e])
        # nothing on the nodes where a quantity does not exist
        assert not gr["phi_s"][fluid].any() and not gr["n"][:, ~fluid].any()
        assert not gr["f"][:, ~fluid].any()
    # the state is back at the end of the record and the record stays usable
    assert np.array_equal(g.qhist()[-1], q_gpu)
    g.step(1)
    with pytest.raises(lbe.LbeError):
        g.adjoint(np.ones(g.ne))


@pytest.mark.parametrize("kind", ["k2_field", "k3_naive"])
def test_momentum_adjoint_matches_tangent_oracle(kind):
    """Gradient of the total fluid momentum sum_r (sum_i f_i c_i + F/2) at the
    end (under the applied field, its component along the field is the
    electro-osmotic flux), each component in turn, against the tangent
    oracle along the voltage, l_B, random phi_s, n(0) and f(0); and the
    gradient of a combined charge + momentum objective is the sum of the
    two.  FP64 multigrid with flexible CG and the extrapolated start.
    Bound 1e-7 of the largest derivative: the momentum is ~1e-4 and its
    derivatives come through the force, which the Poisson tolerance moves by
    ~1e-12 relative, with rounding in sums of ~1e-5-sized terms."""
    case = G.adjoint_case(kind)
    shape, t, ps, n0, f0, kw, flags = case
    steps = 12
    g = _lbe(*case, poisson=lbe.MG, max_iter=400, extra_flags=lbe.KRYLOV | lbe.EXTRAPOLATE)
    g.record(steps, every=5)
    rng = np.random.default_rng(17)
    fluid = t == 0
    dirs = {"V1": dict(dphi_s=(t == 1).astype(float)), "lB": dict(dlB=1.0),
            "phi_s": dict(dphi_s=rng.standard_normal(t.size) * (~fluid)),
            "n0": dict(dn=1e-3 * rng.standard_normal(n0.shape) * fluid),
            "f0": dict(df=1e-2 * rng.standard_normal(f0.shape) * fluid)}
    tp = dict(kw)
    tp["wall"] = 1.0 if flags & lbe.NAIVE_DIRICHLET else 2.0
    dm = {}
    for name, d in dirs.items():
        _, _, s_ = TG.charge_tangent(shape, tp, t, ps, n0, f0, steps, **d)
        dm[name] = s_.momentum().imag / TG.STEP

    def project(gr):
        return {"V1": gr["phi_s"][t == 1].sum(), "lB": gr["lB"],
                "phi_s": gr["phi_s"] @ dirs["phi_s"]["dphi_s"],
                "n0": (gr["n"] * dirs["n0"]["dn"]).sum(), "f0": (gr["f"] * dirs["f0"]["df"]).sum()}

    # the library's own value of the objective (lbe_obs.momentum) is the
    # tangent oracle's real part
    m_ref = s_.momentum().real
    m_lib = np.array(g.totals()["momentum"])
    assert np.abs(m_lib - m_ref).max() <= 1e-10 * np.abs(m_ref).max(), (m_lib, m_ref)
    for a in range(3):
        ubar = np.zeros(3)
        ubar[a] = 1.0
        got = project(g.adjoint(ubar=ubar))
        scale = max(abs(dm[n][a]) for n in dm)
        for name in dm:
            assert abs(got[name] - dm[name][a]) <= 1e-7 * scale, (a, name, got[name], dm[name][a])
    qbar = np.linspace(1.0, -0.5, g.ne)
    ubar = np.array([0.3, -2.0, 1.1])
    both, q_only, u_only = g.adjoint(qbar, ubar), g.adjoint(qbar), g.adjoint(ubar=ubar)
    for key in ("phi_s", "n", "f"):
        ref = q_only[key] + u_only[key]
        assert np.abs(both[key] - ref).max() <= 1e-10 * np.abs(ref).max()


def test_adjoint_porous_crop_matches_tangent_oracle():
    """A 24^3 crop of the porous electrode (sphere caps of electrode 1 and the
    first planes of the counter-electrode), FP64 multigrid with flexible CG
    and the extrapolated start, 20 steps in segments of 8: the voltage,
    l_B and random solid-potential derivatives of both charges against the
    tangent oracle, within RTOL of the largest."""
    w = W.porous_crop()
    t = w.node_type
    rng = np.random.default_rng(7)
    f0 = TG.rest_populations(t) * (1.0 + 1e-3 * rng.uniform(-1, 1, (19, t.size)))
    kw = dict(z=w.z, D=w.D, lB=w.lB, tau=w.tau, Eapp=w.Eapp)
    case = (w.shape, t, w.phi_s, w.n_init, f0, kw, 0)
    steps = 20
    g = _lbe(*case, poisson=lbe.MG, max_iter=400, extra_flags=lbe.KRYLOV | lbe.EXTRAPOLATE)
    g.record(steps, every=8)
    dirs = {"V1": dict(dphi_s=(t == 1).astype(float)), "V2": dict(dphi_s=(t == 2).astype(float)),
            "lB": dict(dlB=1.0), "phi_s": dict(dphi_s=rng.standard_normal(t.size) * (t != 0))}
    tangents = {}
    for name, d in dirs.items():
        q, tangents[name] = _tangent(case, steps, **d)
    assert np.abs(g.qhist()[-1] - q).max() < 1e-11 * np.abs(q).max()
    for e in range(g.ne):
        qbar = np.zeros(g.ne)
        qbar[e] = 1.0
        gr = g.adjoint(qbar, n=False, f=False)
        got = {"V1": gr["phi_s"][t == 1].sum(), "V2": gr["phi_s"][t == 2].sum(), "lB": gr["lB"],
               "phi_s": gr["phi_s"] @ dirs["phi_s"]["dphi_s"]}
        scale = max(abs(tangents[n][e]) for n in tangents)
        for name in tangents:
            assert abs(got[name] - tangents[name][e]) <= RTOL * scale, (e, name, got[name],
                                                                       tangents[name][e])


def test_adjoint_is_linear_in_the_weights():
    case = G.adjoint_case("k2_field")
    g = _lbe(*case, poisson=lbe.MG, max_iter=400)
    g.record(9, every=4)
    a = g.adjoint([1.0, 0.0])
    b = g.adjoint([0.0, 1.0])
    c = g.adjoint([2.0, -3.0])
    for key in ("phi_s", "n", "f"):
        ref = 2 * a[key] - 3 * b[key]
        assert np.abs(c[key] - ref).max() <= 1e-9 * np.abs(ref).max()
    assert abs(c["lB"] - (2 * a["lB"] - 3 * b["lB"])) <= 1e-9 * abs(c["lB"])


def test_reverse_mode_errors():
    case = G.adjoint_case("k2_field")
    shape, t, ps, n0, f0, kw, flags = case
    g = _lbe(*case)
    with pytest.raises(lbe.LbeError) as ei:
        g.adjoint([1.0, 0.0])  # no record yet
    assert ei.value.code == lbe.EINVAL
    with pytest.raises(lbe.LbeError):
        g.record(3, every=0)
    g.record(3, every=2)
    g.set_electrode_potential(ps * 1.1)
    with pytest.raises(lbe.LbeError):
        g.adjoint([1.0, 0.0])  # potentials changed after the record
    with pytest.raises(ValueError):
        g.adjoint([1.0])
    with pytest.raises(lbe.LbeError) as ei:
        g.record(-1)
    assert ei.value.code == lbe.EINVAL


@pytest.mark.parametrize("kind", ["k2_field", "k3_naive"])
def test_mixed_form_adjoint(kind):
    """Reverse mode of an LBE_FP32_MIXED record: the FP64 adjoint along the
    mixed-precision trajectory.  FP32 keeps the deviations h = f - w rho0 and
    nu = n - n_ref to ~6e-8 of themselves, so the trajectory, and with it
    every derivative, moves by ~1e-7 relative: bound 1e-5 against the
    oracle tangent (the FP64 reverse mode meets 2e-9)."""
    case = G.adjoint_case(kind)
    shape, t, ps, n0, f0, kw, flags = case
    steps = 12
    g = _lbe(*case, poisson=lbe.MG, max_iter=400, precision=lbe.FP32_MIXED)
    g.record(steps, every=5)
    rng = np.random.default_rng(41)
    fluid = t == 0
    dirs = {"lB": dict(dlB=1.0), "n0": dict(dn=1e-3 * rng.standard_normal(n0.shape) * fluid),
            "f0": dict(df=1e-2 * rng.standard_normal(f0.shape) * fluid)}
    for e in range(1, g.ne + 1):
        dirs[f"V{e}"] = dict(dphi_s=(t == e).astype(float))
    tangents = {name: _tangent(case, steps, **d)[1] for name, d in dirs.items()}
    for e in range(g.ne):
        qbar = np.zeros(g.ne)
        qbar[e] = 1.0
        gr = g.adjoint(qbar)
        got = {"lB": gr["lB"], "n0": (gr["n"] * dirs["n0"]["dn"]).sum(),
               "f0": (gr["f"] * dirs["f0"]["df"]).sum()}
        for k in range(1, g.ne + 1):
            got[f"V{k}"] = gr["phi_s"][t == k].sum()
        scale = max(abs(tangents[n][e]) for n in tangents)
        for name in tangents:
            assert abs(got[name] - tangents[name][e]) <= 1e-5 * scale, (e, name, got[name],
                                                                       tangents[name][e])


def test_autograd_function():
    """torch.autograd: backward() equals lbe_adjoint; gradcheck in fast mode
    (one random projection checked by central differences of the forward)."""
    import torch
    from paper_1907_04732_amd.autograd import charge_and_momentum, electrode_charge

    shape, t, ps, n0, f0, kw, flags = G.adjoint_case("k2_field")
    kw = dict(kw)
    lB = kw.pop("lB")
    opts = dict(shape=shape, node_type=t, nsteps=6, every=4, tol=1e-13, max_iter=400,
                poisson=lbe.MG, flags=lbe.ALLOW_FLOATING, **kw)
    x = [torch.tensor(ps, dtype=torch.float64, requires_grad=True),
         torch.tensor(lB, dtype=torch.float64, requires_grad=True),
         torch.tensor(n0, dtype=torch.float64, requires_grad=True),
         torch.tensor(f0, dtype=torch.float64, requires_grad=True)]
    q = electrode_charge(*x, **opts)
    w = torch.tensor([0.7, -1.3], dtype=torch.float64)
    (q * w).sum().backward()
    g = _lbe(shape, t, ps, n0, f0, dict(kw, lB=lB), flags, poisson=lbe.MG, max_iter=400)
    g.record(6, every=4)
    ref = g.adjoint(w.numpy())
    assert np.abs(x[0].grad.numpy() - ref["phi_s"]).max() <= 1e-12 * np.abs(ref["phi_s"]).max()
    assert abs(float(x[1].grad) - ref["lB"]) <= 1e-12 * abs(ref["lB"])
    assert np.abs(x[2].grad.numpy() - ref["n"]).max() <= 1e-12 * np.abs(ref["n"]).max()
    assert np.abs(x[3].grad.numpy() - ref["f"]).max() <= 1e-12 * np.abs(ref["f"]).max()
    fn = lambda a, b, c, d: electrode_charge(a, b, c, d, **opts)  # noqa: E731
    assert torch.autograd.gradcheck(fn, tuple(v.detach().requires_grad_() for v in x),
                                    eps=1e-6, atol=1e-7, rtol=1e-5, fast_mode=True)
    # the momentum output: backward equals lbe_adjoint with momentum weights
    y = [v.detach().requires_grad_() for v in x]
    q2, m2 = charge_and_momentum(*y, **opts)
    wm = torch.tensor([1.5, 0.0, -0.7], dtype=torch.float64)
    ((q2 * w).sum() + (m2 * wm).sum()).backward()
    ref = g.adjoint(w.numpy(), wm.numpy())
    assert np.abs(y[0].grad.numpy() - ref["phi_s"]).max() <= 1e-12 * np.abs(ref["phi_s"]).max()
    assert np.abs(y[2].grad.numpy() - ref["n"]).max() <= 1e-12 * np.abs(ref["n"]).max()
    assert np.abs(y[3].grad.numpy() - ref["f"]).max() <= 1e-12 * np.abs(ref["f"]).max()


def test_differential_capacitance_at_steady_state():
    """8000 recorded steps (80 checkpoints) on a 32-plane slab at V = +-0.5:
    dQ_1/dV is the differential capacitance of the discrete non-linear
    Poisson-Boltzmann double layer (Newton, theory.nonlinear_pb_slab), and
    the two plates' derivatives are opposite."""
    nf, V, debye, LB = 32, 0.5, 4.0, 0.4
    salt = W.salt_for_debye(debye, LB)
    shape, t, ps = W.slab(1, 1, nf, 1, V, -V)
    n0 = np.where(t == 0, salt, 0.0)[None, :].repeat(2, 0)
    kw = dict(z=(1, -1), D=(0.2, 0.2), lB=LB, tau=1.0)
    g = _lbe(shape, t, ps, n0, None, kw, 0, poisson=lbe.SOR4, check_every=1)
    g.record(8000, every=100)
    gr = g.adjoint([1.0, 0.0])
    dq_dv = gr["phi_s"][t == 1].sum() - gr["phi_s"][t == 2].sum()
    g2 = g.adjoint([0.0, 1.0])
    dq2_dv = g2["phi_s"][t == 1].sum() - g2["phi_s"][t == 2].sum()
    assert abs(dq2_dv + dq_dv) <= 1e-9 * abs(dq_dv)
    eps = T.permittivity(LB)

    def q1(v):
        phi, _ = T.nonlinear_pb_slab(nf, (1, -1), (salt * nf, salt * nf), LB, v, -v)
        return -eps * 2.0 * (phi[0] - v)

    h = 1e-5
    cdiff = (q1(V + h) - q1(V - h)) / (2 * h)
    assert abs(dq_dv / cdiff - 1) < 1e-6, (dq_dv, cdiff)


POROUS_FORMS = {
    # form: (precision, steps, checkpoint interval, FD step, FD bound, invariant bound)
    "fp64": (lbe.FP64, 24, 10, 1e-3, 1e-6, 1e-7),
    "fp32_mixed": (lbe.FP32_MIXED, 4000, 200, 1e-4, 1e-4, 1e-6),
}


@pytest.mark.parametrize("form", list(POROUS_FORMS))
def test_adjoint_porous_electrode_invariants_and_differences(form):
    """The porous-electrode workload at its full size (192^3, multigrid with
    flexible CG): properties that hold at any size.
    * Gauss's law: sum_e Q_e = -sum rho_el, conserved, so for qbar = (1, 1)
      the phi_s, l_B and population gradients vanish and the concentration
      gradient is -z_k on every fluid node;
    * d Q_1 / d V_1 equals central differences of the GPU forward step.
    FP64: 24 steps, h = 1e-3 (Q is close to linear in V at 0.05, the O(h^2)
    term is ~h^2/24 relative; the solves' residual moves Q by ~1e-8 relative,
    ~1e-7 after the division by 2h).  Mixed form, as the workload is
    configured: 4000 steps checkpointed every 200, h = 1e-4; FP32 rounding
    of the deviations moves Q by ~1e-7 relative at most between the two
    runs, ~5e-5 after the division, within the configuration's 1e-4 bound.
    Invariants: each adjoint solve stops at ||R|| <= 1e-12 with ||A^-1|| ~
    10^3 on this lattice, so lambda carries ~1e-9 and 4 pi l_B lambda ~5e-9
    (FP64); the mixed form's FP32 corrections leave ~1e-7."""
    precision, steps, every, h, fd_bound, inv_bound = POROUS_FORMS[form]
    w = W.porous_electrode(noise=True)
    kw = dict(z=w.z, D=w.D, lB=w.lB, tau=w.tau)
    pk = dict(tol=1e-12, max_iter=200, poisson=lbe.MG, flags=lbe.KRYLOV | lbe.EXTRAPOLATE,
              precision=precision)

    def make(ps):
        return lbe.Lbe(lbe.make_params(w.shape, **kw, **pk), w.node_type, ps, n_init=w.n_init,
                       n_ref=w.n_ref)

    g = make(w.phi_s)
    print(f"porous 192^3 {form}: recording {steps} steps every {every}", flush=True)
    g.record(steps, every)
    print(f"porous 192^3 {form}: adjoint (1, 0)", flush=True)
    a = g.adjoint([1.0, 0.0])
    print(f"porous 192^3 {form}: adjoint (1, 1)", flush=True)
    s = g.adjoint([1.0, 1.0])
    fluid = w.node_type == 0
    scale = np.abs(a["phi_s"]).max()
    assert np.abs(s["phi_s"]).max() <= inv_bound * scale
    assert abs(s["lB"]) <= inv_bound * abs(a["lB"])
    assert np.abs(s["f"]).max() <= inv_bound * np.abs(a["f"]).max()
    z = np.asarray(w.z, float)[:, None]
    assert np.abs(s["n"][:, fluid] + z).max() <= inv_bound
    dv = a["phi_s"][w.node_type == 1].sum()
    del g
    q = []
    for sgn in (1, -1):
        print(f"porous 192^3 {form}: forward at V1 {'+' if sgn > 0 else '-'} h", flush=True)
        f = make(w.phi_s + sgn * h * (w.node_type == 1))
        f.step(steps)
        q.append(f.qhist()[-1][0])
        del f
    fd = (q[0] - q[1]) / (2 * h)
    print(f"porous 192^3 {form}: adjoint {dv:.10e} differences {fd:.10e}", flush=True)
    assert abs(dv - fd) <= fd_bound * abs(fd), (dv, fd)
