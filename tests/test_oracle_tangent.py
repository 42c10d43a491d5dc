"""Pins of the complex-step tangent oracle (oracle/tangent.py).

The tangent oracle is a second, independent statement of the step; these
tests tie it to things other than itself:
* its real part is the trajectory of the pinned C oracle;
* its derivatives equal central finite differences of the C oracle;
* the ion-free slab capacitor has an exact lattice capacitance, so dQ/dV and
  dQ/dl_B are closed forms;
* Gauss's law makes the summed electrode charge equal minus the (conserved)
  ionic charge, which fixes the derivatives of the sum exactly;
* at long times the derivative with respect to the voltage is the differential
  capacitance of the discrete non-linear Poisson-Boltzmann steady state,
  solved independently by Newton's method.
"""
from __future__ import annotations


import numpy as np
import pytest

import gpu_cases as G
import oracle
import theory as T
import workloads as W
from oracle import tangent as TG

LB = 0.4


def _case(kind):
    return G.adjoint_case(kind)


def _oracle(shape, t, ps, n0, f0, kw, flags):
    p = oracle.make_params(shape, kw["z"], kw["D"], kw["lB"], tau=kw["tau"], Eapp=kw["Eapp"],
                           tol=1e-14, flags=flags | oracle.FLAG_ALLOW_FLOATING)
    return oracle.Oracle(p, t, ps, n0, None, f0)


def _tparams(kw, flags):
    d = dict(kw)
    d["wall"] = 1.0 if flags & oracle.FLAG_NAIVE_DIRICHLET else 2.0
    return d


@pytest.mark.parametrize("kind", ["k2_field", "k3_naive"])
def test_real_part_is_the_oracle_trajectory(kind):
    shape, t, ps, n0, f0, kw, flags = _case(kind)
    steps = 15
    o = _oracle(shape, t, ps, n0, f0, kw, flags)
    o.step(steps)
    _, _, s = TG.charge_tangent(shape, _tparams(kw, flags), t, ps, n0, f0, steps,
                                dphi_s=(t == 1).astype(float))
    qh = o.qhist()
    q_t = np.array([q.real for q in s.q_hist])
    assert np.abs(qh - q_t).max() < 1e-12 * np.abs(qh).max()
    F = o.fields()
    assert np.abs(F["phi"] - s.phi.real.reshape(-1)).max() < 1e-12
    assert np.abs(F["n"] - s.n.real.reshape(len(kw["z"]), -1)).max() < 1e-15
    assert np.abs(F["f"] - s.f.real.reshape(19, -1)).max() < 1e-14


@pytest.mark.parametrize("kind", ["k2_field", "k3_naive"])
def test_derivatives_match_central_differences(kind):
    shape, t, ps, n0, f0, kw, flags = _case(kind)
    steps = 12
    rng = np.random.default_rng(21)
    fluid = t == 0
    directions = {
        "V1": dict(dphi_s=(t == 1).astype(float)),
        "lB": dict(dlB=1.0),
        "phi_s": dict(dphi_s=rng.standard_normal(t.size) * (~fluid)),
        "n0": dict(dn=1e-3 * rng.standard_normal(n0.shape) * fluid),
        "f0": dict(df=1e-2 * rng.standard_normal(f0.shape) * fluid),
    }
    for name, d in directions.items():
        _, dq, _ = TG.charge_tangent(shape, _tparams(kw, flags), t, ps, n0, f0, steps, **d)
        h = 1e-5

        def q_at(sgn):
            kk = dict(kw)
            kk["lB"] = kw["lB"] + sgn * h * d.get("dlB", 0.0)
            o = _oracle(shape, t, ps + sgn * h * d.get("dphi_s", 0.0), n0 + sgn * h * d.get("dn", 0.0),
                        f0 + sgn * h * d.get("df", 0.0), kk, flags)
            o.step(steps)
            return o.qhist()[-1]

        fd = (q_at(1) - q_at(-1)) / (2 * h)
        # central differences: O(h^2) truncation plus ~1e-16 |Q| / h rounding
        assert np.abs(dq - fd).max() < 1e-8 * np.abs(fd).max() + 1e-10, (name, dq, fd)


def test_ion_free_slab_capacitance():
    """No ions: nothing moves, Q_1 = C (V1 - V2) with the lattice capacitance
    A / (4 pi l_B L) of L fluid planes between mid-link walls (the potential
    is exactly linear in z).  So dQ_1/dphi_s is 1/(4 pi l_B L) on every node
    of electrode 1's face plane and 0 on the plane behind it, and
    dQ/dl_B = -Q/l_B."""
    nxy, L = 4, 10
    shape, t, ps = W.slab(nxy, nxy, L, 2, 0.05, -0.03)
    n0 = np.zeros((1, t.size))
    f0 = TG.rest_populations(t)
    kw = dict(z=(1,), D=(0.05,), lB=LB, tau=1.0, wall=2.0)
    steps = 3
    C = nxy * nxy * T.dielectric_slab_capacitance(LB, L)
    q, dq, _ = TG.charge_tangent(shape, kw, t, ps, n0, f0, steps, dphi_s=(t == 1).astype(float))
    assert abs(q[0] - C * 0.08) < 1e-14 and abs(dq[0] - C) < 1e-13 * C and abs(dq[1] + C) < 1e-13 * C
    z = np.arange(t.size) // (nxy * nxy)
    for plane, expect in ((1, C / nxy ** 2), (0, 0.0)):
        r = int(np.flatnonzero(z == plane)[5])
        e = np.zeros(t.size)
        e[r] = 1.0
        _, dq, _ = TG.charge_tangent(shape, kw, t, ps, n0, f0, steps, dphi_s=e)
        assert abs(dq[0] - expect) < 1e-14, (plane, dq, expect)
    _, dq, _ = TG.charge_tangent(shape, kw, t, ps, n0, f0, steps, dlB=1.0)
    assert np.abs(dq + q / LB).max() < 1e-13 * np.abs(q).max()


@pytest.mark.parametrize("kind", ["k2_field", "k3_naive"])
def test_gauss_law_fixes_the_summed_charge(kind):
    """Sum_e Q_e = -sum_r rho_el(r) (Gauss's law on the lattice) and the link
    fluxes conserve every species, so the derivative of the summed charge is
    0 along phi_s, l_B and the populations, and -sum z_k dn_k along n(0)."""
    shape, t, ps, n0, f0, kw, flags = _case(kind)
    steps = 10
    rng = np.random.default_rng(5)
    fluid = t == 0
    scale = None
    for d in (dict(dphi_s=rng.standard_normal(t.size) * (~fluid)), dict(dlB=1.0),
              dict(df=1e-2 * rng.standard_normal(f0.shape) * fluid)):
        _, dq, _ = TG.charge_tangent(shape, _tparams(kw, flags), t, ps, n0, f0, steps, **d)
        scale = np.abs(dq).max()
        assert abs(dq.sum()) < 1e-12 * scale + 1e-15, (d.keys(), dq)
    dn = rng.standard_normal(n0.shape) * fluid
    _, dq, _ = TG.charge_tangent(shape, _tparams(kw, flags), t, ps, n0, f0, steps, dn=dn)
    expect = -(np.asarray(kw["z"])[:, None] * dn).sum()
    assert abs(dq.sum() - expect) < 1e-12 * np.abs(dq).max()


def test_differential_capacitance_of_the_nonlinear_steady_state():
    """Long times, beyond the linear regime (V = 0.5): dQ_1/dV for the
    antisymmetric voltage +-V tends to the differential capacitance of the
    discrete non-linear Poisson-Boltzmann double layer (Newton solution of
    theory.nonlinear_pb_slab, differentiated by central differences)."""
    nf, V, debye = 32, 0.5, 4.0
    salt = W.salt_for_debye(debye, LB)
    shape, t, ps = W.slab(1, 1, nf, 1, V, -V)
    n0 = np.where(t == 0, salt, 0.0)[None, :].repeat(2, 0)
    f0 = TG.rest_populations(t)
    kw = dict(z=(1, -1), D=(0.2, 0.2), lB=LB, tau=1.0, wall=2.0)
    direction = np.where(t == 1, 1.0, np.where(t == 2, -1.0, 0.0))
    _, dq, _ = TG.charge_tangent(shape, kw, t, ps, n0, f0, 8000, dphi_s=direction)
    eps = T.permittivity(LB)

    def q1(v):
        phi, _ = T.nonlinear_pb_slab(nf, (1, -1), (salt * nf, salt * nf), LB, v, -v)
        return -eps * 2.0 * (phi[0] - v)

    h = 1e-5
    cdiff = (q1(V + h) - q1(V - h)) / (2 * h)
    assert abs(dq[0] / cdiff - 1) < 1e-6, (dq, cdiff)
    assert abs(dq[1] / dq[0] + 1) < 1e-9
    # and it is not the linear (Debye-Hueckel) value: the pin sees the non-linearity
    assert abs(cdiff / T.dh_slab_capacitance(LB, debye, nf) - 1) > 0.05


def _momentum_c(o, t):
    F = o.fields()
    return (F["u"] * F["rho"])[:, t == 0].sum(1)


@pytest.mark.parametrize("kind", ["k2_field", "k3_naive"])
def test_momentum_matches_oracle_and_differences(kind):
    """The total fluid momentum sum_r (sum_i f_i c_i + F/2) (the mass flux of
    the velocity of Guo forcing; under the applied field its component along
    it is the electro-osmotic flux): real part against the C oracle's rho u,
    derivatives along the voltage, l_B and random n(0), f(0) against central
    differences of the C oracle."""
    shape, t, ps, n0, f0, kw, flags = _case(kind)
    steps = 10
    o = _oracle(shape, t, ps, n0, f0, kw, flags)
    o.step(steps)
    rng = np.random.default_rng(9)
    fluid = t == 0
    dirs = {"V1": dict(dphi_s=(t == 1).astype(float)), "lB": dict(dlB=1.0),
            "n0": dict(dn=1e-3 * rng.standard_normal(n0.shape) * fluid),
            "f0": dict(df=1e-2 * rng.standard_normal(f0.shape) * fluid)}
    m_c = _momentum_c(o, t)
    for name, d in dirs.items():
        _, _, s = TG.charge_tangent(shape, _tparams(kw, flags), t, ps, n0, f0, steps, **d)
        m = s.momentum()
        # rho u from u = (m + F/2) / rho rounds differently from m + F/2: ~1e-16 per site
        assert np.abs(m.real - m_c).max() <= 1e-11 * np.abs(m_c).max() + 1e-15, (name, m, m_c)
        h = 1e-5

        def m_at(sgn):
            kk = dict(kw)
            kk["lB"] = kw["lB"] + sgn * h * d.get("dlB", 0.0)
            oo = _oracle(shape, t, ps + sgn * h * d.get("dphi_s", 0.0),
                         n0 + sgn * h * d.get("dn", 0.0), f0 + sgn * h * d.get("df", 0.0), kk, flags)
            oo.step(steps)
            return _momentum_c(oo, t)

        fd = (m_at(1) - m_at(-1)) / (2 * h)
        dm = m.imag / TG.STEP
        # the momentum sum carries ~4e-16 of rounding, ~3e-11 after / 2h; the
        # solves' 1e-14 residual adds as much
        assert np.abs(dm - fd).max() <= 1e-7 * np.abs(fd).max() + 3e-10, (name, dm, fd)
