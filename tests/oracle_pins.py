"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each function builds a small case, runs the oracle (optionally a modified
build of it, given by `libpath`) and raises AssertionError when the oracle
departs from the closed form, the exact lattice identity or the invariant.
None of them re-types the oracle's own formula: the expected values are
closed forms of the paper (arXiv:1907.04732), exact consequences of them on
the lattice derived by hand, or invariants.
"""
from __future__ import annotations

import math

import numpy as np

import oracle
import theory as T
import workloads as W

LB = 0.4
FLOAT = oracle.FLAG_ALLOW_FLOATING


def _run(shape, t, ps, z, D, lB=LB, n_init=None, n_ref=None, f_init=None, libpath=None, **kw):
    p = oracle.make_params(shape, z, D, lB, **kw)
    return oracle.Oracle(p, t, ps, n_init, n_ref, f_init, libpath=libpath)


def _periodic(shape):
    N = shape[0] * shape[1] * shape[2]
    return np.zeros(N, np.uint8), np.zeros(N)


def _coords(shape):
    nx, ny, nz = shape
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx]
    return x.reshape(-1), y.reshape(-1), z.reshape(-1)


def _equilibrium(rho, u):
    """Second-order equilibrium populations for uniform rho, u (used only to
    build a uniform flow as an input)."""
    c, w = oracle.velocities()
    cu = c @ np.asarray(u, float)
    uu = float(np.dot(u, u))
    return w * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu)


# ---------------------------------------------------------------------------

def pin_velocity_set():
    """Sec. II C sum rules: sum w = 1, sum w c = 0, sum w c c = delta / 3; the
    19 velocities are rest, 6 nearest and 12 next-nearest neighbours."""
    c, w = oracle.velocities()
    assert abs(w.sum() - 1) < 1e-15
    assert np.abs(w @ c).max() < 1e-15
    assert np.abs((w[:, None, None] * c[:, :, None] * c[:, None, :]).sum(0) - np.eye(3) / 3).max() < 1e-15
    n2 = (c * c).sum(1)
    assert sorted(n2.tolist()) == [0] + [1] * 6 + [2] * 12
    assert len({tuple(v) for v in c}) == 19


def pin_neutral_slab(layers=1, nxy=4, libpath=None):
    """Sec. II C, Fig. 1 and Sec. III A 2: in a neutral liquid between plates
    the discrete solution is exactly linear with phi = phi_s half-way between
    the last solid and first fluid node, and the induced charge is the
    dielectric one, Q(0) = C_0 dV per unit area with C_0 = eps / L."""
    nf, V1, V2 = 32, 0.05, -0.05
    shape, t, ps = W.slab(nxy, nxy, nf, layers, V1, V2)
    o = _run(shape, t, ps, (1, -1), (0.05, 0.05), n_ref=(1e-3, 1e-3), tol=1e-14, omega=1.8,
             libpath=libpath)
    phi = o.fields()["phi"].reshape(shape[2], nxy, nxy)
    zc = np.arange(layers, layers + nf) - (layers - 0.5)  # distance from the wall
    exact = V1 + (V2 - V1) * zc / nf
    err = np.abs(phi[layers:layers + nf] - exact[:, None, None]).max()
    assert err < 1e-13, err
    q = o.electrode_charge()
    q0 = T.dielectric_slab_capacitance(LB, nf) * (V1 - V2) * nxy * nxy
    assert abs(q[0] - q0) < 1e-10 * abs(q0) and abs(q[1] + q0) < 1e-10 * abs(q0), (q, q0)
    return q


def pin_uniform_charge(libpath=None):
    """Uniform charge density rho between grounded plates: Poisson's equation
    (Eq. 2) with the modified Laplacian (Eq. 15) has, on the lattice, exactly
    the continuum parabola 2 pi l_B rho (z - 1/2)(L + 1/2 - z) plus the
    constant pi l_B rho / 2 (the second difference of a parabola is exact in
    the bulk; at the first fluid node the doubled wall link sees 3/4 of the
    curvature, which the constant shift compensates).  The relative shift is
    1/L^2: second-order accuracy."""
    nf, q0 = 16, 1e-3
    shape, t, ps = W.slab(2, 2, nf, 1, 0.0, 0.0)
    n0 = np.where(t == 0, q0, 0.0)[None, :]
    o = _run(shape, t, ps, (1,), (0.05,), n_init=n0, tol=1e-15, omega=1.5, max_iter=100000,
             check_every=1, libpath=libpath)
    phi = o.fields()["phi"].reshape(shape[2], 2, 2)[1:nf + 1, 0, 0]
    z = np.arange(1, nf + 1)
    c = 4 * math.pi * LB * q0
    exact = c / 2 * (z - 0.5) * (nf + 0.5 - z) + c / 8
    err = np.abs(phi - exact).max() / exact.max()
    assert err < 1e-12, err


def pin_gauss_identity(libpath=None):
    """Eq. 16 with Eq. 15: summing the modified Laplacian over all nodes
    telescopes (every link difference appears twice with opposite signs), so
    for ANY potential the electrode charges and the ionic charge satisfy
    sum_e Q_e + Q_ion = eps * sum_fluid R exactly, R the Poisson residual.
    Checked on a random, deliberately unconverged state of a coaxial cell."""
    shape, t, ps = W.coax(16, 16, 4, 2.5, 7.0, 0.07, -0.03)
    rng = np.random.default_rng(7)
    N = t.size
    n0 = np.where(t == 0, 1e-3 * (1 + 0.3 * rng.uniform(-1, 1, (2, N))), 0.0)
    o = _run(shape, t, ps, (1, -1), (0.05, 0.05), n_init=n0, tol=0.0, max_iter=3,
             libpath=libpath)
    q = o.electrode_charge()
    n = o.fields()["n"]
    qion = (n[0] - n[1])[t == 0].sum()
    R = o.residual()
    rhs = R[t == 0].sum() / (4 * math.pi * LB)
    assert abs(R).max() > 1e-6  # really unconverged
    assert abs(q.sum() + qion - rhs) < 1e-12 * (abs(q).sum() + abs(qion)), (q.sum() + qion, rhs)


def pin_diffusion_decay(axis=0, libpath=None):
    """Eqs. 9-10 with the prefactor D/A0 (reading R4): a sinusoidal neutral
    solute n = n0 + a cos(k x) in a periodic box decays in one step by exactly
    1 - 2 D (1 - cos k), the factor of the 1-D lattice diffusion equation with
    coefficient D (with the printed factor A0 in front of the sum it would be
    1 - 2 A0 D (1 - cos k))."""
    shape = [4, 4, 4]
    shape[axis] = 16
    shape = tuple(shape)
    t, ps = _periodic(shape)
    xyz = _coords(shape)
    k = 2 * math.pi * 3 / 16
    D, n0, a = 0.07, 1e-2, 1e-4
    n = n0 + a * np.cos(k * xyz[axis])
    o = _run(shape, t, ps, (0,), (D,), n_init=n[None, :], flags=FLOAT, libpath=libpath)
    o.step(1)
    n1 = o.fields()["n"][0]
    expect = n0 + a * (1 - 2 * D * (1 - math.cos(k))) * np.cos(k * xyz[axis])
    err = np.abs(n1 - expect).max() / a
    assert err < 1e-12, err


def pin_diffusion_isotropy(libpath=None):
    """Sec. II C sum rules make the link-flux Laplacian isotropic to second
    order: a long-wavelength mode along the body diagonal decays at D |k|^2
    per step up to O(k^4)."""
    L = 32
    shape = (L, L, L)
    t, ps = _periodic(shape)
    x, y, z = _coords(shape)
    k = 2 * math.pi / L
    D, n0, a = 0.05, 1e-2, 1e-5
    n = n0 + a * np.cos(k * (x + y + z))
    o = _run(shape, t, ps, (0,), (D,), n_init=n[None, :], flags=FLOAT, libpath=libpath)
    o.step(1)
    n1 = o.fields()["n"][0]
    amp = np.dot(n1 - n0, np.cos(k * (x + y + z))) / np.dot(np.cos(k * (x + y + z)), np.cos(k * (x + y + z)))
    rate = 1 - amp / a
    expect = D * 3 * k * k
    assert abs(rate - expect) < 0.05 * expect, (rate, expect)


def pin_debye_relaxation(libpath=None):
    """Eqs. 1-2 on the lattice: in a periodic box of a 1:1 electrolyte a small
    charge mode c = n+ - n- ~ cos(k x) relaxes in one step by
    1 - 2 D (1 - cos k) - D kappa^2 at linear order: along an axis the link-flux
    divergence and the Poisson stencil have the same symbol 2 (cos k - 1),
    so the migration term is exactly -D kappa^2 (kappa^2 = 8 pi l_B rho_s)."""
    shape = (16, 2, 2)
    t, ps = _periodic(shape)
    x, _, _ = _coords(shape)
    k = 2 * math.pi * 2 / 16
    D, rs, a = 0.05, 5e-3, 1e-9
    c = a * np.cos(k * x)
    n = np.stack([rs + c / 2, rs - c / 2])
    o = _run(shape, t, ps, (1, -1), (D, D), n_init=n, flags=FLOAT, tol=1e-17, max_iter=20000,
             omega=1.5, libpath=libpath)
    o.step(1)
    n1 = o.fields()["n"]
    c1 = n1[0] - n1[1]
    kappa2 = 8 * math.pi * LB * rs
    expect = (1 - 2 * D * (1 - math.cos(k)) - D * kappa2) * c
    err = np.abs(c1 - expect).max() / a
    assert err < 1e-5, err


def pin_advection_translation(libpath=None):
    """Advection (reading R5): a uniform flow u_x carries n0 + a cos(k x) in
    one step to n0 + a [(1 - 2 D (1 - cos k)) cos(k x) + u_x sin k sin(k x)],
    i.e. the central-difference translation of the profile by u_x."""
    shape = (16, 2, 2)
    t, ps = _periodic(shape)
    x, _, _ = _coords(shape)
    k = 2 * math.pi / 16
    D, n0, a, ux = 0.05, 1e-2, 1e-4, 0.02
    n = n0 + a * np.cos(k * x)
    f = np.repeat(_equilibrium(1.0, (ux, 0, 0))[:, None], t.size, axis=1)
    o = _run(shape, t, ps, (0,), (D,), n_init=n[None, :], f_init=f, flags=FLOAT, libpath=libpath)
    o.step(1)
    n1 = o.fields()["n"][0]
    expect = n0 + a * ((1 - 2 * D * (1 - math.cos(k))) * np.cos(k * x) + ux * math.sin(k) * np.sin(k * x))
    err = np.abs(n1 - expect).max() / a
    assert err < 1e-11, err


def pin_uniform_field_force(libpath=None):
    """Force on the fluid (Eq. 3: e rho_el E_app; reading R3): one species of
    valency z at uniform n in a field E along x, with no Poisson coupling
    (l_B = 0), gives the force density n sinh(z E) along x (z n E at linear
    order; the sinh is the exact link form) and nothing across, and Guo
    forcing adds exactly that momentum per step."""
    shape = (4, 4, 4)
    t, ps = _periodic(shape)
    n0, E, zv = 2e-2, 3e-2, 2
    o = _run(shape, t, ps, (zv,), (0.05,), lB=0.0, n_init=np.full((1, t.size), n0),
             Eapp=(E, 0, 0), flags=FLOAT, libpath=libpath)
    F = o.fields()["force"]
    assert np.abs(F[0] - n0 * math.sinh(zv * E)).max() < 1e-16
    assert np.abs(F[1:]).max() < 1e-18
    o.step(1)
    fld = o.fields()
    c, _ = oracle.velocities()
    mom = (fld["f"] * c[:, 0:1]).sum(0)
    assert np.abs(mom - n0 * math.sinh(zv * E)).max() < 1e-16, mom[:3]


def pin_shear_wave(libpath=None):
    """LB viscosity (Eq. 8, Sec. III A: nu = (tau - 1/2)/3): a small shear wave
    u_x = U sin(k y) decays as exp(-nu k^2 t) up to O(k^2) relative."""
    L = 32
    shape = (2, L, 2)
    t, ps = _periodic(shape)
    _, y, _ = _coords(shape)
    k = 2 * math.pi / L
    U, tau = 1e-4, 0.8
    c, w = oracle.velocities()
    f = np.empty((19, t.size))
    for r in range(t.size):
        f[:, r] = _equilibrium(1.0, (U * math.sin(k * y[r]), 0, 0))
    o = _run(shape, t, ps, (0,), (0.0,), n_init=np.zeros((1, t.size)), f_init=f, tau=tau,
             flags=FLOAT, libpath=libpath)
    nsteps = 200
    o.step(nsteps)
    ux = o.fields()["u"][0]
    amp = np.dot(ux, np.sin(k * y)) / np.dot(np.sin(k * y), np.sin(k * y))
    nu = (tau - 0.5) / 3
    expect = U * math.exp(-nu * k * k * nsteps)
    assert abs(amp - expect) < 0.01 * (U - expect), (amp, expect)


def run_slab(nf=32, debye=4.0, V=0.05, nxy=1, steps=0, D=0.05, E=(0, 0, 0), tau=1.0, layers=1,
             shift=0.0, noise=None, tol=1e-12, libpath=None):
    rs = W.salt_for_debye(debye, LB)
    shape, t, ps = W.slab(nxy, nxy, nf, layers, V + shift, -V + shift)
    o = _run(shape, t, ps, (1, -1), (D, D), n_init=noise, n_ref=(rs, rs), Eapp=E, tau=tau,
             tol=tol, omega=1.8, check_every=1, libpath=libpath)
    if steps:
        o.step(steps)
    return o, shape, t


def pin_charging(libpath=None):
    """Sec. III A 2-3 on the 32-plane slab (lambda_D = 4, dV = 0.1):
    Q(0) = C_0 dV; Q(t) relaxes exponentially with the slowest charging
    time of the linearised Poisson-Nernst-Planck cell within 3%; the final
    charge gives the Debye-Hueckel capacitance (finite-gap form of Eq. 18)
    within 1.5% (second-order lattice error at lambda_D = 4 grid spacings)."""
    o, shape, t = run_slab(steps=20000, libpath=libpath)
    q = o.qhist()[:, 0]
    q0 = T.dielectric_slab_capacitance(LB, 32) * 0.1
    assert abs(q[0] / q0 - 1) < 1e-9, (q[0], q0)
    d = q[-1] - q
    tt = np.arange(q.size)
    m = (d < 0.2 * d[0]) & (d > 1e-4 * d[0])
    slope = np.polyfit(tt[m], np.log(d[m]), 1)[0]
    tau = -1 / slope
    tau_th = 1 / T.charging_rate_slab(4.0, 32.0, 0.05)
    assert abs(tau / tau_th - 1) < 0.03, (tau, tau_th)
    C = q[-1] / 0.1
    C_th = T.dh_slab_capacitance(LB, 4.0, 32.0)
    assert abs(C / C_th - 1) < 0.015, (C, C_th)
    return o


def pin_boltzmann(o):
    """Sec. II A: at equilibrium every ionic flux vanishes and
    n_k = n_k^0 exp(-z_k phi), i.e. ln n_k + z_k phi is uniform."""
    fld = o.fields()
    t = o._keep[0]
    for k, zk in enumerate((1, -1)):
        g = np.log(fld["n"][k][t == 0]) + zk * fld["phi"][t == 0]
        assert np.ptp(g) < 1e-7, np.ptp(g)


def pin_dh_profiles(o):
    """Eq. 17 and the linearised Boltzmann profiles rho_+- = rho_s (1 -+ phi)
    (Fig. 3) at steady state, within the O(dx^2) lattice error."""
    fld = o.fields()
    t = o._keep[0]
    phi = fld["phi"][t == 0]
    z = np.arange(phi.size) + 0.5 - phi.size / 2
    th = T.dh_slab_potential(z, phi.size, 0.25, 0.05, -0.05)
    assert np.abs(phi - th).max() < 0.01 * 0.1, np.abs(phi - th).max()


def pin_capacitance_order(libpath=None):
    """Fig. 4b: the error of the steady-state capacitance with respect to
    Debye-Hueckel falls as (dx/lambda_D)^2.  Two resolutions of the same
    physical cell (L = 8 lambda_D): the error ratio is 4 within 10%."""
    errs = []
    for debye in (2.0, 4.0):
        nf = int(8 * debye)
        o, shape, t = run_slab(nf=nf, debye=debye, V=0.005, D=0.2, steps=int(60 * debye * nf / 2 / 0.2 / 4),
                               libpath=libpath)
        q = o.qhist()[:, 0]
        C = q[-1] / 0.01
        C_th = T.dh_slab_capacitance(LB, debye, nf)
        errs.append(abs(C / C_th - 1))
    ratio = errs[0] / errs[1]
    assert 3.6 < ratio < 4.4, (errs, ratio)


def pin_eo_slab(libpath=None):
    """Eq. 20: steady electro-osmotic velocity along an applied field between
    charged plates (32 fluid planes, lambda_D = 4, E_x = 1e-3), within 3% of
    the peak velocity."""
    o, shape, t = run_slab(steps=14000, E=(1e-3, 0, 0), libpath=libpath)
    fld = o.fields()
    ux = fld["u"][0][t == 0]
    z = np.arange(ux.size) + 0.5 - ux.size / 2
    th = T.eo_slab_velocity(z, ux.size, 0.25, 0.05, -0.05, 1e-3, LB, 1.0)
    err = np.abs(ux - th).max() / np.abs(th).max()
    assert err < 0.03, err
    assert np.abs(fld["u"][1:]).max() < 1e-6 * np.abs(th).max()


def pin_coax_neutral(libpath=None):
    """Eq. 21 and C_0^cyl = 2 pi eps / ln(R2/R1) (Sec. III B 1-2): the t = 0
    potential of the staircase coaxial capacitor follows the logarithmic
    profile and its charge the dielectric capacitance, within the few-percent
    error of the voxelised cylinders."""
    R1, R2 = 4.0, 25.0
    shape, t, ps = W.coax(54, 54, 2, R1, R2, 0.05, -0.05)
    o = _run(shape, t, ps, (1, -1), (0.05, 0.05), n_ref=(1e-3, 1e-3), tol=1e-12, omega=1.9,
             libpath=libpath)
    phi = o.fields()["phi"]
    r = W.radial_distance(shape)
    sel = (t == 0) & (r > R1 + 1.5) & (r < R2 - 1.5)
    th = T.coax_neutral_potential(r[sel], R1, R2, 0.05, -0.05)
    err = np.abs(phi[sel] - th).max() / 0.1
    assert err < 0.02, err
    q = o.electrode_charge()
    C = q[0] / 0.1 / shape[2]
    C_th = T.coax_capacitance_neutral(LB, R1, R2)
    assert abs(C / C_th - 1) < 0.05, (C, C_th)
    assert abs(q[0] + q[1]) < 1e-9 * abs(q[0])


def pin_equilibrium_moments(libpath=None):
    """Eq. 8 with tau = 1 replaces the populations by the equilibrium, and in
    a uniform periodic box streaming leaves them in place.  Whatever the
    equilibrium's form, the Navier-Stokes limit needs its moments to be
    rho, rho u and rho (c_s^2 delta + u u); checked for a random, far from
    equilibrium start with |u| ~ 0.1."""
    shape = (2, 2, 2)
    t, ps = _periodic(shape)
    rng = np.random.default_rng(3)
    f0 = rng.uniform(0.02, 0.1, 19)
    f = np.repeat(f0[:, None], t.size, axis=1)
    o = _run(shape, t, ps, (0,), (0.0,), n_init=np.zeros((1, t.size)), f_init=f, tau=1.0,
             flags=FLOAT, libpath=libpath)
    c, _ = oracle.velocities()
    rho = f0.sum()
    u = (f0 @ c) / rho
    o.step(1)
    f1 = o.fields()["f"][:, 0]
    assert abs(f1.sum() - rho) < 1e-15
    assert np.abs(f1 @ c - rho * u).max() < 1e-15
    second = (f1[:, None, None] * c[:, :, None] * c[:, None, :]).sum(0)
    assert np.abs(second - rho * (np.eye(3) / 3 + np.outer(u, u))).max() < 1e-15


def pin_advection_shear(libpath=None):
    """Advection (reading R5) in a shear flow u_x = U sin(q y) of a solute
    n0 + a cos(k x): summing the central link fluxes over D3Q19 gives exactly
    n(1) = n0 + a (1 - 2 D (1 - cos k)) cos(k x)
                + a U sin k (2 + cos q)/3 sin(k x) sin(q y),
    the lattice form of -u . grad n (the factor (2 + cos q)/3 -> 1 as q -> 0
    comes from the diagonal links reading u at the neighbour)."""
    shape = (16, 8, 2)
    t, ps = _periodic(shape)
    x, y, _ = _coords(shape)
    k, q = 2 * math.pi / 16, 2 * math.pi / 8
    D, n0, a, U = 0.05, 1e-2, 1e-4, 0.02
    n = n0 + a * np.cos(k * x)
    f = np.stack([_equilibrium(1.0, (U * math.sin(q * yy), 0, 0)) for yy in y], axis=1)
    o = _run(shape, t, ps, (0,), (D,), n_init=n[None, :], f_init=f, flags=FLOAT, libpath=libpath)
    o.step(1)
    n1 = o.fields()["n"][0]
    expect = (n0 + a * (1 - 2 * D * (1 - math.cos(k))) * np.cos(k * x)
              + a * U * math.sin(k) * (2 + math.cos(q)) / 3 * np.sin(k * x) * np.sin(q * y))
    err = np.abs(n1 - expect).max() / (a * U)
    assert err < 1e-9, err


# ---- first-order scheme, electrode potentials, non-linear steady state ------

NAIVE = oracle.FLAG_NAIVE_DIRICHLET


def pin_naive_neutral_slab(layers=1, nxy=2, libpath=None):
    """The first-order scheme the paper contrasts with (Sec. II C, Fig. 1):
    phi_s held on the solid nodes and the plain Laplacian of Eq. 12 on every
    link.  In a neutral liquid the discrete solution is then exactly linear
    through the last solid node of each electrode, nf + 1 spacings apart, and
    Gauss's law with the same Laplacian gives Q(0) = eps dV / (nf + 1) per
    unit area: the dielectric capacitance with a gap one spacing too wide, a
    first-order error."""
    nf, V1, V2 = 32, 0.05, -0.05
    shape, t, ps = W.slab(nxy, nxy, nf, layers, V1, V2)
    o = _run(shape, t, ps, (1, -1), (0.05, 0.05), n_ref=(1e-3, 1e-3), tol=1e-14, omega=1.8,
             flags=NAIVE, libpath=libpath)
    phi = o.fields()["phi"].reshape(shape[2], nxy, nxy)
    zc = np.arange(layers, layers + nf) - (layers - 1)  # distance from the last solid node
    exact = V1 + (V2 - V1) * zc / (nf + 1)
    err = np.abs(phi[layers:layers + nf] - exact[:, None, None]).max()
    assert err < 1e-13, err
    q = o.electrode_charge()
    q0 = T.permittivity(LB) / (nf + 1) * (V1 - V2) * nxy * nxy
    assert abs(q[0] - q0) < 1e-10 * abs(q0) and abs(q[1] + q0) < 1e-10 * abs(q0), (q, q0)
    return q


def pin_naive_gauss_identity(libpath=None):
    """Gauss's law telescopes with the plain Laplacian too: with factor 1 on
    both ends of every solid-fluid link, sum_e Q_e + Q_ion = eps sum_fluid R
    for any potential."""
    shape, t, ps = W.coax(16, 16, 4, 2.5, 7.0, 0.07, -0.03)
    rng = np.random.default_rng(8)
    N = t.size
    n0 = np.where(t == 0, 1e-3 * (1 + 0.3 * rng.uniform(-1, 1, (2, N))), 0.0)
    o = _run(shape, t, ps, (1, -1), (0.05, 0.05), n_init=n0, tol=0.0, max_iter=3, flags=NAIVE,
             libpath=libpath)
    q = o.electrode_charge()
    n = o.fields()["n"]
    qion = (n[0] - n[1])[t == 0].sum()
    R = o.residual()
    rhs = R[t == 0].sum() / (4 * math.pi * LB)
    assert abs(R).max() > 1e-6
    assert abs(q.sum() + qion - rhs) < 1e-12 * (abs(q).sum() + abs(qion)), (q.sum() + qion, rhs)


def pin_set_potential(libpath=None):
    """New electrode potentials in a neutral slab: after the call the
    potential is the new linear profile with phi_s at mid-link and the charge
    recorded for the current step is the new dielectric charge (Sec. III A 2);
    the history keeps its length."""
    nf, nxy = 16, 2
    shape, t, ps = W.slab(nxy, nxy, nf, 1, 0.05, -0.05)
    # no ions: the liquid stays neutral through the steps taken first
    o = _run(shape, t, ps, (1, -1), (0.05, 0.05), n_ref=(0.0, 0.0), tol=1e-14, omega=1.8,
             check_every=1, libpath=libpath)
    o.step(3)
    len0 = o.qhist().shape[0]
    V1, V2 = 0.2, -0.1
    o.set_electrode_potential(np.where(t == 1, V1, np.where(t == 2, V2, 0.0)))
    phi = o.fields()["phi"].reshape(shape[2], nxy, nxy)[1:nf + 1]
    exact = V1 + (V2 - V1) * (np.arange(1, nf + 1) - 0.5) / nf
    assert np.abs(phi - exact[:, None, None]).max() < 1e-13
    qh = o.qhist()
    q0 = T.dielectric_slab_capacitance(LB, nf) * (V1 - V2) * nxy * nxy
    assert qh.shape[0] == len0
    assert abs(qh[-1, 0] - q0) < 1e-10 * q0 and abs(qh[-1, 1] + q0) < 1e-10 * q0
    assert np.allclose(qh[:-1, 0], qh[0, 0], rtol=1e-9)  # earlier entries untouched


def pin_nonlinear_steady_state(z=(1, -1), D=(0.2, 0.2), V=0.5, debye=4.0, flags=0, steps=8000,
                               libpath=None):
    """Exact steady state beyond the linear regime (Sec. II C: the voltage need
    not be small): on a 32-plane slab the LBE relaxes to the Boltzmann
    distribution in the discrete non-linear Poisson-Boltzmann potential,
    computed independently by Newton's method (theory.nonlinear_pb_slab);
    the potential, the concentrations and the electrode charge agree.  Works
    for any valences (salt of valences z with bulk concentrations in the
    ratio that makes it neutral), unequal D and either wall scheme."""
    nf = 32
    zz = np.asarray(z, float)
    # neutral salt: concentrations ~ 1/|z_k|, scaled to the requested Debye length
    ratio = 1.0 / np.abs(zz)
    rs = ratio / (4 * math.pi * LB * debye * debye * float((zz * zz * ratio).sum()))
    shape, t, ps = W.slab(1, 1, nf, 1, V, -V)
    o = _run(shape, t, ps, tuple(z), tuple(D), n_ref=tuple(rs), tol=1e-13, omega=1.8,
             check_every=1, max_iter=100000, flags=flags, libpath=libpath)
    o.step(steps)
    f = o.fields()
    phi = f["phi"][1:nf + 1]
    n = f["n"][:, 1:nf + 1]
    wall = 1.0 if flags & NAIVE else 2.0
    phi_th, n_th = T.nonlinear_pb_slab(nf, z, rs * nf, LB, V, -V, wall=wall)
    assert np.abs(phi - phi_th).max() < 1e-8 * V, np.abs(phi - phi_th).max()
    assert np.abs(n / n_th - 1).max() < 1e-7, np.abs(n / n_th - 1).max()
    eps = T.permittivity(LB)
    q1 = -eps * wall * (phi_th[0] - V)  # Eq. 16 on the column, c_z = +1 links weigh 1/6
    q = o.electrode_charge()
    assert abs(q[0] / q1 - 1) < 1e-7 and abs(q[1] / q[0] + 1) < 1e-6, (q, q1)
    return o


def pin_sor_rate(libpath=None):
    """The SOR iteration itself, not only its fixed point (Sec. II C, Eq. 13
    with Eq. 15).  On a 1 x 1 x 32 slab every in-plane link of the D3Q19 set
    joins a node to itself and is left out, the five links along each z
    direction sum to the weight 1/6, and the four colour classes reduce to
    two alternating planes: the sweep is SOR on the tridiagonal operator with
    diagonal 2 (3 next to a wall, the doubled wall link) and off-diagonal 1,
    in red-black order, a consistently ordered matrix.  Young's theorem then
    gives the asymptotic contraction per sweep from the Jacobi spectral
    radius mu (computed here as an eigenvalue): ((omega mu + sqrt(omega^2
    mu^2 - 4 (omega - 1))) / 2)^2 below the optimal omega.  The residual's
    decay between sweeps 100 and 160 after a change of the electrode
    potentials (one that excites the slowest mode) must show it, for omega
    1.8 (the configured value) and 1.5."""
    nf = 32
    shape, t, ps = W.slab(1, 1, nf, 1, 0.05, -0.05)
    rs = W.salt_for_debye(4.0, LB)
    n0 = W.noisy_concentrations(t, [rs, rs], 1e-3, seed=1)
    diag = np.full(nf, 2.0)
    diag[0] = diag[-1] = 3.0
    off = np.diag(np.ones(nf - 1), 1) + np.diag(np.ones(nf - 1), -1)
    mu = float(np.abs(np.linalg.eigvals(off / diag[:, None])).max())
    new_ps = np.where(t == 1, 0.1, 0.0)

    def resid_after(sweeps, omega):
        o = _run(shape, t, ps, (1, -1), (0.05, 0.05), n_init=n0, n_ref=(rs, rs), omega=omega,
                 tol=1e-14, max_iter=100000, check_every=1, libpath=libpath)
        o.set_solver(0.0, sweeps)
        o.set_electrode_potential(new_ps)
        return float(np.abs(o.residual()).max())

    rates = {}
    for omega in (1.8, 1.5):
        assert omega < 2.0 / (1.0 + math.sqrt(1.0 - mu * mu))  # below the optimum
        young = ((omega * mu + math.sqrt(omega ** 2 * mu ** 2 - 4.0 * (omega - 1.0))) / 2.0) ** 2
        rate = (resid_after(160, omega) / resid_after(100, omega)) ** (1.0 / 60.0)
        assert abs(rate / young - 1.0) < 1e-4, (omega, rate, young)
        rates[omega] = rate
    return rates
