"""Closed forms from arXiv:1907.04732 used to pin the oracle and the GPU path.

Lattice units: Delta x = Delta t = k_B T = e = 1, phi = beta e psi,
epsilon = 1 / (4 pi l_B), c_s^2 = 1/3, kinematic viscosity nu = (tau - 1/2)/3.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import optimize, special


def permittivity(lB):
    """epsilon_0 epsilon_r in lattice units: l_B = beta e^2 / (4 pi eps)."""
    return 1.0 / (4.0 * math.pi * lB)


def debye_length(lB, rho, z):
    """Eq. 6: lambda_D = (4 pi l_B sum_k rho_k z_k^2)^(-1/2)."""
    return (4.0 * math.pi * lB * sum(r * q * q for r, q in zip(rho, z))) ** -0.5


def viscosity(tau, rho0=1.0):
    """Dynamic viscosity of BGK LB, eta = rho nu with nu = (tau - 1/2)/3
    (Sec. III A: tau = 1 gives nu = 1/6)."""
    return rho0 * (tau - 0.5) / 3.0


# ---- parallel plates (Sec. III A) -------------------------------------------

def dh_slab_potential(z, L, kappa, psi1, psi2):
    """Eq. 17: Debye-Hueckel potential between plates at z = -L/2 (psi1) and
    z = +L/2 (psi2)."""
    z = np.asarray(z, dtype=float)
    return 0.5 * (psi1 + psi2) + 0.5 * (psi2 - psi1) * np.sinh(kappa * z) / math.sinh(kappa * L / 2)


def dh_slab_capacitance(lB, debye, L=None):
    """Eq. 18: C_DH = eps / (2 lambda_D) per unit area.  With L given, the
    finite-gap value that follows from Eq. 17, (eps kappa / 2) coth(kappa L / 2)."""
    eps = permittivity(lB)
    kappa = 1.0 / debye
    if L is None:
        return eps * kappa / 2.0
    return eps * kappa / 2.0 / math.tanh(kappa * L / 2.0)


def dielectric_slab_capacitance(lB, L):
    """C_0 = eps / L, the capacitance of the neutral liquid (Sec. III A 2)."""
    return permittivity(lB) / L


def charging_rate_slab(debye, L, D):
    """Slowest relaxation rate of the charge of a blocking parallel-plate cell
    under a small step voltage (Sec. III A 3).  Linearising Eqs. 1-2 for the
    charge density c = n+ - n- of a symmetric electrolyte gives
    dc/dt = D (c'' - kappa^2 c) with zero ionic flux at the walls and the
    potential fixed there.  Its odd eigenmode c ~ sinh(q z) decays at
    lambda = D (kappa^2 - q^2), with q solving
        kappa^2 - q^2 = (2 kappa^2 / (q L)) tanh(q L / 2),
    whose large-L limit is tau = L lambda_D / (2 D) (the paper's time unit).
    Returns lambda (1/time)."""
    kappa = 1.0 / debye
    if kappa * L > math.sqrt(12.0) + 1e-9:
        # q = 0 is a spurious root; g > 0 just above it and g(kappa) < 0
        g = lambda q: kappa ** 2 - q ** 2 - 2 * kappa ** 2 / (q * L) * math.tanh(q * L / 2)
        qs = kappa * np.logspace(-6, 0, 2001)[:-1]
        vals = np.array([g(q) for q in qs])
        i = int(np.nonzero((vals[:-1] > 0) & (vals[1:] <= 0))[0][-1])
        q = optimize.brentq(g, qs[i], qs[i + 1])
        return D * (kappa ** 2 - q ** 2)
    # otherwise the mode is oscillatory: q = i p
    g = lambda p: kappa ** 2 + p ** 2 - 2 * kappa ** 2 / (p * L) * math.tan(p * L / 2)
    p = optimize.brentq(g, 1e-9, math.pi / L * (1 - 1e-12))
    return D * (kappa ** 2 + p ** 2)


def eo_slab_velocity(z, L, kappa, psi1, psi2, E, lB, tau, rho0=1.0):
    """Eq. 20: electro-osmotic velocity along the applied field between the
    plates (no slip at z = +-L/2)."""
    eps = permittivity(lB)
    eta = viscosity(tau, rho0)
    z = np.asarray(z, dtype=float)
    return eps * E * (psi2 - psi1) / eta * 0.5 * (np.sinh(kappa * z) / math.sinh(kappa * L / 2) - 2 * z / L)


# ---- coaxial cylinders (Sec. III B) -----------------------------------------

def coax_neutral_potential(r, R1, R2, psi1, psi2):
    """Eq. 21: potential of the neutral coaxial capacitor."""
    r = np.asarray(r, dtype=float)
    return psi1 + (psi2 - psi1) * np.log(r / R1) / math.log(R2 / R1)


def coax_f(r, R1, R2, kappa):
    """Eq. 23: the Debye-Hueckel shape function f(r; R1, R2, kappa)."""
    r = np.asarray(r, dtype=float)
    I0, I1, K0, K1 = special.i0, special.i1, special.k0, special.k1
    a = R2 * K1(kappa * R2) - R1 * K1(kappa * R1)
    b = R2 * I1(kappa * R2) - R1 * I1(kappa * R1)
    num = a * (I0(kappa * r) - I0(kappa * R1)) + b * (K0(kappa * r) - K0(kappa * R1))
    den = a * (I0(kappa * R2) - I0(kappa * R1)) + b * (K0(kappa * R2) - K0(kappa * R1))
    return num / den


def coax_f_prime(r, R1, R2, kappa):
    """d f / d r of Eq. 23 (I0' = I1, K0' = -K1)."""
    I0, I1, K0, K1 = special.i0, special.i1, special.k0, special.k1
    a = R2 * K1(kappa * R2) - R1 * K1(kappa * R1)
    b = R2 * I1(kappa * R2) - R1 * I1(kappa * R1)
    den = a * (I0(kappa * R2) - I0(kappa * R1)) + b * (K0(kappa * R2) - K0(kappa * R1))
    return kappa * (a * I1(kappa * r) - b * K1(kappa * r)) / den


def coax_dh_potential(r, R1, R2, kappa, psi1, psi2):
    """Eq. 22."""
    return psi1 + (psi2 - psi1) * coax_f(r, R1, R2, kappa)


def coax_capacitance_neutral(lB, R1, R2):
    """C_0^cyl = 2 pi eps / ln(R2/R1) per unit length (Sec. III B 2)."""
    return 2 * math.pi * permittivity(lB) / math.log(R2 / R1)


def coax_capacitance_dh(lB, R1, R2, kappa):
    """Eq. 24: C_DH^cyl = 2 pi eps R1 f'(R1) per unit length."""
    return 2 * math.pi * permittivity(lB) * R1 * float(coax_f_prime(R1, R1, R2, kappa))


def coax_eo_velocity(r, R1, R2, kappa, psi1, psi2, E, lB, tau, rho0=1.0):
    """Eq. 25: axial electro-osmotic velocity in the coaxial capacitor."""
    eps = permittivity(lB)
    eta = viscosity(tau, rho0)
    r = np.asarray(r, dtype=float)
    return eps * E * (psi2 - psi1) / eta * (coax_f(r, R1, R2, kappa) - np.log(r / R1) / math.log(R2 / R1))


def nonlinear_pb_slab(nf, z, amounts, lB, phi1, phi2, wall=2.0, tol=1e-15, max_newton=100):
    """Steady state of the LBE between parallel plates, reduced to z.

    With no flow every link flux of Eq. 10 vanishes when n'/n = exp(-z (phi' -
    phi)), i.e. n_k = A_k exp(-z_k phi) (Boltzmann), with A_k set by the
    conserved amount per lattice column `amounts[k]`.  For a laterally uniform
    field the D3Q19 Laplacian of Eq. 12 / 15 reduces to a second difference
    along z (the five links with c_z = +1 carry total weight 1/6, so
    6 sum_i w_i s_i (phi' - phi) = s_+ (phi(z+1) - phi) + s_- (phi(z-1) - phi));
    a link into an electrode plane has s = `wall` (2 for Eq. 15, 1 for the
    first-order scheme with phi_s on the solid node).  phi on the nf fluid
    planes solves the discrete non-linear Poisson-Boltzmann equation
      L phi + 4 pi l_B sum_k z_k A_k(phi) exp(-z_k phi) = 0,
    by Newton's method with the exact Jacobian (A_k depends on phi through the
    normalisation).  Returns phi (nf,), n (K, nf)."""
    z = np.asarray(z, dtype=float)
    amounts = np.asarray(amounts, dtype=float)
    c = 4.0 * math.pi * lB
    # linear operator with the wall terms moved to b: L phi = M phi + b
    M = np.zeros((nf, nf))
    b = np.zeros(nf)
    for i in range(nf):
        M[i, i] = -2.0
        if i > 0:
            M[i, i - 1] = 1.0
        else:
            M[i, i] += 1.0 - wall
            b[i] += wall * phi1
        if i < nf - 1:
            M[i, i + 1] = 1.0
        else:
            M[i, i] += 1.0 - wall
            b[i] += wall * phi2
    phi = phi1 + (phi2 - phi1) * (np.arange(nf) + 0.5) / nf
    for _ in range(max_newton):
        E = np.exp(-np.outer(z, phi))            # (K, nf)
        S = E.sum(axis=1)
        A = amounts / S
        n = A[:, None] * E
        F = M @ phi + b + c * (z[:, None] * n).sum(axis=0)
        J = M.copy()
        for k in range(z.size):
            # d n_k(i) / d phi_j = -z_k n_k(i) delta_ij + n_k(i) z_k E_k(j) / S_k
            J += c * z[k] * (np.diag(-z[k] * n[k]) + np.outer(n[k], z[k] * E[k] / S[k]))
        step = np.linalg.solve(J, -F)
        phi = phi + step
        if np.abs(step).max() < tol:
            break
    E = np.exp(-np.outer(z, phi))
    n = (amounts / E.sum(axis=1))[:, None] * E
    return phi, n
