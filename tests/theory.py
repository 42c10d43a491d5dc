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
