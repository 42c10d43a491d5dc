"""Seeded parity cases shared by the GPU tests, the smoke check and the bench:
the same inputs go to the GPU library and to the oracle."""
from __future__ import annotations

import numpy as np

import workloads as W

LB = 0.4


def random_geometry(shape, nelec=3, seed=5, fill=0.2):
    """Random solid blobs (cubes of side 1-3) assigned to `nelec` electrodes at
    different potentials; the lattice need not be a multiple of any tile."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    t = np.zeros((nz, ny, nx), np.uint8)
    while (t != 0).mean() < fill:
        s = rng.integers(1, 4, 3)
        o = rng.integers(0, [nz, ny, nx])
        e = rng.integers(1, nelec + 1)
        zz = (o[0] + np.arange(s[0])) % nz
        yy = (o[1] + np.arange(s[1])) % ny
        xx = (o[2] + np.arange(s[2])) % nx
        t[np.ix_(zz, yy, xx)] = e
    volts = np.linspace(-0.08, 0.1, nelec)
    ps = np.where(t > 0, volts[np.maximum(t.astype(int) - 1, 0)], 0.0)
    return t.reshape(-1), ps.reshape(-1)


def case(name):
    """Return (kwargs for make_params without shape, shape, type, phi_s, n_init, n_ref, nsteps,
    fixed_sweeps)."""
    if name == "slab_4x4x34":
        rs = W.salt_for_debye(4.0, LB)
        shape, t, ps = W.slab(4, 4, 32, 1, 0.05, -0.05)
        n0 = W.noisy_concentrations(t, [rs, rs], 1e-6, seed=1)
        kw = dict(z=(1, -1), D=(0.05, 0.05), lB=LB, tau=1.0, Eapp=(1e-3, 0, 0), omega=1.8)
        return kw, shape, t, ps, n0, (rs, rs), 40, 80
    if name == "slab_1x1x34":
        rs = W.salt_for_debye(4.0, LB)
        shape, t, ps = W.slab(1, 1, 32, 1, 0.05, -0.05)
        n0 = W.noisy_concentrations(t, [rs, rs], 1e-3, seed=1)
        kw = dict(z=(1, -1), D=(0.05, 0.05), lB=LB, tau=1.0, Eapp=(0, 2e-3, 0), omega=1.8)
        return kw, shape, t, ps, n0, (rs, rs), 30, 80
    if name == "coax_16x16x4":
        rs = W.salt_for_debye(3.0, LB)
        shape, t, ps = W.coax(16, 16, 4, 2.5, 7.0, 0.05, -0.05)
        n0 = W.noisy_concentrations(t, [rs, rs], 1e-2, seed=3)
        kw = dict(z=(1, -1), D=(0.05, 0.08), lB=LB, tau=0.8, Eapp=(0, 0, 1e-3), omega=1.7)
        return kw, shape, t, ps, n0, (rs, rs), 25, 40
    if name == "random_6x10x14_k3":
        shape = (6, 10, 14)
        t, ps = random_geometry(shape, 3, seed=5)
        rs = np.array([2e-3, 3e-3, 0.5e-3])
        n0 = W.noisy_concentrations(t, rs, 5e-2, seed=6)
        kw = dict(z=(1, -1, 2), D=(0.05, 0.03, 0.02), lB=LB, tau=0.9, Eapp=(2e-3, -1e-3, 5e-4),
                  omega=1.6, flags=1)
        return kw, shape, t, ps, n0, tuple(rs), 15, 30
    if name == "random_8x6x10_k4":
        shape = (8, 6, 10)
        t, ps = random_geometry(shape, 2, seed=9, fill=0.15)
        rs = np.array([1e-3, 1e-3, 0.5e-3, 0.5e-3])
        n0 = W.noisy_concentrations(t, rs, 1e-1, seed=10)
        kw = dict(z=(1, -1, 2, -2), D=(0.05, 0.05, 0.02, 0.04), lB=LB, tau=1.2,
                  Eapp=(0, 0, 0), omega=1.5, flags=1)
        return kw, shape, t, ps, n0, tuple(rs), 10, 30
    if name == "slab_2x2x18_k1":
        shape, t, ps = W.slab(2, 2, 16, 2, 0.03, 0.01)
        n0 = W.noisy_concentrations(t, [1e-3], 1e-1, seed=12)
        kw = dict(z=(1,), D=(0.1,), lB=LB, tau=0.7, Eapp=(0, 0, 0), omega=1.8)
        return kw, shape, t, ps, n0, (1e-3,), 20, 60
    raise KeyError(name)


PARITY_CASES = ["slab_4x4x34", "slab_1x1x34", "coax_16x16x4", "random_6x10x14_k3",
                "random_8x6x10_k4", "slab_2x2x18_k1"]


def _rest(node_type, rho0=1.0):
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    return np.where(np.asarray(node_type).reshape(-1)[None, :] == 0, w[:, None] * rho0, 0.0)


def adjoint_case(kind):
    """Small cases of the reverse-mode tests: (shape, type, phi_s, n_init (K, N),
    f_init (19, N), parameters, flags); "k2_field": two electrodes, 1:1 salt
    and an applied field; "k3_naive": three electrodes, a divalent species and
    the first-order wall scheme."""
    if kind == "k2_field":
        shape = (6, 6, 12)
        t, ps = random_geometry(shape, 2, seed=7, fill=0.15)
        n0 = W.noisy_concentrations(t, (3e-3, 3e-3), 5e-2, seed=2)
        kw = dict(z=(1, -1), D=(0.05, 0.08), lB=0.4, tau=0.9, Eapp=(2e-3, 0.0, 1e-3))
        flags = 0
    else:  # multivalent, three electrodes, first-order wall scheme
        shape = (4, 6, 10)
        t, ps = random_geometry(shape, 3, seed=11, fill=0.2)
        n0 = W.noisy_concentrations(t, (2e-3, 3e-3, 0.5e-3), 5e-2, seed=4)
        kw = dict(z=(1, -1, 2), D=(0.05, 0.03, 0.02), lB=0.4, tau=1.1, Eapp=(0.0, -1e-3, 5e-4))
        flags = 4  # first-order wall scheme (the same bit in the oracle and the library)
    rng = np.random.default_rng(3)
    f0 = _rest(t) * (1.0 + 1e-3 * rng.uniform(-1, 1, (19, t.size)))
    return shape, t, ps, n0, f0, kw, flags
