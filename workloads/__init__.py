"""Seeded synthetic inputs shared by the GPU library's tests/bench and the oracle.

This module only builds inputs: node-type maps of the paper's geometries
(parallel plates, coaxial cylinders, a packing of spheres), electrode
potentials, seeded concentration noise, and the parameter sets of the
benchmark workloads.  It holds none of the method's arithmetic.

Geometries follow arXiv:1907.04732, Sec. III: electrodes are solid nodes of a
periodic box, type 0 = fluid, type e >= 1 = electrode e held at phi_s.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def salt_for_debye(debye, lB):
    """1:1 salt concentration rho_s giving Debye length `debye` at Bjerrum
    length `lB` (Sec. III: lambda_D = (8 pi l_B rho_s)^(-1/2))."""
    return 1.0 / (8.0 * math.pi * lB * debye * debye)


def slab(nx, ny, nfluid, layers=1, phi1=0.05, phi2=-0.05):
    """Parallel plates normal to z (Sec. III A): `layers` solid planes of
    electrode 1 at the bottom, `nfluid` fluid planes, `layers` planes of
    electrode 2 at the top.  Returns (shape, type, phi_s) with arrays in site
    order x + nx*(y + ny*z)."""
    nz = nfluid + 2 * layers
    t = np.zeros((nz, ny, nx), dtype=np.uint8)
    ps = np.zeros((nz, ny, nx))
    t[:layers] = 1
    ps[:layers] = phi1
    t[layers + nfluid:] = 2
    ps[layers + nfluid:] = phi2
    return (nx, ny, nz), t.reshape(-1), ps.reshape(-1)


def coax(nx, ny, nz, R1, R2, phi1=0.05, phi2=-0.05):
    """Coaxial cylinders along z (Sec. III B, Fig. 7), voxelised as a staircase:
    axis at ((nx-1)/2, (ny-1)/2); a node is electrode 1 if its distance to the
    axis is < R1 and electrode 2 if it is > R2."""
    cx, cy = (nx - 1) / 2.0, (ny - 1) / 2.0
    y, x = np.mgrid[0:ny, 0:nx]
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    t2 = np.zeros((ny, nx), dtype=np.uint8)
    ps2 = np.zeros((ny, nx))
    t2[r < R1] = 1
    ps2[r < R1] = phi1
    t2[r > R2] = 2
    ps2[r > R2] = phi2
    t = np.broadcast_to(t2, (nz, ny, nx)).copy()
    ps = np.broadcast_to(ps2, (nz, ny, nx)).copy()
    return (nx, ny, nz), t.reshape(-1), ps.reshape(-1)


def radial_distance(shape):
    """Distance of every site to the coaxial axis used by `coax`."""
    nx, ny, nz = shape
    cx, cy = (nx - 1) / 2.0, (ny - 1) / 2.0
    y, x = np.mgrid[0:ny, 0:nx]
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    return np.broadcast_to(r, (nz, ny, nx)).reshape(-1).copy()


def sphere_packing(n=192, zlo=16, zhi=159, counter=(176, 191), rmin=6.0, rmax=10.0,
                   fraction=0.3, phi_spheres=0.05, phi_counter=-0.05, seed=5, max_tries=200000):
    """Porous electrode: random sequential addition of non-overlapping spheres
    (radius uniform in [rmin, rmax], periodic in x and y, at least one lattice
    spacing apart) inside the slab zlo <= z <= zhi until the solid fraction of
    that slab reaches `fraction`; all spheres are electrode 1.  Planes
    counter[0]..counter[1] are electrode 2."""
    rng = np.random.default_rng(seed)
    t = np.zeros((n, n, n), dtype=np.uint8)
    target = fraction * n * n * (zhi - zlo + 1)
    centres = np.zeros((0, 3))
    radii = np.zeros(0)
    solid = 0
    tries = 0
    while solid < target and tries < max_tries:
        tries += 1
        rad = rng.uniform(rmin, rmax)
        c = np.array([rng.uniform(0, n), rng.uniform(0, n),
                      rng.uniform(zlo + rad, zhi + 1 - rad)])
        if len(radii):
            d = centres - c
            d[:, :2] -= n * np.round(d[:, :2] / n)
            if np.any((d * d).sum(1) < (radii + rad + 1.0) ** 2):
                continue
        centres = np.vstack([centres, c])
        radii = np.append(radii, rad)
        lo = np.floor(c - rad).astype(int)
        hi = np.ceil(c + rad).astype(int) + 1
        zz, yy, xx = np.mgrid[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        inside = (xx - c[0]) ** 2 + (yy - c[1]) ** 2 + (zz - c[2]) ** 2 < rad * rad
        zi, yi, xi = zz[inside], yy[inside] % n, xx[inside] % n
        fresh = t[zi, yi, xi] == 0
        t[zi[fresh], yi[fresh], xi[fresh]] = 1
        solid += int(fresh.sum())
    t[counter[0]:counter[1] + 1] = 2
    ps = np.where(t == 1, phi_spheres, np.where(t == 2, phi_counter, 0.0))
    return (n, n, n), t.reshape(-1), ps.reshape(-1)


def porous_electrode(noise=True, n=192):
    """Porous electrode: 192^3 lattice, seeded packing of spheres (radius
    6-10, solid fraction 0.3 of z in [16, 159]) at +0.05 facing a flat
    counter-electrode (z in [176, 191]) at -0.05, 1:1 salt with Debye length 4,
    tau = 1, D = 0.05."""
    lB, debye = 0.4, 4.0
    rs = salt_for_debye(debye, lB)
    scale = n / 192.0
    shape, t, ps = sphere_packing(n=n, zlo=int(16 * scale), zhi=int(159 * scale),
                                  counter=(int(176 * scale), n - 1), seed=5)
    n_init = noisy_concentrations(t, [rs, rs], 1e-6, seed=5) if noise else None
    return Workload(f"porous_electrode_{n}^3", shape, t, ps, (1, -1), (0.05, 0.05), lB, 1.0, 1.0,
                    (0.0, 0.0, 0.0), (rs, rs), n_init, 1.8, 1e-10, 4000, dict(debye=debye))


def porous_crop(n=24, z0=156, noise=True):
    """An n^3 crop of the porous electrode (x, y in [0, n), z in [z0, z0 + n)),
    periodic as a box of its own: with the default z0 it holds the caps of
    the top spheres (electrode 1, +0.05) and the first planes of the
    counter-electrode (z >= 176, -0.05) with the electrolyte between."""
    w = porous_electrode(noise=False)
    N = w.shape[0]
    t3 = w.node_type.reshape(N, N, N)[z0:z0 + n, :n, :n].copy()
    p3 = w.phi_s.reshape(N, N, N)[z0:z0 + n, :n, :n].copy()
    t = t3.reshape(-1)
    ps = p3.reshape(-1)
    n_init = noisy_concentrations(t, w.n_ref, 1e-6, seed=5) if noise else None
    return Workload(f"porous_crop_{n}^3", (n, n, n), t, ps, w.z, w.D, w.lB, w.tau, w.rho0, w.Eapp,
                    w.n_ref, n_init, w.omega, w.tol, w.steps, dict(w.extra))


def porous_column(nxy=32, noise=True):
    """A lateral crop of the porous electrode that keeps its whole height:
    x, y in [0, nxy), every z (sphere packing, gap and counter-electrode),
    periodic as a box of its own."""
    w = porous_electrode(noise=False)
    N = w.shape[0]
    t = w.node_type.reshape(N, N, N)[:, :nxy, :nxy].copy().reshape(-1)
    ps = w.phi_s.reshape(N, N, N)[:, :nxy, :nxy].copy().reshape(-1)
    n_init = noisy_concentrations(t, w.n_ref, 1e-6, seed=5) if noise else None
    return Workload(f"porous_column_{nxy}x{nxy}x{N}", (nxy, nxy, N), t, ps, w.z, w.D, w.lB,
                    w.tau, w.rho0, w.Eapp, w.n_ref, n_init, w.omega, w.tol, w.steps,
                    dict(w.extra))


def noisy_concentrations(node_type, rho, rel=1e-6, seed=1):
    """n_k(r) = rho_k (1 + rel * U(-1, 1)) on fluid nodes, 0 on solid nodes,
    drawn from a PCG64 stream seeded with `seed`.  Returns (K, N)."""
    rng = np.random.default_rng(seed)
    rho = np.asarray(rho, dtype=np.float64)
    N = node_type.size
    out = np.empty((rho.size, N))
    for k in range(rho.size):
        out[k] = rho[k] * (1.0 + rel * rng.uniform(-1.0, 1.0, N))
    out[:, node_type != 0] = 0.0
    return out


@dataclass
class Workload:
    """One benchmark or parity workload."""
    name: str
    shape: tuple
    node_type: np.ndarray
    phi_s: np.ndarray
    z: tuple
    D: tuple
    lB: float
    tau: float
    rho0: float
    Eapp: tuple
    n_ref: tuple
    n_init: np.ndarray | None
    omega: float
    tol: float
    steps: int
    extra: dict = field(default_factory=dict)


def parallel_plate_small(noise=True):
    """Parallel-plate nanocapacitor, 4x4x34 (one electrode plane each end, 32
    fluid planes), tau = 1, D = 0.05, Debye length 4 at l_B = 0.4, electrode
    potentials +/-0.05, SOR omega 1.8 to residual 1e-10, 20000 steps."""
    lB, debye = 0.4, 4.0
    rs = salt_for_debye(debye, lB)
    shape, t, ps = slab(4, 4, 32, layers=1, phi1=0.05, phi2=-0.05)
    n_init = noisy_concentrations(t, [rs, rs], 1e-6, seed=1) if noise else None
    return Workload("parallel_plate_4x4x34", shape, t, ps, (1, -1), (0.05, 0.05), lB, 1.0, 1.0,
                    (0.0, 0.0, 0.0), (rs, rs), n_init, 1.8, 1e-10, 20000,
                    dict(debye=debye, dV=-0.1))


def eo_slab(noise=True, nx=64, ny=64, nfluid=128):
    """Parallel-plate electro-osmosis slab, 64x64x130 (128 fluid planes),
    Debye length 8 at l_B = 0.4, electrode potentials +/-0.1, tangential field
    E_x = 1e-3, tau = 1, D = 0.05, 50000 steps."""
    lB, debye = 0.4, 8.0
    rs = salt_for_debye(debye, lB)
    shape, t, ps = slab(nx, ny, nfluid, layers=1, phi1=0.1, phi2=-0.1)
    n_init = noisy_concentrations(t, [rs, rs], 1e-6, seed=2) if noise else None
    return Workload(f"eo_slab_{nx}x{ny}x{nfluid + 2}", shape, t, ps, (1, -1), (0.05, 0.05), lB,
                    1.0, 1.0, (1e-3, 0.0, 0.0), (rs, rs), n_init, 1.8, 1e-10, 50000,
                    dict(debye=debye, dV=-0.2))


def coaxial(noise=True, nx=160, ny=160, nz=64, R1=8.0, R2=72.0):
    """Coaxial electrodes, 160x160x64 periodic along z, inner radius 8 at
    +0.05, outer radius 72 at -0.05, Debye length 6, tau = 0.8, E_z = 1e-3."""
    lB, debye = 0.4, 6.0
    rs = salt_for_debye(debye, lB)
    shape, t, ps = coax(nx, ny, nz, R1, R2, 0.05, -0.05)
    n_init = noisy_concentrations(t, [rs, rs], 1e-6, seed=3) if noise else None
    return Workload(f"coaxial_{nx}x{ny}x{nz}", shape, t, ps, (1, -1), (0.05, 0.05), lB, 0.8, 1.0,
                    (0.0, 0.0, 1e-3), (rs, rs), n_init, 1.8, 1e-10, 30000,
                    dict(debye=debye, R1=R1, R2=R2, dV=-0.1))


@dataclass
class Batch:
    """Independent parallel-plate systems stacked along z in one lattice."""
    name: str
    shape: tuple
    node_type: np.ndarray
    phi_s: np.ndarray
    system: np.ndarray          # system index of every node (0 on solid nodes)
    n_ref: np.ndarray           # (nsys, K) salt concentration of each system
    n_init: np.ndarray | None
    z: tuple
    D: tuple
    lB: float
    tau: float
    L: np.ndarray               # fluid planes of each system
    V: np.ndarray               # voltage across each system
    debye: np.ndarray           # Debye length of each system
    z0: np.ndarray              # first fluid plane of each system


def batch_slabs(nsys=96, nxy=8, Lmin=16, Lmax=256, Vmin=0.01, Vmax=0.2, dmin=2.0, dmax=16.0,
                seed=4, noise=True, lB=0.4, D=0.05):
    """Parameter sweep of parallel-plate capacitors (Sec. III A): nsys systems,
    each nxy x nxy periodic with L fluid planes (L uniform in Lmin..Lmax),
    voltage V uniform in [Vmin, Vmax] (+V/2 and -V/2 on its electrodes),
    Debye length uniform in [dmin, dmax] (1:1 salt, l_B = 0.4).  Each system
    is one electrode plane, L fluid planes and one or two electrode planes
    (an even number of planes in all, so the four-colour order of each
    system is the one it has alone), stacked along z; system s owns
    electrodes 2s + 1 (bottom) and 2s + 2 (top).  Seeded."""
    rng = np.random.default_rng(seed)
    L = rng.integers(Lmin, Lmax + 1, nsys)
    V = rng.uniform(Vmin, Vmax, nsys)
    debye = rng.uniform(dmin, dmax, nsys)
    planes = L + 2 + ((L + 2) % 2)
    nz = int(planes.sum())
    t = np.zeros((nz, nxy, nxy), np.uint8)
    ps = np.zeros((nz, nxy, nxy))
    sy = np.zeros((nz, nxy, nxy), np.uint16)
    z0 = np.zeros(nsys, int)
    z = 0
    for s in range(nsys):
        t[z] = 2 * s + 1
        ps[z] = 0.5 * V[s]
        z0[s] = z + 1
        sy[z + 1:z + 1 + L[s]] = s
        t[z + 1 + L[s]:z + planes[s]] = 2 * s + 2
        ps[z + 1 + L[s]:z + planes[s]] = -0.5 * V[s]
        z += planes[s]
    rs = np.array([salt_for_debye(d, lB) for d in debye])
    n_ref = np.stack([rs, rs], axis=1)
    t = t.reshape(-1)
    sy = sy.reshape(-1)
    n_init = None
    if noise:
        rng2 = np.random.default_rng(seed + 1000)
        n_init = np.empty((2, t.size))
        for k in range(2):
            n_init[k] = rs[sy] * (1.0 + 1e-6 * rng2.uniform(-1.0, 1.0, t.size))
        n_init[:, t != 0] = 0.0
    return Batch(f"batched_{nsys}_slabs_{nxy}x{nxy}", (nxy, nxy, nz), t, ps.reshape(-1), sy,
                 n_ref, n_init, (1, -1), (D, D), lB, 1.0, L, V, debye, z0)
