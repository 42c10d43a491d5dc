"""Directional derivatives of the electrode charge by complex-step
differentiation (test infrastructure only).

A plain numpy restatement of the LBE time step of arXiv:1907.04732 that runs on
complex numbers:

* link fluxes of Eq. 10 (excess part written with expm1) and the force they
  exert on the fluid, the velocity of Eq. 7 with the half-force shift of Guo
  forcing, the ion update of Eq. 9 with diffusion-migration and advective
  link fluxes on fluid-fluid links only;
* BGK collision towards the second-order equilibrium with the Guo source term,
  streaming with halfway bounce-back (Eq. 8);
* Poisson with the Laplacian of Eq. 15 (Eq. 12 in the first-order mode), the
  electrode potential at the mid-link, solved EXACTLY by a sparse LU
  factorisation of the fluid-node operator (the same equations the iterative
  solvers approach);
* the electrode charges of Eq. 16.

Every operation above is analytic in its inputs (sums, products, quotients,
expm1 and a linear solve).  Evaluating the step sequence at x + i h v with a
real direction v and h = 1e-30 therefore gives Im Q / h = dQ/dx . v to
rounding, with no subtractive cancellation (the complex-step method of Squire
and Trapp, SIAM Review 40 (1998); Martins, Sturdza and Alonso, ACM TOMS 29
(2003)).  The real part is the forward trajectory itself.

This is an independent restatement: it shares no code with the C oracle or
with the GPU library.  Parity pinned by ``tests/test_oracle_tangent.py``:
the real part against the pinned C oracle, the derivative against central
finite differences of the C oracle, the ion-free slab capacitor's closed
form, and Gauss's-law invariants of the summed charge.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as sla

# D3Q19 in the documented order; weights and link lengths (Sec. II B)
_C = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
               [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1],
               [1, 0, -1], [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]])
_W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
_LEN = np.sqrt((_C * _C).sum(1).astype(float))
_OPP = np.array([int(np.flatnonzero((_C == -_C[i]).all(1))[0]) for i in range(19)])
_A0 = 1.0 + 2.0 * math.sqrt(2.0)  # lattice factor of Eq. 9 for D3Q19

STEP = 1e-30  # imaginary step


class ComplexLBE:
    """Complex-valued LBE state.  Fields are arrays over (z, y, x); site
    r = x + nx*(y + ny*z) is their C-order flattening.

    params: dict with z, D, lB, tau, Eapp, wall (2 = Eq. 15, 1 = Eq. 12).
    node_type: N uint8 (0 fluid, e >= 1 electrode e); phi_s: N values (solid
    entries used); n_init: (K, N); f_init: (19, N) pre-collision populations.
    Any of phi_s, lB, n_init, f_init may be complex.
    """

    def __init__(self, shape, params, node_type, phi_s, n_init, f_init):
        nx, ny, nz = shape
        self.shape3 = (nz, ny, nx)
        self.N = nx * ny * nz
        self.t = np.asarray(node_type, np.uint8).reshape(self.shape3)
        self.fluid = self.t == 0
        self.ne = int(self.t.max())
        self.z = np.asarray(params["z"], int)
        self.K = len(self.z)
        self.d = np.asarray(params["D"], float) / _A0
        self.lB = complex(params["lB"])
        self.tau = float(params["tau"])
        self.E = np.asarray(params.get("Eapp", (0.0, 0.0, 0.0)), float)
        self.wall = float(params.get("wall", 2.0))
        ps = np.asarray(phi_s).reshape(self.shape3).astype(complex)
        self.phi_s = np.where(self.fluid, 0.0, ps)
        self.n = np.where(self.fluid, np.asarray(n_init).reshape((self.K,) + self.shape3), 0.0)
        self.n = self.n.astype(complex)
        self.f = np.where(self.fluid, np.asarray(f_init).reshape((19,) + self.shape3), 0.0)
        self.f = self.f.astype(complex)
        # fluid-fluid links and links from a fluid node to a solid one
        self.ff = [None] + [self.fluid & self._at(self.fluid, i) for i in range(1, 19)]
        self.fs = [None] + [self.fluid & ~self._at(self.fluid, i) for i in range(1, 19)]
        self._factor_poisson()
        self.phi = self._solve_poisson()
        self.q_hist = [self.charges()]

    # value at r + c_i of every site (periodic)
    def _at(self, a, i):
        cx, cy, cz = _C[i]
        return np.roll(a, shift=(-cz, -cy, -cx), axis=(-3, -2, -1))

    # value at r - c_i: the inverse shift
    def _from(self, a, i):
        cx, cy, cz = _C[i]
        return np.roll(a, shift=(cz, cy, cx), axis=(-3, -2, -1))

    # ---- Poisson (Eqs. 12-15) ------------------------------------------------
    def _factor_poisson(self):
        """L_h phi = A phi_fluid + B phi_s at fluid nodes; A is factorised once
        (it does not depend on time, l_B or phi_s)."""
        N = self.N
        idx = np.full(N, -1)
        fl = self.fluid.reshape(-1)
        self.fidx = np.flatnonzero(fl)
        idx[self.fidx] = np.arange(self.fidx.size)
        site = np.arange(N).reshape(self.shape3)
        rows, cols, vals = [], [], []
        diag = np.zeros(self.fidx.size)
        brow, bcol, bval = [], [], []
        for i in range(1, 19):
            nb = self._at(site, i).reshape(-1)
            r = self.fidx
            rn = nb[r]
            keep = rn != r  # a link from a node to itself carries no difference
            r, rn = r[keep], rn[keep]
            is_f = fl[rn]
            s = np.where(is_f, 1.0, self.wall) * 6.0 * _W[i]
            np.add.at(diag, idx[r], -s)
            rows.append(idx[r[is_f]])
            cols.append(idx[rn[is_f]])
            vals.append(s[is_f])
            brow.append(idx[r[~is_f]])
            bcol.append(rn[~is_f])
            bval.append(s[~is_f])
        nf = self.fidx.size
        A = sp.coo_matrix((np.concatenate(vals + [diag]),
                           (np.concatenate(rows + [np.arange(nf)]),
                            np.concatenate(cols + [np.arange(nf)]))), shape=(nf, nf))
        self.A = A.tocsc()
        self.B = sp.coo_matrix((np.concatenate(bval), (np.concatenate(brow), np.concatenate(bcol))),
                               shape=(nf, N)).tocsr()
        self.lu = sla.splu(self.A)

    def _solve_poisson(self):
        """Fluid potential from A phi = -4 pi l_B rho_el - B phi_s (exact)."""
        rho = np.tensordot(self.z, self.n, axes=1).reshape(-1)[self.fidx]
        rhs = -4.0 * math.pi * self.lB * rho - self.B @ self.phi_s.reshape(-1)
        sol = self.lu.solve(np.ascontiguousarray(rhs.real)) + 1j * self.lu.solve(
            np.ascontiguousarray(rhs.imag))
        phi = self.phi_s.reshape(-1).copy()
        phi[self.fidx] = sol
        return phi.reshape(self.shape3)

    # ---- Gauss's law (Eq. 16) ------------------------------------------------
    def charges(self):
        """Q_e = -(1/(4 pi l_B)) sum over electrode e's nodes of L_h phi, the
        difference doubled (factor `wall`) on each solid-fluid link."""
        lap = np.zeros(self.shape3, complex)
        solid = ~self.fluid
        for i in range(1, 19):
            to_fluid = solid & self._at(self.fluid, i)
            lap += np.where(to_fluid, _W[i] * self.wall * (self._at(self.phi, i) - self.phi), 0.0)
        lap *= 6.0
        q = np.zeros(self.ne, complex)
        for e in range(1, self.ne + 1):
            q[e - 1] = -lap[self.t == e].sum() / (4.0 * math.pi * self.lB)
        return q

    # ---- one time step (Eqs. 7-10) ------------------------------------------
    def _link_terms(self):
        """Force on the fluid (excess link fluxes projected on the node) and
        the sum over links of each species' diffusion-migration flux."""
        n, phi = self.n, self.phi
        force = np.zeros((3,) + self.shape3, complex)
        flux = np.zeros_like(n)
        for i in range(1, 19):
            link = self.ff[i]
            Ec = float(self.E @ _C[i])
            n_there = self._at(n, i)
            g_sum = 0.0
            for k in range(self.K):
                delta = self.z[k] * (self._at(phi, i) - phi - Ec)
                g = -(n_there[k] * np.expm1(delta) - n[k] * np.expm1(-delta)) / (2.0 * _LEN[i])
                g = np.where(link, g, 0.0)
                g_sum = g_sum + g
                flux[k] += self.d[k] * np.where(link, g - (n_there[k] - n[k]) / _LEN[i], 0.0)
            for a in range(3):
                force[a] += 3.0 * _W[i] * _C[i, a] * _LEN[i] * g_sum
        return force, flux

    def momentum(self):
        """Total fluid momentum sum_r (sum_i f_i c_i + F/2) of the current
        state (the mass flux of the velocity of Guo forcing), 3 values."""
        force, _ = self._link_terms()
        mom = np.tensordot(_C.T.astype(float), self.f, axes=1) + 0.5 * force
        return np.array([mom[a][self.fluid].sum() for a in range(3)])

    def step(self):
        fl = self.fluid
        n, f = self.n, self.f
        force, flux = self._link_terms()
        rho = f.sum(0)
        mom = np.tensordot(_C.T.astype(float), f, axes=1)
        safe = np.where(fl, rho, 1.0)
        u = np.where(fl, (mom + 0.5 * force) / safe, 0.0)
        # advective link fluxes with this step's velocity
        for i in range(1, 19):
            link = self.ff[i]
            cu_here = np.tensordot(_C[i].astype(float), u, axes=1)
            cu_there = self._at(cu_here, i)
            n_there = self._at(n, i)
            for k in range(self.K):
                J = 3.0 * _W[i] * (n[k] * cu_here + n_there[k] * cu_there)
                flux[k] += np.where(link, J, 0.0)
        n_new = np.where(fl, n - flux, 0.0)
        # BGK + Guo source, then streaming with halfway bounce-back
        uu = (u * u).sum(0)
        f_new = np.zeros_like(f)
        for i in range(19):
            cu = np.tensordot(_C[i].astype(float), u, axes=1)
            feq = _W[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu)
            src = sum((3.0 * (_C[i, a] - u[a]) + 9.0 * cu * _C[i, a]) * force[a] for a in range(3))
            src = src * (1.0 - 0.5 / self.tau) * _W[i]
            post = np.where(fl, f[i] - (f[i] - feq) / self.tau + src, 0.0)
            if i == 0:
                f_new[0] += post
                continue
            f_new[i] += self._from(np.where(self.ff[i], post, 0.0), i)
            f_new[_OPP[i]] += np.where(self.fs[i], post, 0.0)
        self.n, self.f = n_new, f_new
        self.phi = self._solve_poisson()
        self.q_hist.append(self.charges())


def charge_tangent(shape, params, node_type, phi_s, n_init, f_init, nsteps, dphi_s=None,
                   dlB=0.0, dn=None, df=None):
    """Q(nsteps) and its directional derivative along (dphi_s, dlB, dn, df)
    (None = 0), both per electrode, by one complex-step evaluation."""
    h = STEP
    ps = np.asarray(phi_s, float) + (0 if dphi_s is None else 1j * h * np.asarray(dphi_s, float))
    pr = dict(params)
    pr["lB"] = complex(params["lB"]) + 1j * h * float(dlB)
    n0 = np.asarray(n_init, float) + (0 if dn is None else 1j * h * np.asarray(dn, float))
    f0 = np.asarray(f_init, float) + (0 if df is None else 1j * h * np.asarray(df, float))
    s = ComplexLBE(shape, pr, node_type, ps, n0, f0)
    for _ in range(nsteps):
        s.step()
    q = s.q_hist[-1]
    return q.real.copy(), q.imag / h, s


def rest_populations(node_type, rho0=1.0):
    """w_i rho0 on fluid nodes, 0 on solid nodes: (19, N)."""
    fl = np.asarray(node_type).reshape(-1) == 0
    return np.where(fl[None, :], _W[:, None] * rho0, 0.0)
