"""Plain FP64 CPU oracle of the LBE time step (test infrastructure only).

The C source ``lbe_oracle.c`` holds the arithmetic; this module builds it with
gcc and drives it through ctypes.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the GPU
library and imports nothing from it.

Parity pinned: every function is checked in ``tests/test_oracle_pins.py``
against closed forms and exact lattice identities that follow from the paper
(arXiv:1907.04732, Secs. II-III).  The transient electro-osmotic profiles have
no closed form and are "parity unpinned" beyond conservation and symmetry.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbe_oracle.c")
_LIB = os.path.join(_HERE, "liblbe_oracle.so")
# the same source built with OpenMP: the independent per-site loops run on
# several threads, every value bit for bit the single-threaded one
_LIB_OMP = os.path.join(_HERE, "liblbe_oracle_omp.so")

FLAG_ALLOW_FLOATING = 1
FLAG_NAIVE_DIRICHLET = 4  # first-order scheme: potential on the solid nodes, Eq. 12 everywhere

OK, EINVAL, EGEOM, ENOMEM, ENOCONV, ENONFINITE = 0, -1, -2, -3, -5, -6


class OracleParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("nspecies", C.c_int32),
        ("z", C.c_int32 * 4),
        ("D", C.c_double * 4),
        ("lB", C.c_double), ("tau", C.c_double), ("rho0", C.c_double),
        ("Eapp", C.c_double * 3),
        ("omega", C.c_double), ("tol", C.c_double),
        ("max_iter", C.c_int32), ("check_every", C.c_int32),
        ("flags", C.c_int32), ("reserved", C.c_int32),
    ]


def build() -> str:
    """Compile the oracle into shared libraries next to its source: the
    single-threaded one and the OpenMP one."""
    base = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared"]
    subprocess.run(base + ["-o", _LIB, _SRC, "-lm"], check=True)
    subprocess.run(base + ["-fopenmp", "-o", _LIB_OMP, _SRC, "-lm"], check=True)
    return _LIB


_libs = {}


def build_variant(src_text: str, out_path: str) -> str:
    """Compile a modified copy of the oracle source (used by the tests that
    plant mistakes in the oracle to show that the pins catch them)."""
    src_path = out_path + ".c"
    with open(src_path, "w") as fh:
        fh.write(src_text)
    subprocess.run(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-o", out_path,
                    src_path, "-lm"], check=True)
    return out_path


def source_text() -> str:
    with open(_SRC) as fh:
        return fh.read()


def _stale(lib_path):
    return not os.path.exists(lib_path) or os.path.getmtime(lib_path) < os.path.getmtime(_SRC)


def _load(path=None):
    key = path or _LIB
    if key in _libs:
        return _libs[key]
    if key in (_LIB, _LIB_OMP) and (_stale(_LIB) or _stale(_LIB_OMP)):
        build()
    lib = C.CDLL(key)
    P = C.POINTER
    d = P(C.c_double)
    lib.orc_init.argtypes = [P(OracleParams), P(C.c_uint8), d, d, d, d, P(C.c_void_p),
                             C.c_char_p, C.c_int]
    lib.orc_init.restype = C.c_int
    lib.orc_step.argtypes = [C.c_void_p, C.c_long]
    lib.orc_step.restype = C.c_int
    lib.orc_set_solver.argtypes = [C.c_void_p, C.c_double, C.c_int]
    lib.orc_set_solver.restype = C.c_int
    lib.orc_poisson.argtypes = [C.c_void_p, P(C.c_int), d]
    lib.orc_poisson.restype = C.c_int
    lib.orc_set_electrode_potential.argtypes = [C.c_void_p, d]
    lib.orc_set_electrode_potential.restype = C.c_int
    lib.orc_electrode_charge.argtypes = [C.c_void_p, d, C.c_int]
    lib.orc_electrode_charge.restype = C.c_int
    lib.orc_num_electrodes.argtypes = [C.c_void_p]
    lib.orc_num_electrodes.restype = C.c_int
    lib.orc_step_count.argtypes = [C.c_void_p]
    lib.orc_step_count.restype = C.c_long
    lib.orc_last_iters.argtypes = [C.c_void_p]
    lib.orc_last_iters.restype = C.c_int
    lib.orc_last_resid.argtypes = [C.c_void_p]
    lib.orc_last_resid.restype = C.c_double
    lib.orc_fields.argtypes = [C.c_void_p, d, d, d, d, d, d]
    lib.orc_fields.restype = C.c_int
    lib.orc_residual.argtypes = [C.c_void_p, d]
    lib.orc_residual.restype = C.c_int
    lib.orc_qhist.argtypes = [C.c_void_p, d, C.c_long]
    lib.orc_qhist.restype = C.c_long
    lib.orc_free.argtypes = [C.c_void_p]
    lib.orc_free.restype = None
    lib.orc_last_error.argtypes = [C.c_void_p]
    lib.orc_last_error.restype = C.c_char_p
    lib.orc_strerror.argtypes = [C.c_int]
    lib.orc_strerror.restype = C.c_char_p
    lib.orc_velocities.argtypes = [P(C.c_int), d]
    lib.orc_velocities.restype = None
    lib.orc_set_threads.argtypes = [C.c_int]
    lib.orc_set_threads.restype = C.c_int
    _libs[key] = lib
    return lib


def _dptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


def make_params(shape, z, D, lB, tau=1.0, rho0=1.0, Eapp=(0.0, 0.0, 0.0), omega=1.8,
                tol=1e-10, max_iter=200000, check_every=4, flags=0) -> OracleParams:
    nx, ny, nz = shape
    p = OracleParams()
    p.nx, p.ny, p.nz = nx, ny, nz
    p.nspecies = len(z)
    for k in range(len(z)):
        p.z[k] = int(z[k])
        p.D[k] = float(D[k])
    p.lB, p.tau, p.rho0 = float(lB), float(tau), float(rho0)
    for a in range(3):
        p.Eapp[a] = float(Eapp[a])
    p.omega, p.tol = float(omega), float(tol)
    p.max_iter, p.check_every, p.flags = int(max_iter), int(check_every), int(flags)
    return p


class Oracle:
    """One oracle state.  Arrays use site index x + nx*(y + ny*z)."""

    def __init__(self, params: OracleParams, node_type, phi_s, n_init=None, n_ref=None,
                 f_init=None, libpath=None, threads=None):
        """threads: run the per-site loops on that many OpenMP threads (the
        same values bit for bit; None = the single-threaded build)."""
        lib = _load(_LIB_OMP if threads and libpath is None else libpath)
        if threads and libpath is None:
            self.threads = lib.orc_set_threads(int(threads))
        else:
            self.threads = 1
        self._lib = lib
        self.p = params
        self.N = params.nx * params.ny * params.nz
        self.K = params.nspecies
        t = np.ascontiguousarray(node_type, dtype=np.uint8).reshape(-1)
        ps = np.ascontiguousarray(phi_s, dtype=np.float64).reshape(-1)
        assert t.size == self.N and ps.size == self.N
        ni = None if n_init is None else np.ascontiguousarray(n_init, dtype=np.float64).reshape(-1)
        nr = None if n_ref is None else np.ascontiguousarray(n_ref, dtype=np.float64).reshape(-1)
        fi = None if f_init is None else np.ascontiguousarray(f_init, dtype=np.float64).reshape(-1)
        if ni is not None:
            assert ni.size == self.K * self.N
        if fi is not None:
            assert fi.size == 19 * self.N
        self._keep = (t, ps, ni, nr, fi)
        h = C.c_void_p()
        err = C.create_string_buffer(256)
        rc = lib.orc_init(C.byref(params), t.ctypes.data_as(C.POINTER(C.c_uint8)), _dptr(ps),
                          _dptr(ni), _dptr(nr), _dptr(fi), C.byref(h), err, 256)
        if rc:
            raise OracleError(rc, err.value.decode())
        self.h = h
        self.ne = lib.orc_num_electrodes(h)

    def close(self):
        if getattr(self, "h", None):
            self._lib.orc_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc:
            raise OracleError(rc, self._lib.orc_last_error(self.h).decode())

    def step(self, nsteps=1):
        if self.threads > 1:
            self._lib.orc_set_threads(self.threads)
        self._check(self._lib.orc_step(self.h, int(nsteps)))

    def set_solver(self, tol, max_iter):
        """New Poisson stopping rule for later solves."""
        self._check(self._lib.orc_set_solver(self.h, float(tol), int(max_iter)))

    def poisson(self):
        it = C.c_int()
        res = C.c_double()
        self._check(self._lib.orc_poisson(self.h, C.byref(it), C.byref(res)))
        return it.value, res.value

    def set_electrode_potential(self, phi_s):
        """New potentials of the solid nodes (length N, fluid entries ignored);
        re-solves Poisson and replaces the current step's recorded charge."""
        ps = np.ascontiguousarray(phi_s, dtype=np.float64)
        if ps.size != self.N:
            raise ValueError("phi_s must have one entry per lattice site")
        self._check(self._lib.orc_set_electrode_potential(self.h, _dptr(ps)))

    def electrode_charge(self):
        q = np.zeros(max(self.ne, 1))
        self._check(self._lib.orc_electrode_charge(self.h, _dptr(q), len(q)))
        return q[: self.ne]

    @property
    def step_count(self):
        return self._lib.orc_step_count(self.h)

    @property
    def last_iters(self):
        return self._lib.orc_last_iters(self.h)

    @property
    def last_resid(self):
        return self._lib.orc_last_resid(self.h)

    def fields(self):
        """Return dict with phi, n (K,N), f (19,N), rho, u (3,N), force (3,N)."""
        N, K = self.N, self.K
        phi = np.empty(N)
        n = np.empty(K * N)
        f = np.empty(19 * N)
        rho = np.empty(N)
        u = np.empty(3 * N)
        force = np.empty(3 * N)
        self._lib.orc_fields(self.h, _dptr(phi), _dptr(n), _dptr(f), _dptr(rho), _dptr(u),
                           _dptr(force))
        return dict(phi=phi, n=n.reshape(K, N), f=f.reshape(19, N), rho=rho,
                    u=u.reshape(3, N), force=force.reshape(3, N))

    def residual(self):
        r = np.empty(self.N)
        self._lib.orc_residual(self.h, _dptr(r))
        return r

    def qhist(self):
        lib = self._lib
        n = lib.orc_qhist(self.h, None, 0)
        out = np.empty(max(n * self.ne, 1))
        lib.orc_qhist(self.h, _dptr(out), n)
        return out[: n * self.ne].reshape(n, self.ne)


def velocities():
    lib = _load()
    c = (C.c_int * 57)()
    w = np.empty(19)
    lib.orc_velocities(c, _dptr(w))
    return np.array(list(c), dtype=np.int64).reshape(19, 3), w
