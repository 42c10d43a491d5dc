"""Python binding of liblbe.so, the gfx950 Lattice Boltzmann Electrokinetics
library (arXiv:1907.04732).  Argument marshalling only: every step of the
method runs in the HIP kernels behind include/lbe.h.  There is no CPU
fallback; importing works without a GPU, creating a context needs one.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbe.so")

OK, EINVAL, EGEOM, ENOMEM, EDEVICE, ENOCONV, ENONFINITE = 0, -1, -2, -3, -4, -5, -6
FP64, FP32_MIXED = 0, 1
SOR4, MG = 0, 1
MG_JACOBI, MG_GS4 = 0, 1
ALLOW_FLOATING = 1
EXTRAPOLATE = 2
NAIVE_DIRICHLET = 4
KRYLOV = 8
NOALLOC_MAX_ELECTRODES = 16

# public entry points of include/lbe.h
ENTRY_POINTS = (
    "lbe_init", "lbe_init_batch", "lbe_init_device", "lbe_step", "lbe_step_chunk",
    "lbe_set_solver",
    "lbe_poisson", "lbe_set_electrode_potential", "lbe_record", "lbe_adjoint",
    "lbe_electrode_charge", "lbe_observables", "lbe_fields_device",
    "lbe_destroy", "lbe_strerror", "lbe_last_error", "lbe_profile", "lbe_kernel_times",
    "lbe_kernel_name", "lbe_num_kernel_kinds", "lbe_velocities", "lbe_build_id",
    "lbe_electrode_charge_noalloc", "lbe_launch_shape",
)


class Params(C.Structure):
    """Mirror of lbe_params."""
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("nspecies", C.c_int32),
        ("z", C.c_int32 * 4),
        ("D", C.c_double * 4),
        ("lB", C.c_double), ("tau", C.c_double), ("rho0", C.c_double),
        ("Eapp", C.c_double * 3),
        ("omega", C.c_double), ("tol", C.c_double),
        ("max_iter", C.c_int32), ("check_every", C.c_int32),
        ("flags", C.c_int32), ("precision", C.c_int32), ("poisson", C.c_int32),
        ("mg_levels", C.c_int32), ("mg_nu1", C.c_int32), ("mg_nu2", C.c_int32),
        ("mg_smoother", C.c_int32), ("mg_nu1_coarse", C.c_int32), ("mg_nu2_coarse", C.c_int32),
        ("stream", C.c_void_p),
    ]


class Obs(C.Structure):
    """Mirror of lbe_obs."""
    _fields_ = [
        ("step", C.c_int64), ("nelectrodes", C.c_int32), ("poisson_iters", C.c_int32),
        ("poisson_resid", C.c_double), ("mass", C.c_double), ("nk", C.c_double * 4),
        ("q_ion", C.c_double), ("poisson_total", C.c_int64), ("momentum", C.c_double * 3),
    ]


class LbeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lbe error {code}: {msg}")
        self.code = code


_lib = None


def _bring_up_torch_first():
    """torch ships its own HIP runtime beside the system one the library links.
    Both work in one process only when torch's initialises the device first
    (the other order leaves torch with no GPU), so when torch is installed
    and sees a GPU it is brought up before the library is loaded."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


def load(path: str = LIB_PATH):
    """Load liblbe.so (built by paper_1907_04732_amd.build); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"{path} is missing: build it with `python -m paper_1907_04732_amd.build` "
                      "(there is no CPU fallback)")
    _bring_up_torch_first()
    lib = C.CDLL(path)
    lib.lbe_build_id.argtypes = []
    lib.lbe_build_id.restype = C.c_char_p
    if os.path.isdir(os.path.join(_HERE, "csrc")):
        from .build import source_hash
        have, want = lib.lbe_build_id().decode(), source_hash()
        if have != want:
            raise OSError(f"{path} was built from other sources (build {have}, sources {want}): "
                          "rebuild it with `python -m paper_1907_04732_amd.build`")
    P = C.POINTER
    d = P(C.c_double)
    lib.lbe_init.argtypes = [P(Params), P(C.c_uint8), d, d, d, d, P(C.c_void_p)]
    lib.lbe_init.restype = C.c_int
    lib.lbe_init_batch.argtypes = [P(Params), P(C.c_uint8), d, d, d, P(C.c_uint16), C.c_int32,
                                   P(C.c_void_p)]
    lib.lbe_init_batch.restype = C.c_int
    v = C.c_void_p
    lib.lbe_init_device.argtypes = [P(Params), v, v, v, v, v, P(C.c_void_p)]
    lib.lbe_init_device.restype = C.c_int
    lib.lbe_set_solver.argtypes = [C.c_void_p, C.c_double, C.c_int32]
    lib.lbe_set_solver.restype = C.c_int
    lib.lbe_fields_device.argtypes = [C.c_void_p, v, v, v, v]
    lib.lbe_fields_device.restype = C.c_int
    lib.lbe_step.argtypes = [C.c_void_p, C.c_int64]
    lib.lbe_step.restype = C.c_int
    lib.lbe_step_chunk.argtypes = [C.c_void_p, C.c_int64, C.c_int32]
    lib.lbe_step_chunk.restype = C.c_int
    lib.lbe_poisson.argtypes = [C.c_void_p, P(C.c_int32), d]
    lib.lbe_poisson.restype = C.c_int
    lib.lbe_set_electrode_potential.argtypes = [C.c_void_p, d]
    lib.lbe_set_electrode_potential.restype = C.c_int
    lib.lbe_record.argtypes = [C.c_void_p, C.c_int64, C.c_int32]
    lib.lbe_record.restype = C.c_int
    lib.lbe_adjoint.argtypes = [C.c_void_p, d, d, d, d, d, d]
    lib.lbe_adjoint.restype = C.c_int
    lib.lbe_electrode_charge.argtypes = [C.c_void_p, d, C.c_int32]
    lib.lbe_electrode_charge.restype = C.c_int
    lib.lbe_observables.argtypes = [C.c_void_p, P(Obs), d, d, d, d, d, C.c_int64, P(C.c_int64)]
    lib.lbe_observables.restype = C.c_int
    lib.lbe_destroy.argtypes = [C.c_void_p]
    lib.lbe_destroy.restype = None
    lib.lbe_strerror.argtypes = [C.c_int]
    lib.lbe_strerror.restype = C.c_char_p
    lib.lbe_last_error.argtypes = [C.c_void_p]
    lib.lbe_last_error.restype = C.c_char_p
    lib.lbe_profile.argtypes = [C.c_void_p, C.c_int]
    lib.lbe_profile.restype = C.c_int
    lib.lbe_kernel_times.argtypes = [C.c_void_p, d, P(C.c_int64), P(C.c_int64), C.c_int32]
    lib.lbe_kernel_times.restype = C.c_int
    lib.lbe_kernel_name.argtypes = [C.c_int32]
    lib.lbe_kernel_name.restype = C.c_char_p
    lib.lbe_num_kernel_kinds.argtypes = []
    lib.lbe_num_kernel_kinds.restype = C.c_int32
    i32p = P(C.c_int32)
    lib.lbe_launch_shape.argtypes = [v, i32p, i32p, i32p]
    lib.lbe_launch_shape.restype = C.c_int
    lib.lbe_velocities.argtypes = [P(C.c_int32), d]
    lib.lbe_velocities.restype = None
    lib.lbe_electrode_charge_noalloc.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_double,
                                                 C.c_int32, v, v, v, C.c_int32, v]
    lib.lbe_electrode_charge_noalloc.restype = C.c_int
    _lib = lib
    return lib


def _dptr(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(shape, z, D, lB, tau=1.0, rho0=1.0, Eapp=(0.0, 0.0, 0.0), omega=1.8, tol=1e-10,
                max_iter=200000, check_every=4, flags=0, precision=FP64, poisson=SOR4,
                mg_levels=0, mg_nu1=2, mg_nu2=2, mg_smoother=MG_JACOBI, mg_nu1_coarse=0,
                mg_nu2_coarse=0, stream=None) -> Params:
    p = Params()
    p.nx, p.ny, p.nz = (int(v) for v in shape)
    if not 1 <= len(z) <= 4 or len(D) != len(z):
        raise ValueError("1..4 species with one valency and one D each")
    p.nspecies = len(z)
    for k in range(len(z)):
        p.z[k] = int(z[k])
        p.D[k] = float(D[k])
    p.lB, p.tau, p.rho0 = float(lB), float(tau), float(rho0)
    for a in range(3):
        p.Eapp[a] = float(Eapp[a])
    p.omega, p.tol = float(omega), float(tol)
    p.max_iter, p.check_every, p.flags = int(max_iter), int(check_every), int(flags)
    p.precision, p.poisson = int(precision), int(poisson)
    p.mg_levels, p.mg_nu1, p.mg_nu2 = int(mg_levels), int(mg_nu1), int(mg_nu2)
    p.mg_smoother = int(mg_smoother)
    p.mg_nu1_coarse, p.mg_nu2_coarse = int(mg_nu1_coarse), int(mg_nu2_coarse)
    p.stream = stream
    return p


def electrode_charge_noalloc(shape, lB, node_type, phi, q, naive=False, stream=None):
    """lbe_electrode_charge_noalloc: electrode charges of the potential `phi`
    (float64 GPU tensor, N) on the node types `node_type` (uint8 GPU tensor,
    N) into `q` (float64 GPU tensor, one entry per electrode 1..len(q)),
    launched on `stream` (a torch stream; None = torch's current stream) and
    not waited for.  Nothing is allocated."""
    import torch

    lib = load()
    for name, a, dt in (("node_type", node_type, torch.uint8), ("phi", phi, torch.float64),
                        ("q", q, torch.float64)):
        if not _is_gpu_tensor(a) or a.dtype != dt or not a.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dt} GPU tensor")
    nx, ny, nz = (int(v) for v in shape)
    if node_type.numel() != nx * ny * nz or phi.numel() != nx * ny * nz:
        raise ValueError("node_type and phi need nx*ny*nz entries")
    s = stream if stream is not None else torch.cuda.current_stream(q.device)
    with torch.cuda.device(q.device):
        rc = lib.lbe_electrode_charge_noalloc(nx, ny, nz, float(lB),
                                              NAIVE_DIRICHLET if naive else 0,
                                              _tptr(node_type), _tptr(phi), _tptr(q), q.numel(),
                                              C.c_void_p(s.cuda_stream))
    if rc:
        raise LbeError(rc, lib.lbe_last_error(None).decode())


def velocities():
    lib = load()
    c = (C.c_int32 * 57)()
    w = np.empty(19)
    lib.lbe_velocities(c, _dptr(w))
    return np.array(list(c), dtype=np.int64).reshape(19, 3), w


def kernel_names():
    lib = load()
    return [lib.lbe_kernel_name(k).decode() for k in range(lib.lbe_num_kernel_kinds())]


def _is_gpu_tensor(a):
    return getattr(a, "is_cuda", False)


def _tptr(a):
    return None if a is None else C.c_void_p(a.data_ptr())


class Lbe:
    """One LBE context on the current HIP device (see include/lbe.h)."""

    def __init__(self, params: Params, node_type, phi_s, n_init=None, n_ref=None, f_init=None,
                 system=None, nsys=None):
        """system (N ints) and nsys select lbe_init_batch: independent systems
        in one lattice, n_ref then holding nsys x nspecies values.  With
        node_type a GPU tensor, every array is read from device memory
        (lbe_init_device)."""
        lib = load()
        self._lib = lib
        self.p = params
        self.N = params.nx * params.ny * params.nz
        self.K = params.nspecies
        self.h = None
        if _is_gpu_tensor(node_type):
            if system is not None:
                raise ValueError("batched systems take host arrays")
            self._init_device(node_type, phi_s, n_init, n_ref, f_init)
            return
        t = np.ascontiguousarray(node_type, dtype=np.uint8).reshape(-1)
        ps = np.ascontiguousarray(phi_s, dtype=np.float64).reshape(-1)
        if t.size != self.N or ps.size != self.N:
            raise ValueError("node_type and phi_s need nx*ny*nz entries")
        ni = None if n_init is None else np.ascontiguousarray(n_init, dtype=np.float64).reshape(-1)
        nr = None if n_ref is None else np.ascontiguousarray(n_ref, dtype=np.float64).reshape(-1)
        fi = None if f_init is None else np.ascontiguousarray(f_init, dtype=np.float64).reshape(-1)
        if ni is not None and ni.size != self.K * self.N:
            raise ValueError("n_init needs nspecies*N entries")
        nsys = 1 if system is None else int(nsys if nsys is not None else np.max(system) + 1)
        if nr is not None and nr.size < self.K * nsys:
            raise ValueError("n_ref needs nspecies (x nsys) entries")
        if fi is not None and fi.size != 19 * self.N:
            raise ValueError("f_init needs 19*N entries")
        h = C.c_void_p()
        if system is None:
            rc = lib.lbe_init(C.byref(params), t.ctypes.data_as(C.POINTER(C.c_uint8)), _dptr(ps),
                              _dptr(ni), _dptr(nr), _dptr(fi), C.byref(h))
        else:
            if fi is not None:
                raise ValueError("batched systems start from rest populations")
            sy = np.ascontiguousarray(system, dtype=np.uint16).reshape(-1)
            if sy.size != self.N:
                raise ValueError("system needs N entries")
            rc = lib.lbe_init_batch(C.byref(params), t.ctypes.data_as(C.POINTER(C.c_uint8)),
                                    _dptr(ps), _dptr(ni), _dptr(nr),
                                    sy.ctypes.data_as(C.POINTER(C.c_uint16)), nsys, C.byref(h))
        if rc:
            raise LbeError(rc, lib.lbe_last_error(None).decode())
        self.h = h
        self.ne = int(t.max()) if t.size else 0

    def _init_device(self, node_type, phi_s, n_init, n_ref, f_init):
        import torch

        dev = node_type.device
        sizes = {"node_type": self.N, "phi_s": self.N, "n_init": self.K * self.N,
                 "n_ref": self.K, "f_init": 19 * self.N}
        args = {}
        for name, a in (("node_type", node_type), ("phi_s", phi_s), ("n_init", n_init),
                        ("n_ref", n_ref), ("f_init", f_init)):
            if a is None:
                args[name] = None
                continue
            dtype = torch.uint8 if name == "node_type" else torch.float64
            t = torch.as_tensor(a, device=dev).to(dtype).contiguous().reshape(-1)
            if t.numel() != sizes[name]:
                raise ValueError(f"{name} needs {sizes[name]} entries")
            args[name] = t
        # the library reads on its own stream: finish the work that made the inputs
        torch.cuda.current_stream(dev).synchronize()
        h = C.c_void_p()
        with torch.cuda.device(dev):
            rc = self._lib.lbe_init_device(C.byref(self.p), _tptr(args["node_type"]),
                                           _tptr(args["phi_s"]), _tptr(args["n_init"]),
                                           _tptr(args["n_ref"]), _tptr(args["f_init"]), C.byref(h))
        if rc:
            raise LbeError(rc, self._lib.lbe_last_error(None).decode())
        self.h = h
        self.ne = int(args["node_type"].max().item()) if self.N else 0
        self.device = dev

    def close(self):
        if getattr(self, "h", None):
            self._lib.lbe_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc):
        if rc:
            raise LbeError(rc, self._lib.lbe_last_error(self.h).decode())

    def step(self, nsteps=1):
        self._check(self._lib.lbe_step(self.h, int(nsteps)))

    def step_chunk(self, nsteps, units):
        """nsteps steps replayed from captured 16-step graphs with `units`
        solver units per step (lbe_step_chunk)."""
        self._check(self._lib.lbe_step_chunk(self.h, int(nsteps), int(units)))

    def set_solver(self, tol=None, max_iter=None):
        """New Poisson stopping rule for later solves (None keeps a value)."""
        tol = self.p.tol if tol is None else float(tol)
        max_iter = self.p.max_iter if max_iter is None else int(max_iter)
        self._check(self._lib.lbe_set_solver(self.h, tol, max_iter))
        self.p.tol, self.p.max_iter = tol, max_iter

    def poisson(self):
        it = C.c_int32()
        res = C.c_double()
        self._check(self._lib.lbe_poisson(self.h, C.byref(it), C.byref(res)))
        return it.value, res.value

    def set_electrode_potential(self, phi_s):
        """New solid-node potentials (N values, fluid entries ignored); Poisson
        is re-solved and the current step's recorded charge replaced."""
        ps = np.ascontiguousarray(phi_s, dtype=np.float64)
        if ps.size != self.N:
            raise ValueError("phi_s must have one entry per lattice site")
        self._check(self._lib.lbe_set_electrode_potential(self.h, _dptr(ps)))

    def record(self, nsteps, every=64):
        """Advance nsteps steps keeping checkpoints every `every` steps for
        adjoint() (FP64 form)."""
        self._check(self._lib.lbe_record(self.h, int(nsteps), int(every)))

    def adjoint(self, qbar=None, ubar=None, phi_s=True, lB=True, n=True, f=True):
        """Gradient of sum_e qbar[e] Q_e + ubar . M at the end of the record
        (M: total fluid momentum, sum_i f_i c_i + F/2 over fluid nodes): dict
        with phi_s (N), lB (float), n (K, N) at the record's start and f
        (19, N), the pre-collision populations at its start (each only if
        asked)."""
        qb = None if qbar is None else np.ascontiguousarray(qbar, dtype=np.float64).reshape(-1)
        ub = None if ubar is None else np.ascontiguousarray(ubar, dtype=np.float64).reshape(-1)
        if qb is not None and qb.size != self.ne:
            raise ValueError("one weight per electrode")
        if ub is not None and ub.size != 3:
            raise ValueError("three momentum weights")
        g_ps = np.empty(self.N) if phi_s else None
        g_lb = np.zeros(1) if lB else None
        g_n = np.empty(self.K * self.N) if n else None
        g_f = np.empty(19 * self.N) if f else None
        self._check(self._lib.lbe_adjoint(self.h, _dptr(qb), _dptr(ub), _dptr(g_ps), _dptr(g_lb),
                                          _dptr(g_n), _dptr(g_f)))
        out = {}
        if phi_s:
            out["phi_s"] = g_ps
        if lB:
            out["lB"] = float(g_lb[0])
        if n:
            out["n"] = g_n.reshape(self.K, self.N)
        if f:
            out["f"] = g_f.reshape(19, self.N)
        return out

    def electrode_charge(self):
        q = np.zeros(max(self.ne, 1))
        self._check(self._lib.lbe_electrode_charge(self.h, _dptr(q), len(q)))
        return q[: self.ne]

    def totals(self):
        o = Obs()
        self._check(self._lib.lbe_observables(self.h, C.byref(o), None, None, None, None, None, 0,
                                              None))
        return dict(step=o.step, nelectrodes=o.nelectrodes, poisson_iters=o.poisson_iters,
                    poisson_resid=o.poisson_resid, mass=o.mass, nk=list(o.nk)[: self.K],
                    q_ion=o.q_ion, poisson_total=o.poisson_total, momentum=list(o.momentum))

    def fields(self, f=True, device=None):
        """dict with phi (N), n (K,N), u (3,N) and, if f, populations (19,N).
        device (a torch device): float64 tensors written there by
        lbe_fields_device instead of numpy arrays."""
        N, K = self.N, self.K
        if device is not None:
            import torch

            out = dict(phi=torch.empty(N, dtype=torch.float64, device=device),
                       n=torch.empty(K, N, dtype=torch.float64, device=device),
                       u=torch.empty(3, N, dtype=torch.float64, device=device))
            if f:
                out["f"] = torch.empty(19, N, dtype=torch.float64, device=device)
            # the library writes on its own stream
            torch.cuda.current_stream(device).synchronize()
            self._check(self._lib.lbe_fields_device(self.h, _tptr(out["phi"]), _tptr(out["n"]),
                                                    _tptr(out["u"]), _tptr(out.get("f"))))
            return out
        phi = np.empty(N)
        n = np.empty(K * N)
        u = np.empty(3 * N)
        fp = np.empty(19 * N) if f else None
        self._check(self._lib.lbe_observables(self.h, None, _dptr(phi), _dptr(n), _dptr(u),
                                              _dptr(fp), None, 0, None))
        out = dict(phi=phi, n=n.reshape(K, N), u=u.reshape(3, N))
        if f:
            out["f"] = fp.reshape(19, N)
        return out

    def qhist(self):
        ln = C.c_int64()
        self._check(self._lib.lbe_observables(self.h, None, None, None, None, None, None, 0,
                                              C.byref(ln)))
        rows = ln.value
        out = np.empty(max(rows * self.ne, 1))
        self._check(self._lib.lbe_observables(self.h, None, None, None, None, None, _dptr(out),
                                              rows, None))
        return out[: rows * self.ne].reshape(rows, self.ne)

    def profile(self, enable=True):
        self._check(self._lib.lbe_profile(self.h, 1 if enable else 0))

    def pass_blocks(self):
        """(block of pass A, block of pass B (1: LDS tiles), non-temporal
        streams: bit 0 pass A, bit 1 pass B) as the context chose them."""
        a, b, nt = C.c_int32(), C.c_int32(), C.c_int32()
        self._check(self._lib.lbe_launch_shape(self.h, C.byref(a), C.byref(b), C.byref(nt)))
        return a.value, b.value, nt.value

    def kernel_times(self):
        """{kind: (total ms, launches, cells covered)} since profile(True)."""
        n = self._lib.lbe_num_kernel_kinds()
        ms = np.zeros(n)
        cnt = np.zeros(n, dtype=np.int64)
        cells = np.zeros(n, dtype=np.int64)
        i64 = C.POINTER(C.c_int64)
        self._check(self._lib.lbe_kernel_times(self.h, _dptr(ms), cnt.ctypes.data_as(i64),
                                               cells.ctypes.data_as(i64), n))
        return {kernel_names()[k]: (float(ms[k]), int(cnt[k]), int(cells[k])) for k in range(n)}
