"""lbe_electrode_charge_noalloc (the allocation-free entry point, for
callers that cannot allocate device memory) against lbe_electrode_charge of
a context holding the same potential: the same Gauss's-law charges (Eq. 16)
to FP64 rounding, on two calls in a row, the second on a smaller lattice
with fewer electrodes and the first-order wall factor, so that nothing of
the first call's scratch contents can stand in for the second's."""
import numpy as np
import pytest

import gpu_cases as G
import paper_1907_04732_amd as lbe
import workloads as W

pytestmark = pytest.mark.gpu

# FP64: both sides form each node's term by the same expression and sum the
# terms with compensation, in different orders
RTOL = 1e-12


def _context_and_fields(shape, nelec, seed, naive):
    import torch

    t, ps = G.random_geometry(shape, nelec, seed=seed, fill=0.15)
    rs = W.salt_for_debye(3.0, G.LB)
    n0 = W.noisy_concentrations(t, [rs, rs], 5e-2, seed=seed + 1)
    # Krylov acceleration: plain V-cycles can diverge around random blobs
    flags = lbe.ALLOW_FLOATING | lbe.KRYLOV | (lbe.NAIVE_DIRICHLET if naive else 0)
    g = lbe.Lbe(lbe.make_params(shape, (1, -1), (0.05, 0.08), G.LB, tau=0.9, Eapp=(1e-3, 0, 0),
                                tol=1e-12, max_iter=400, poisson=lbe.MG, flags=flags),
                t, ps, n0, (rs, rs))
    g.step(6)
    q_ref = g.electrode_charge()
    phi = g.fields(f=False, device="cuda")["phi"]
    g.close()
    return torch.tensor(t, dtype=torch.uint8, device="cuda"), phi, q_ref


def test_noalloc_charge_matches_context_charge_twice():
    import torch

    for shape, nelec, seed, naive in (((24, 20, 18), 3, 21, False), ((8, 6, 10), 2, 9, True)):
        t_d, phi_d, q_ref = _context_and_fields(shape, nelec, seed, naive)
        ne = len(q_ref)
        assert ne == nelec
        q_d = torch.full((ne,), float("nan"), dtype=torch.float64, device="cuda")
        lbe.electrode_charge_noalloc(shape, G.LB, t_d, phi_d, q_d, naive=naive)
        torch.cuda.synchronize()
        q = q_d.cpu().numpy()
        err = np.abs(q - q_ref).max() / np.abs(q_ref).max()
        print(shape, "charges", q, "context", q_ref, "relative difference", err)
        assert np.all(np.isfinite(q)) and err <= RTOL


def test_noalloc_charge_rejects_bad_arguments():
    import torch

    shape = (4, 4, 6)
    t_d = torch.zeros(96, dtype=torch.uint8, device="cuda")
    phi_d = torch.zeros(96, dtype=torch.float64, device="cuda")
    lib = lbe.load()
    for ne in (0, lbe.NOALLOC_MAX_ELECTRODES + 1):
        q_d = torch.zeros(max(ne, 1), dtype=torch.float64, device="cuda")
        with pytest.raises(lbe.LbeError) as ei:
            lbe.electrode_charge_noalloc(shape, G.LB, t_d, phi_d, q_d[:ne] if ne else q_d[:0])
        assert ei.value.code == lbe.EINVAL
    # host memory for q: refused before anything is launched
    import ctypes as C
    q_h = np.zeros(2)
    rc = lib.lbe_electrode_charge_noalloc(4, 4, 6, G.LB, 0, C.c_void_p(t_d.data_ptr()),
                                          C.c_void_p(phi_d.data_ptr()),
                                          q_h.ctypes.data_as(C.c_void_p), 2, None)
    assert rc == lbe.EINVAL
    assert b"device memory" in lib.lbe_last_error(None)
