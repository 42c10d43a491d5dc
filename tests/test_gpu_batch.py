"""Many independent parallel-plate systems in one context (lbe_init_batch):
the parameter sweeps of Sec. III A (widths, Debye lengths, voltages) run as
one lattice whose every kernel launch advances all systems.  Checked against
the oracle on the same packed lattice, and against each system run alone."""
import numpy as np
import pytest

import oracle
import paper_1907_04732_amd as lbe
import workloads as W
from test_gpu_parity import compare, rel

pytestmark = pytest.mark.gpu


def small_batch():
    # Debye lengths 2..16: salt concentrations 64x apart
    return W.batch_slabs(nsys=5, nxy=4, Lmin=16, Lmax=40, dmin=2.0, dmax=16.0, seed=7)


def gpu_batch(b, **kw):
    p = lbe.make_params(b.shape, b.z, b.D, b.lB, tau=b.tau, omega=1.8, **kw)
    return lbe.Lbe(p, b.node_type, b.phi_s, b.n_init, b.n_ref.reshape(-1), system=b.system,
                   nsys=len(b.L))


def oracle_packed(b, **kw):
    p = oracle.make_params(b.shape, b.z, b.D, b.lB, tau=b.tau, omega=1.8, **kw)
    return oracle.Oracle(p, b.node_type, b.phi_s, b.n_init, None)


def test_batch_fp64_parity_with_oracle():
    """FP64 SOR, same sweeps: the packed lattice matches the oracle run on the
    same lattice to <= 1e-12 (the systems' electrodes are separate nodes, so
    the oracle needs nothing batch-specific)."""
    b = small_batch()
    kw = dict(tol=0.0, max_iter=60, check_every=4)
    o, g = oracle_packed(b, **kw), gpu_batch(b, **kw)
    compare(o, g, b.node_type)
    o.step(20)
    g.step(20)
    compare(o, g, b.node_type)


def _alone(b, s, **kw):
    """System s cut out of the packed lattice, electrodes renumbered 1, 2."""
    nxy = b.shape[0]
    z1 = b.z0[s] - 1
    z2 = b.z0[s + 1] - 1 if s + 1 < len(b.L) else b.shape[2]
    sl = slice(z1 * nxy * nxy, z2 * nxy * nxy)
    t = b.node_type[sl].copy()
    t[t == 2 * s + 1] = 1
    t[t == 2 * s + 2] = 2
    shape = (nxy, nxy, z2 - z1)
    n0 = b.n_init[:, sl]
    p = lbe.make_params(shape, b.z, b.D, b.lB, tau=b.tau, omega=1.8, **kw)
    return lbe.Lbe(p, t, b.phi_s[sl], n0, tuple(b.n_ref[s])), sl


@pytest.mark.parametrize("precision", [lbe.FP64, lbe.FP32_MIXED])
def test_batch_systems_are_independent(precision):
    """Each system of the packed run equals the same system run alone
    (multigrid at tol 1e-13): no coupling through the stacked electrodes,
    and in the mixed form each system keeps its own deviation reference.
    The two runs converge along different multigrid paths, so they agree to
    the solver bound: |A^-1| tol <= L^2/8 * 1e-13 = 2e-11 on phi (L <= 40),
    and on the charge, which is set by phi(first plane) - phi_s ~ V/(2L), to
    2e-11 / 1.2e-3 ~ 2e-8 relative."""
    b = small_batch()
    kw = dict(tol=1e-13, max_iter=200, poisson=lbe.MG, precision=precision)
    g = gpu_batch(b, **kw)
    g.step(30)
    fg = g.fields(f=False)
    qg = g.qhist()
    tol, qtol = (1e-10, 2e-8) if precision == lbe.FP64 else (1e-6, 1e-6)
    for s in range(len(b.L)):
        a, sl = _alone(b, s, **kw)
        a.step(30)
        fa = a.fields(f=False)
        assert rel(fg["phi"][sl], fa["phi"], 0.2) <= tol, s
        assert rel(fg["n"][:, sl], fa["n"]) <= tol, s
        assert rel(qg[:, 2 * s:2 * s + 2], a.qhist()) <= qtol, s


def test_batch_mixed_form_against_oracle():
    """FP32-mixed packed run against the FP64 oracle on the packed lattice at
    solver tolerance 1e-13: potential within 1e-5 of the largest voltage and
    every electrode's charge history within 1e-5 of its own scale, for salt
    concentrations 64x apart."""
    b = small_batch()
    o = oracle_packed(b, tol=1e-13, max_iter=10**6, check_every=1)
    g = gpu_batch(b, tol=1e-13, max_iter=200, poisson=lbe.MG, precision=lbe.FP32_MIXED)
    o.step(30)
    g.step(30)
    fo, fg = o.fields(), g.fields(f=False)
    assert rel(fg["phi"], fo["phi"], float(b.V.max())) <= 1e-5
    qo, qg = o.qhist(), g.qhist()
    for e in range(qo.shape[1]):
        assert rel(qg[:, e], qo[:, e]) <= 1e-5, e
    # concentrations relative to each system's own salt level
    for s in range(len(b.L)):
        m = (b.system == s) & (b.node_type == 0)
        assert rel(fg["n"][:, m], fo["n"][:, m]) <= 1e-5, s


@pytest.mark.parametrize("precision", [lbe.FP64, lbe.FP32_MIXED])
def test_batch_reverse_mode(precision):
    """Reverse mode on the packed lattice: the gradient of one system's
    charge is that system's own gradient (its run alone, same multigrid
    settings, to the solver bound) and exactly zero on every other system's
    nodes and on l_B's share from other systems (the systems do not couple,
    and the coarse levels never merge two of them)."""
    b = small_batch()
    kw = dict(tol=1e-13, max_iter=200, poisson=lbe.MG, precision=precision)
    g = gpu_batch(b, **kw)
    g.record(24, every=10)
    s = 2
    qbar = np.zeros(2 * len(b.L))
    qbar[2 * s] = 1.0  # bottom electrode of system s
    gr = g.adjoint(qbar)
    a, sl = _alone(b, s, **kw)
    a.record(24, every=10)
    ga = a.adjoint([1.0, 0.0])
    inside = np.zeros(b.node_type.size, bool)
    inside[sl] = True
    assert not gr["phi_s"][~inside].any() and not gr["n"][:, ~inside].any()
    assert not gr["f"][:, ~inside].any()
    tol = 1e-9 if precision == lbe.FP64 else 1e-5
    assert rel(gr["phi_s"][sl], ga["phi_s"]) <= tol
    assert rel(gr["n"][:, sl], ga["n"]) <= tol
    assert abs(gr["lB"] - ga["lB"]) <= tol * abs(ga["lB"])


@pytest.mark.parametrize("krylov", [False, True])
@pytest.mark.parametrize("precision", [lbe.FP64, lbe.FP32_MIXED])
def test_small_levels_split_by_system_same_results(precision, krylov, monkeypatch):
    """On the coarse levels that one work-group handles in LDS, independent
    systems (no fluid cell next to another system's, the exact coarsest solve
    block-diagonal) get a work-group each; every cell's arithmetic is that of
    one work-group doing all of them, so a run with the split (the default)
    and one without (LBE_NO_SMALL_GROUPS=1) must agree bit for bit.  24
    systems of 8 x 8 x L (L 16..64; the small levels are 1 x 1 columns whose
    systems wrap through the periodic boundary on some levels)."""
    b = W.batch_slabs(nsys=24, nxy=8, Lmin=16, Lmax=64, seed=11)
    flags = lbe.EXTRAPOLATE | (lbe.KRYLOV if krylov else 0)
    out = []
    for off in ("0", "1"):
        monkeypatch.setenv("LBE_NO_SMALL_GROUPS", off)
        g = gpu_batch(b, tol=1e-11, max_iter=400, precision=precision, poisson=lbe.MG,
                      flags=flags)
        g.step(8)
        out.append((g.fields(), g.qhist(), g.totals()["poisson_total"]))
        g.close()
    (fa, qa, ia), (fb, qb, ib) = out
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k
    assert np.array_equal(qa, qb) and ia == ib
