"""Multigrid Poisson (LBE_MG) on the GPU against the FP64 oracle's SOR.

Both solve the same linear system (Eq. 2 with the Laplacian of Eq. 15) to a
residual tol; they differ by at most |A^-1| tol in the potential.  For a gap
of L lattice units |A^-1| <= L^2/8, so with tol = 1e-14 and L <= 32 the
potentials agree to 1.3e-11 absolute; the tests allow 2e-11 relative to the
electrode voltage scale 0.1 for phi and the same relative bound for n, f.
The electrode charge is set by the potential drop between the wall and the
first fluid plane, about dV/(2L) = 1.6e-3 here, so its bound is
1.3e-11 / 1.6e-3 ~ 1e-8 relative.
"""
import numpy as np
import pytest

import gpu_cases as G
import oracle
import paper_1907_04732_amd as lbe
import workloads as W
from test_gpu_parity import U_SCALE, rel, residual_numpy

pytestmark = pytest.mark.gpu

MG_TOL = 2e-11
MG_QTOL = 1e-8


def mg_pair(name, tol=1e-14, steps=None, **sweeps):
    kw, shape, t, ps, n0, nref, nsteps, _ = G.case(name)
    o = oracle.Oracle(oracle.make_params(shape, **kw, tol=tol, max_iter=10**6, check_every=1), t,
                      ps, n0, nref)
    nu = dict(mg_nu1=2, mg_nu2=2)
    nu.update(sweeps)
    g = lbe.Lbe(lbe.make_params(shape, **kw, tol=tol, max_iter=200, poisson=lbe.MG, mg_levels=0,
                                **nu), t, ps, n0, nref)
    return o, g, (nsteps if steps is None else steps), t


@pytest.mark.parametrize("sweeps", [dict(mg_nu1_coarse=1, mg_nu2_coarse=1),
                                    dict(mg_nu1=1, mg_nu2=3, mg_nu1_coarse=3, mg_nu2_coarse=1)])
@pytest.mark.parametrize("name", ["slab_4x4x34", "coax_16x16x4"])
def test_mg_sweep_counts_same_fixed_point(name, sweeps):
    """Other smoothing counts (odd ones, and fewer sweeps on the coarser
    levels) change the cycle, not its fixed point: the oracle's within the
    multigrid bounds."""
    o, g, nsteps, t = mg_pair(name, **sweeps)
    o.step(nsteps)
    g.step(nsteps)
    fo, fg = o.fields(), g.fields()
    assert rel(fg["phi"], fo["phi"], 0.1) <= MG_TOL
    assert rel(fg["n"], fo["n"]) <= MG_TOL
    assert rel(g.qhist(), o.qhist()) <= MG_QTOL


@pytest.mark.parametrize("name", ["slab_4x4x34", "coax_16x16x4", "random_6x10x14_k3",
                                  "slab_1x1x34"])
def test_mg_matches_oracle(name):
    o, g, nsteps, t = mg_pair(name)
    o.step(nsteps)
    g.step(nsteps)
    fo, fg = o.fields(), g.fields()
    vscale = 0.1
    errs = dict(phi=rel(fg["phi"], fo["phi"], vscale), n=rel(fg["n"], fo["n"]),
                f=rel(fg["f"], fo["f"]), q=rel(g.qhist(), o.qhist()),
                u=rel(fg["u"], fo["u"], max(np.abs(fo["u"]).max(), U_SCALE)))
    tot = g.totals()
    print(name, {k: f"{v:.2e}" for k, v in errs.items()}, "cycles", tot["poisson_iters"])
    for k, v in errs.items():
        assert v <= (MG_QTOL if k == "q" else MG_TOL), (k, errs)
    assert tot["poisson_resid"] <= 1e-14


def test_mg_converges_fast_on_full_slab():
    """64x64x130 electro-osmosis slab at the production tolerance: the
    multigrid solve reaches ||R|| <= 1e-10 in a few V-cycles per step, and the
    returned potential satisfies Poisson's equation (residual recomputed)."""
    w = W.eo_slab(noise=True)
    p = lbe.make_params(w.shape, w.z, w.D, w.lB, tau=w.tau, Eapp=w.Eapp, omega=w.omega,
                        tol=1e-10, max_iter=100, poisson=lbe.MG, mg_levels=0)
    g = lbe.Lbe(p, w.node_type, w.phi_s, w.n_init, w.n_ref)
    init_cycles = g.totals()["poisson_iters"]
    cyc = []
    for _ in range(5):
        g.step(1)
        cyc.append(g.totals()["poisson_iters"])
    print("init cycles", init_cycles, "per step", cyc)
    assert init_cycles <= 40 and max(cyc) <= 10
    fg = g.fields(f=False)
    R = residual_numpy(w.shape, w.node_type, fg["phi"], fg["n"], w.z, w.lB)
    assert np.abs(R).max() <= 1.01e-10


def test_mg_and_sor_agree_on_full_slab():
    """FP64 SOR and multigrid from the same input, 2 steps at tol 1e-12."""
    w = W.eo_slab(noise=True)
    common = dict(tau=w.tau, Eapp=w.Eapp, omega=1.9, tol=1e-12)
    a = lbe.Lbe(lbe.make_params(w.shape, w.z, w.D, w.lB, max_iter=10**6, **common), w.node_type,
                w.phi_s, w.n_init, w.n_ref)
    b = lbe.Lbe(lbe.make_params(w.shape, w.z, w.D, w.lB, max_iter=200, poisson=lbe.MG, **common),
                w.node_type, w.phi_s, w.n_init, w.n_ref)
    a.step(2)
    b.step(2)
    fa, fb = a.fields(f=False), b.fields(f=False)
    # |A^-1| <= L^2/8 = 2048 for the 128-plane gap: 2e-9 absolute on phi
    assert rel(fb["phi"], fa["phi"], 0.2) <= 2e-8
    assert rel(fb["n"], fa["n"]) <= 2e-8


@pytest.mark.parametrize("precision", [lbe.FP64, lbe.FP32_MIXED])
def test_extrapolated_warm_start_same_fixed_point(precision):
    """LBE_EXTRAPOLATE only changes the initial guess of each solve
    (3 phi(t) - 3 phi(t-1) + phi(t-2)); at tol = 1e-13 the trajectory matches
    the FP64 oracle to the solver-tolerance bound (FP32 bars for the mixed
    form), with fewer cycles than the plain warm start from phi(t)."""
    kw, shape, t, ps, n0, nref, _, _ = G.case("slab_4x4x34")
    o = oracle.Oracle(oracle.make_params(shape, **kw, tol=1e-13, max_iter=10**6, check_every=1),
                      t, ps, n0, nref)
    g = lbe.Lbe(lbe.make_params(shape, **kw, tol=1e-13, max_iter=200, poisson=lbe.MG,
                                precision=precision, flags=lbe.EXTRAPOLATE), t, ps, n0, nref)
    plain = lbe.Lbe(lbe.make_params(shape, **kw, tol=1e-13, max_iter=200, poisson=lbe.MG,
                                    precision=precision), t, ps, n0, nref)
    o.step(300)
    g.step(300)
    plain.step(300)
    fo, fg = o.fields(), g.fields(f=False)
    tol = 1e-10 if precision == lbe.FP64 else 1e-5
    assert rel(fg["phi"], fo["phi"], 0.1) <= tol
    assert rel(g.qhist(), o.qhist()) <= tol
    cyc, cyc_plain = g.totals()["poisson_total"], plain.totals()["poisson_total"]
    print("cycles in 300 steps: extrapolated", cyc, "plain", cyc_plain)
    assert cyc < cyc_plain


@pytest.mark.parametrize("name", ["slab_4x4x34", "coax_16x16x4", "random_6x10x14_k3"])
def test_krylov_matches_oracle(name):
    """LBE_KRYLOV (V-cycle preconditioned flexible CG) solves the same system
    to the same tolerance: the oracle's SOR fixed point within the MG bounds."""
    kw, shape, t, ps, n0, nref, nsteps, _ = G.case(name)
    kw = dict(kw)
    flags = kw.pop("flags", 0)
    o = oracle.Oracle(oracle.make_params(shape, **kw, flags=flags, tol=1e-14, max_iter=10**6,
                                         check_every=1), t, ps, n0, nref)
    g = lbe.Lbe(lbe.make_params(shape, **kw, flags=flags | lbe.KRYLOV, tol=1e-14, max_iter=200,
                                poisson=lbe.MG), t, ps, n0, nref)
    o.step(nsteps)
    g.step(nsteps)
    fo, fg = o.fields(), g.fields()
    errs = dict(phi=rel(fg["phi"], fo["phi"], 0.1), n=rel(fg["n"], fo["n"]),
                f=rel(fg["f"], fo["f"]), q=rel(g.qhist(), o.qhist()))
    print(name, {k: f"{v:.2e}" for k, v in errs.items()}, "cycles", g.totals()["poisson_iters"])
    for k, v in errs.items():
        assert v <= (MG_QTOL if k == "q" else MG_TOL), (k, errs)
    assert g.totals()["poisson_resid"] <= 1e-14


def test_krylov_mixed_form_extrapolated():
    """Mixed form with Krylov acceleration and the extrapolated warm start
    (the production combination) against the oracle: FP32 bars."""
    kw, shape, t, ps, n0, nref, _, _ = G.case("slab_4x4x34")
    o = oracle.Oracle(oracle.make_params(shape, **kw, tol=1e-13, max_iter=10**6, check_every=1),
                      t, ps, n0, nref)
    g = lbe.Lbe(lbe.make_params(shape, **kw, tol=1e-13, max_iter=200, poisson=lbe.MG,
                                precision=lbe.FP32_MIXED,
                                flags=lbe.EXTRAPOLATE | lbe.KRYLOV), t, ps, n0, nref)
    o.step(300)
    g.step(300)
    fo, fg = o.fields(), g.fields(f=False)
    assert rel(fg["phi"], fo["phi"], 0.1) <= 1e-5
    assert rel(g.qhist(), o.qhist()) <= 1e-5


def test_krylov_fewer_cycles_on_the_coaxial_cell():
    """160x160x64 coaxial cell, mixed form, warm start from phi(t): the
    curved electrodes are poorly represented on coarse levels, so plain
    V-cycles converge slowly; with the Krylov acceleration fewer cycles per
    step reach the same tolerance, and the potential agrees to the solver
    bound."""
    w = W.coaxial(noise=True)
    res = {}
    for flags in (0, lbe.KRYLOV):
        p = lbe.make_params(w.shape, w.z, w.D, w.lB, tau=w.tau, Eapp=w.Eapp, omega=w.omega,
                            tol=1e-10, max_iter=200, precision=lbe.FP32_MIXED, poisson=lbe.MG,
                            flags=flags)
        g = lbe.Lbe(p, w.node_type, w.phi_s, w.n_init, w.n_ref)
        t0 = g.totals()["poisson_total"]
        g.step(20)
        res[flags] = ((g.totals()["poisson_total"] - t0) / 20, g.fields(f=False)["phi"])
    plain, kry = res[0][0], res[lbe.KRYLOV][0]
    print("cycles per step: V-cycles", plain, "Krylov", kry)
    assert kry < plain
    # |A^-1| <= (R2 - R1)^2 / 8 ~ 512 for the 64-wide gap: 5e-8 on phi at tol 1e-10
    assert rel(res[lbe.KRYLOV][1], res[0][1], 0.1) <= 1e-6


@pytest.mark.parametrize("geometry", ["slab", "random"])
@pytest.mark.parametrize("precision", [lbe.FP32_MIXED, lbe.FP64])
def test_tiled_kernels_match_untiled(geometry, precision, monkeypatch):
    """On levels wide enough for it the restriction runs in row order with
    the children of a coarse cell combined in LDS, claiming the eight-lane
    kernel's values and summation order; a run with it (the default) and one
    without (LBE_NO_TILES=1) must agree bit for bit, here on a 64 x 8 x 34
    lattice (both restrictions below it are tiled)."""
    if geometry == "slab":
        shape, t, ps = W.slab(64, 8, 32, 1, 0.05, -0.05)
        flags = lbe.EXTRAPOLATE
    else:
        shape = (64, 8, 34)
        t, ps = G.random_geometry(shape, 3, seed=13, fill=0.12)
        # plain cycles can diverge around blobs: Krylov acceleration
        flags = lbe.EXTRAPOLATE | lbe.ALLOW_FLOATING | lbe.KRYLOV
    rs = W.salt_for_debye(4.0, G.LB)
    n0 = W.noisy_concentrations(t, [rs, rs], 1e-2, seed=8)
    p = dict(z=(1, -1), D=(0.05, 0.08), lB=G.LB, tau=0.9, Eapp=(1e-3, 0.0, 5e-4), tol=1e-11,
             max_iter=1000, precision=precision, poisson=lbe.MG, flags=flags)
    out = []
    for no_tiles in ("0", "1"):
        monkeypatch.setenv("LBE_NO_TILES", no_tiles)
        g = lbe.Lbe(lbe.make_params(shape, **p), t, ps, n0, (rs, rs))
        g.step(12)
        out.append((g.fields(), g.qhist(), g.totals()["poisson_total"]))
        g.close()
    (fa, qa, ia), (fb, qb, ib) = out
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k
    assert np.array_equal(qa, qb) and ia == ib


@pytest.mark.parametrize("geometry", ["slab", "random"])
@pytest.mark.parametrize("precision", [lbe.FP32_MIXED, lbe.FP64])
@pytest.mark.parametrize("cycle", ["V(2,2)", "V(1,1)"])
def test_coarse_first_sweep_in_restriction_same_results(geometry, precision, cycle, monkeypatch):
    """A correction that starts from zero makes the first Jacobi sweep
    pointwise, so the kernel writing a level's right-hand side writes it (the
    restriction on coarse levels; on the finest level the residual check,
    and under Krylov acceleration the update kernel); a run with that (the
    default) and one with every such sweep as its own launch
    (LBE_NO_COARSE_START=1) must agree bit for bit.  On 64 x 64 x 34 the two
    levels below the finest (32 x 32 x 17, 16 x 16 x 9) are smoothed by the
    global kernels and the rest by the one-work-group kernel."""
    shape = (64, 64, 34)
    if geometry == "slab":
        _, t, ps = W.slab(64, 64, 32, 1, 0.05, -0.05)
        flags = lbe.EXTRAPOLATE
    else:
        t, ps = G.random_geometry(shape, 3, seed=29, fill=0.12)
        flags = lbe.EXTRAPOLATE | lbe.ALLOW_FLOATING | lbe.KRYLOV
    rs = W.salt_for_debye(4.0, G.LB)
    n0 = W.noisy_concentrations(t, [rs, rs], 1e-2, seed=9)
    nu = 1 if cycle == "V(1,1)" else 2
    p = dict(z=(1, -1), D=(0.05, 0.08), lB=G.LB, tau=0.9, Eapp=(1e-3, 0.0, 5e-4), tol=1e-11,
             max_iter=1000, precision=precision, poisson=lbe.MG, flags=flags, mg_nu1=nu,
             mg_nu2=nu, mg_nu1_coarse=nu, mg_nu2_coarse=nu)
    out = []
    for off in ("0", "1"):
        monkeypatch.setenv("LBE_NO_COARSE_START", off)
        g = lbe.Lbe(lbe.make_params(shape, **p), t, ps, n0, (rs, rs))
        g.step(10)
        out.append((g.fields(), g.qhist(), g.totals()["poisson_total"]))
        g.close()
    (fa, qa, ia), (fb, qb, ib) = out
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k
    assert np.array_equal(qa, qb) and ia == ib


@pytest.mark.parametrize("precision", [lbe.FP64, lbe.FP32_MIXED])
@pytest.mark.parametrize("solver", ["mg", "mg+krylov", "sor"])
def test_fixed_iteration_count_follows_the_tolerance_schedule(solver, precision):
    """tol <= 0 runs exactly max_iter cycles (or sweeps) with the residual
    checks of a tolerance-driven solve between them (the defect correction's
    V-cycle, the mixed SOR sweeps and the Krylov iteration take their
    right-hand side from the check before them).  So a solve at tol = 0 with
    max_iter = k must give the potential, bit for bit, of the same solve at a
    tolerance it cannot reach, stopped by the same limit (LBE_ENOCONV), and
    the residual must have fallen.  A 64 x 8 x 34 slab with 1% noise on the
    concentrations, so the finest level and the one below it run in the
    global multigrid kernels."""
    shape, t, ps = W.slab(64, 8, 32, 1, 0.05, -0.05)
    rs = W.salt_for_debye(4.0, G.LB)
    n0 = W.noisy_concentrations(t, [rs, rs], 1e-2, seed=8)
    flags = lbe.KRYLOV if solver == "mg+krylov" else 0
    k = 3 if solver != "sor" else 12
    p = dict(z=(1, -1), D=(0.05, 0.08), lB=G.LB, tau=0.9, Eapp=(1e-3, 0.0, 5e-4),
             tol=1e-4, max_iter=5000, check_every=4, precision=precision,
             poisson=lbe.SOR4 if solver == "sor" else lbe.MG, flags=flags)
    out = []
    for tol in (0.0, 1e-300):
        g = lbe.Lbe(lbe.make_params(shape, **p), t, ps, n0, (rs, rs))
        r0 = g.totals()["poisson_resid"]
        g.set_solver(tol=tol, max_iter=k)
        if tol > 0:
            with pytest.raises(lbe.LbeError) as ei:
                g.poisson()
            assert ei.value.code == lbe.ENOCONV
        else:
            it, _ = g.poisson()
            assert it == k
        tot = g.totals()
        out.append((g.fields(f=False)["phi"], tot["poisson_iters"], tot["poisson_resid"], r0))
        g.close()
    (pa, ia, ra, r0), (pb, ib, rb, _) = out
    print(solver, precision, "residual", r0, "->", ra, "iterations", ia, ib)
    assert ia == ib == k
    assert np.array_equal(pa, pb)
    assert ra == rb and ra < r0


@pytest.mark.parametrize("solver", ["mg", "mg+krylov", "sor"])
@pytest.mark.parametrize("precision", [lbe.FP32_MIXED, lbe.FP64])
def test_die_contiguous_block_order_same_results(solver, precision, monkeypatch):
    """The LB pass, the residual checks and the Krylov operator hand each of
    the part's eight dies the same eighth of every plane (neighbouring rows
    and planes then share one L2); the map is a bijection and reduction
    partials keep their logical order, so a run with it (the default) and
    one without (LBE_NO_XCD_MAP=1) must agree bit for bit, on a 64 x 64 x 34
    lattice with random electrodes (a slab for plain cycles)."""
    shape = (64, 64, 34)
    t, ps = G.random_geometry(shape, 3, seed=31, fill=0.1)
    rs = W.salt_for_debye(4.0, G.LB)
    n0 = W.noisy_concentrations(t, [rs, rs], 1e-2, seed=4)
    flags = lbe.EXTRAPOLATE | lbe.ALLOW_FLOATING
    if solver == "mg+krylov":
        flags |= lbe.KRYLOV
    p = dict(z=(1, -1), D=(0.05, 0.08), lB=G.LB, tau=0.9, Eapp=(1e-3, 0.0, 5e-4),
             tol=1e-10 if solver == "sor" else 1e-11, max_iter=100000, precision=precision,
             poisson=lbe.SOR4 if solver == "sor" else lbe.MG, flags=flags)
    if solver == "mg":
        # plain cycles diverge around random blobs: a slab in the same box
        _, t, ps = W.slab(64, 64, 32, 1, 0.05, -0.05)
        n0 = W.noisy_concentrations(t, [rs, rs], 1e-2, seed=4)
        p["flags"] = lbe.EXTRAPOLATE
    out = []
    for off in ("0", "1"):
        monkeypatch.setenv("LBE_NO_XCD_MAP", off)
        g = lbe.Lbe(lbe.make_params(shape, **p), t, ps, n0, (rs, rs))
        g.step(6)
        out.append((g.fields(), g.qhist(), g.totals()["poisson_total"]))
        g.close()
    (fa, qa, ia), (fb, qb, ib) = out
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k
    assert np.array_equal(qa, qb) and ia == ib


@pytest.mark.parametrize("solver", ["mg", "mg+krylov"])
@pytest.mark.parametrize("precision", [lbe.FP32_MIXED, lbe.FP64])
@pytest.mark.parametrize("shape,zrun", [((64, 64, 34), 16), ((128, 8, 22), 5)])
def test_plane_ring_stencils_same_results(solver, precision, shape, zrun, monkeypatch):
    """On a level whose nx is a multiple of 64 and ny of 4, the residual
    check, the Jacobi sweeps and the Krylov operator can stage their
    gathered array in LDS planes (a tile marching along z through a run of
    planes; on their own they do so on levels large enough to fill the
    part, so here the run length is forced, with z extents that leave a
    ragged last run, and on 128 x 8 x 22 the level below fits too).  A cell
    sees the values the global gathers load, so with plain cycles a run with
    the rings and one without (LBE_NO_RINGS=1) agree bit for bit.  The
    Krylov sums then add a block's cells plane by plane, another order: the
    two runs take the same number of cycles and agree to rounding."""
    nx, ny, nz = shape
    rs = W.salt_for_debye(4.0, G.LB)
    if solver == "mg":
        _, t, ps = W.slab(nx, ny, nz - 2, 1, 0.05, -0.05)
        flags = lbe.EXTRAPOLATE
    else:
        t, ps = G.random_geometry(shape, 3, seed=37, fill=0.1)
        flags = lbe.EXTRAPOLATE | lbe.ALLOW_FLOATING | lbe.KRYLOV
    n0 = W.noisy_concentrations(t, [rs, rs], 1e-2, seed=6)
    p = dict(z=(1, -1), D=(0.05, 0.08), lB=G.LB, tau=0.9, Eapp=(1e-3, 0.0, 5e-4), tol=1e-11,
             max_iter=1000, precision=precision, poisson=lbe.MG, flags=flags)
    out = []
    monkeypatch.setenv("LBE_RING_ZRUN", str(zrun))
    for off in ("0", "1"):
        monkeypatch.setenv("LBE_NO_RINGS", off)
        g = lbe.Lbe(lbe.make_params(shape, **p), t, ps, n0, (rs, rs))
        g.step(8)
        out.append((g.fields(), g.qhist(), g.totals()["poisson_total"]))
        g.close()
    (fa, qa, ia), (fb, qb, ib) = out
    print(shape, solver, precision, "cycles", ia, ib)
    if solver == "mg":
        for k in fa:
            assert np.array_equal(fa[k], fb[k]), k
        assert np.array_equal(qa, qb) and ia == ib
    else:
        assert ia == ib
        assert rel(fa["phi"], fb["phi"], 0.1) <= 1e-9
        assert np.abs(qa - qb).max() <= 1e-9 * np.abs(qb).max()


@pytest.mark.parametrize("precision", [lbe.FP32_MIXED, lbe.FP64])
@pytest.mark.parametrize("shape", [(64, 8, 24), (128, 16, 36), (96, 12, 20)])
def test_tiled_step_passes_same_bits(monkeypatch, shape, precision):
    """The step passes on LDS-staged tiles of 32 x 8 nodes marching through
    runs of 8 planes do the arithmetic of the per-node kernels on the same
    values: pass B with the velocity and concentrations (deviations in the
    mixed form) of three planes in LDS (with a periodic halo), in both
    forms; pass A with the potential and deviations, in the mixed form.  So
    a run forced onto them where they fit (LBE_PASS_TILE=1) and one kept off
    them (LBE_PASS_TILE=0) must agree bit for bit: random electrodes, an
    applied field, two species of unequal D, the quadratic warm start.
    64 x 8 x 24 and 128 x 16 x 36 (four tiles across x, two along y, a last
    run of 4 planes) take them; 96 x 12 x 20 does not."""
    fit = shape[0] % 32 == 0 and shape[1] % 8 == 0
    fit_a, fit_b = fit and precision == lbe.FP32_MIXED, fit
    t, ps = G.random_geometry(shape, 3, seed=7, fill=0.1)
    rs = W.salt_for_debye(4.0, G.LB)
    n0 = W.noisy_concentrations(t, [rs, rs], 1e-2, seed=5)
    p = lbe.make_params(shape, (1, -1), (0.05, 0.08), G.LB, tau=0.9, Eapp=(1e-3, 0.0, 5e-4),
                        tol=1e-11, max_iter=100000, precision=precision, poisson=lbe.MG,
                        flags=lbe.EXTRAPOLATE | lbe.ALLOW_FLOATING | lbe.KRYLOV)
    out = []
    for tile in ("1", "0"):
        monkeypatch.setenv("LBE_PASS_TILE", tile)
        g = lbe.Lbe(p, t, ps, n0, (rs, rs))
        blk_a, blk_b, _ = g.pass_blocks()
        assert (blk_a == 1) == (tile == "1" and fit_a) and (blk_b == 1) == (tile == "1" and fit_b)
        g.step(8)
        out.append((g.fields(), g.qhist(), g.totals()))
        g.close()
    (fa, qa, ta), (fb, qb, tb) = out
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k
    assert np.array_equal(qa, qb) and ta["poisson_total"] == tb["poisson_total"]
    assert ta["nk"] == tb["nk"]
