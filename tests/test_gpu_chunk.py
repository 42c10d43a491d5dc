"""Time steps replayed from captured graphs (lbe_step_chunk): 16 whole steps,
each with a fixed number of solver units gated on the device's stop flag,
captured once and replayed without the host waiting between steps.  When
every replayed solve converges within its units, the result is the same bit
for bit as stepping one by one (lbe_step), whose parity with the oracle the
other tests establish; a solve that does not converge is reported after the
replays."""
import numpy as np
import pytest

import gpu_cases as G
import paper_1907_04732_amd as lbe
import workloads as W

pytestmark = pytest.mark.gpu


def small_batch():
    return W.batch_slabs(nsys=5, nxy=4, Lmin=16, Lmax=40, dmin=2.0, dmax=16.0, seed=7)


def batch_ctx(b, **kw):
    p = lbe.make_params(b.shape, b.z, b.D, b.lB, tau=b.tau, omega=1.8, **kw)
    return lbe.Lbe(p, b.node_type, b.phi_s, b.n_init, b.n_ref.reshape(-1), system=b.system,
                   nsys=len(b.L))


def same_state(g1, g2):
    f1, f2 = g1.fields(), g2.fields()
    for k in ("phi", "n", "u", "f"):
        assert np.array_equal(f1[k], f2[k]), k
    assert np.array_equal(g1.qhist(), g2.qhist())
    t1, t2 = g1.totals(), g2.totals()
    assert t1["step"] == t2["step"]
    assert t1["poisson_total"] == t2["poisson_total"]


@pytest.mark.parametrize("precision", [lbe.FP64, lbe.FP32_MIXED])
@pytest.mark.parametrize("krylov", [False, True])
def test_chunk_same_bits_as_steps(precision, krylov):
    """Batch of five slabs, multigrid with the extrapolated start (the
    benchmark's solver): two first steps one by one (the extrapolation
    history fills), two replays of 16 steps, five more one by one; then a
    second call on the same graph.  Everything equal to lbe_step."""
    b = small_batch()
    flags = lbe.EXTRAPOLATE | (lbe.KRYLOV if krylov else 0)
    kw = dict(tol=1e-10, max_iter=200, poisson=lbe.MG, precision=precision, flags=flags)
    g1, g2 = batch_ctx(b, **kw), batch_ctx(b, **kw)
    print(f"chunk parity: batch {b.shape}, precision {precision}, krylov {krylov}", flush=True)
    g1.step(39)
    g2.step_chunk(39, units=24)
    same_state(g1, g2)
    g1.step(32)
    g2.step_chunk(32, units=24)
    same_state(g1, g2)


def test_chunk_on_a_curved_lattice_same_bits():
    """Random electrodes at three potentials (blobs across the periodic
    boundary), three species with a divalent one, FP32-mixed, multigrid with
    Krylov acceleration on a lattice large enough for the global multigrid
    kernels."""
    shape = (40, 36, 24)
    t, ps = G.random_geometry(shape, 3, seed=11, fill=0.15)
    rs = np.array([2e-3, 3e-3, 0.5e-3])
    n0 = W.noisy_concentrations(t, rs, 5e-2, seed=12)
    p = lbe.make_params(shape, (1, -1, 2), (0.05, 0.03, 0.02), G.LB, tau=0.9,
                        Eapp=(2e-3, -1e-3, 5e-4), tol=1e-10, max_iter=200, poisson=lbe.MG,
                        precision=lbe.FP32_MIXED,
                        flags=lbe.ALLOW_FLOATING | lbe.EXTRAPOLATE | lbe.KRYLOV)
    print(f"chunk parity: random geometry {shape}", flush=True)
    g1 = lbe.Lbe(p, t, ps, n0, tuple(rs))
    g2 = lbe.Lbe(p, t, ps, n0, tuple(rs))
    g1.step(34)
    g2.step_chunk(34, units=24)
    same_state(g1, g2)


def test_chunk_with_the_papers_sor_same_bits():
    """FP64 four-colour SOR (the paper's solver, the path the oracle
    reproduces sweep for sweep), four sweeps per unit: replayed steps equal
    lbe_step bit for bit."""
    kwc, shape, t, ps, n0, nref, _, _ = G.case("slab_4x4x34")
    kwc = dict(kwc)
    kwc.update(tol=1e-10, max_iter=2000, check_every=4)
    print("chunk parity: slab 4x4x34, FP64 SOR", flush=True)
    g1 = lbe.Lbe(lbe.make_params(shape, **kwc), t, ps, n0, nref)
    g2 = lbe.Lbe(lbe.make_params(shape, **kwc), t, ps, n0, nref)
    g1.step(35)
    g2.step_chunk(35, units=150)
    same_state(g1, g2)


def test_chunk_graph_kept_across_a_potential_change():
    """A new set of electrode potentials restarts the extrapolation history:
    the next call takes two steps one by one and then replays the graph
    captured before the change (same buffers, same unit count)."""
    b = small_batch()
    kw = dict(tol=1e-10, max_iter=200, poisson=lbe.MG, precision=lbe.FP32_MIXED,
              flags=lbe.EXTRAPOLATE | lbe.KRYLOV)
    g1, g2 = batch_ctx(b, **kw), batch_ctx(b, **kw)
    print(f"chunk parity: batch {b.shape}, potential change between calls", flush=True)
    g1.step(18)
    g2.step_chunk(18, units=24)
    same_state(g1, g2)
    ps = np.where(b.node_type > 0, 1.5 * b.phi_s, 0.0)
    g1.set_electrode_potential(ps)
    g2.set_electrode_potential(ps)
    g1.step(34)
    g2.step_chunk(34, units=24)
    same_state(g1, g2)


def test_chunk_reports_an_unconverged_solve():
    """SOR with one sweep per unit and a single unit per step cannot reach
    1e-10: the replays run to the end and the call reports LBE_ENOCONV, with
    the step count advanced by the replayed steps."""
    kwc, shape, t, ps, n0, nref, _, _ = G.case("slab_4x4x34")
    kwc = dict(kwc)
    kwc.update(tol=1e-10, max_iter=1000, check_every=1)
    print("chunk error path: slab 4x4x34, SOR, one sweep per step", flush=True)
    g = lbe.Lbe(lbe.make_params(shape, **kwc), t, ps, n0, nref)
    s0 = g.totals()["step"]
    with pytest.raises(lbe.LbeError) as ei:
        g.step_chunk(20, units=1)
    assert ei.value.code == lbe.ENOCONV
    assert g.totals()["step"] == s0 + 16
    # every replayed step still appended the charges of its last potential
    assert np.isfinite(g.qhist()).all()
    with pytest.raises(lbe.LbeError) as ei:
        g.step_chunk(16, units=0)
    assert ei.value.code == lbe.EINVAL
    g.set_solver(tol=0.0, max_iter=10)
    with pytest.raises(lbe.LbeError) as ei:
        g.step_chunk(16, units=1)
    assert ei.value.code == lbe.EINVAL
    g.set_solver(tol=1e-10, max_iter=2000)
    g.step(1)  # the context still steps one by one after a failed replay
