"""The FP64 oracle against closed forms and exact lattice identities (CPU)."""
import numpy as np
import pytest

import gpu_cases as G
import oracle
import oracle_pins as P
import workloads as W


def test_velocity_set():
    P.pin_velocity_set()


@pytest.mark.parametrize("layers,nxy", [(1, 4), (3, 2), (1, 1)])
def test_neutral_slab_linear_and_dielectric_charge(layers, nxy):
    P.pin_neutral_slab(layers, nxy)


def test_electrode_thickness_does_not_matter():
    # Sec. III A: 1 or 3 electrode layers give the same induced charge
    q1 = P.pin_neutral_slab(1, 2)
    q3 = P.pin_neutral_slab(3, 2)
    assert np.allclose(q1, q3, rtol=1e-12, atol=0)


def test_uniform_charge_exact_parabola():
    P.pin_uniform_charge()


def test_gauss_law_identity():
    P.pin_gauss_identity()


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_diffusion_decay(axis):
    P.pin_diffusion_decay(axis)


def test_diffusion_isotropy():
    P.pin_diffusion_isotropy()


def test_debye_relaxation():
    P.pin_debye_relaxation()


def test_advection_translation():
    P.pin_advection_translation()


def test_uniform_field_force_and_momentum():
    P.pin_uniform_field_force()


def test_shear_wave_viscosity():
    P.pin_shear_wave()


def test_charging_boltzmann_and_dh_profiles():
    o = P.pin_charging()
    P.pin_boltzmann(o)
    P.pin_dh_profiles(o)


def test_capacitance_second_order():
    P.pin_capacitance_order()


def test_eo_slab_profile():
    P.pin_eo_slab()


def test_coax_neutral_profile():
    P.pin_coax_neutral()


def test_conservation_with_field_and_noise():
    """Mass and per-species ion number are conserved to rounding (Sec. I: the
    link fluxes are antisymmetric, bounce-back returns every population)."""
    rs = W.salt_for_debye(4.0, P.LB)
    shape, t, ps = W.coax(12, 12, 4, 2.0, 5.0, 0.1, -0.1)
    n0 = W.noisy_concentrations(t, [rs, rs], 1e-2, seed=11)
    o = P._run(shape, t, ps, (1, -1), (0.05, 0.05), n_init=n0, Eapp=(1e-3, 2e-3, 3e-3), tol=1e-11)
    N0 = n0.sum(1)
    M0 = o.fields()["rho"].sum()
    o.step(200)
    fl = o.fields()
    assert np.abs(fl["n"].sum(1) / N0 - 1).max() < 1e-13
    assert abs(fl["rho"].sum() / M0 - 1) < 1e-13
    assert (fl["n"][:, t != 0] == 0).all()


def test_gauge_invariance():
    """Sec. III A: results do not depend on the absolute electrode potentials."""
    a, _, t = P.run_slab(nf=16, steps=300, tol=1e-13, E=(1e-3, 0, 0))
    b, _, _ = P.run_slab(nf=16, steps=300, tol=1e-13, E=(1e-3, 0, 0), shift=0.15)
    fa, fb = a.fields(), b.fields()
    assert np.abs(fa["n"] - fb["n"]).max() < 1e-10 * fa["n"].max()
    assert np.abs(fa["u"] - fb["u"]).max() < 1e-8 * np.abs(fa["u"]).max()
    assert np.abs(a.qhist() - b.qhist()).max() < 1e-9 * np.abs(a.qhist()).max()


def test_mirror_symmetry():
    """A +V/-V slab with equal D is mirror symmetric: n+(z) = n-(L-z)."""
    o, shape, t = P.run_slab(nf=16, steps=500, tol=1e-14)
    n = o.fields()["n"][:, t == 0]
    assert np.abs(n[0] - n[1][::-1]).max() < 1e-11 * n.max()


def test_lateral_independence():
    """Sec. III A: Nx = Ny = 1 already describes infinite plates."""
    a, _, ta = P.run_slab(nf=16, steps=300, nxy=1, tol=1e-14)
    b, sb, tb = P.run_slab(nf=16, steps=300, nxy=4, tol=1e-14)
    na = a.fields()["n"][:, ta == 0]
    nb = b.fields()["n"].reshape(2, sb[2], 4, 4)[:, 1:-1]
    for y in range(4):
        for x in range(4):
            assert np.abs(nb[:, :, y, x] - na).max() < 1e-11 * na.max()
    assert np.allclose(a.qhist() * 16, b.qhist(), rtol=1e-9, atol=0)


# ---- error handling ---------------------------------------------------------

def _params(**kw):
    shape, t, ps = W.slab(2, 2, 8, 1)
    base = dict(shape=shape, z=(1, -1), D=(0.05, 0.05), lB=0.4)
    base.update(kw)
    return oracle.make_params(**base), t, ps


@pytest.mark.parametrize("kw", [dict(tau=0.5), dict(omega=2.0), dict(omega=0.0),
                                dict(check_every=0), dict(lB=-1.0)])
def test_invalid_parameters(kw):
    p, t, ps = _params(**kw)
    with pytest.raises(oracle.OracleError) as e:
        oracle.Oracle(p, t, ps, None, (1e-3, 1e-3))
    assert e.value.code == oracle.EINVAL


def test_invalid_dimensions():
    p = oracle.make_params((0, 2, 10), (1, -1), (0.05, 0.05), 0.4)
    with pytest.raises(oracle.OracleError) as e:
        oracle.Oracle(p, np.zeros(0, np.uint8), np.zeros(0), None, (1e-3, 1e-3))
    assert e.value.code == oracle.EINVAL


def test_nan_initial_concentration():
    p, t, ps = _params()
    n0 = np.full((2, t.size), 1e-3)
    n0[0, 20] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        oracle.Oracle(p, t, ps, n0)
    assert e.value.code == oracle.EINVAL


def test_floating_region_rejected():
    shape = (4, 4, 4)
    t = np.zeros(64, np.uint8)
    p = oracle.make_params(shape, (1, -1), (0.05, 0.05), 0.4)
    with pytest.raises(oracle.OracleError) as e:
        oracle.Oracle(p, t, np.zeros(64), None, (1e-3, 1e-3))
    assert e.value.code == oracle.EGEOM


def test_odd_periodic_extent_rejected():
    shape, t, ps = W.slab(3, 2, 8, 1)
    p = oracle.make_params(shape, (1, -1), (0.05, 0.05), 0.4)
    with pytest.raises(oracle.OracleError) as e:
        oracle.Oracle(p, t, ps, None, (1e-3, 1e-3))
    assert e.value.code == oracle.EGEOM


def test_no_convergence_reported():
    p, t, ps = _params(max_iter=1, tol=1e-12)
    with pytest.raises(oracle.OracleError) as e:
        oracle.Oracle(p, t, ps, None, (1e-3, 1e-3))
    assert e.value.code == oracle.ENOCONV


def test_failed_step_goes_back_to_its_start():
    """A step whose solve hits max_iter leaves n, f, phi, the step count and
    the charge history as they were before it; with the limit raised the
    same steps then give exactly the uninterrupted trajectory."""
    kw, shape, t, ps, n0, nref, _, _ = G.case("slab_2x2x18_k1")
    pk = dict(tol=1e-12, max_iter=100000, check_every=2)
    a = oracle.Oracle(oracle.make_params(shape, **kw, **pk), t, ps, n0, nref)
    b = oracle.Oracle(oracle.make_params(shape, **kw, **pk), t, ps, n0, nref)
    a.step(4)
    before = a.fields(), a.qhist(), a.step_count
    a.set_solver(1e-14, 1)
    with pytest.raises(oracle.OracleError) as e:
        a.step(3)
    assert e.value.code == oracle.ENOCONV
    after = a.fields(), a.qhist(), a.step_count
    for k in before[0]:
        assert np.array_equal(before[0][k], after[0][k]), k
    assert np.array_equal(before[1], after[1]) and before[2] == after[2] == 4
    a.set_solver(1e-12, 100000)
    a.step(3)
    b.step(7)
    fa, fb = a.fields(), b.fields()
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k
    assert np.array_equal(a.qhist(), b.qhist())
    with pytest.raises(oracle.OracleError):
        a.set_solver(float("nan"), 10)


def test_equilibrium_moments():
    P.pin_equilibrium_moments()


def test_advection_shear():
    P.pin_advection_shear()


@pytest.mark.parametrize("layers,nxy", [(1, 2), (3, 1)])
def test_naive_neutral_slab_first_order(layers, nxy):
    P.pin_naive_neutral_slab(layers, nxy)


def test_naive_gauss_identity():
    P.pin_naive_gauss_identity()


def test_set_electrode_potential():
    P.pin_set_potential()


@pytest.mark.parametrize("z,D,V,flags", [((1, -1), (0.2, 0.2), 0.5, 0),
                                         ((2, -1), (0.2, 0.35), 0.25, 0),
                                         ((1, -1), (0.2, 0.2), 0.5, P.NAIVE)])
def test_nonlinear_steady_state(z, D, V, flags):
    P.pin_nonlinear_steady_state(z, D, V, flags=flags)


def test_sor_contraction_follows_young():
    P.pin_sor_rate()
