"""Plant plausible mistakes in a copy of the oracle and check that the pins
catch each one (CPU only; the planted copies live in a temporary folder)."""
import pytest

import oracle
import oracle_pins as P

# (name, original text, planted text, pins expected to notice)
MUTATIONS = [
    ("wall factor 1 in the Laplacian",
     "double factor = is_fluid(s, rn) ? 1.0 : wall_factor(s);", "double factor = 1.0;",
     [P.pin_neutral_slab, P.pin_uniform_charge]),
    ("wall factor 1 in the SOR update",
     "double ws = weight(i) * (is_fluid(s, rn) ? 1.0 : wall_factor(s));", "double ws = weight(i);",
     [P.pin_neutral_slab, P.pin_uniform_charge]),
    ("source term off by 2",
     "num += 4.0 * M_PI * s->p.lB / 6.0 * charge_density(s, r);",
     "num += 4.0 * M_PI * s->p.lB / 3.0 * charge_density(s, r);",
     [P.pin_uniform_charge]),
    ("electrode charge without the wall factor",
     "lap += weight(i) * wall_factor(s) * (s->phi[rn] - s->phi[r]);",
     "lap += weight(i) * (s->phi[rn] - s->phi[r]);",
     [P.pin_neutral_slab, P.pin_gauss_identity]),
    ("electrode charge with the wrong sign",
     "q[e - 1] += -(6.0 * lap) / (4.0 * M_PI * s->p.lB);",
     "q[e - 1] += (6.0 * lap) / (4.0 * M_PI * s->p.lB);",
     [P.pin_neutral_slab, P.pin_gauss_identity]),
    ("printed A0 kept in front of the flux sum",
     "double dk = p->D[k] / A0;", "double dk = p->D[k];",
     [P.pin_diffusion_decay]),
    ("diagonal links at unit length in the flux",
     "double j = dk * (g - (nk[rn] - nk[r]) / len);", "double j = dk * (g - (nk[rn] - nk[r]));",
     [P.pin_diffusion_decay, P.pin_diffusion_isotropy]),
    ("migration with the wrong sign",
     "double delta = p->z[k] * (s->phi[rn] - s->phi[r] - Ec);\n        double g = excess_link",
     "double delta = p->z[k] * (s->phi[r] - s->phi[rn] - Ec);\n        double g = excess_link",
     [P.pin_debye_relaxation]),
    ("applied field tilt with the wrong sign",
     "double delta = p->z[k] * (s->phi[rn] - s->phi[r] - Ec);\n          gsum",
     "double delta = p->z[k] * (s->phi[rn] - s->phi[r] + Ec);\n          gsum",
     [P.pin_uniform_field_force]),
    ("advection subtracted",
     "sum += j + J;", "sum += j - J;",
     [P.pin_advection_translation, P.pin_advection_shear]),
    ("advection from the local velocity only",
     "cu_there += C[i][a] * s->u[3 * rn + a];", "cu_there += C[i][a] * s->u[3 * r + a];",
     [P.pin_advection_shear]),
    ("force projected without the link length",
     "F[a] += 3.0 * weight(i) * C[i][a] * len * gsum;", "F[a] += 3.0 * weight(i) * C[i][a] * gsum;",
     [P.pin_uniform_field_force]),
    ("Guo source without the (1 - 1/2tau) factor",
     "src *= (1.0 - 0.5 / tau) * weight(i);", "src *= weight(i);",
     [P.pin_uniform_field_force]),
    ("velocity without the half-force shift",
     "(m[a] + 0.5 * s->force[3 * r + a]) / rho;", "(m[a]) / rho;",
     [P.pin_uniform_field_force, P.pin_eo_slab]),
    ("equilibrium quadratic term 3 instead of 9/2",
     "(1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu)", "(1.0 + 3.0 * cu + 3.0 * cu * cu - 1.5 * uu)",
     [P.pin_equilibrium_moments]),
    ("relaxation time ignored",
     "double post = fi - (fi - feq) / tau + src;", "double post = fi - (fi - feq) + src;",
     [P.pin_shear_wave]),
    ("first-order scheme keeps the factor 2 in Gauss's law",
     "lap += weight(i) * wall_factor(s) * (s->phi[rn] - s->phi[r]);",
     "lap += weight(i) * 2.0 * (s->phi[rn] - s->phi[r]);",
     [P.pin_naive_neutral_slab, P.pin_naive_gauss_identity]),
    ("first-order flag ignored",
     "return (s->p.flags & ORC_FLAG_NAIVE_DIRICHLET) ? 1.0 : 2.0;", "return 2.0;",
     [P.pin_naive_neutral_slab]),
    ("new electrode potential not applied before the solve",
     "      s->phi_s[r] = phi_s[r];\n      s->phi[r] = phi_s[r];\n    }\n  int rc = poisson_solve(s);",
     "      s->phi_s[r] = phi_s[r];\n    }\n  int rc = poisson_solve(s);",
     [P.pin_set_potential]),
    ("charge of the new potential not recorded",
     "if (s->ne && s->qlen > 0) electrode_charges(s, s->qhist + (s->qlen - 1) * s->ne);",
     "",
     [P.pin_set_potential]),
    ("excess flux linearised in delta",
     "return -(n_there * expm1(delta) - n_here * expm1(-delta)) / (2.0 * len);",
     "return -(n_there * delta + n_here * delta) / (2.0 * len);",
     [P.pin_nonlinear_steady_state]),
    ("SOR relaxation factor ignored (Gauss-Seidel)",
     "s->phi[r] = (1.0 - s->p.omega) * s->phi[r] + s->p.omega * gs;", "s->phi[r] = gs;",
     [P.pin_sor_rate]),
    ("SOR relaxation weights swapped",
     "s->phi[r] = (1.0 - s->p.omega) * s->phi[r] + s->p.omega * gs;",
     "s->phi[r] = s->p.omega * s->phi[r] + (1.0 - s->p.omega) * gs;",
     [P.pin_sor_rate]),
    ("bounce-back into the same direction",
     "s->fnew[(long)opposite(i) * s->N + r] = post;", "s->fnew[(long)i * s->N + r] = post;",
     [P.pin_eo_slab, P.pin_equilibrium_moments]),
]


@pytest.mark.parametrize("name,old,new,pins", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(tmp_path, name, old, new, pins):
    src = oracle.source_text()
    assert src.count(old) == 1, f"mutation site not unique: {old!r}"
    lib = oracle.build_variant(src.replace(old, new), str(tmp_path / "liboracle_planted.so"))
    caught = []
    for pin in pins:
        try:
            pin(libpath=lib)
        except (AssertionError, oracle.OracleError, FloatingPointError, ValueError):
            caught.append(pin.__name__)
    assert caught, f"no pin noticed: {name}"
