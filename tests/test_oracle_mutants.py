"""Planted mistakes in the oracle: every pin set must reject them.

Each case rewrites one line of ``oracle/mns_oracle.c`` into a plausible
mistake (a dropped term, a wrong sign, a transposed index, a wrong constant),
compiles that copy on the CPU, routes the oracle calls to it, and runs the
pins of ``test_oracle_pins.py`` that are meant to catch it: at least one of
them must fail.  The real oracle passes all of them (``test_oracle_pins.py``).
"""
import os

import pytest

import oracle
from tests import test_oracle_iso as iso
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "mns_oracle.c")

# (name, original text, mistaken text, pins expected to catch it)
MUTANTS = [
    ("SUPG weight derivative dropped",
     "C->Gv[m][e] += tau * Rp[m] * a[e] + tau * R[m] * T->u[e];",
     "C->Gv[m][e] += tau * Rp[m] * a[e];",
     [(pins.test_jacobian_is_derivative_of_residual, dict(dim=2, steady=1))]),
    ("pressure term of the momentum test with the wrong sign",
     "C->Gv[m][e] = nu * T->gu[m][e] - (m == e ? T->p : 0.0);",
     "C->Gv[m][e] = nu * T->gu[m][e] + (m == e ? T->p : 0.0);",
     [(pins.test_galerkin_saddle_structure, dict(dim=2))]),
    ("reaction term with the transposed velocity gradient",
     "reac += S->gu[m][e] * T->u[e];",
     "reac += S->gu[e][m] * T->u[e];",
     [(pins.test_jacobian_is_derivative_of_residual, dict(dim=2, steady=1))]),
    ("convection of the increment by u instead of u - u_ALE",
     "conv += T->gu[m][e] * a[e];",
     "conv += T->gu[m][e] * S->u[e];",
     [(pins.test_ale_convection_of_rigid_rotation, {})]),
    ("mesh velocity rotating the wrong way",
     "w[0] = -M->P.omega * x[1];",
     "w[0] = M->P.omega * x[1];",
     [(pins.test_ale_convection_of_rigid_rotation, {}),
      (pins.test_taylor_green_transient_with_rotating_rotor, {})]),
    ("mapping term missing from the physical Hessian",
     "for (int m = 0; m < d; ++m) s -= gp[m] * X2[m][p][q];",
     "(void)X2;",
     [(pins.test_physical_derivatives_of_polar_polynomials, dict(dim=2, k=2))]),
    ("BDF2 coefficient 1/dt instead of 3/(2 dt)",
     "return M->P.steady ? 0.0 : 1.5 / M->P.dt;",
     "return M->P.steady ? 0.0 : 1.0 / M->P.dt;",
     [(pins.test_mass_and_viscous_coefficients, dict(steady=0)),
      (pins.test_taylor_green_transient_with_rotating_rotor, {})]),
    ("tau: viscous factor 3 instead of 9",
     "9.0 * (4.0 * nu / (h * h))",
     "3.0 * (4.0 * nu / (h * h))",
     [(pins.test_tau_closed_form, dict(U=0.0, steady=1))]),
    ("tau: convective part |a|^2/h^2 instead of (2|a|/h)^2",
     "4.0 * an2 / (h * h)",
     "an2 / (h * h)",
     [(pins.test_tau_closed_form, dict(U=0.7, steady=1))]),
    ("PSPG with grad dp only (velocity part of R' dropped)",
     "C->Gq[m] = stab ? tau * Rp[m] : 0.0;",
     "C->Gq[m] = stab ? tau * T->gp[m] : 0.0;",
     [(pins.test_jacobian_is_derivative_of_residual, dict(dim=2, steady=1)),
      (pins.test_supg_pspg_adjoint_identity, dict(dim=2))]),
    ("mortar jump taken as other - own",
     "j[m] = Fs->u[m] - Fo->u[m];",
     "j[m] = Fo->u[m] - Fs->u[m];",
     [(pins.test_galerkin_saddle_structure, dict(dim=2)), (pins.test_sipg_symmetry, dict(dim=2))]),
    ("mortar Jacobian with the arc length (extra factor R)",
     "M->P.r_if * len * ((d == 3) ? M->gw[qz] * M->dz : 1.0);\n        field_t F[2];",
     "M->P.r_if * M->P.r_if * len * ((d == 3) ? M->gw[qz] * M->dz : 1.0);\n        field_t F[2];",
     [(pins.test_matrix_free_equals_assembled, dict(dim=2)), (pins.test_interface_penalty_closed_form, {})]),
    ("interface penalty without nu",
     "C->gv[m] = pbar * ns[m] - nu * gn + nu * tau * j[m];",
     "C->gv[m] = pbar * ns[m] - nu * gn + tau * j[m];",
     [(pins.test_interface_penalty_closed_form, {})]),
    ("interface penalty taken from the other side's cell",
     "double nu = M->P.nu, tau = M->tau_side[side];",
     "double nu = M->P.nu, tau = M->tau_side[1 - side];",
     [(pins.test_interface_penalty_closed_form, {})]),
    ("SIPG symmetric term without the 1/2",
     "C->Gv[m][e] = -0.5 * nu * j[m] * ns[e];",
     "C->Gv[m][e] = -nu * j[m] * ns[e];",
     [(pins.test_sipg_symmetry, dict(dim=2))]),
    ("mortar mass term without the 1/2",
     "C->gq = -0.5 * jn;",
     "C->gq = -jn;",
     [(pins.test_galerkin_saddle_structure, dict(dim=2))]),
    ("Picard option keeping the reaction term",
     "    if (M->P.picard) reac = 0.0;\n",
     "\n",
     [(pins.test_picard_jacobian_applied_to_state_is_residual, dict(dim=2, steady=1))]),
    ("Picard option keeping the SUPG weight derivative",
     "for (int m = 0; m < d; ++m) R[m] = 0.0; /* no SUPG weight derivative */",
     "(void)0;",
     [(pins.test_picard_jacobian_applied_to_state_is_residual, dict(dim=2, steady=1))]),
    ("mortar pressure average taken from the own side only",
     "double pbar = 0.5 * (Fs->p + Fo->p);",
     "double pbar = Fs->p;",
     [(pins.test_galerkin_saddle_structure, dict(dim=2)),
      (pins.test_aligned_mortar_reduces_to_conforming_cg, dict(dim=2))]),
    ("inward interface normals in the face coefficients (n = -n_outward on both sides)",
     "static void mortar_coef(const mesh_t *M, int side, const field_t *Fs, const field_t *Fo, const double ns[3],\n"
     "                        testcoef_t *C) {\n",
     "static void mortar_coef(const mesh_t *M, int side, const field_t *Fs, const field_t *Fo, const double nso[3],\n"
     "                        testcoef_t *C) {\n  const double ns[3] = {-nso[0], -nso[1], -nso[2]};\n",
     [(pins.test_discrete_mass_conservation, dict(dim=2)), (pins.test_pressure_nullspace_up_to_quadrature, {})]),
    ("iso-parametric map without its Hessian",
     "for (int q = 0; q < d; ++q) X2[m][p][q] += X[m] * H[p][q];",
     "(void)H;",
     [(iso.test_affine_fields_are_exact, dict(dim=2, k=2))]),
    ("iso-parametric Jacobian accumulated transposed",
     "J[m][p] += X[m] * g[p];",
     "J[p][m] += X[m] * g[p];",
     [(iso.test_affine_fields_are_exact, dict(dim=2, k=2))]),
    ("node perturbation that does not vanish on the rotor's side of the interface",
     "const double ra = rotor_side ? P->r_in : P->r_if, rb = rotor_side ? P->r_if : P->r_out;",
     "const double ra = rotor_side ? P->r_in : P->r_if, rb = rotor_side ? P->r_out : P->r_out;",
     [(iso.test_node_perturbation_keeps_boundaries, {}),
      (iso.test_aligned_mortar_reduces_to_conforming_cg_on_perturbed_mesh, dict(dim=2))]),
    ("rotor nodes of the iso-parametric mesh left unrotated",
     "const double rr = r + dr, th = thm + dt + rot;",
     "const double rr = r + dr, th = thm + dt;",
     [(iso.test_mass_balance_on_iso_mesh, dict(dim=2)), (iso.test_mms_convergence_q2_perturbed_iso, {})]),
]


@pytest.fixture(scope="module")
def source():
    with open(SRC) as f:
        return f.read()


@pytest.mark.parametrize("name,old,new,catchers", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_reject_planted_mistake(tmp_path, source, name, old, new, catchers):
    assert source.count(old) == 1, f"mutation site not unique: {old!r}"
    path = oracle.build_variant(source.replace(old, new), str(tmp_path / "libmutant.so"))
    oracle.swap_library(path)
    failed = []
    try:
        for fn, kw in catchers:
            try:
                fn(**kw)
            except AssertionError:
                failed.append(fn.__name__)
    finally:
        oracle.swap_library(None)
    assert failed, f"no pin rejects the planted mistake: {name}"
