"""Strength of the oracle's pins (CPU only).

Each case plants one plausible mistake in a copy of the oracle package: a dropped factor, a
flipped sign, a transposed operand or index, a misplaced quadrature point or weight, a wrong
update in the Newton loop. The copy's C source is built with gcc (the loader takes the library
from ``BSC_ORACLE_LIB``) and the oracle's pin tests (``tests/test_oracle_*.py``) run in a child
process that imports the copy as ``oracle``. Every mutant must make at least one pin fail, and
the unmodified copy, built and imported the same way, must pass all of them. The pins compare
the oracle with closed forms, brute force, finite differences, library routines and the
invariants of the method, never with the oracle itself, so a mutant that no pin catches would be
a mistake that the GPU parity tests inherit unseen.
"""
from __future__ import annotations

import os
import re
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (name, [(old, new), ...]) in the C source: each old text must occur; its first occurrence is
# replaced (an edit listed twice replaces two occurrences).
C_MUTANTS = [
    # basis (Sec. 3.1.1)
    ("basis_right_term_index",
     [("* or_basis(xi, i + 1, p - 1, u);", "* or_basis(xi, i, p - 1, u);")]),
    ("basis_derivative_sign", [("    return left - right;\n}", "    return left + right;\n}")]),
    ("dv_along_u", [("B->Nv[m] = Ru[a][0] * Rv[b][1] * hv;", "B->Nv[m] = Ru[a][1] * Rv[b][0] * hv;")]),
    ("duv_missing_v_derivative",
     [("B->Nuv[m] = Ru[a][1] * hu * Rv[b][1] * hv;", "B->Nuv[m] = Ru[a][1] * hu * Rv[b][0] * hv;")]),
    ("du_missing_knot_spacing", [("B->Nu[m] = Ru[a][1] * hu * Rv[b][0];", "B->Nu[m] = Ru[a][1] * Rv[b][0];")]),
    # rest geometry (Sec. 4.1 inverse function theorem, Sec. 4.2 second derivatives)
    ("inverse_jacobian_transposed",
     [("K[0][1] = -J[0][1] / det;", "K[0][1] = -J[1][0] / det;"),
      ("K[1][0] = -J[1][0] / det;", "K[1][0] = -J[0][1] / det;")]),
    ("inverse_derivative_sign", [("dK[p][r][c] = -s;", "dK[p][r][c] = s;")]),
    ("laplacian_cross_term_halved", [("lap[4] = 2.0 * (", "lap[4] = (")]),
    ("weight_without_jacobian", [("return wbar * fabs(detJ);", "return wbar;")]),
    # membrane densities (Sec. 4.1)
    ("stvk_energy_lambda_doubled",
     [("*psi = mu * EE + 0.5 * lam * trE * trE;", "*psi = mu * EE + lam * trE * trE;")]),
    ("stvk_hessian_term_transposed", [("mu * F[i][d] * F[j][g]", "mu * F[i][g] * F[j][d]")]),
    ("green_strain_offdiagonal_unhalved", [("0.5 * C[0][1]}", "C[0][1]}")]),
    ("shear_modulus_unhalved",
     [("double mu = S->young * S->thickness / (2.0 * (1.0 + S->poisson));",
       "double mu = S->young * S->thickness / (1.0 + S->poisson);")]),
    ("lambda_of_3d_elasticity",
     [("double lam = S->young * S->thickness * S->poisson / (1.0 - S->poisson * S->poisson);",
       "double lam = S->young * S->thickness * S->poisson / ((1.0 + S->poisson) * (1.0 - 2.0 * S->poisson));")]),
    ("fbw_stretch_stress_halved",
     [("2.0 * mu[g] * (1.0 - 1.0 / len[g]) * f[g][i];", "mu[g] * (1.0 - 1.0 / len[g]) * f[g][i];")]),
    ("fbw_shear_hessian_transposed",
     [("(f[d][i] * f[g][j] + (i == j ? I6 : 0.0))", "(f[g][i] * f[d][j] + (i == j ? I6 : 0.0))")]),
    # projection (Sec. 5.1)
    ("projection_absolute_eigenvalues", [("lam[r] = A[r][r] > 0.0 ? A[r][r] : 0.0;", "lam[r] = fabs(A[r][r]);")]),
    # element gradient and Hessian (Sec. 4.1, 4.2)
    ("membrane_gradient_wrong_direction",
     [("P[i][0] * dN[m][0] + P[i][1] * dN[m][1]", "P[i][0] * dN[m][0] + P[i][1] * dN[m][0]")]),
    ("membrane_hessian_operands_transposed",
     [("s += dN[m][ga] * A[3 * ga + i][3 * de + j] * dN[n][de];",
       "s += dN[m][de] * A[3 * ga + i][3 * de + j] * dN[n][ga];")]),
    ("bending_laplacian_first_order_swapped",
     [("lap[2] * B.Nu[m] + lap[3] * B.Nv[m]", "lap[3] * B.Nu[m] + lap[2] * B.Nv[m]")]),
    ("bending_energy_unhalved", [("*E += w * 0.5 * mu * (dphi[0]", "*E += w * mu * (dphi[0]")]),
    # quadrature (Appendix A)
    ("gauss2_offset_not_in_span_units", [("G2 = 0.28867513459481288225", "G2 = 0.57735026918962576451")]),
    ("gauss3_equal_weights",
     [("w[0] = 5.0 / 18.0; w[1] = 8.0 / 18.0; w[2] = 5.0 / 18.0;", "w[0] = 1.0 / 3.0; w[1] = 1.0 / 3.0; w[2] = 1.0 / 3.0;")]),
    ("side_spans_points_swapped", [("nu = bu ? 3 : 2; nv = bv ? 3 : 2;", "nu = bu ? 2 : 3; nv = bv ? 2 : 3;")]),
    ("checkerboard_flipped", [("} else if ((a + b) % 2 == 0) {", "} else if ((a + b) % 2 == 1) {")]),
    ("edge_half_cell_full_weight", [("np = 2; w = 0.25;", "np = 2; w = 0.5;")]),
    ("bending_knot_weight_not_quartered", [("double w = lu * lv * 0.25;", "double w = lu * lv;")]),
    ("bending_knot_wrong_span",
     [("cnt = push(out, cap, cnt, a, b, w, a - 1, b);", "cnt = push(out, cap, cnt, a, b, w, a - 1, b - 1);")]),
    # mass, inertia, gravity, assembly and pins (Sec. 3.2, 5.1)
    ("mass_diagonal_instead_of_row_sum",
     [("row += S->rho_area * B.N[m] * B.N[n];", "row += S->rho_area * B.N[m] * B.N[m];")]),
    ("inertia_energy_unhalved", [("E += 0.5 * M[a] * inv_dt2 * d * d;", "E += M[a] * inv_dt2 * d * d;")]),
    ("inertia_hessian_without_dt", [("+= M[a] * inv_dt2;", "+= M[a];")]),
    ("gravity_gradient_sign", [("g[3 * a + i] -= M[a] * grav[i];", "g[3 * a + i] += M[a] * grav[i];")]),
    ("stencil_slot_transposed",
     [("int s = (bn - bm + 2) * 5 + (an - am + 2);", "int s = (an - am + 2) * 5 + (bn - bm + 2);")]),
    ("pin_mirror_block_not_mirrored",
     [("int sb = (-dj + 2) * 5 + (-di + 2);", "int sb = (dj + 2) * 5 + (di + 2);")]),
    ("pinned_gradient_kept",
     [("for (int i = 0; i < 3; ++i) g[3 * a + i] = 0.0;", "for (int i = 0; i < 3; ++i) g[3 * a + i] += 0.0;")]),
    # further consistent mistakes (energy, gradient and Hessian all agree) and variant rules
    ("laplacian_u_term_transposed",
     [("lap[0] = K[0][0] * K[0][0] + K[0][1] * K[0][1];", "lap[0] = K[0][0] * K[0][0] + K[1][0] * K[1][0];")]),
    ("bending_modulus_doubled", [("double mu = S->mu_bend;", "double mu = 2.0 * S->mu_bend;")]),
    ("stvk_stress_mu_halved", [("Sm[g][d] = 2.0 * mu * E[g][d]", "Sm[g][d] = mu * E[g][d]")]),
    ("green_strain_diagonal_sign", [("0.5 * (C[0][0] - 1.0)", "0.5 * (1.0 - C[0][0])")]),
    ("fbw_moduli_swapped_at_points",
     [("fbw_density(F, S->mu_st1, S->mu_st2, S->mu_sh, &psi, P, A);",
       "fbw_density(F, S->mu_st2, S->mu_st1, S->mu_sh, &psi, P, A);")]),
    ("jacobi_single_sweep", [("sweep < 100;", "sweep < 1;")]),
    ("jacobi_rotation_sign", [("A[k][p] = c * akp - s * akq;", "A[k][p] = c * akp + s * akq;")]),
    ("bending_boundary_span_half_weight",
     [("cnt = push(out, cap, cnt, k + 0.5, l + 0.5, 1.0, k, l);\n    if (quad == OR_QUAD_GAUSS2) {",
       "cnt = push(out, cap, cnt, k + 0.5, l + 0.5, 0.5, k, l);\n    if (quad == OR_QUAD_GAUSS2) {")]),
    ("interior1_midpoint_half_weight",
     [("cnt = push(out, cap, cnt, k + 0.5, l + 0.5, 1.0, k, l);   /* span midpoint */",
       "cnt = push(out, cap, cnt, k + 0.5, l + 0.5, 0.5, k, l);   /* span midpoint */")]),
    ("corner2_rule_ignored", [("nu = nv = (quad == OR_QUAD_CORNER2) ? 2 : 3;", "nu = nv = 3;")]),
    ("gauss2_bending_interior_weight",
     [("l + 0.5 + o[b], w[a] * w[b], k, l);", "l + 0.5 + o[b], w[a], k, l);")]),
    ("surface_top_edge_not_clamped", [("if (v >= vmax) v = vmax * (1.0 - 1e-15);", "(void)vmax;")]),
    ("surface_basis_in_wrong_parameter",
     [("double Ni = or_basis(S->knots_u, i, 2, u);", "double Ni = or_basis(S->knots_u, i, 2, v);")]),
]

# (name, file of the package, [(old, new), ...]) in the Python parts
PY_MUTANTS = [
    # projected Newton (Sec. 3.2, 5.1)
    ("predictor_sign", "__init__.py", [("xhat = x_n + dt * v_n", "xhat = x_n - dt * v_n")]),
    ("velocity_from_predictor", "__init__.py", [("v=(x - x_n) / dt", "v=(x - xhat) / dt")]),
    ("pins_left_at_previous_position", "__init__.py",
     [("x[pins] = _f64(pin_targets).reshape(-1, 3)", "x[pins] = x[pins]")]),
    ("step_rule_without_dt", "__init__.py",
     [("np.abs(p).max() / dt <= atol", "np.abs(p).max() <= atol")]),
    ("gradient_rule_absolute", "__init__.py", [("gn <= rtol * g0", "gn <= rtol")]),
    ("newton_without_projection", "__init__.py",
     [("assemble(sheet, x, xhat, dt, gravity, mask, project=True)",
       "assemble(sheet, x, xhat, dt, gravity, mask, project=False)")]),
    ("line_search_never_halves", "__init__.py", [("alpha *= 0.5", "alpha *= 1.0")]),
    ("inertia_over_dt", "__init__.py",
     [("inv_dt2 = 0.0 if dt is None else 1.0 / (dt * dt)", "inv_dt2 = 0.0 if dt is None else 1.0 / dt"),
      ("inv_dt2 = 0.0 if dt is None else 1.0 / (dt * dt)", "inv_dt2 = 0.0 if dt is None else 1.0 / dt")]),
    ("csr_blocks_transposed", "__init__.py",
     [("rows.append(3 * A + r)\n                cols.append(3 * B + c)",
       "rows.append(3 * A + c)\n                cols.append(3 * B + r)")]),
    # contact conversion (Sec. 4.3)
    ("contact_right_end_not_clamped", "contact_ref.py",
     [("k = min(int(math.floor(u / hu)), Nu - 1)", "k = int(math.floor(u / hu))")]),
    ("contact_weights_transposed", "contact_ref.py", [("w = wu[c] * wv[b]", "w = wu[b] * wv[c]")]),
    ("contact_cp_index_swapped", "contact_ref.py",
     [("cols.append((l + b) * sheet.n_u + (k + c))", "cols.append((l + c) * sheet.n_u + (k + b))")]),
    ("contact_gradient_sign", "contact_ref.py",
     [("g[a] += pair_grad[c, 3 * s:3 * s + 3]", "g[a] -= pair_grad[c, 3 * s:3 * s + 3]")]),
    # learned warm start (network reference)
    ("net_taps_flipped", "net_ref.py",
     [("out += np.tensordot(W[:, :, ky, kx], patch", "out += np.tensordot(W[:, :, 2 - ky, 2 - kx], patch")]),
    ("net_backward_relu_derivative", "net_ref.py",
     [("np.where(inputs[l] > 0, 1.0, SLOPE)", "np.where(inputs[l] > 0, 1.0, 0.0)")]),
    ("net_input_not_normalised", "net_ref.py", [("s = 1.0 / rms if rms > 0 else 0.0", "s = 1.0")]),
    ("net_loss_mask_inverted", "net_ref.py",
     [("m = (np.abs(x[b]).sum(axis=0) != 0)", "m = (np.abs(x[b]).sum(axis=0) == 0)")]),
    # partial factorization (Sec. 5.3)
    ("neumann_term_sign", "partial_ref.py", [("t = -lu.solve(B @ t)", "t = lu.solve(B @ t)")]),
    ("gershgorin_without_abs", "partial_ref.py", [("A = abs(B).tolil()", "A = B.tolil()")]),
    ("lambda_min_mass_over_dt", "partial_ref.py",
     [("best = min(best, mass[a] / (dt * dt) + max(0.0, g))", "best = min(best, mass[a] / dt + max(0.0, g))")]),
    ("barrier_pins_not_dropped", "partial_ref.py",
     [("P = sp.diags(dof_mask(n_cp, pinned))", "P = sp.identity(3 * n_cp)")]),
    ("merged_branch_drops_b", "partial_ref.py",
     [("x = spla.spsolve((D + B).tocsc(), bb)", "x = spla.spsolve(D, bb)")]),
]

MUTANTS = [(name, "bsc_oracle.c", edits) for name, edits in C_MUTANTS] + PY_MUTANTS

PIN_FILES = sorted(f for f in os.listdir(os.path.join(ROOT, "tests"))
                   if f.startswith("test_oracle_") and f.endswith(".py"))


def _mutate(text: str, edits) -> str:
    for old, new in edits:
        assert old in text, "mutation site not found: %r" % old
        text = text.replace(old, new, 1)
    return text


# The child imports the copy as the package ``oracle`` before pytest starts, so every later
# ``import oracle`` (and its submodules) resolves to the copy.
_BOOT = """
import importlib.util, sys
pkg = sys.argv[1]
spec = importlib.util.spec_from_file_location("oracle", pkg + "/__init__.py", submodule_search_locations=[pkg])
mod = importlib.util.module_from_spec(spec)
sys.modules["oracle"] = mod
spec.loader.exec_module(mod)
assert mod.__file__.startswith(pkg)
import pytest
sys.exit(pytest.main(sys.argv[2:]))
"""

PKG_FILES = ("__init__.py", "bsc_oracle.c", "contact_ref.py", "net_ref.py", "partial_ref.py")


def _run_pins(tmp: str, name: str, fname: str | None, edits):
    """Copies the package, plants the edits, builds the copy's C source and runs the pin tests
    against the copy; returns (return code, first failing test or None, tail of the output)."""
    pkg = os.path.join(tmp, name, "oracle")
    os.makedirs(pkg)
    for f in PKG_FILES:
        text = open(os.path.join(ROOT, "oracle", f)).read()
        if f == fname:
            text = _mutate(text, edits)
        with open(os.path.join(pkg, f), "w") as fh:
            fh.write(text)
    lib = oracle.build(os.path.join(pkg, "bsc_oracle.c"), os.path.join(tmp, name, "liboracle.so"))
    env = dict(os.environ, BSC_ORACLE_LIB=lib, PYTHONDONTWRITEBYTECODE="1")
    env.setdefault("OMP_NUM_THREADS", "1")
    args = ["-x", "-q", "-rf", "-p", "no:cacheprovider", "-m", "not gpu"]
    args += [os.path.join("tests", f) for f in PIN_FILES]
    res = subprocess.run([sys.executable, "-c", _BOOT, pkg] + args, cwd=ROOT, env=env,
                         capture_output=True, text=True, timeout=600)
    out = res.stdout + res.stderr
    m = re.search(r"^FAILED (\S+)", out, re.M)
    return res.returncode, (m.group(1) if m else None), out[-1500:]


@pytest.fixture(scope="module")
def mutant_results():
    tmp = tempfile.mkdtemp(prefix="bsc_mutants_")
    jobs = [("control", None, [])] + MUTANTS
    try:
        with ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
            futs = {name: ex.submit(_run_pins, tmp, name, f, edits) for name, f, edits in jobs}
            res = {name: fut.result() for name, fut in futs.items()}
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    for name, (rc, first, _) in res.items():
        print("%-40s rc=%d  %s" % (name, rc, first or "-"))
    return res


def test_every_mutation_site_exists():
    for name, f, edits in MUTANTS:
        base = open(os.path.join(ROOT, "oracle", f)).read()
        assert _mutate(base, edits) != base, name


def test_unmodified_copy_passes_every_pin(mutant_results):
    rc, first, tail = mutant_results["control"]
    assert rc == 0, tail


@pytest.mark.parametrize("name", [m[0] for m in MUTANTS])
def test_pins_catch_mutant(mutant_results, name):
    rc, first, tail = mutant_results[name]
    # 1 = some test failed (an assertion or an error raised by the oracle); anything else would
    # be a crash or a collection problem, which says nothing about the pins
    assert rc == 1 and first is not None, "mutant %s survived the pins (rc=%d):\n%s" % (name, rc, tail)
