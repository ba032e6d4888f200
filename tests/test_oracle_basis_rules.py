"""Pins for the oracle's B-spline basis, quadrature rules and lumped mass (CPU only).

Each check compares against something other than the oracle's own formula: library B-splines
(scipy), B-spline identities (partition of unity, Greville and Marsden reproduction), the
closed-form pieces of the quadratic basis, the quadrature points printed in the paper's
figure, and the closed-form lumped mass."""
import os

import numpy as np
import pytest

import oracle
import synthetic as syn

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "quadrature_n5.txt")


def read_golden():
    sec, out = None, {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("["):
            sec = line.strip("[]")
            out[sec] = []
            continue
        out[sec].append([float(t) for t in line.split()])
    return {k: np.array(v) for k, v in out.items()}


# ---- basis --------------------------------------------------------------------------------

@pytest.mark.parametrize("n", [5, 8, 13])
def test_basis_matches_scipy_bspline(n):
    from scipy.interpolate import BSpline
    kn = syn.open_uniform_knots(n)
    us = np.linspace(0.0, kn[-1], 57, endpoint=False)
    for i in range(n):
        ref = BSpline.basis_element(kn[i:i + 4], extrapolate=False)
        for u in us:
            want = ref(u)
            want = 0.0 if np.isnan(want) else float(want)
            assert abs(oracle.basis(kn, i, u) - want) < 1e-14


@pytest.mark.parametrize("n", [5, 9])
def test_partition_of_unity_and_reproduction(n):
    kn = syn.open_uniform_knots(n, spacing=1)
    grev = syn.greville(kn, n)
    marsden = kn[1:n + 1] * kn[2:n + 2]
    for u in np.random.default_rng(0).uniform(0, kn[-1], 40):
        N = np.array([oracle.basis(kn, i, u) for i in range(n)])
        assert abs(N.sum() - 1.0) < 1e-14
        assert abs(N @ grev - u) < 1e-13                  # linear precision (Greville)
        assert abs(N @ marsden - u * u) < 1e-12           # Marsden's identity for u^2
        assert (N >= -1e-15).all()


def test_values_at_knots_and_open_end():
    n = 9
    kn = syn.open_uniform_knots(n)
    assert oracle.basis(kn, 0, 0.0) == 1.0
    for a in range(1, n - 2):
        vals = np.array([oracle.basis(kn, i, float(a)) for i in range(n)])
        nz = np.nonzero(np.abs(vals) > 1e-15)[0]
        assert list(nz) == [a, a + 1]
        assert np.allclose(vals[nz], [0.5, 0.5], atol=1e-15)


def _piece(kn, n, k, t, d):
    s = k + 2
    return np.array([oracle.basis_piece(kn, k + a, s, k + t, d) for a in range(3)])


def test_closed_form_pieces():
    n = 9
    N = n - 2
    kn = syn.open_uniform_knots(n)
    for t in (0.0, 0.17, 0.5, 0.93, 1.0):
        # uniform interior span
        want = [0.5 * (1 - t) ** 2, 0.5 * (-2 * t * t + 2 * t + 1), 0.5 * t * t]
        assert np.allclose(_piece(kn, n, 3, t, 0), want, atol=1e-15)
        assert np.allclose(_piece(kn, n, 3, t, 1), [-(1 - t), 1 - 2 * t, t], atol=1e-14)
        # first span of the open knot vector
        want0 = [(1 - t) ** 2, 2 * t - 1.5 * t * t, 0.5 * t * t]
        assert np.allclose(_piece(kn, n, 0, t, 0), want0, atol=1e-15)
        # last span mirrors the first
        wantL = [0.5 * (1 - t) ** 2, 2 * (1 - t) - 1.5 * (1 - t) ** 2, t * t]
        assert np.allclose(_piece(kn, n, N - 1, t, 0), wantL, atol=1e-14)
    # one-sided second derivatives: interior (1,-2,1), next to the ends (2,-3,1) / (1,-3,2)
    assert np.allclose(_piece(kn, n, 3, 0.3, 2), [1, -2, 1], atol=1e-14)
    assert np.allclose(_piece(kn, n, 0, 0.3, 2), [2, -3, 1], atol=1e-14)
    assert np.allclose(_piece(kn, n, N - 1, 0.3, 2), [1, -3, 2], atol=1e-14)
    assert np.allclose(_piece(kn, n, 1, 0.3, 2), [1, -2, 1], atol=1e-14)


def test_c1_continuity_across_knots():
    n = 8
    kn = syn.open_uniform_knots(n)
    for a in range(1, n - 2):
        for i in range(n):
            for d in (0, 1):
                left = oracle.basis_piece(kn, i, a - 1 + 2, float(a), d)
                right = oracle.basis_piece(kn, i, a + 2, float(a), d)
                assert abs(left - right) < 1e-13


def test_basis_piece_equals_literal_inside_span():
    n = 8
    kn = syn.open_uniform_knots(n)
    for u in np.random.default_rng(3).uniform(0, n - 2, 30):
        k = int(np.floor(u))
        for i in range(n):
            lit = oracle.basis(kn, i, u)
            pc = oracle.basis_piece(kn, i, k + 2, u, 0)
            assert abs(lit - pc) < 1e-14


def test_knot_validation():
    assert oracle.check_knots(syn.open_uniform_knots(6), 6) == (4, 1.0)
    assert oracle.check_knots(syn.open_uniform_knots(6, spacing=2), 6) == (4, 2.0)
    bad = syn.open_uniform_knots(6).copy()
    bad[4] += 0.5
    assert oracle.check_knots(bad, 6) == (None, None)
    nonopen = np.arange(9, dtype=float)
    assert oracle.check_knots(nonopen, 6) == (None, None)


# ---- quadrature rules ---------------------------------------------------------------------

def _as_set(pts, nd=3):
    return sorted((round(float(a), nd), round(float(b), nd)) for a, b in pts)


def test_membrane_rule_matches_figure_n5():
    gold = read_golden()
    r = oracle.membrane_rule(5, 5)
    # boundary-span Gauss points never sit on a knot line; interior-region points always do
    interior = r[(r[:, 0] % 1 == 0) | (r[:, 1] % 1 == 0)]
    want = _as_set(gold["membrane_interior"])
    got = _as_set(interior[:, :2])
    assert len(got) == 28
    assert np.allclose(np.array(got), np.array(want), atol=1.5e-3)


def test_membrane_reference_cells_match_figure():
    gold = read_golden()
    r = oracle.membrane_rule(5, 5)
    def cell(k, l):
        sel = r[(r[:, 3] == k) & (r[:, 4] == l) & (r[:, 0] > k) & (r[:, 0] < k + 1) & (r[:, 1] > l) & (r[:, 1] < l + 1)]
        return (sel[:, :2] - [k, l]) * 1.25
    for name, origin, span in (("membrane_corner_cell", (6, 4), (0, 0)),
                               ("membrane_bottom_top_cell", (6, 2), (2, 0)),
                               ("membrane_left_right_cell", (6, 0), (0, 2))):
        want = _as_set(gold[name] - np.array(origin))
        got = _as_set(cell(*span))
        assert np.allclose(np.array(got), np.array(want), atol=1.5e-3), name


def test_bending_rule_matches_figure_n5():
    gold = read_golden()
    b = oracle.bending_rule(5, 5)
    pts = sorted(set((float(u), float(v)) for u, v in b[:, :2]))
    assert np.allclose(np.array(pts), np.array(_as_set(gold["bending"])), atol=1e-12)
    assert len(pts) == 32


@pytest.mark.parametrize("Nu,Nv", [(3, 3), (4, 4), (5, 5), (6, 9), (12, 7), (18, 18)])
def test_rule_counts_and_weights(Nu, Nv):
    r = oracle.membrane_rule(Nu, Nv)
    b = oracle.bending_rule(Nu, Nv)
    assert abs(r[:, 2].sum() - Nu * Nv) < 1e-12
    assert abs(b[:, 2].sum() - Nu * Nv) < 1e-12
    if Nu == Nv:
        N = Nu
        assert len(r) == 36 + 24 * (N - 2) + 2 * (N - 3) ** 2 + 8 * (N - 3) + 4
        assert len(set(map(tuple, b[:, :2]))) == (N - 1) * (N + 3)
    # every point lies in (the closure of) the span it is evaluated in
    for rule in (r, b):
        assert (rule[:, 0] >= rule[:, 3] - 1e-12).all() and (rule[:, 0] <= rule[:, 3] + 1 + 1e-12).all()
        assert (rule[:, 1] >= rule[:, 4] - 1e-12).all() and (rule[:, 1] <= rule[:, 4] + 1 + 1e-12).all()


def test_membrane_interior_stencil_is_2x3():
    """Interior points on knot lines touch only two bases across the line (Sec. 4.1)."""
    n = 10
    kn = syn.open_uniform_knots(n)
    r = oracle.membrane_rule(n - 2, n - 2)
    for u, v, w, k, l in r:
        if 1 <= u <= n - 3 and 1 <= v <= n - 3 and (u % 1 == 0 or v % 1 == 0):
            coord = u if u % 1 == 0 else v
            span = int(k if u % 1 == 0 else l)
            active = [a for a in range(3)
                      if abs(oracle.basis_piece(kn, span + a, span + 2, coord, 0)) > 1e-15
                      or abs(oracle.basis_piece(kn, span + a, span + 2, coord, 1)) > 1e-15]
            assert len(active) == 2


# ---- lumped mass --------------------------------------------------------------------------

@pytest.mark.parametrize("n_u,n_v,Lu,Lv,shear,spacing", [(8, 8, 1.0, 1.0, 0.0, 1), (10, 7, 2.0, 0.5, 0.0, 2),
                                                          (6, 9, 1.0, 1.5, 0.3, 3)])
def test_lumped_mass_closed_form(n_u, n_v, Lu, Lv, shear, spacing):
    """Knot spacing only reparametrises the sheet: mass and area must not depend on it."""
    ku, kv, rest = syn.flat_sheet(n_u, n_v, Lu, Lv, shear=shear, spacing=spacing)
    rho = 0.37
    sh = oracle.Sheet(n_u, n_v, ku, kv, rest, rho_area=rho)
    M = oracle.lumped_mass(sh).reshape(n_v, n_u)
    def a(n):
        v = np.ones(n)
        v[0] = v[-1] = 1 / 3
        v[1] = v[-2] = 2 / 3
        return v
    hu, hv = Lu / (n_u - 2), Lv / (n_v - 2)
    want = rho * hu * hv * np.outer(a(n_v), a(n_u))
    assert np.allclose(M, want, rtol=1e-13, atol=0)
    assert abs(M.sum() - rho * Lu * Lv) < 1e-13 * rho * Lu * Lv
