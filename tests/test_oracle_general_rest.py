"""Pins for the oracle on general (non-affine) rest shapes: the distorted patches of the paper's
robustness study of its reduced quadrature (Sec. 6.2, "Support of Non-Rectangular Domains":
aspect ratio, skewed corners, sharp turns within an edge) and a curved quarter annulus.

Checked against what the definitions fix, independently of the oracle's code:
- the lumped mass against a brute-force Gauss integral of rho N_a |det J| built on the
  Cox-de Boor recursion (3-point Gauss per span is exact here: the integrand is a polynomial of
  degree 5 per direction);
- the membrane energy against a brute-force evaluation on the same reduced points, with the
  inverse map K = J^{-1} taken from the brute-force rest derivatives;
- the affine patch test: an affine deformation has a constant energy density, so the exact
  membrane energy is area x Psi(A). The reduced rule passes it exactly for rest maps whose
  det J it integrates exactly (rectangles, bilinear skews) and with an error that falls under
  refinement on curved patches, below 1e-3 at 20 x 20 CPs for edge turns down to 90 degrees,
  in line with the paper's report that the quadrature errors stay below 1e-3 and grow for sharp
  turns.
The inverse-map second derivatives behind the bending term are pinned in test_oracle_energy.py
(finite differences of a Newton-inverted map, and zero bending for an affine field on a curved
rest)."""
import numpy as np
import pytest

import oracle
import synthetic as syn
from tests._bruteforce import Tiny

CASES = [("aspect", 10.0), ("skew", 45.0), ("bend", 120.0), ("annulus", 0.5)]


def _gauss_rule(Nu, Nv, npt):
    t, w = np.polynomial.legendre.leggauss(npt)
    t, w = 0.5 * (t + 1.0), 0.5 * w
    return [(k + t[a], l + t[b], w[a] * w[b], k, l) for l in range(Nv) for k in range(Nu)
            for b in range(npt) for a in range(npt)]


def _jac(tiny, rest, k, l, u, v):
    d = tiny.derivs(rest, k, l, u, v)
    return np.stack([d["u"], d["v"]], axis=1)


def _sheet(n_u, n_v, rest, mu_bend=0.0):
    ku, kv = syn.open_uniform_knots(n_u), syn.open_uniform_knots(n_v)
    return oracle.Sheet(n_u, n_v, ku, kv, rest, 0, 1e4, 0.3, 1e-3, 0.0, 0.0, 0.0, mu_bend, 0.2)


@pytest.mark.parametrize("kind,param", CASES)
def test_lumped_mass_matches_bruteforce_integral(kind, param):
    n_u, n_v = 9, 7
    _, _, rest = syn.mapped_sheet(n_u, n_v, kind, param)
    sh = _sheet(n_u, n_v, rest)
    tiny = Tiny(n_u, n_v, rest, (1e4, 0.3, 1e-3), 0.0, 0.2)
    want = np.zeros(n_u * n_v)
    for u, v, w, k, l in _gauss_rule(n_u - 2, n_v - 2, 5):
        detJ = np.linalg.det(_jac(tiny, rest, k, l, u, v))
        for b in range(3):
            for a in range(3):
                i, j = k + a, l + b
                N = tiny.surface(np.eye(n_u * n_v)[j * n_u + i][:, None], u, v)
                want[j * n_u + i] += 0.2 * w * detJ * float(N[0])
    got = oracle.lumped_mass(sh)
    assert np.abs(got - want).max() < 1e-13 * want.max()


@pytest.mark.parametrize("kind,param", CASES)
def test_membrane_energy_matches_bruteforce_on_mapped_rest(kind, param):
    n_u, n_v = 8, 7
    _, _, rest = syn.mapped_sheet(n_u, n_v, kind, param)
    sh = _sheet(n_u, n_v, rest)
    tiny = Tiny(n_u, n_v, rest, (1e4, 0.3, 1e-3), 0.0, 0.2)
    x = syn.embed(rest) + syn.smooth_field(n_u, n_v, 5, amp=0.05)
    want = 0.0
    for u, v, w, k, l in tiny.membrane_points():
        J = _jac(tiny, rest, k, l, u, v)
        K = np.linalg.inv(J)
        d = tiny.derivs(x, k, l, u, v)
        F = np.stack([d["u"] * K[0, 0] + d["v"] * K[1, 0], d["u"] * K[0, 1] + d["v"] * K[1, 1]], axis=1)
        want += w * np.linalg.det(J) * tiny.stvk(F)
    got = oracle.energy(sh, x)
    assert abs(got - want) < 1e-12 * abs(want)


def _patch_error(kind, param, n):
    _, _, rest = syn.mapped_sheet(n, n, kind, param)
    sh = _sheet(n, n, rest, mu_bend=1.0)
    area = oracle.lumped_mass(sh).sum() / 0.2           # exact (pinned above)
    A = np.array([[1.05, 0.1], [0.02, 0.97], [0.2, -0.1]])
    x = rest @ A.T + np.array([0.1, 0.2, 0.3])
    Eg = 0.5 * (A.T @ A - np.eye(2))
    mu, lam = 1e4 * 1e-3 / 2.6, 1e4 * 1e-3 * 0.3 / 0.91
    psi = mu * np.sum(Eg * Eg) + 0.5 * lam * np.trace(Eg) ** 2
    return abs(oracle.energy(sh, x) - area * psi) / (area * psi)


@pytest.mark.parametrize("kind,param", [("aspect", 1.0), ("aspect", 10.0), ("skew", 60.0), ("skew", 30.0)])
def test_patch_test_exact_when_det_j_is_bilinear(kind, param):
    assert _patch_error(kind, param, 10) < 1e-13


@pytest.mark.parametrize("kind,param", [("bend", 150.0), ("bend", 120.0), ("bend", 90.0), ("annulus", 0.5)])
def test_patch_test_error_on_curved_patches(kind, param):
    e10, e20 = _patch_error(kind, param, 10), _patch_error(kind, param, 20)
    print(f"[patch test] {kind} {param}: relative membrane energy error {e10:.2e} (10x10), {e20:.2e} (20x20)")
    assert 1e-8 < e20 < 1e-3
    assert e20 < e10 / 3.0
