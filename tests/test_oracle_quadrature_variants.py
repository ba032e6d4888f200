"""Pins for the oracle's comparison quadrature rules (Sec. 6.5, "Effectiveness and Minimality of
Reduced Integration"): the standard 2x2 Gauss rule on the interior knot spans for membrane and
bending (configuration (A) of the timing breakdown), a single midpoint per interior span for
the membrane (the "1x1" rule that admits hourglass modes), and 2x2 instead of 3x3 Gauss on the
four corner spans. Boundary spans keep the placement of Fig. "quadrature" unless stated.

Checked against what the definitions fix: closed-form point counts, the total weight, exact
integration of polynomials of the degree each Gauss rule is exact for, an independent
brute-force evaluator of the energy, and the hourglass modes the paper reports for the 1x1 rule
(an oscillating displacement whose membrane stiffness vanishes relative to the other rules as
the sheet is refined)."""
import numpy as np
import pytest

import oracle
import synthetic as syn
from tests._bruteforce import Tiny

RULES = ("reduced", "gauss2", "interior1", "corner2")


def m_count(rule, Nu, Nv):
    boundary = 36 + 12 * (Nu - 2) + 12 * (Nv - 2)
    dual = 4 + 4 * (Nu - 3) + 4 * (Nv - 3) + 2 * (Nu - 3) * (Nv - 3)
    return {"reduced": boundary + dual, "gauss2": boundary + 4 * (Nu - 2) * (Nv - 2),
            "interior1": boundary + (Nu - 2) * (Nv - 2), "corner2": boundary - 20 + dual}[rule]


def b_count(rule, Nu, Nv):
    ring = 2 * Nu + 2 * Nv - 4
    if rule == "gauss2":
        return ring + 4 * (Nu - 2) * (Nv - 2)
    return ring + 4 * (Nu - 1) * (Nv - 1)


@pytest.mark.parametrize("rule", RULES)
@pytest.mark.parametrize("Nu,Nv", [(3, 3), (5, 7), (8, 4), (6, 6)])
def test_counts_weights_and_spans(rule, Nu, Nv):
    m = oracle.membrane_rule(Nu, Nv, rule)
    b = oracle.bending_rule(Nu, Nv, rule)
    assert len(m) == m_count(rule, Nu, Nv)
    assert len(b) == b_count(rule, Nu, Nv)
    for pts in (m, b):
        assert abs(pts[:, 2].sum() - Nu * Nv) < 1e-12
        u, v, k, l = pts[:, 0], pts[:, 1], pts[:, 3], pts[:, 4]
        assert np.all((u >= k - 1e-12) & (u <= k + 1 + 1e-12) & (v >= l - 1e-12) & (v <= l + 1 + 1e-12))


def _integrate(pts, i, j):
    return float(np.sum(pts[:, 2] * pts[:, 0] ** i * pts[:, 1] ** j))


@pytest.mark.parametrize("Nu,Nv", [(5, 7), (9, 6)])
def test_polynomial_exactness(Nu, Nv):
    """All rules integrate bilinear functions exactly; the membrane rule with 2x2 Gauss on the
    interior spans (and 3x3 / 3x2 on the boundary) is exact for bicubics, and the reduced rule
    is not (its interior cells use one point across)."""
    def exact(i, j):
        return Nu ** (i + 1) / (i + 1) * Nv ** (j + 1) / (j + 1)
    for rule in RULES:
        for pts in (oracle.membrane_rule(Nu, Nv, rule), oracle.bending_rule(Nu, Nv, rule)):
            for i in range(2):
                for j in range(2):
                    assert abs(_integrate(pts, i, j) / exact(i, j) - 1) < 1e-13, (rule, i, j)
    g2 = oracle.membrane_rule(Nu, Nv, "gauss2")
    for i in range(4):
        for j in range(4):
            assert abs(_integrate(g2, i, j) / exact(i, j) - 1) < 1e-13, (i, j)
    red = oracle.membrane_rule(Nu, Nv, "reduced")
    assert abs(_integrate(red, 2, 2) / exact(2, 2) - 1) > 1e-6


def _sheet(n_u, n_v, rule, mu_bend=3e-3, shear=0.0):
    ku, kv, rest = syn.flat_sheet(n_u, n_v, 1.0, 1.2, shear=shear)
    return oracle.Sheet(n_u, n_v, ku, kv, rest, 0, 2e4, 0.25, 1e-3, 0.0, 0.0, 0.0, mu_bend, 0.2, quadrature=rule)


@pytest.mark.parametrize("rule", ("gauss2", "interior1", "corner2"))
@pytest.mark.parametrize("n_u,n_v,shear", [(6, 7, 0.0), (7, 5, 0.3)])
def test_energy_matches_bruteforce(rule, n_u, n_v, shear):
    sh = _sheet(n_u, n_v, rule, shear=shear)
    tiny = Tiny(n_u, n_v, sh.rest, (2e4, 0.25, 1e-3), 3e-3, 0.2)
    for seed in (3, 4):
        x = syn.embed(sh.rest) + syn.smooth_field(n_u, n_v, seed, amp=0.1)
        x += 0.01 * np.random.default_rng(seed).standard_normal(x.shape)
        want = tiny.elastic_energy(x, rule=rule)
        got = oracle.energy(sh, x)
        assert abs(got - want) < 1e-12 * abs(want)
    # and the rules really differ
    assert abs(oracle.energy(sh, x) - oracle.energy(_sheet(n_u, n_v, "reduced", shear=shear), x)) > 1e-9 * abs(want)


def _inplane_stiffness(rule, n):
    """In-plane block of the membrane stiffness at the rest state (no bending, no inertia)."""
    sh = _sheet(n, n, rule, mu_bend=0.0)
    _, _, H = oracle.assemble(sh, syn.embed(sh.rest), project=False)
    K = oracle.stencil_to_csr(sh, H).toarray()
    idx = np.array([3 * a + c for a in range(sh.n_cp) for c in (0, 1)])
    return K[np.ix_(idx, idx)]


def _alternating_mode_stiffness(rule, n):
    """Rayleigh quotient of d_ij = (-1)^i e_1. Its gradient vanishes at every span midpoint
    (the midpoint derivative of a quadratic B-spline is (d_{k+2} - d_k)/2), so a midpoint rule
    sees it only through the boundary ring."""
    K = _inplane_stiffness(rule, n)
    m = np.zeros(K.shape[0])
    m[0::2] = (-1.0) ** (np.arange(n * n) % n)
    return m @ K @ m / (m @ m)


def test_rigid_motions_are_the_only_zero_modes():
    for rule in RULES:
        lam = np.linalg.eigvalsh(_inplane_stiffness(rule, 8))
        assert int(np.sum(np.abs(lam) < 1e-9 * lam.max())) == 3, rule


def test_interior_1x1_rule_has_hourglass_modes():
    """Sec. 6.5: one point per interior span lets an oscillating displacement escape the
    membrane energy everywhere but on the boundary ring, so its stiffness relative to the
    reduced rule falls as the sheet is refined; under the reduced rule and the denser
    comparison rules it stays of the same order."""
    ratios = {}
    for n in (10, 20):
        red = _alternating_mode_stiffness("reduced", n)
        ratios[n] = _alternating_mode_stiffness("interior1", n) / red
        for rule in ("gauss2", "corner2"):
            assert _alternating_mode_stiffness(rule, n) / red > 0.5, (rule, n)
    assert ratios[20] < 0.3
    assert ratios[20] < 0.6 * ratios[10]


def test_unknown_rule_is_rejected():
    with pytest.raises(ValueError):
        oracle.membrane_rule(5, 5, 7)
