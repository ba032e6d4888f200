"""Pins for the oracle's implicit-Euler / projected-Newton step (CPU only).

Pinned against: conservation of linear momentum without pins or gravity (the contact-free
form of the paper's two-plate test, Sec. 6.1), the Kirchhoff simply-supported plate closed
form of the paper's bending benchmark (Sec. 6.2, "Convergence under Refinement (Bending)"),
one-iteration exactness on a quadratic energy checked by an independent dense solve, pinned
CPs at moved targets, the step rule's stop against dense-solve directions, and the first
direction against a dense solve with the projected Hessian where projection matters."""
import numpy as np
import pytest

import oracle
import synthetic as syn


def sheet_from_scene(sc):
    m = sc.material
    return oracle.Sheet(sc.n_u, sc.n_v, sc.knots_u, sc.knots_v, sc.rest, m.membrane, m.young, m.poisson,
                        m.thickness, m.mu_st1, m.mu_st2, m.mu_sh, m.mu_bend, m.rho_area)


def test_momentum_is_conserved_without_pins_or_gravity():
    sc = syn.hanging_sheet(10, seed=3)
    sh = sheet_from_scene(sc)
    rng = np.random.default_rng(4)
    x = sc.x0 + syn.smooth_field(10, 10, 6, amp=0.02)
    v = 0.3 * rng.standard_normal(x.shape)
    M = oracle.lumped_mass(sh)
    p0 = (M[:, None] * v).sum(axis=0)
    res = oracle.newton_step(sh, x, v, 0.01, np.zeros(3), rtol=1e-8)
    p1 = (M[:, None] * res.v).sum(axis=0)
    # internal forces sum to zero, so sum_a M_a (x_a - xhat_a) = dt^2 sum_a g_a at the end
    bound = 0.01 * np.sqrt(x.size) * res.g_norm + 1e-14 * np.abs(M[:, None] * v).sum()
    assert np.abs(p1 - p0).max() <= bound
    assert res.g_norm <= 1e-8 * res.g0_norm


def test_hanging_step_converges_and_is_a_stationary_point():
    sc = syn.hanging_sheet(12, seed=1)
    sh = sheet_from_scene(sc)
    res = oracle.newton_step(sh, sc.x0, sc.v0, sc.dt, sc.gravity, sc.pins, sc.pin_targets(0), rtol=1e-9)
    assert res.g_norm <= 1e-9 * res.g0_norm
    assert np.allclose(res.x[sc.pins], sc.pin_targets(0))
    mask = np.zeros(sh.n_cp, dtype=bool)
    mask[sc.pins] = True
    E, g, _ = oracle.assemble(sh, res.x, sc.x0 + sc.dt * sc.v0, sc.dt, sc.gravity, mask, want_hessian=False)
    assert np.linalg.norm(g) <= 1e-9 * res.g0_norm
    # the sheet falls: free CPs move along gravity (-y)
    assert res.v[~mask, 1].mean() < 0


def test_both_starts_reach_the_same_step():
    """The paper leaves the first Newton iterate open: x_n and the inertial prediction
    xhat = x_n + dt v_n start the same minimisation. On a sheet moving with a smooth velocity
    field both reach the same stationary point, and the predictor start, where the inertia term's
    gradient vanishes, begins with a smaller gradient."""
    sc = syn.hanging_sheet(10, seed=2)
    sh = sheet_from_scene(sc)
    v = syn.smooth_field(10, 10, 8, amp=0.3)
    v[sc.pins] = 0.0
    # (1e-7: tighter, the oracle's plain energy comparison meets FP64 rounding of E)
    a = oracle.newton_step(sh, sc.x0, v, sc.dt, sc.gravity, sc.pins, sc.pin_targets(0), rtol=1e-7)
    b = oracle.newton_step(sh, sc.x0, v, sc.dt, sc.gravity, sc.pins, sc.pin_targets(0), rtol=1e-7,
                           start="predictor")
    d = np.linalg.norm(b.x - a.x) / np.linalg.norm(a.x - sc.x0)
    assert d < 1e-5
    assert b.g0_norm < a.g0_norm
    with pytest.raises(ValueError):
        oracle.newton_step(sh, sc.x0, v, sc.dt, sc.gravity, sc.pins, sc.pin_targets(0), start="xhat")


def test_quadratic_energy_needs_one_newton_iteration():
    """Bending plus inertia only (zero membrane stiffness) is quadratic: one Newton iteration
    lands on the minimiser, which equals a dense solve of the same linear system."""
    n = 8
    sc = syn.hanging_sheet(n, seed=2, material=syn.stvk_material(young=0.0, mu_bend=0.05))
    sh = sheet_from_scene(sc)
    x0 = sc.x0 + syn.smooth_field(n, n, 2, amp=0.05)
    res = oracle.newton_step(sh, x0, sc.v0, sc.dt, sc.gravity, sc.pins, x0[sc.pins], fixed_iters=1)
    mask = np.zeros(sh.n_cp, dtype=bool)
    mask[sc.pins] = True
    E, g, H = oracle.assemble(sh, res.x, x0, sc.dt, sc.gravity, mask, want_hessian=True)
    assert np.linalg.norm(g) < 1e-10 * res.g0_norm
    E0, g0, H0 = oracle.assemble(sh, x0, x0, sc.dt, sc.gravity, mask)
    dense = oracle.stencil_to_csr(sh, H0).toarray()
    p = np.linalg.solve(dense, -g0.reshape(-1))
    assert np.allclose(res.x.reshape(-1), x0.reshape(-1) + p, atol=1e-12 * np.abs(x0).max())


def test_pinned_cps_reach_moved_targets():
    """Dirichlet conditions (Sec. 5.1): pinned CPs end at their targets whatever x_n was, and
    their velocity is (target - x_n) / dt; the free CPs end at a stationary point."""
    sc = syn.hanging_sheet(10, seed=5)
    sh = sheet_from_scene(sc)
    targets = sc.x0[sc.pins] + np.array([[0.02, -0.01, 0.015], [-0.02, 0.005, 0.01]])
    # (1e-6: tighter, the oracle's plain energy comparison meets FP64 rounding of E)
    res = oracle.newton_step(sh, sc.x0, sc.v0, sc.dt, sc.gravity, sc.pins, targets, rtol=1e-6)
    assert np.array_equal(res.x[sc.pins], targets)
    assert np.allclose(res.v[sc.pins], (targets - sc.x0[sc.pins]) / sc.dt, rtol=1e-12, atol=0)
    assert res.g_norm <= 1e-6 * res.g0_norm


def _dense_direction(sh, x, xhat, dt, gravity, mask, project=True):
    _, g, H = oracle.assemble(sh, x, xhat, dt, gravity, mask, project=project)
    A = oracle.stencil_to_csr(sh, H).toarray()
    return np.linalg.solve(A, -g.reshape(-1)).reshape(-1, 3), A


def test_step_rule_stops_at_the_first_small_direction():
    """The paper's stopping rule (Sec. 6): stop once the Newton direction p at the current
    iterate has |p|_inf / dt <= atol. At the returned iterate the direction (recomputed by a
    dense solve) meets the bound and at the iterate before it does not; dt = 0.01 makes the
    division by dt matter."""
    sc = syn.compressed_sheet(10, seed=3)
    sh = sheet_from_scene(sc)
    v = syn.smooth_field(10, 10, 9, amp=0.5)
    v[sc.pins] = 0.0
    xhat = sc.x0 + sc.dt * v
    mask = np.zeros(sh.n_cp, dtype=bool)
    mask[sc.pins] = True
    atol = 1e-3
    res = oracle.newton_step(sh, sc.x0, v, sc.dt, sc.gravity, sc.pins, sc.pin_targets(0), atol=atol)
    assert res.iters >= 2
    p, _ = _dense_direction(sh, res.x, xhat, sc.dt, sc.gravity, mask)
    assert np.abs(p).max() / sc.dt <= atol
    prev = oracle.newton_step(sh, sc.x0, v, sc.dt, sc.gravity, sc.pins, sc.pin_targets(0),
                              fixed_iters=res.iters - 1)
    p, _ = _dense_direction(sh, prev.x, xhat, sc.dt, sc.gravity, mask)
    assert np.abs(p).max() / sc.dt > atol


def test_newton_direction_uses_the_projected_hessian():
    """Projected Newton (Sec. 5.1): on a compressed sheet, where per-point projection changes
    the Hessian and the unprojected system is indefinite, the first step is alpha_0 times the
    dense solve with the projected Hessian, and that direction descends."""
    sc = syn.compressed_sheet(10, seed=4, compression=0.2)
    sh = sheet_from_scene(sc)
    mask = np.zeros(sh.n_cp, dtype=bool)
    mask[sc.pins] = True
    p, A = _dense_direction(sh, sc.x0, sc.x0, 1.0, sc.gravity, mask)
    _, A_raw = _dense_direction(sh, sc.x0, sc.x0, 1.0, sc.gravity, mask, project=False)
    assert np.linalg.eigvalsh(A).min() > 0 > np.linalg.eigvalsh(A_raw).min()
    _, g, _ = oracle.assemble(sh, sc.x0, sc.x0, 1.0, sc.gravity, mask, want_hessian=False)
    assert float(np.sum(g * p)) < 0
    res = oracle.newton_step(sh, sc.x0, sc.v0, 1.0, sc.gravity, sc.pins, sc.pin_targets(0), fixed_iters=1)
    step = res.x - sc.x0
    assert np.allclose(step, res.alphas[0] * p, rtol=0, atol=1e-10 * np.abs(step).max())


def plate_deflection(N):
    """Square plate, bending only, boundary CPs fixed (simply supported: the edge is held,
    slopes are free), uniform load q = 9.81 per unit area; static solve (no inertia)."""
    n = N + 2
    E, nu, h, q = 2e6, 0.03, 0.01, 9.81
    D = syn.plate_bending_stiffness(E, nu, h)
    ku, kv, rest = syn.flat_sheet(n)
    # rho_area = 1 turns "gravity" into a load of q per unit area through the lumped mass
    sh = oracle.Sheet(n, n, ku, kv, rest, 0, 0.0, nu, h, 0, 0, 0, D, 1.0)
    x = syn.embed(rest)
    pins = np.array([a for a in range(n * n) if a % n in (0, n - 1) or a // n in (0, n - 1)])
    mask = np.zeros(n * n, dtype=bool)
    mask[pins] = True
    _, g, H = oracle.assemble(sh, x, None, None, np.array([0.0, 0.0, -q]), mask)
    A = oracle.stencil_to_csr(sh, H)
    import scipy.sparse.linalg as spla
    p = spla.spsolve(A.tocsc(), -g.reshape(-1)).reshape(-1, 3)
    xs = x + p
    return -oracle.surface_point(sh, xs, N / 2, N / 2)[2]


def test_plate_benchmark_converges_to_kirchhoff_solution():
    """Max deflection 0.048744 q a^4 (1 - nu^2) / (E h^3) (Sec. 6.2; 0.23887 m here)."""
    exact = 0.048744 * 9.81 * (1 - 0.03 ** 2) / (2e6 * 0.01 ** 3)
    errs = [abs(plate_deflection(N) - exact) / exact for N in (8, 16, 32)]
    assert errs[2] < 0.01
    assert errs[0] > errs[1] > errs[2]
