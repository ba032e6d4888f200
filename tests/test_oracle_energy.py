"""Pins for the oracle's membrane/bending energies, derivatives and projection (CPU only).

Pinned against: small-strain elasticity (plane-stress Young's modulus and Poisson contraction,
shear modulus), finite differences, exact results for affine and quadratic deformation fields
(linear precision and Marsden's identity), rigid-motion invariance, reflection symmetry,
LAPACK eigen-decomposition, an independent brute-force evaluator and full Gauss quadrature."""
import numpy as np
import pytest

import oracle
import synthetic as syn
from tests._bruteforce import Tiny


def make_sheet(n_u=8, n_v=None, L_u=1.0, L_v=None, shear=0.0, young=1e4, poisson=0.3, thickness=1e-3,
               mu_bend=1e-3, rho=0.2, membrane=0, mu_fbw=(0.0, 0.0, 0.0), spacing=1):
    n_v = n_u if n_v is None else n_v
    ku, kv, rest = syn.flat_sheet(n_u, n_v, L_u, L_v, spacing=spacing, shear=shear)
    return oracle.Sheet(n_u, n_v, ku, kv, rest, membrane, young, poisson, thickness,
                        mu_fbw[0], mu_fbw[1], mu_fbw[2], mu_bend, rho)


def rand_F(rng):
    return np.array([[1.0, 0.0], [0.0, 1.0], [0.0, 0.0]]) + 0.3 * rng.standard_normal((3, 2))


# ---- densities ----------------------------------------------------------------------------

def test_stvk_small_strain_uniaxial_stress_gives_young_modulus():
    """Uniaxial stress: minimising over the lateral stretch leaves Psi = E t eps^2 / 2 and a
    lateral strain of -nu eps (plane stress), to O(eps^3)."""
    from scipy.optimize import minimize_scalar
    E, nu, t = 2.5e4, 0.31, 1.3e-3
    eps = 1e-4
    f = lambda s2: oracle.membrane_density([[1 + eps, 0], [0, s2], [0, 0]], 0, E, nu, t)[0]
    res = minimize_scalar(f, bracket=(0.99, 1.0, 1.01), tol=1e-14)
    assert abs(res.fun / (0.5 * E * t * eps ** 2) - 1) < 1e-3
    assert abs((res.x - 1) / eps + nu) < 1e-3


def test_stvk_small_shear_gives_shear_modulus():
    E, nu, t = 1e4, 0.3, 1e-3
    gam = 1e-5
    psi = oracle.membrane_density([[1, gam], [0, 1], [0, 0]], 0, E, nu, t)[0]
    G = E / (2 * (1 + nu))
    assert abs(psi / (0.5 * G * t * gam ** 2) - 1) < 1e-4


def test_fbw_reduces_to_its_invariants():
    """Pure stretch of f1 only: Psi = mu_st1 (s - 1)^2; orthogonal columns carry no shear."""
    s = 1.2
    psi = oracle.membrane_density([[s, 0], [0, 1], [0, 0]], 1, mu_st1=3.0, mu_st2=5.0, mu_sh=7.0)[0]
    assert abs(psi - 3.0 * (s - 1) ** 2) < 1e-14
    c = 0.1
    psi = oracle.membrane_density([[1, c], [0, 1], [0, 0]], 1, mu_st1=0.0, mu_st2=0.0, mu_sh=7.0)[0]
    assert abs(psi - 7.0 * c * c) < 1e-14


@pytest.mark.parametrize("model", [0, 1])
def test_density_derivatives_by_finite_differences(model):
    rng = np.random.default_rng(11 + model)
    kw = dict(young=1e4, poisson=0.3, thickness=1e-3) if model == 0 else dict(mu_st1=3.0, mu_st2=2.0, mu_sh=0.7)
    for _ in range(5):
        F = rand_F(rng)
        psi, P, A = oracle.membrane_density(F, model, **kw)
        vecF = F.T.reshape(-1)              # column-major: r = 3*gamma + i
        h = 1e-6
        Pfd = np.zeros(6)
        Afd = np.zeros((6, 6))
        for r in range(6):
            dv = np.zeros(6)
            dv[r] = h
            Fp = (vecF + dv).reshape(2, 3).T
            Fm = (vecF - dv).reshape(2, 3).T
            Pfd[r] = (oracle.membrane_density(Fp, model, **kw)[0] - oracle.membrane_density(Fm, model, **kw)[0]) / (2 * h)
            Afd[:, r] = (oracle.membrane_density(Fp, model, **kw)[1].T.reshape(-1)
                         - oracle.membrane_density(Fm, model, **kw)[1].T.reshape(-1)) / (2 * h)
        assert np.allclose(P.T.reshape(-1), Pfd, rtol=1e-6, atol=1e-8 * np.abs(Pfd).max())
        assert np.allclose(A, Afd, rtol=1e-6, atol=1e-7 * np.abs(A).max())
        assert np.allclose(A, A.T, atol=1e-13 * np.abs(A).max())


def test_projection_matches_lapack():
    rng = np.random.default_rng(5)
    for _ in range(20):
        B = rng.standard_normal((6, 6))
        A = B + B.T
        w, V = np.linalg.eigh(A)
        want = (V * np.maximum(w, 0)) @ V.T
        got = oracle.project_psd6(A)
        assert np.allclose(got, want, atol=1e-13 * np.abs(A).max())
    # compressed StVK point: indefinite before, PSD after
    psi, P, A = oracle.membrane_density([[0.8, 0], [0, 0.9], [0, 0]], 0, 1e4, 0.3, 1e-3)
    assert np.linalg.eigvalsh(A).min() < 0
    assert np.linalg.eigvalsh(oracle.project_psd6(A)).min() > -1e-12 * np.abs(A).max()


# ---- whole-sheet invariants ---------------------------------------------------------------

@pytest.mark.parametrize("shear,spacing", [(0.0, 1), (0.35, 1), (0.2, 2)])
def test_affine_deformation_is_exact(shear, spacing):
    """phi = A X + b is reproduced exactly (linear precision), so F = A at every point, the
    membrane energy is area * Psi(A) and the bending energy vanishes, for any knot spacing."""
    sh = make_sheet(9, 7, 1.0, 0.8, shear=shear, spacing=spacing)
    A = np.array([[1.1, 0.2], [-0.1, 0.95], [0.3, -0.2]])
    x = sh.rest @ A.T + np.array([0.5, -1.0, 2.0])
    E, g, _ = oracle.assemble(sh, x, want_hessian=False)
    psi = oracle.membrane_density(A, 0, sh.young, sh.poisson, sh.thickness)[0]
    area = 1.0 * 0.8
    assert abs(E - area * psi) < 1e-12 * area * psi


def test_fbw_affine_field_energy_closed_form():
    """FBW on a whole sheet (Sec. 4.1, warp along u, weft along v): x = (s1 X + c Y, s2 Y, 0)
    gives f1 = (s1, 0, 0), f2 = (c, s2, 0) at every point, so E = area * (mu_sh (s1 c)^2 +
    mu_st1 (s1 - 1)^2 + mu_st2 (sqrt(c^2 + s2^2) - 1)^2), with three distinct moduli so that
    each is matched to its own invariant."""
    mu1, mu2, msh = 2.0, 5.0, 0.7
    sh = make_sheet(9, 7, 1.0, 0.8, membrane=1, mu_fbw=(mu1, mu2, msh))
    s1, s2, c = 1.15, 0.9, 0.25
    X, Y = sh.rest[:, 0], sh.rest[:, 1]
    x = np.stack([s1 * X + c * Y, s2 * Y, np.zeros_like(X)], axis=1)
    E, _, _ = oracle.assemble(sh, x, want_hessian=False)
    psi = msh * (s1 * c) ** 2 + mu1 * (s1 - 1) ** 2 + mu2 * (np.hypot(c, s2) - 1) ** 2
    area = 1.0 * 0.8
    assert abs(E - area * psi) < 1e-12 * area * psi


def test_rigid_motion_has_zero_energy_and_gradient():
    sh = make_sheet(10, shear=0.2)
    from scipy.spatial.transform import Rotation
    R = Rotation.from_rotvec([0.3, -0.7, 0.4]).as_matrix()
    x = syn.embed(sh.rest) @ R.T + np.array([1.0, 2.0, -3.0])
    E, g, _ = oracle.assemble(sh, x, want_hessian=False)
    assert abs(E) < 1e-20
    assert np.abs(g).max() < 1e-13


def test_paraboloid_bending_energy_closed_form():
    """phi = (X1, X2, kappa (X1^2 + X2^2) / 2) from Greville / Marsden coefficients has
    Laplacian (0, 0, 2 kappa) everywhere: E_bend = 2 mu kappa^2 L^2, independently of the
    bending quadrature. A saddle kappa X1 X2 has zero Laplacian."""
    n, L, kap, mu = 12, 1.0, 0.7, 0.013
    sh = make_sheet(n, young=0.0, mu_bend=mu)
    kn = syn.open_uniform_knots(n)
    N = n - 2
    h = L / N
    g = syn.greville(kn, n) * h
    m = kn[1:n + 1] * kn[2:n + 2] * h * h          # coefficients reproducing X^2
    x = syn.embed(sh.rest)
    mi, mj = np.meshgrid(m, m)
    x[:, 2] = 0.5 * kap * (mi + mj).ravel()
    E, _, _ = oracle.assemble(sh, x, want_hessian=False)
    assert abs(E - 2 * mu * kap ** 2 * L ** 2) < 1e-12 * E
    gi, gj = np.meshgrid(g, g)
    x[:, 2] = kap * (gi * gj).ravel()
    E, _, _ = oracle.assemble(sh, x, want_hessian=False)
    assert abs(E) < 1e-24


def test_curved_rest_geometry_against_numerical_inverse():
    """Inverse-map derivatives (Sec. 4.1) and the Laplacian coefficients (Sec. 4.2) on a
    curved rest shape against finite differences of a Newton-inverted rest map."""
    n = 7
    ku, kv, rest = syn.flat_sheet(n)
    rng = np.random.default_rng(2)
    rest = rest + 0.02 * rng.standard_normal(rest.shape)
    sh = oracle.Sheet(n, n, ku, kv, rest, 0, 1e4, 0.3, 1e-3, 0, 0, 0, 1e-3, 0.2)

    def X_of(u, v):   # span units == knot units here
        return oracle.surface_point(sh, syn.embed(rest), u, v)[:2]

    def uv_of(X, guess):
        uv = np.array(guess, dtype=float)
        for _ in range(50):
            r = X_of(*uv) - X
            h = 1e-7
            J = np.stack([(X_of(uv[0] + h, uv[1]) - X_of(uv[0] - h, uv[1])) / (2 * h),
                          (X_of(uv[0], uv[1] + h) - X_of(uv[0], uv[1] - h)) / (2 * h)], axis=1)
            uv = uv - np.linalg.solve(J, r)
            if np.abs(r).max() < 1e-15:
                break
        return uv

    for (k, l, u, v) in [(2, 2, 2.37, 2.61), (1, 3, 1.5, 3.2), (0, 0, 0.4, 0.7)]:
        K, detJ, lap = oracle.point_geometry(sh, k, l, u, v)
        X0 = X_of(u, v)
        h = 1e-4
        Kfd = np.zeros((2, 2))
        for b in range(2):
            e = np.zeros(2)
            e[b] = h
            Kfd[:, b] = (uv_of(X0 + e, (u, v)) - uv_of(X0 - e, (u, v))) / (2 * h)
        assert np.allclose(K, Kfd, rtol=1e-6)
        lapfd = np.zeros(2)
        hh = 2e-3
        for b in range(2):
            e = np.zeros(2)
            e[b] = hh
            lapfd += (uv_of(X0 + e, (u, v)) - 2 * np.array([u, v]) + uv_of(X0 - e, (u, v))) / hh ** 2
        assert np.allclose(lap[2:4], lapfd, rtol=2e-3, atol=2e-3 * np.abs(K).max() ** 2)
        assert abs(lap[0] - (K[0] @ K[0])) < 1e-12 and abs(lap[1] - (K[1] @ K[1])) < 1e-12


def test_affine_field_on_curved_rest_has_no_bending():
    """phi = A X + b on a curved rest shape: Laplacian(phi) = 0 at every point only if the
    inverse-map second derivatives are right."""
    n = 8
    ku, kv, rest = syn.flat_sheet(n)
    rng = np.random.default_rng(9)
    rest = rest + 0.015 * rng.standard_normal(rest.shape)
    sh = oracle.Sheet(n, n, ku, kv, rest, 0, 0.0, 0.3, 1e-3, 0, 0, 0, 1.0, 0.2)
    A = np.array([[1.0, 0.3], [0.2, 0.9], [0.5, -0.4]])
    x = rest @ A.T
    E, g, _ = oracle.assemble(sh, x, want_hessian=False)
    assert abs(E) < 1e-22
    x2 = x + 1e-3 * syn.smooth_field(n, n, 4)
    assert oracle.assemble(sh, x2, want_hessian=False)[0] > 1e-10


def fd_check(sh, x, dt=None, xhat=None, grav=None, h=1e-6, ntest=12, seed=0):
    rng = np.random.default_rng(seed)
    E, g, H = oracle.assemble(sh, x, xhat, dt, grav, project=False)
    Hd = oracle.stencil_to_csr(sh, H).toarray()
    idx = rng.choice(x.size, size=ntest, replace=False)
    for r in idx:
        d = np.zeros(x.size)
        d[r] = h
        Ep = oracle.energy(sh, x.reshape(-1) + d, xhat, dt, grav)
        Em = oracle.energy(sh, x.reshape(-1) - d, xhat, dt, grav)
        assert abs((Ep - Em) / (2 * h) - g.reshape(-1)[r]) < 1e-6 * max(1e-3, np.abs(g).max())
        gp = oracle.assemble(sh, x.reshape(-1) + d, xhat, dt, grav, project=False, want_hessian=False)[1].reshape(-1)
        gm = oracle.assemble(sh, x.reshape(-1) - d, xhat, dt, grav, project=False, want_hessian=False)[1].reshape(-1)
        col = (gp - gm) / (2 * h)
        assert np.allclose(Hd[:, r], col, atol=1e-6 * np.abs(Hd).max())
    assert np.allclose(Hd, Hd.T, atol=1e-12 * np.abs(Hd).max())


@pytest.mark.parametrize("membrane", [0, 1])
def test_gradient_and_hessian_by_finite_differences(membrane):
    sh = make_sheet(7, 6, 1.0, 0.9, membrane=membrane, mu_fbw=(2.0, 3.0, 0.5), mu_bend=0.01)
    x = syn.embed(sh.rest) + syn.smooth_field(7, 6, 3, amp=0.08)
    xhat = x + 0.01 * syn.smooth_field(7, 6, 8)
    fd_check(sh, x, dt=0.01, xhat=xhat, grav=np.array([0.0, -9.81, 1.0]), seed=membrane)


def test_projected_hessian_is_psd_and_symmetric():
    sh = make_sheet(8, mu_bend=1e-4)
    x = syn.embed(sh.rest)
    x[:, 0] *= 0.85                                # compression makes StVK indefinite
    x += syn.smooth_field(8, 8, 1, amp=0.03)
    _, _, H0 = oracle.assemble(sh, x, project=False)
    _, _, H1 = oracle.assemble(sh, x, project=True)
    D0 = oracle.stencil_to_csr(sh, H0).toarray()
    D1 = oracle.stencil_to_csr(sh, H1).toarray()
    assert np.linalg.eigvalsh(D0).min() < -1e-6 * np.abs(D0).max()
    assert np.linalg.eigvalsh(D1).min() > -1e-12 * np.abs(D1).max()
    assert np.allclose(D1, D1.T, atol=1e-14 * np.abs(D1).max())
    E, g, He = oracle.element_egh(sh, x, project=True)
    for e in range(0, len(E), 7):
        assert np.linalg.eigvalsh(He[e]).min() > -1e-12 * np.abs(He[e]).max()


def test_reflection_symmetry_even_spans():
    """For an even number of spans the rules map onto themselves under u -> N - u and
    v -> N - v, so the energy of a reflected state is unchanged (R2 is symmetric)."""
    n = 10
    sh = make_sheet(n, mu_bend=0.02)
    x = syn.embed(sh.rest) + syn.smooth_field(n, n, 21, amp=0.06)
    E0 = oracle.energy(sh, x)
    X = x.reshape(n, n, 3)
    xr = X[:, ::-1, :].copy()
    xr[..., 0] = 1.0 - xr[..., 0]
    E1 = oracle.energy(sh, xr.reshape(-1, 3))
    xr2 = X[::-1, :, :].copy()
    xr2[..., 1] = 1.0 - xr2[..., 1]
    E2 = oracle.energy(sh, xr2.reshape(-1, 3))
    assert abs(E1 - E0) < 1e-12 * E0 and abs(E2 - E0) < 1e-12 * E0


# ---- independent brute force --------------------------------------------------------------

@pytest.mark.parametrize("n_u,n_v,shear", [(6, 6, 0.0), (7, 5, 0.0), (6, 8, 0.25)])
def test_bruteforce_energy_matches(n_u, n_v, shear):
    E_, nu_, t_, mub = 2e4, 0.25, 1e-3, 3e-3
    sh = make_sheet(n_u, n_v, 1.0, 1.2, shear=shear, young=E_, poisson=nu_, thickness=t_, mu_bend=mub)
    tiny = Tiny(n_u, n_v, sh.rest, (E_, nu_, t_), mub, 0.2)
    for seed in (1, 2):
        x = syn.embed(sh.rest) + syn.smooth_field(n_u, n_v, seed, amp=0.1)
        x += 0.01 * np.random.default_rng(seed).standard_normal(x.shape)
        want = tiny.elastic_energy(x)
        got = oracle.energy(sh, x)
        assert abs(got - want) < 1e-12 * abs(want)


def test_bruteforce_fd_gradient_matches_oracle():
    n = 6
    sh = make_sheet(n, young=1e4, poisson=0.3, thickness=1e-3, mu_bend=2e-3)
    tiny = Tiny(n, n, sh.rest, (1e4, 0.3, 1e-3), 2e-3, 0.2)
    x = syn.embed(sh.rest) + syn.smooth_field(n, n, 5, amp=0.1)
    _, g, _ = oracle.assemble(sh, x, want_hessian=False)
    h = 1e-6
    for r in np.random.default_rng(0).choice(x.size, 8, replace=False):
        d = np.zeros(x.size)
        d[r] = h
        fd = (tiny.elastic_energy((x.reshape(-1) + d).reshape(-1, 3)) - tiny.elastic_energy((x.reshape(-1) - d).reshape(-1, 3))) / (2 * h)
        assert abs(fd - g.reshape(-1)[r]) < 1e-6 * np.abs(g).max()


def test_reduced_rules_agree_with_full_gauss_on_exact_fields():
    """Affine fields (membrane) and quadratic fields (bending) are integrated exactly by the
    reduced rules, so they equal a full 3x3 Gauss rule on every span."""
    n = 7
    sh = make_sheet(n, young=1e4, mu_bend=0.0)
    tiny = Tiny(n, n, sh.rest, (1e4, 0.3, 1e-3), 0.0, 0.2)
    A = np.array([[1.05, 0.1], [0.0, 0.97], [0.2, 0.1]])
    x = sh.rest @ A.T
    assert abs(tiny.elastic_energy(x) - tiny.elastic_energy(x, full_gauss=True)) < 1e-13 * tiny.elastic_energy(x)
    tb = Tiny(n, n, sh.rest, (0.0, 0.3, 1e-3), 0.05, 0.2)
    kn = syn.open_uniform_knots(n)
    h = 1.0 / (n - 2)
    m = kn[1:n + 1] * kn[2:n + 2] * h * h
    mi, mj = np.meshgrid(m, m)
    xq = syn.embed(sh.rest)
    xq[:, 2] = (0.3 * mi + 0.8 * mj).ravel()
    a, b = tb.elastic_energy(xq), tb.elastic_energy(xq, full_gauss=True)
    assert abs(a - b) < 1e-12 * b
