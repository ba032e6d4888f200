"""Pins for the oracle's partial factorization (Sec. 5.3: Eq. "per iteration solve", Eq. "Woodbury",
Eq. "Neumann expansion", the Gershgorin bound).

Checked against what the mathematics fixes, not against the oracle's own steps:
- the two bounds against dense spectra computed by LAPACK: |lambda(B)| <= Gershgorin radius,
  lambda_min(D) on the free DOFs >= the diagonal-pass lower bound, |D^-1 B|_2 <= their ratio;
- the series against a dense solve of the merged Newton matrix assembled directly (inertia plus
  elasticity plus the whole barrier Hessian, pinned rows and columns removed), within the
  truncation bound rho^(K+1) / (1 - rho) |D^-1 b| that the series must meet, and with an error
  that shrinks as terms are added;
- the special cases: no contact (one term, a plain solve), the merged branch (the dense solve),
  pinned control points (identity rows: x = b there).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synthetic as syn
from oracle import contact_ref as cr
from oracle import partial_ref as pr


def _system(n_u=9, n_v=8, n_pairs=40, scale=1.0, seed=3, pins=True):
    ku, kv, rest = syn.flat_sheet(n_u, n_v)
    m = syn.stvk_material(young=1e4, thickness=1e-3)
    sh = oracle.Sheet(n_u, n_v, ku, kv, rest, m.membrane, m.young, m.poisson, m.thickness, m.mu_st1, m.mu_st2,
                      m.mu_sh, m.mu_bend, m.rho_area)
    x = syn.embed(rest) + syn.smooth_field(n_u, n_v, seed, amp=0.03)
    x[:, 0] *= 0.95                                   # some compression: projected membrane points
    dt = 0.01
    mask = np.zeros(sh.n_cp, dtype=bool)
    if pins:
        mask[[0, n_u - 1]] = True
    _, _, H = oracle.assemble(sh, x, x, dt, np.array([0.0, 0.0, -9.81]), mask)
    A = oracle.stencil_to_csr(sh, H)
    uv, tris, grid = syn.contact_mesh(n_u, n_v)
    pv, Hp, _ = syn.contact_pairs(uv, tris, grid, n_pairs, seed=seed, scale=scale)
    Hc, _ = cr.contact_to_cp(sh, uv, pv, Hp)
    mass = oracle.lumped_mass(sh)
    b = np.random.default_rng(seed).standard_normal((sh.n_cp, 3))
    return sh, A, Hc, mass, dt, mask, b


def _dense_merged(A, Hc, mask):
    """The merged Newton matrix written directly: A + P Hc P with P the free-DOF projector."""
    P = np.diag(pr.dof_mask(len(mask), mask))
    return A.toarray() + P @ Hc.toarray() @ P


@pytest.mark.parametrize("scale", [0.05, 1.0, 30.0])
def test_bounds_hold_against_dense_spectra(scale):
    sh, A, Hc, mass, dt, mask, b = _system(scale=scale)
    Hd, Ho = pr.split_barrier(Hc, sh.n_cp, mask)
    D = (A + Hd).toarray()
    B = Ho.toarray()
    r_b = pr.gershgorin_radius_max(Ho)
    d_lo = pr.lambda_min_lower(mass, dt, Hd, mask)
    lam_b = np.abs(np.linalg.eigvalsh(B)).max()
    free = pr.dof_mask(sh.n_cp, mask) > 0
    Dff = D[np.ix_(free, free)]
    lam_d = np.linalg.eigvalsh(0.5 * (Dff + Dff.T)).min()
    op = np.linalg.norm(np.linalg.solve(D, B), 2)
    print(f"scale {scale}: |lambda(B)| {lam_b:.4g} <= {r_b:.4g}; lambda_min(D) {lam_d:.4g} >= {d_lo:.4g}; "
          f"|D^-1 B| {op:.4g} <= {r_b / d_lo:.4g}")
    assert lam_b <= r_b * (1 + 1e-12)
    assert lam_d >= d_lo * (1 - 1e-10)
    assert op <= r_b / d_lo * (1 + 1e-10)
    # the split: D keeps the elasticity block pattern, and the two parts add up to the barrier
    Dp = sp.csr_matrix(A + Hd)
    assert set(zip(*Dp.nonzero())) <= set(zip(*sp.csr_matrix(A).nonzero())) | set(zip(*np.nonzero(np.kron(np.eye(sh.n_cp), np.ones((3, 3))))))
    P = np.diag(pr.dof_mask(sh.n_cp, mask))
    assert np.allclose((Hd + Ho).toarray(), P @ Hc.toarray() @ P, rtol=0, atol=1e-14)


def test_series_meets_its_truncation_bound_against_the_merged_solve():
    sh, A, Hc, mass, dt, mask, b = _system(scale=0.05)
    xs = np.linalg.solve(_dense_merged(A, Hc, mask), b.reshape(-1))
    Hd, _ = pr.split_barrier(Hc, sh.n_cp, mask)
    t0 = np.linalg.solve((A + Hd).toarray(), b.reshape(-1))
    errs = []
    for terms in (1, 2, 3, 5):
        res = pr.solve(A, Hc, mass, dt, b, mask, rho_max=0.9, max_terms=terms, series_tol=0.0)
        assert res.triggered and res.terms == terms and res.rho_bound < 0.9
        err = np.linalg.norm(res.x.reshape(-1) - xs)
        bound = res.rho_bound ** terms / (1.0 - res.rho_bound) * np.linalg.norm(t0)
        print(f"terms {terms}: rho {res.rho_bound:.3e} err {err:.3e} bound {bound:.3e}")
        assert err <= bound * (1 + 1e-9) + 1e-13 * np.linalg.norm(xs)
        errs.append(err)
    assert errs[0] > 0 and all(e1 < e0 for e0, e1 in zip(errs, errs[1:]))
    full = pr.solve(A, Hc, mass, dt, b, mask, rho_max=0.9, series_tol=1e-13)
    assert full.triggered
    assert np.linalg.norm(full.x.reshape(-1) - xs) <= 1e-11 * np.linalg.norm(xs)


def test_merged_branch_is_the_dense_solve():
    sh, A, Hc, mass, dt, mask, b = _system(scale=30.0)
    res = pr.solve(A, Hc, mass, dt, b, mask, rho_max=0.5)
    assert not res.triggered and res.rho_bound > 0.5
    xs = np.linalg.solve(_dense_merged(A, Hc, mask), b.reshape(-1))
    assert np.linalg.norm(res.x.reshape(-1) - xs) <= 1e-11 * np.linalg.norm(xs)


def test_no_contact_is_one_plain_solve():
    sh, A, Hc, mass, dt, mask, b = _system()
    res = pr.solve(A, sp.csr_matrix(Hc.shape), mass, dt, b, mask)
    assert res.triggered and res.terms == 1 and res.rho_bound == 0.0
    xs = np.linalg.solve(A.toarray(), b.reshape(-1))
    assert np.linalg.norm(res.x.reshape(-1) - xs) <= 1e-12 * np.linalg.norm(xs)


@pytest.mark.parametrize("force", ["series", "merged"])
def test_pinned_rows_are_identity_rows(force):
    sh, A, Hc, mass, dt, mask, b = _system(scale=0.05)
    res = pr.solve(A, Hc, mass, dt, b, mask, force=force, series_tol=1e-13)
    assert np.array_equal(res.x[mask], b[mask])
