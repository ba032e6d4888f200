"""GPU parity of the partial factorization (Sec. 5.3: Eq. "per iteration solve", Eq. "Neumann
expansion", the Gershgorin trigger) against oracle/partial_ref.py, through the C ABI.

Both sides build their own inputs from the same seeded scene: the GPU assembles H with
bsc_assemble and converts the contact pairs with bsc_contact_hessian; the oracle assembles with
its C kernels and converts with contact_ref. FP64 with every PCG solve at 1e-14: the result
within 1e-10 of the oracle (LU solves), the bound within 1e-12, the same branch and number of
terms. FP32-mixed (D in float, every PCG solve at 1e-6): within 1e-4."""
import numpy as np
import pytest

import oracle
import synthetic as syn
from oracle import contact_ref as cr
from oracle import partial_ref as pr
from tests.helpers import oracle_sheet, relerr

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_2506_18867_amd import bsc  # noqa: E402

DT = 0.01
GRAV = (0.0, 0.0, -9.81)


def _scene(n_u, n_v, seed):
    ku, kv, rest = syn.flat_sheet(n_u, n_v)
    mat = syn.stvk_material(young=1e4, thickness=1e-3)
    x0 = syn.embed(rest) + syn.smooth_field(n_u, n_v, seed, amp=0.03)
    x0[:, 0] *= 0.95
    pins = np.array([0, n_u - 1, n_u * n_v - 1])
    return syn.Scene("contact", n_u, n_v, ku, kv, rest, mat, x0, np.zeros_like(x0), pins, x0[pins].copy(), DT,
                     np.array(GRAV))


def _case(n_u=21, n_v=17, n_pairs=300, scale=0.002, seed=4, precision=bsc.BSC_FP64):
    sc = _scene(n_u, n_v, seed)
    uv, tris, grid = syn.contact_mesh(n_u, n_v)
    pv, Hp, _ = syn.contact_pairs(uv, tris, grid, n_pairs, seed=seed, scale=scale)
    b = np.random.default_rng(seed).standard_normal((sc.n_cp, 3))
    # GPU inputs
    ctx = bsc.context_for_scene(sc)
    xg = bsc.to_soa(sc.x0)
    _, _, Hg = ctx.bsc_assemble(xg, xg, DT, GRAV, precision)
    ctx.bsc_contact_setup(uv, n_pairs)
    rp, ci, cv, _ = ctx.bsc_contact_hessian(torch.from_numpy(pv).cuda(), torch.from_numpy(Hp).cuda(), want_grad=False)
    # oracle inputs
    sh = oracle_sheet(sc)
    mask = np.zeros(sc.n_cp, dtype=bool)
    mask[sc.pins] = True
    _, _, H = oracle.assemble(sh, sc.x0, sc.x0, DT, np.array(GRAV), mask)
    A = oracle.stencil_to_csr(sh, H)
    Hc, _ = cr.contact_to_cp(sh, uv, pv, Hp)
    mass = oracle.lumped_mass(sh)
    return sc, ctx, Hg, (rp, ci, cv), b, (A, Hc, mass, mask)


def _gpu(ctx, Hg, csr, b, precision=bsc.BSC_FP64, pcg_rtol=1e-14, **kw):
    x, st = ctx.bsc_contact_solve(Hg, DT, *csr, bsc.to_soa(b), precision=precision, pcg_rtol=pcg_rtol, **kw)
    torch.cuda.synchronize()
    return bsc.to_aos(x), st


# contact scales: 0.002 gives a bound of about 0.2 on this sheet (the series, about 18 terms),
# 30 a bound far above 1 (the merged solve)
@pytest.mark.parametrize("scale,branch", [(0.002, "series"), (30.0, "merged")])
def test_trigger_and_result_match_oracle(scale, branch):
    sc, ctx, Hg, csr, b, (A, Hc, mass, mask) = _case(scale=scale)
    ref = pr.solve(A, Hc, mass, DT, b, mask, rho_max=0.5, series_tol=1e-12)
    got, st = _gpu(ctx, Hg, csr, b, rho_max=0.5, series_tol=1e-12)
    err = relerr(got, ref.x)
    print(f"[partial] {branch}: rho gpu {st.rho_bound:.6e} oracle {ref.rho_bound:.6e}, terms {st.terms}/{ref.terms}, "
          f"pcg {st.pcg_iters}, rel err {err:.2e}")
    assert bool(st.triggered) == ref.triggered == (branch == "series")
    assert st.terms == ref.terms
    assert abs(st.rho_bound - ref.rho_bound) <= 1e-12 * ref.rho_bound
    assert abs(st.d_bound - ref.d_bound) <= 1e-12 * ref.d_bound
    assert err < 1e-10
    # pinned control points: identity rows, solved by PCG (so to rounding, not bit for bit)
    assert np.abs(got[mask] - b[mask]).max() <= 1e-12 * np.abs(b).max()


@pytest.mark.parametrize("terms", [1, 2, 4])
def test_truncated_series_matches_oracle_term_for_term(terms):
    """Forced series with a fixed number of terms: the same truncated sum, not only the limit (a
    contact scale whose bound is above 1 while the series still contracts)."""
    sc, ctx, Hg, csr, b, (A, Hc, mass, mask) = _case(scale=0.05)
    ref = pr.solve(A, Hc, mass, DT, b, mask, force="series", max_terms=terms, series_tol=0.0)
    got, st = _gpu(ctx, Hg, csr, b, force=1, max_terms=terms, series_tol=0.0)
    err = relerr(got, ref.x)
    print(f"[partial] forced series, {terms} terms: rho {st.rho_bound:.3e}, rel err {err:.2e}")
    assert st.triggered == 1 and st.terms == terms == ref.terms
    assert err < 1e-10


def test_no_contact_is_one_stencil_solve():
    sc, ctx, Hg, csr, b, (A, Hc, mass, mask) = _case()
    rp = torch.zeros(sc.n_cp + 1, dtype=torch.int32, device="cuda")
    empty = torch.zeros(0, dtype=torch.int32, device="cuda")
    got, st = _gpu(ctx, Hg, (rp, empty, None), b)
    ref = pr.solve(A, Hc * 0.0, mass, DT, b, mask)
    assert st.triggered == 1 and st.terms == 1 and st.rho_bound == 0.0
    assert relerr(got, ref.x) < 1e-10


def test_fp32_mixed_within_bound():
    sc, ctx, Hg, csr, b, (A, Hc, mass, mask) = _case(precision=bsc.BSC_FP32_MIXED)
    ref = pr.solve(A, Hc, mass, DT, b, mask, rho_max=0.5, series_tol=1e-12)
    # an FP32 SpMV cannot drive the residual below about 1e-7 relative; 1e-6 per solve
    got, st = _gpu(ctx, Hg, csr, b, precision=bsc.BSC_FP32_MIXED, pcg_rtol=1e-6, rho_max=0.5, series_tol=1e-12)
    err = relerr(got, ref.x)
    print(f"[partial] FP32-mixed: triggered {st.triggered}, terms {st.terms}, rel err {err:.2e}")
    assert bool(st.triggered) == ref.triggered and err < 1e-4


def test_larger_sheet_both_branches_agree():
    """100 x 100 control points, 3000 pairs (bound about 0.09): the series and the merged solve give
    the oracle's x."""
    sc, ctx, Hg, csr, b, (A, Hc, mass, mask) = _case(100, 100, 3000, scale=3e-5, seed=6)
    ref = pr.solve(A, Hc, mass, DT, b, mask, rho_max=0.5, series_tol=1e-12)
    assert ref.triggered
    xs, s1 = _gpu(ctx, Hg, csr, b, rho_max=0.5, series_tol=1e-12)
    xm, s2 = _gpu(ctx, Hg, csr, b, force=2)
    print(f"[partial] 100x100: rho {s1.rho_bound:.3e}, series {s1.terms} terms {s1.pcg_iters} it "
          f"{s1.ms_total:.1f} ms; merged {s2.pcg_iters} it {s2.ms_total:.1f} ms")
    exact = pr.solve(A, Hc, mass, DT, b, mask, force="merged")
    assert s1.triggered == 1 and s1.terms == ref.terms
    assert relerr(xm, exact.x) < 1e-10
    assert relerr(xs, ref.x) < 1e-10


def test_bad_column_index_is_refused():
    sc, ctx, Hg, (rp, ci, cv), b, _ = _case(n_pairs=20)
    bad = ci.clone()
    bad[0] = sc.n_cp + 5
    with pytest.raises(bsc.BscError) as e:
        ctx.bsc_contact_solve(Hg, DT, rp, bad, cv, bsc.to_soa(b))
    assert e.value.status == bsc.BSC_E_INVAL
    x, st = ctx.bsc_contact_solve(Hg, DT, rp, ci, cv, bsc.to_soa(b), pcg_rtol=1e-12)   # still usable
    assert torch.isfinite(x).all()
