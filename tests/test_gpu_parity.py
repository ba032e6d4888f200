"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

FP64 bar: normwise relative error <= 1e-10 for energies, gradients, element and assembled
Hessians and Newton iterates, and the same bound on every entry against the size of its own
row (one element, or one CP: ``rowwise_err``), so that an error confined to a few elements
cannot hide in a norm over the whole array. FP32-mixed bar: gradient within 1e-4 relative of the FP64
oracle, Hessian within 1e-5, and the Newton step reaching the same FP64 residual tolerance.
Sizes span several tiles with ragged tails (n = 5..23 and non-square), the 100 x 100 sheet,
and the full 226 x 226 sheet compared element by element."""
import numpy as np
import pytest

import oracle
import synthetic as syn
from tests.helpers import deformed, oracle_sheet, oracle_stencil_to_upper, relerr, rowwise_err, upper27

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2506_18867_amd import bsc  # noqa: E402

TOL64 = 1e-10


def check64(got, ref, axis, what=""):
    """FP64 bar, normwise and row by row (``axis`` indexes the rows: elements or CPs)."""
    got = np.asarray(got.cpu().numpy() if hasattr(got, "cpu") else got, dtype=np.float64)
    en, er = relerr(got, ref), rowwise_err(got, ref, axis=axis)
    if what:
        print(f"  {what}: normwise {en:.2e}, worst row {er:.2e}")
    assert en < TOL64, (what, en)
    assert er < TOL64, (what, er)


def _scene(kind, n, seed=1, **kw):
    if kind == "hanging":
        return syn.hanging_sheet(n, seed=seed, **kw)
    if kind == "compressed":
        return syn.compressed_sheet(n, seed=seed, **kw)
    return syn.driven_sheet(n, seed=seed, **kw)


def _ctx(sc):
    return bsc.context_for_scene(sc)


# ---- element-level E/g/H ----------------------------------------------------------------------

@pytest.mark.parametrize("n_u,n_v,shear,spacing", [(5, 5, 0.0, 1), (7, 6, 0.0, 1), (11, 11, 0.3, 2), (20, 20, 0.0, 1), (23, 9, 0.1, 1)])
def test_eval_egh_fp64_matches_oracle(n_u, n_v, shear, spacing):
    print(f"[eval_egh fp64] n={n_u}x{n_v} shear={shear} spacing={spacing}", flush=True)
    ku, kv, rest = syn.flat_sheet(n_u, n_v, 1.0, 0.8, spacing=spacing, shear=shear)
    mat = syn.stvk_material(young=1e4, thickness=1e-3, mu_bend=2e-3)
    sh = oracle_sheet((n_u, n_v, ku, kv, rest), mat)
    x = syn.embed(rest) + syn.smooth_field(n_u, n_v, 7, amp=0.05)
    x[:, 0] *= 0.93                                            # some compression: indefinite points
    ctx = bsc.Context(n_u, n_v, ku, kv, rest, bsc.make_material(0, mat.young, mat.poisson, mat.thickness,
                                                               mu_bend=mat.mu_bend, rho_area=mat.rho_area))
    E, eE, eg, eH = ctx.bsc_eval_egh(bsc.to_soa(x), bsc.BSC_FP64)
    torch.cuda.synchronize()
    rE, rg, rH = oracle.element_egh(sh, x, project=True)
    assert relerr(E.item(), rE.sum()) < TOL64
    check64(eE, rE, 0, "element energy")
    check64(eg, rg.T, 1, "element gradient")
    check64(eH, upper27(rH), 1, "element Hessian")


def test_eval_egh_fbw_matches_oracle():
    n = 9
    ku, kv, rest = syn.flat_sheet(n)
    mat = syn.Material(1, 0, 0, 0, 3.0, 2.0, 0.7, 1e-3, 0.2)
    sh = oracle_sheet((n, n, ku, kv, rest), mat)
    x = syn.embed(rest) + syn.smooth_field(n, n, 3, amp=0.08)
    x[:, 1] *= 0.9
    ctx = bsc.Context(n, n, ku, kv, rest, bsc.make_material(1, 0, 0, 0, 3.0, 2.0, 0.7, 1e-3, 0.2))
    E, eE, eg, eH = ctx.bsc_eval_egh(bsc.to_soa(x), bsc.BSC_FP64)
    rE, rg, rH = oracle.element_egh(sh, x, project=True)
    check64(eE, rE, 0, "element energy")
    check64(eg, rg.T, 1, "element gradient")
    check64(eH, upper27(rH), 1, "element Hessian")


# ---- assembled incremental potential ----------------------------------------------------------

@pytest.mark.parametrize("kind,n", [("hanging", 5), ("hanging", 12), ("hanging", 20), ("compressed", 17)])
def test_assemble_fp64_matches_oracle(kind, n):
    print(f"[assemble fp64] {kind} n={n}", flush=True)
    sc = _scene(kind, n)
    sh = oracle_sheet(sc)
    x = deformed(sc, 4, amp=0.03)
    x[sc.pins] = sc.pin_targets(0)
    xhat = sc.x0 + sc.dt * syn.smooth_field(n, n, 9, amp=0.5)
    ctx = _ctx(sc)
    E, g, H = ctx.bsc_assemble(bsc.to_soa(x), bsc.to_soa(xhat), sc.dt, tuple(sc.gravity), bsc.BSC_FP64)
    torch.cuda.synchronize()
    mask = np.zeros(sc.n_cp, dtype=bool)
    mask[sc.pins] = True
    rE, rg, rH = oracle.assemble(sh, x, xhat, sc.dt, sc.gravity, mask)
    assert relerr(E.item(), rE) < TOL64
    check64(bsc.to_aos(g), rg, 0, "gradient")
    check64(H, oracle_stencil_to_upper(rH, n, n), 1, "Hessian")


def test_assemble_without_inertia_or_gravity():
    sc = syn.hanging_sheet(8, seed=3)
    sh = oracle_sheet(sc)
    x = deformed(sc, 2)
    ctx = bsc.Context(sc.n_u, sc.n_v, sc.knots_u, sc.knots_v, sc.rest,
                      bsc.make_material(0, 1e4, 0.3, 1e-3, mu_bend=sc.material.mu_bend, rho_area=0.2))
    E, g, H = ctx.bsc_assemble(bsc.to_soa(x), None, 0.0, None, bsc.BSC_FP64)
    rE, rg, rH = oracle.assemble(sh, x)
    assert relerr(E.item(), rE) < TOL64
    check64(bsc.to_aos(g), rg, 0, "gradient")
    check64(H, oracle_stencil_to_upper(rH, 8, 8), 1, "Hessian")


def test_full_size_226_matches_oracle():
    """The full 226 x 226 sheet (50,176 elements), compared entry by entry."""
    print("[assemble fp64] driven n=226", flush=True)
    sc = syn.driven_sheet(226, seed=300)
    sh = oracle_sheet(sc)
    x = deformed(sc, 11, amp=0.02)
    x[sc.pins] = sc.pin_targets(0)
    ctx = _ctx(sc)
    E, g, H = ctx.bsc_assemble(bsc.to_soa(x), bsc.to_soa(sc.x0), sc.dt, tuple(sc.gravity), bsc.BSC_FP64)
    torch.cuda.synchronize()
    mask = np.zeros(sc.n_cp, dtype=bool)
    mask[sc.pins] = True
    rE, rg, rH = oracle.assemble(sh, x, sc.x0, sc.dt, sc.gravity, mask)
    assert relerr(E.item(), rE) < TOL64
    check64(bsc.to_aos(g), rg, 0, "gradient")
    check64(H, oracle_stencil_to_upper(rH, 226, 226), 1, "Hessian")


def test_spmv_and_bsr_export_match_oracle_matrix():
    sc = syn.hanging_sheet(13, seed=5)
    sh = oracle_sheet(sc)
    x = deformed(sc, 1)
    ctx = _ctx(sc)
    E, g, H = ctx.bsc_assemble(bsc.to_soa(x), bsc.to_soa(sc.x0), sc.dt, tuple(sc.gravity), bsc.BSC_FP64)
    mask = np.zeros(sc.n_cp, dtype=bool)
    mask[sc.pins] = True
    _, _, rH = oracle.assemble(sh, x, sc.x0, sc.dt, sc.gravity, mask)
    A = oracle.stencil_to_csr(sh, rH)
    v = np.random.default_rng(0).standard_normal((sc.n_cp, 3))
    y = ctx.bsc_spmv(H, bsc.to_soa(v), bsc.BSC_FP64)
    want = (A @ v.reshape(-1)).reshape(-1, 3)
    assert relerr(bsc.to_aos(y), want) < TOL64
    rp, ci, vals = ctx.bsc_export_bsr(H, bsc.BSC_FP64)
    vals = vals.cpu().numpy()
    dense = A.toarray()
    for a in range(0, sc.n_cp, 7):
        for k in range(rp[a], rp[a + 1]):
            b = ci[k]
            assert np.allclose(vals[k], dense[3 * a:3 * a + 3, 3 * b:3 * b + 3], rtol=0, atol=1e-12 * np.abs(dense).max())


def test_results_are_bitwise_deterministic():
    sc = syn.compressed_sheet(31, seed=6)
    x = bsc.to_soa(deformed(sc, 2))
    ctx = _ctx(sc)
    outs = []
    for _ in range(2):
        E, g, H = ctx.bsc_assemble(x, x, sc.dt, tuple(sc.gravity), bsc.BSC_FP64)
        outs.append((E.cpu().numpy().copy(), g.cpu().numpy().copy(), H.cpu().numpy().copy()))
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


# ---- FP32-mixed path --------------------------------------------------------------------------

@pytest.mark.parametrize("kind,n", [("hanging", 20), ("compressed", 40)])
def test_fp32_gradient_and_hessian_within_bounds(kind, n):
    sc = _scene(kind, n)
    sh = oracle_sheet(sc)
    x = deformed(sc, 8, amp=0.02)
    x[sc.pins] = sc.pin_targets(0)
    ctx = _ctx(sc)
    E, g, H = ctx.bsc_assemble(bsc.to_soa(x), bsc.to_soa(sc.x0), sc.dt, tuple(sc.gravity), bsc.BSC_FP32_MIXED)
    assert g.dtype == torch.float32 and H.dtype == torch.float32
    mask = np.zeros(sc.n_cp, dtype=bool)
    mask[sc.pins] = True
    rE, rg, rH = oracle.assemble(sh, x, sc.x0, sc.dt, sc.gravity, mask)
    eg = relerr(bsc.to_aos(g), rg)
    eh = relerr(H.cpu().numpy(), oracle_stencil_to_upper(rH, n, n))
    print(f"[fp32] {kind} n={n}: grad rel err {eg:.2e}, hessian rel err {eh:.2e}, energy rel err {relerr(E.item(), rE):.2e}")
    assert eg < 1e-4
    assert eh < 1e-5
    assert relerr(E.item(), rE) < 1e-5


@pytest.mark.parametrize("delta", [0.15, 0.05, 1e-6])
def test_nearly_parallel_columns_match_oracle(delta):
    """Every element sheared and flattened to F = [[1, 1/2], [0, delta], [0, 0]], so that
    r = |f1 x f2| / (|f1| |f2|) is about 1.9 delta: at 0.15 the FP32 structured projection takes
    the points, at 0.05 it declines (r < 0.1) and the FP64 one does, at 1e-6 that declines too
    (r < 1e-5) and the full 6x6 matrix is projected. FP64 at the FP64 bar, FP32-mixed at its own."""
    sc = syn.hanging_sheet(12, seed=3)
    sh = oracle_sheet(sc)
    X = np.asarray(sc.rest, dtype=np.float64).reshape(-1, 2)     # CP rest positions: F is exact
    x = np.stack([X[:, 0] + 0.5 * X[:, 1], delta * X[:, 1], np.zeros(X.shape[0])], axis=1)
    mask = np.zeros(sc.n_cp, dtype=bool)
    mask[sc.pins] = True
    rE, rg, rH = oracle.assemble(sh, x, sc.x0, sc.dt, sc.gravity, mask)
    rHu = oracle_stencil_to_upper(rH, sc.n_u, sc.n_v)
    ctx = _ctx(sc)
    E, g, H = ctx.bsc_assemble(bsc.to_soa(x), bsc.to_soa(sc.x0), sc.dt, tuple(sc.gravity), bsc.BSC_FP64)
    torch.cuda.synchronize()
    print(f"[parallel columns] delta={delta:g}", flush=True)
    assert relerr(E.item(), rE) < TOL64
    check64(bsc.to_aos(g), rg, 0, "gradient")
    check64(H, rHu, 1, "Hessian")
    E, g, H = ctx.bsc_assemble(bsc.to_soa(x), bsc.to_soa(sc.x0), sc.dt, tuple(sc.gravity), bsc.BSC_FP32_MIXED)
    eg, eh = relerr(bsc.to_aos(g), rg), relerr(H.cpu().numpy(), rHu)
    print(f"  fp32: grad rel err {eg:.2e}, hessian rel err {eh:.2e}")
    assert eg < 1e-4
    assert eh < 1e-5


def test_compressed_100_sheet_matches_oracle():
    """The 100 x 100 CP sheet with 10% in-plane compression and +-2 mm z-noise, both side
    columns held (the workload of the FP64 against FP32 comparison): FP64 assembly within 1e-10
    of the oracle, FP32-mixed gradient and Hessian within their bars, and the first FP64 Newton
    iterate within 1e-10 of the oracle's exact solve."""
    n = 100
    print(f"[compressed {n}] assembly in both precisions and one Newton iterate", flush=True)
    sc = syn.compressed_sheet(n, seed=2)
    sh = oracle_sheet(sc)
    ctx = _ctx(sc)
    mask = np.zeros(sc.n_cp, dtype=bool)
    mask[sc.pins] = True
    xhat = sc.x0 + sc.dt * sc.v0
    rE, rg, rH = oracle.assemble(sh, sc.x0, xhat, sc.dt, sc.gravity, mask)
    rHu = oracle_stencil_to_upper(rH, n, n)
    E, g, H = ctx.bsc_assemble(bsc.to_soa(sc.x0), bsc.to_soa(xhat), sc.dt, tuple(sc.gravity), bsc.BSC_FP64)
    assert relerr(E.item(), rE) < TOL64
    check64(bsc.to_aos(g), rg, 0, "gradient")
    check64(H, rHu, 1, "Hessian")
    E, g, H = ctx.bsc_assemble(bsc.to_soa(sc.x0), bsc.to_soa(xhat), sc.dt, tuple(sc.gravity), bsc.BSC_FP32_MIXED)
    assert relerr(bsc.to_aos(g), rg) < 1e-4
    assert relerr(H.cpu().numpy(), rHu) < 1e-5
    x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
    opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), fixed_newton_iters=1, pcg_rtol=1e-14, max_pcg=50000)
    st, stats = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(0)), opts)
    ref = oracle.newton_step(sh, sc.x0, sc.v0, sc.dt, sc.gravity, sc.pins, sc.pin_targets(0), fixed_iters=1)
    err = relerr(bsc.to_aos(x) - sc.x0, ref.x - sc.x0)
    print(f"[compressed {n}] pcg={stats.pcg_iters_total} rel err of x - x0: {err:.2e}", flush=True)
    check64(bsc.to_aos(x) - sc.x0, ref.x - sc.x0, 0, "x - x0")


# ---- Newton step --------------------------------------------------------------------------

@pytest.mark.parametrize("iters", [1, 2])
def test_newton_fp64_iterates_match_oracle(iters):
    """Same iteration count on both sides; GPU PCG to 1e-14 against the oracle's sparse LU.
    Compared while the energy decrease of each iteration is far above FP64 rounding of E
    (the oracle compares the two energies directly, so once the decrease falls below the
    rounding of E its backtracking becomes arbitrary; the library evaluates the difference)."""
    sc = syn.hanging_sheet(20, seed=1)
    sh = oracle_sheet(sc)
    ctx = _ctx(sc)
    x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
    opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), fixed_newton_iters=iters, pcg_rtol=1e-14, max_pcg=20000)
    st, stats = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(0)), opts)
    ref = oracle.newton_step(sh, sc.x0, sc.v0, sc.dt, sc.gravity, sc.pins, sc.pin_targets(0), fixed_iters=iters)
    got = bsc.to_aos(x)
    err = relerr(got - sc.x0, ref.x - sc.x0)
    print(f"[newton fp64] iters={iters} pcg={stats.pcg_iters_total} rel err of x - x0: {err:.2e}")
    check64(got - sc.x0, ref.x - sc.x0, 0, "x - x0")
    assert relerr(bsc.to_aos(v), ref.v) < TOL64
    assert abs(stats.g0_norm - ref.g0_norm) < 1e-10 * ref.g0_norm


@pytest.mark.parametrize("iters", [1, 2])
def test_newton_fbw_iterates_match_oracle(iters):
    """The FBW membrane (Sec. 4.1) through the whole Newton step: assembly, PCG and the line
    search's per-point energy difference, FP64 iterates against the oracle's exact solves. A
    hanging sheet compressed by 10% across, so that the projection clamps at many points."""
    sc = syn.hanging_sheet(14, seed=6, material=syn.Material(1, 0.0, 0.0, 0.0, 3.0, 2.0, 0.7, 1e-3, 0.2))
    sc.x0[:, 0] *= 0.9
    sc.pin_rest = sc.x0[sc.pins].copy()
    sh = oracle_sheet(sc)
    ctx = _ctx(sc)
    x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
    opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), fixed_newton_iters=iters, pcg_rtol=1e-14, max_pcg=20000)
    st, stats = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(0)), opts)
    assert st == 0
    ref = oracle.newton_step(sh, sc.x0, sc.v0, sc.dt, sc.gravity, sc.pins, sc.pin_targets(0), fixed_iters=iters)
    err = relerr(bsc.to_aos(x) - sc.x0, ref.x - sc.x0)
    print(f"[newton fbw fp64] iters={iters} halvings={stats.ls_halvings} (oracle {ref.alphas}) rel err of x - x0: {err:.2e}")
    assert err < TOL64
    assert relerr(bsc.to_aos(v), ref.v) < TOL64


@pytest.mark.parametrize("variant", ["spacing2_sheared", "gauss2", "corner2"])
def test_newton_iterates_match_oracle_on_variants(variant):
    """Two Newton iterates (FP64, PCG to 1e-14) against the oracle on a knot spacing of 2 with a
    sheared, non-square rest, and on two of the ablation's comparison rules (the line search then
    sums the energy difference over those rules' points)."""
    n_u, n_v = 11, 9
    spacing, shear, rule = (2, 0.25, bsc.BSC_QUAD_REDUCED) if variant == "spacing2_sheared" else \
        (1, 0.0, bsc.BSC_QUAD_GAUSS2 if variant == "gauss2" else bsc.BSC_QUAD_CORNER2)
    ku, kv, rest = syn.flat_sheet(n_u, n_v, 1.0, 0.8, spacing=spacing, shear=shear)
    mat = syn.stvk_material(young=1e4, thickness=1e-3, mu_bend=2e-3)
    x0 = syn.embed(rest)
    x0[:, 2] += 0.002 * syn.smooth_field(n_u, n_v, 11, amp=1.0)[:, 2]
    pins = np.array([0, n_u - 1], dtype=np.int64)
    sc = syn.Scene(variant, n_u, n_v, ku, kv, rest, mat, x0, np.zeros_like(x0), pins, x0[pins].copy(), 0.01,
                   np.array([0.0, -9.81, 0.0]))
    sh = oracle_sheet(sc)
    sh.quadrature = rule
    ctx = bsc.context_for_scene(sc, quadrature=rule)
    x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
    opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), fixed_newton_iters=2, pcg_rtol=1e-14, max_pcg=20000)
    st, _ = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(0)), opts)
    assert st == 0
    ref = oracle.newton_step(sh, sc.x0, sc.v0, sc.dt, sc.gravity, sc.pins, sc.pin_targets(0), fixed_iters=2)
    err = relerr(bsc.to_aos(x) - sc.x0, ref.x - sc.x0)
    print(f"[newton {variant}] rel err of x - x0: {err:.2e}")
    assert err < TOL64


@pytest.mark.parametrize("precision", [bsc.BSC_FP64, bsc.BSC_FP32_MIXED])
def test_newton_fbw_converges(precision):
    sc = syn.hanging_sheet(20, seed=7, material=syn.Material(1, 0.0, 0.0, 0.0, 3.0, 2.0, 0.7, 1e-3, 0.2))
    ctx = _ctx(sc)
    x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
    opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), precision=precision, rtol=1e-6, pcg_rtol=1e-3,
                         pcg_adaptive=1, max_newton=200)
    st, stats = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(0)), opts)
    assert st == 0
    assert stats.g_norm <= 1e-6 * stats.g0_norm


@pytest.mark.parametrize("iters", [1, 2])
def test_newton_predictor_start_iterates_match_oracle(iters):
    """BSC_START_PREDICTOR: the first iterate is xhat = x_n + dt v_n (pins at their targets).
    A hanging sheet moving with a smooth velocity field; FP64 iterates against the oracle's exact
    solves from the same start."""
    sc = syn.hanging_sheet(20, seed=1)
    v0 = syn.smooth_field(20, 20, 9, amp=0.3)
    v0[sc.pins] = 0.0
    sh = oracle_sheet(sc)
    ctx = _ctx(sc)
    x, v = bsc.to_soa(sc.x0), bsc.to_soa(v0)
    opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), fixed_newton_iters=iters, pcg_rtol=1e-14, max_pcg=20000,
                         start=bsc.BSC_START_PREDICTOR)
    st, stats = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(0)), opts)
    assert st == 0
    ref = oracle.newton_step(sh, sc.x0, v0, sc.dt, sc.gravity, sc.pins, sc.pin_targets(0), fixed_iters=iters,
                             start="predictor")
    err = relerr(bsc.to_aos(x) - sc.x0, ref.x - sc.x0)
    print(f"[newton predictor fp64] iters={iters} rel err of x - x0: {err:.2e}")
    assert err < TOL64
    assert relerr(bsc.to_aos(v), ref.v) < TOL64
    assert abs(stats.g0_norm - ref.g0_norm) < 1e-10 * ref.g0_norm


@pytest.mark.parametrize("precision", [bsc.BSC_FP64, bsc.BSC_FP32_MIXED])
@pytest.mark.parametrize("start", [bsc.BSC_START_PREVIOUS, bsc.BSC_START_PREDICTOR])
def test_predictor_start_step_rule_converges(precision, start):
    """Both starts under the paper's step rule on the driven sheet over three steps (velocities
    from the previous steps): every step meets |p|_inf / dt <= atol with status OK."""
    sc = syn.driven_sheet(60, seed=305)
    ctx = _ctx(sc)
    x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
    opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), precision=precision, stop_mode=bsc.BSC_STOP_STEP,
                         atol=1e-2, pcg_adaptive=1, pcg_rtol=1e-3, start=start)
    its = []
    for k in range(3):
        st, stats = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(k)), opts)
        assert st == 0
        its.append(stats.newton_iters)
    print(f"[start {start} precision {precision}] Newton iterations per step {its}")


@pytest.mark.parametrize("precision", [bsc.BSC_FP64, bsc.BSC_FP32_MIXED])
@pytest.mark.parametrize("scene", ["compressed2", "driven"])
def test_newton_converges_to_fp64_tolerance(precision, scene):
    sc = syn.compressed_sheet(40, seed=2, compression=0.02) if scene == "compressed2" else syn.driven_sheet(40, seed=301)
    sh = oracle_sheet(sc)
    ctx = _ctx(sc)
    x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
    opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), precision=precision, rtol=1e-6, pcg_rtol=1e-3)
    st, stats = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(0)), opts)
    assert st == 0
    mask = np.zeros(sc.n_cp, dtype=bool)
    mask[sc.pins] = True
    xhat = sc.x0 + sc.dt * sc.v0
    E, g, _ = oracle.assemble(sh, bsc.to_aos(x), xhat, sc.dt, sc.gravity, mask, want_hessian=False)
    x_init = sc.x0.copy()
    x_init[sc.pins] = sc.pin_targets(0)
    E0, g0, _ = oracle.assemble(sh, x_init, xhat, sc.dt, sc.gravity, mask, want_hessian=False)
    print(f"[newton] precision={precision} iters={stats.newton_iters} pcg={stats.pcg_iters_total} "
          f"|g|/|g0| oracle={np.linalg.norm(g) / stats.g0_norm:.2e}")
    assert np.linalg.norm(g) <= 1.01e-6 * stats.g0_norm
    assert abs(stats.g0_norm - np.linalg.norm(g0)) < 1e-8 * stats.g0_norm


def test_newton_step_paper_stop_rule():
    sc = syn.hanging_sheet(16, seed=4)
    ctx = _ctx(sc)
    x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
    opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), stop_mode=bsc.BSC_STOP_STEP, atol=1e-2, pcg_rtol=1e-6)
    st, stats = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(0)), opts)
    assert st == 0 and stats.newton_iters >= 1


def test_newton_reports_errors():
    sc = syn.hanging_sheet(8, seed=4)
    ctx = _ctx(sc)
    x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
    opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), max_newton=1, rtol=1e-12, pcg_rtol=1e-2)
    st, stats = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(0)), opts, raise_on_error=False)
    assert st == -5                                                   # BSC_E_NOT_CONVERGED
    xb = bsc.to_soa(sc.x0)
    xb[0, 5] = float("nan")
    st, _ = ctx.bsc_newton_step(xb, bsc.to_soa(sc.v0), bsc.to_soa(sc.pin_targets(0)), bsc.make_opts(dt=sc.dt), raise_on_error=False)
    assert st == -7                                                   # BSC_E_NONFINITE
    bad = bsc.make_opts(dt=-1.0)
    st, _ = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(0)), bad, raise_on_error=False)
    assert st == -1


def test_cg_graph_replays_match_eager_launches(monkeypatch):
    """The CG chunk replayed from a HIP graph gives bitwise the same steps as eager launches,
    over several solves with eager work and synchronisations between the replays."""
    sc = syn.driven_sheet(48, seed=303)
    results = []
    for no_graph in ("1", "0"):
        monkeypatch.setenv("BSC_GRAPHS", "0" if no_graph == "1" else "1")
        ctx = _ctx(sc)
        x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
        for prec in (bsc.BSC_FP64, bsc.BSC_FP32_MIXED):
            opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), precision=prec, rtol=1e-7, pcg_rtol=1e-4)
            for step in range(3):
                ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(step)), opts)
                torch.cuda.synchronize()
        results.append((x.cpu().numpy(), v.cpu().numpy()))
    assert np.array_equal(results[0][0], results[1][0])
    assert np.array_equal(results[0][1], results[1][1])


# ---- quadrature variants (the comparison rules of the reduced-integration ablation) -----------

@pytest.mark.parametrize("rule", [bsc.BSC_QUAD_GAUSS2, bsc.BSC_QUAD_INTERIOR1, bsc.BSC_QUAD_CORNER2])
def test_quadrature_variants_match_oracle(rule):
    """The same kernels on the comparison tables: point counts, element E/g/H and the assembled
    incremental potential against the oracle's rule, FP64, on a sheared 9 x 7 sheet with pins."""
    n_u, n_v = 9, 7
    print(f"[quadrature variant] rule={rule} {n_u}x{n_v}", flush=True)
    ku, kv, rest = syn.flat_sheet(n_u, n_v, 1.0, 0.8, shear=0.2)
    mat = syn.stvk_material(young=1e4, thickness=1e-3, mu_bend=2e-3)
    sh = oracle_sheet((n_u, n_v, ku, kv, rest), mat)
    sh.quadrature = rule
    ctx = bsc.Context(n_u, n_v, ku, kv, rest, bsc.make_material(0, mat.young, mat.poisson, mat.thickness,
                                                               mu_bend=mat.mu_bend, rho_area=mat.rho_area,
                                                               quadrature=rule))
    assert ctx.sizes.n_membrane_pts == len(oracle.membrane_rule(n_u - 2, n_v - 2, rule))
    x = syn.embed(rest) + syn.smooth_field(n_u, n_v, 5, amp=0.05)
    x[:, 0] *= 0.94
    E, eE, eg, eH = ctx.bsc_eval_egh(bsc.to_soa(x), bsc.BSC_FP64)
    rE, rg, rH = oracle.element_egh(sh, x, project=True)
    assert relerr(eE.cpu().numpy(), rE) < TOL64
    assert relerr(eg.cpu().numpy(), rg.T) < TOL64
    assert relerr(eH.cpu().numpy(), upper27(rH)) < TOL64
    pins = np.array([0, n_u - 1, n_u * n_v - 1])
    ctx.bsc_set_pins(pins)
    mask = np.zeros(n_u * n_v, dtype=bool)
    mask[pins] = True
    xhat = syn.embed(rest) + 0.01 * syn.smooth_field(n_u, n_v, 6, amp=0.5)
    Ea, ga, Ha = ctx.bsc_assemble(bsc.to_soa(x), bsc.to_soa(xhat), 0.01, (0.0, 0.0, -9.81), bsc.BSC_FP64)
    rEa, rga, rHa = oracle.assemble(sh, x, xhat, 0.01, np.array([0.0, 0.0, -9.81]), mask)
    assert relerr(Ea.item(), rEa) < TOL64
    assert relerr(bsc.to_aos(ga), rga) < TOL64
    assert relerr(Ha.cpu().numpy(), oracle_stencil_to_upper(rHa, n_u, n_v)) < TOL64


def test_standard_2x2_rule_needs_as_many_newton_iterations():
    """Sec. 6.5: reduced integration converges in about as many Newton iterations as the
    standard 2x2 rule on the interior spans (paper's stopping rule, dt = 0.01 s). Driven sheet,
    60 x 60 CPs, 8 steps, FP64, same start state."""
    sc = syn.driven_sheet(60, seed=12, cell=7)
    iters = {}
    for rule in (bsc.BSC_QUAD_REDUCED, bsc.BSC_QUAD_GAUSS2):
        ctx = bsc.context_for_scene(sc, quadrature=rule)
        x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
        opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), precision=bsc.BSC_FP64, stop_mode=bsc.BSC_STOP_STEP,
                             max_newton=60, pcg_rtol=1e-6, max_pcg=4000)
        per = []
        for step in range(8):
            st, s = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(step)), opts)
            assert st == 0
            per.append(s.newton_iters)
        iters[rule] = per
    print(f"[quadrature] Newton iterations per step: reduced {iters[0]} | 2x2 interior {iters[1]}")
    assert abs(sum(iters[0]) - sum(iters[1])) <= max(4, 0.25 * sum(iters[1]))


def test_step_rule_device_tolerance_equals_host_tolerance():
    """With the paper's step rule the Eisenstat-Walker tolerance is formed on the device and the
    solve follows the assembly without a host round trip; with a warm start the same tolerance
    is formed on the host. All-zero warm-start weights always fall back to a zero start, so both
    paths must give bitwise the same steps."""
    from oracle import net_ref
    sc = syn.driven_sheet(40, seed=21)
    res = []
    for ws in (0, 1):
        ctx = _ctx(sc)
        if ws:
            ctx.bsc_warmstart_load(torch.zeros(net_ref.N_PARAMS, dtype=torch.float32, device="cuda"))
        x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
        opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), precision=bsc.BSC_FP32_MIXED, warm_start=ws,
                             stop_mode=bsc.BSC_STOP_STEP, atol=1e-2, pcg_rtol=1e-3, pcg_adaptive=1, max_pcg=4000)
        iters = []
        for step in range(3):
            st, stt = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(step)), opts)
            assert st == 0
            iters.append((stt.newton_iters, stt.pcg_iters_total))
        res.append((x.cpu().numpy(), iters))
    print(f"[step rule] device tolerance {res[0][1]} | host tolerance {res[1][1]}")
    assert res[0][1] == res[1][1]
    assert np.array_equal(res[0][0], res[1][0])


def test_step_rule_stops_within_its_tolerance():
    """The step rule |p|_inf / dt <= atol leaves the state within about atol dt of the converged
    implicit-Euler step (Newton converges quadratically near the solution)."""
    sc = syn.hanging_sheet(24, seed=5)
    out = {}
    for mode, extra in (("step", dict(stop_mode=bsc.BSC_STOP_STEP, atol=1e-2, pcg_adaptive=1)),
                        ("grad", dict(stop_mode=bsc.BSC_STOP_GRAD, rtol=1e-10))):
        ctx = _ctx(sc)
        x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
        opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), precision=bsc.BSC_FP64, pcg_rtol=1e-8,
                             max_newton=60, max_pcg=4000, **extra)
        for step in range(3):
            st, _ = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(step)), opts)
            assert st == 0
        out[mode] = x.cpu().numpy()
    assert np.abs(out["step"] - out["grad"]).max() <= 1e-2 * sc.dt


# ---- a whole time step, and the FP32 element and SpMV paths -------------------------------------

def test_hanging_20_full_time_step_matches_oracle():
    """One complete implicit-Euler step of the 20 x 20 hanging sheet (E = 1e4 Pa, t = 1 mm, two
    top corners pinned, dt = 0.01 s), each side under its own stopping test
    |g| <= 1e-6 |g0| (Sec. 3.2, Eq. "incremental_potential"; Sec. 5.1): the same number of Newton
    iterations, and C^{n+1} - C^n and the new velocity within 1e-10 of the oracle's (GPU PCG to
    1e-14 against the oracle's sparse LU), normwise and CP by CP."""
    sc = syn.hanging_sheet(20, seed=1)
    sh = oracle_sheet(sc)
    ctx = _ctx(sc)
    x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
    opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), precision=bsc.BSC_FP64, stop_mode=bsc.BSC_STOP_GRAD,
                         rtol=1e-6, pcg_rtol=1e-14, max_pcg=20000, max_newton=50)
    st, stats = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(0)), opts)
    assert st == 0
    ref = oracle.newton_step(sh, sc.x0, sc.v0, sc.dt, sc.gravity, sc.pins, sc.pin_targets(0), rtol=1e-6)
    print(f"[hanging 20x20 step] Newton gpu {stats.newton_iters} oracle {ref.iters} (alphas {ref.alphas}); "
          f"|g|/|g0| gpu {stats.g_norm / stats.g0_norm:.2e} oracle {ref.g_norm / ref.g0_norm:.2e}")
    assert stats.newton_iters == ref.iters
    check64(bsc.to_aos(x) - sc.x0, ref.x - sc.x0, 0, "C^{n+1} - C^n")
    check64(bsc.to_aos(v), ref.v, 0, "v^{n+1}")
    assert stats.g_norm <= 1e-6 * stats.g0_norm


# FP32 element bar: the element gradient within 1e-4 of the FP64 oracle (the FP32 path's bar),
# the element Hessian within 1e-5 normwise; row by row both within 1e-4 of their element's size
# (floor 1e-2 of the array's largest entry: FP32 rounds each of the ~30 terms of an entry at
# u = 6e-8 of the terms' size, which can exceed a near-zero entry's size)
TOL32_G, TOL32_H, TOL32_ROW = 1e-4, 1e-5, 1e-4


@pytest.mark.parametrize("n_u,n_v,shear", [(20, 20, 0.0), (23, 9, 0.1)])
def test_eval_egh_fp32_within_bounds(n_u, n_v, shear):
    """bsc_eval_egh in BSC_FP32_MIXED (points evaluated and accumulated in float, PSD eigen-problem
    in double) against the FP64 oracle on a compressed, bent sheet."""
    print(f"[eval_egh fp32] n={n_u}x{n_v} shear={shear}", flush=True)
    ku, kv, rest = syn.flat_sheet(n_u, n_v, 1.0, 0.8, shear=shear)
    mat = syn.stvk_material(young=1e4, thickness=1e-3, mu_bend=2e-3)
    sh = oracle_sheet((n_u, n_v, ku, kv, rest), mat)
    x = syn.embed(rest) + syn.smooth_field(n_u, n_v, 7, amp=0.05)
    x[:, 0] *= 0.93
    ctx = bsc.Context(n_u, n_v, ku, kv, rest, bsc.make_material(0, mat.young, mat.poisson, mat.thickness,
                                                               mu_bend=mat.mu_bend, rho_area=mat.rho_area))
    E, eE, eg, eH = ctx.bsc_eval_egh(bsc.to_soa(x), bsc.BSC_FP32_MIXED)
    assert eE.dtype == torch.float32 and eg.dtype == torch.float32 and eH.dtype == torch.float32
    rE, rg, rH = oracle.element_egh(sh, x, project=True)
    eg_n, eh_n = relerr(eg.cpu().numpy(), rg.T), relerr(eH.cpu().numpy(), upper27(rH))
    eg_r = rowwise_err(eg.cpu().numpy(), rg.T, axis=1, floor=1e-2)
    eh_r = rowwise_err(eH.cpu().numpy(), upper27(rH), axis=1, floor=1e-2)
    ee = relerr(E.item(), rE.sum())
    print(f"  energy {ee:.2e}; gradient normwise {eg_n:.2e} worst element {eg_r:.2e}; "
          f"Hessian normwise {eh_n:.2e} worst element {eh_r:.2e}")
    assert ee < TOL32_H
    assert relerr(eE.cpu().numpy(), rE) < TOL32_H
    assert eg_n < TOL32_G and eh_n < TOL32_H
    assert eg_r < TOL32_ROW and eh_r < TOL32_ROW


def test_spmv_fp32_within_rounding_bound():
    """bsc_spmv in BSC_FP32_MIXED: the input vector rounded to float and the 75 products of a row
    summed in float. Input: the oracle's Hessian rounded to float32 (an input array of the call,
    in its upper-stencil layout). Reference: the same float32 values times the FP64 vector in
    FP64. Every entry must meet the standard bound for a rounded dot product,
    |y - A v| <= gamma_{n+1} (|A| |v|) with n = 75 terms (one more rounding for v), u = 2^-24."""
    sc = syn.compressed_sheet(37, seed=4)
    sh = oracle_sheet(sc)
    x = deformed(sc, 3, amp=0.03)
    mask = np.zeros(sc.n_cp, dtype=bool)
    mask[sc.pins] = True
    _, _, rH = oracle.assemble(sh, x, sc.x0, sc.dt, sc.gravity, mask)
    H32 = oracle_stencil_to_upper(rH, sc.n_u, sc.n_v).astype(np.float32)
    # the same float32 values back in the oracle's stencil form, as a sparse matrix
    rH32 = rH.astype(np.float32).astype(np.float64)
    A = oracle.stencil_to_csr(sh, rH32)
    v = np.random.default_rng(3).standard_normal((sc.n_cp, 3))
    ctx = _ctx(sc)
    y = ctx.bsc_spmv(torch.from_numpy(H32).cuda(), bsc.to_soa(v), bsc.BSC_FP32_MIXED)
    want = (A @ v.reshape(-1)).reshape(-1, 3)
    bound_terms = (abs(A) @ np.abs(v).reshape(-1)).reshape(-1, 3)
    u = 2.0 ** -24
    n = 76
    gamma = n * u / (1 - n * u)
    got = bsc.to_aos(y)
    ratio = np.abs(got - want) / np.maximum(gamma * bound_terms, 1e-300)
    print(f"[spmv fp32] normwise {relerr(got, want):.2e}; worst entry at {ratio.max():.3f} of the rounding bound")
    assert ratio.max() <= 1.0
    # and against the FP64 product of the unrounded matrix: the float storage of H adds u |A| |v|
    want64 = (oracle.stencil_to_csr(sh, rH) @ v.reshape(-1)).reshape(-1, 3)
    assert np.all(np.abs(got - want64) <= (gamma + 2 * u) * bound_terms + 1e-300)
