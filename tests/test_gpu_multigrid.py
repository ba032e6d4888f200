"""The multigrid-preconditioned CG path of the Newton step (BSC_PRECOND_MULTIGRID): exact
B-spline prolongation between knot halvings, Galerkin coarse operators, symmetric V(1,1) cycles.

The preconditioner changes the iterates of the linear solver, not the Newton iterates it is
asked for: solved to the same relative residual, the step must match the oracle's exact solves
as the block-Jacobi path does (FP64 within 1e-10 with PCG to 1e-14), Newton steps must reach the
FP64 stopping tolerance in both precisions, graph replays must equal eager launches bitwise, and
grids whose span counts are odd fall back to block Jacobi. The point of the hierarchy is the
iteration count, checked against block Jacobi on the full 226 x 226 sheet."""
import numpy as np
import pytest

import oracle
import synthetic as syn
from tests.helpers import oracle_sheet, relerr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2506_18867_amd import bsc  # noqa: E402

MG = bsc.BSC_PRECOND_MULTIGRID


@pytest.mark.parametrize("kind,n", [("hanging", 20), ("driven", 40), ("annulus", 38)])
def test_multigrid_newton_iterates_match_oracle(kind, n):
    print(f"[mg newton fp64] {kind} n={n}", flush=True)
    if kind == "hanging":
        sc = syn.hanging_sheet(n, seed=1)
    elif kind == "driven":
        sc = syn.driven_sheet(n, seed=301)
    else:
        sc = syn.mapped_hanging_sheet(n, "annulus", 0.5, seed=3)
    sh = oracle_sheet(sc)
    ctx = bsc.context_for_scene(sc)
    x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
    opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), fixed_newton_iters=2, pcg_rtol=1e-14, max_pcg=2000,
                         preconditioner=MG)
    st, stats = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(0)), opts)
    assert st == 0
    ref = oracle.newton_step(sh, sc.x0, sc.v0, sc.dt, sc.gravity, sc.pins, sc.pin_targets(0), fixed_iters=2)
    err = relerr(bsc.to_aos(x) - sc.x0, ref.x - sc.x0)
    print(f"[mg newton fp64] {kind} n={n}: pcg={stats.pcg_iters_total} rel err of x - x0: {err:.2e}")
    assert err < 1e-10
    assert relerr(bsc.to_aos(v), ref.v) < 1e-10


@pytest.mark.parametrize("precision", [bsc.BSC_FP64, bsc.BSC_FP32_MIXED])
def test_multigrid_newton_converges(precision):
    sc = syn.driven_sheet(66, seed=302)
    sh = oracle_sheet(sc)
    ctx = bsc.context_for_scene(sc)
    x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
    opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), precision=precision, rtol=1e-6, pcg_rtol=1e-3,
                         pcg_adaptive=1, preconditioner=MG)
    st, stats = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(0)), opts)
    assert st == 0
    mask = np.zeros(sc.n_cp, dtype=bool)
    mask[sc.pins] = True
    _, g, _ = oracle.assemble(sh, bsc.to_aos(x), sc.x0 + sc.dt * sc.v0, sc.dt, sc.gravity, mask, want_hessian=False)
    print(f"[mg newton] precision={precision} newton={stats.newton_iters} pcg={stats.pcg_iters_total} "
          f"|g|/|g0| = {np.linalg.norm(g) / stats.g0_norm:.2e}")
    assert np.linalg.norm(g) <= 1.01e-6 * stats.g0_norm


def test_multigrid_needs_far_fewer_iterations_at_full_size():
    """First two Newton iterations of the 226 x 226 driven sheet, PCG to 1e-6, FP32-mixed."""
    sc = syn.driven_sheet(226, seed=304)
    counts = {}
    for pre in (bsc.BSC_PRECOND_JACOBI, MG):
        ctx = bsc.context_for_scene(sc)
        x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
        opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), precision=bsc.BSC_FP32_MIXED, fixed_newton_iters=2,
                             pcg_rtol=1e-6, max_pcg=4000, preconditioner=pre)
        st, stats = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(0)), opts)
        assert st == 0
        counts[pre] = stats.pcg_iters_total
    print(f"[mg] PCG iterations over two Newton iterations at 1e-6: block Jacobi {counts[0]}, multigrid {counts[MG]}")
    assert counts[MG] * 5 <= counts[bsc.BSC_PRECOND_JACOBI]


def test_multigrid_graph_replays_match_eager_launches(monkeypatch):
    sc = syn.driven_sheet(42, seed=303)
    results = []
    for no_graph in ("1", "0"):
        monkeypatch.setenv("BSC_GRAPHS", "0" if no_graph == "1" else "1")
        ctx = bsc.context_for_scene(sc)
        x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
        for prec in (bsc.BSC_FP64, bsc.BSC_FP32_MIXED):
            opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), precision=prec, stop_mode=bsc.BSC_STOP_STEP,
                                 pcg_rtol=1e-5, pcg_adaptive=1, preconditioner=MG)
            for step in range(3):
                st, _ = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(step)), opts)
                assert st == 0
                torch.cuda.synchronize()
        results.append((x.cpu().numpy(), v.cpu().numpy()))
    assert np.array_equal(results[0][0], results[1][0])
    assert np.array_equal(results[0][1], results[1][1])


def test_odd_span_counts_fall_back_to_block_jacobi():
    sc = syn.driven_sheet(21, seed=305)          # 19 spans: no knot halving
    out = []
    for pre in (bsc.BSC_PRECOND_JACOBI, MG):
        ctx = bsc.context_for_scene(sc)
        x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
        opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), rtol=1e-6, pcg_rtol=1e-4, preconditioner=pre)
        st, stats = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(0)), opts)
        assert st == 0
        out.append((x.cpu().numpy(), stats.pcg_iters_total))
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]
