"""The recycled PCG warm start (BSC_WARM_PREVIOUS): the previous Newton direction, scaled by its
energy-optimal multiple and kept only when it lowers the initial residual, decided on the device.

- With PCG solved to 1e-14 the start cannot change the Newton iterates: three FP64 iterates on a
  compressed sheet match the oracle's exact Newton iterates to 1e-10, and the stats show the
  path ran (the first iteration of a fresh context has no previous direction and falls back,
  later ones keep the start).
- At the gradient stop |g| <= 1e-6 |g0| with the adaptive tolerance, both precisions reach the
  oracle-checked residual over three steps; under compression with fewer PCG iterations than the
  zero start, on the driven sheet with no more; under the step rule (the deferred read-back
  path) the steps also converge.
- With the learned start the decision is the same device rule; a prediction that does not lower
  the residual falls back to the zero start bitwise (covered in the net tests).
"""
import numpy as np
import pytest

import oracle
import synthetic as syn
from tests.helpers import oracle_sheet, relerr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2506_18867_amd import bsc  # noqa: E402

TOL64 = 1e-10


def _compressed_14():
    sc = syn.hanging_sheet(14, seed=6)
    sc.x0[:, 0] *= 0.9
    sc.pin_rest = sc.x0[sc.pins].copy()
    return sc


def test_recycled_start_leaves_exact_newton_iterates_unchanged():
    sc = _compressed_14()
    sh = oracle_sheet(sc)
    ctx = bsc.context_for_scene(sc)
    x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
    opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), fixed_newton_iters=3, pcg_rtol=1e-14, max_pcg=20000,
                         warm_start=bsc.BSC_WARM_PREVIOUS)
    st, stats = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(0)), opts)
    assert st == 0
    ref = oracle.newton_step(sh, sc.x0, sc.v0, sc.dt, sc.gravity, sc.pins, sc.pin_targets(0), fixed_iters=3)
    err = relerr(bsc.to_aos(x) - sc.x0, ref.x - sc.x0)
    print(f"[warm previous] used {stats.warm_start_used} fallbacks {stats.warm_start_fallbacks} "
          f"pcg {stats.pcg_iters_total} rel err of x - x0: {err:.2e}")
    assert err < TOL64
    assert relerr(bsc.to_aos(v), ref.v) < TOL64
    # a fresh context has no previous direction: the first iteration falls back
    assert stats.warm_start_fallbacks >= 1
    assert stats.warm_start_used + stats.warm_start_fallbacks == 3
    assert stats.warm_start_used >= 1


@pytest.mark.parametrize("precision", [bsc.BSC_FP64, bsc.BSC_FP32_MIXED])
@pytest.mark.parametrize("scene", ["driven", "compressed"])
def test_recycled_start_reaches_the_residual_with_fewer_pcg_iterations(precision, scene):
    """Three steps from the same start with each start mode; every step reaches the oracle-checked
    residual. Under compression (projected Newton converging linearly, many iterations) the
    recycled start needs fewer PCG iterations (1043 against 687 when written); on the driven
    sheet, whose steps take two or three Newton iterations, not more."""
    sc = syn.driven_sheet(40, seed=301) if scene == "driven" else syn.compressed_sheet(40, seed=2, compression=0.05)
    sh = oracle_sheet(sc)
    res = {}
    for warm in (bsc.BSC_WARM_NONE, bsc.BSC_WARM_PREVIOUS):
        ctx = bsc.context_for_scene(sc)
        x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
        tot = {"newton": 0, "pcg": 0, "used": 0, "fallbacks": 0}
        for k in range(3):
            xs, vs = x.clone(), v.clone()
            opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), precision=precision, rtol=1e-6, pcg_rtol=1e-3,
                                 max_newton=400, warm_start=warm)
            st, stats = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(k)), opts)
            assert st == 0
            mask = np.zeros(sc.n_cp, dtype=bool)
            mask[sc.pins] = True
            xn, vn = bsc.to_aos(xs), bsc.to_aos(vs)
            _, g, _ = oracle.assemble(sh, bsc.to_aos(x), xn + sc.dt * vn, sc.dt, sc.gravity, mask, want_hessian=False)
            assert np.linalg.norm(g) <= 1.01e-6 * stats.g0_norm
            for key, val in (("newton", stats.newton_iters), ("pcg", stats.pcg_iters_total),
                             ("used", stats.warm_start_used), ("fallbacks", stats.warm_start_fallbacks)):
                tot[key] += val
        res[warm] = (tot, x.clone())
        print(f"[warm {warm}] {scene} prec {precision}: {tot}")
    t0, x0 = res[bsc.BSC_WARM_NONE]
    t2, x2 = res[bsc.BSC_WARM_PREVIOUS]
    assert t0["used"] == 0 and t0["fallbacks"] == 0
    assert t2["used"] > 0
    assert t2["pcg"] <= t0["pcg"]
    if scene != "driven":
        assert t2["pcg"] < 0.8 * t0["pcg"]
    # both trajectories are the steps' solutions to the Newton tolerance
    d = bsc.to_aos(x2) - bsc.to_aos(x0)
    step = bsc.to_aos(x0) - sc.x0
    print(f"  |x_warm - x_zero| / |x - x0| = {np.linalg.norm(d) / np.linalg.norm(step):.2e}")
    assert np.linalg.norm(d) <= 1e-3 * np.linalg.norm(step)


@pytest.mark.parametrize("precision", [bsc.BSC_FP64, bsc.BSC_FP32_MIXED])
def test_recycled_start_under_the_step_rule(precision):
    sc = syn.driven_sheet(40, seed=301)
    ctx = bsc.context_for_scene(sc)
    x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
    for k in range(3):
        opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), precision=precision, stop_mode=bsc.BSC_STOP_STEP,
                             atol=1e-2, pcg_rtol=1e-3, warm_start=bsc.BSC_WARM_PREVIOUS)
        st, stats = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(k)), opts)
        assert st == 0
        print(f"[warm previous, step rule] step {k}: newton {stats.newton_iters} pcg {stats.pcg_iters_total} "
              f"used {stats.warm_start_used}")
        # one decision per solved direction: every Newton iteration, plus the one whose direction met the stop
        assert stats.newton_iters <= stats.warm_start_used + stats.warm_start_fallbacks <= stats.newton_iters + 1
    assert torch.isfinite(x).all()


def test_bad_warm_start_mode_is_rejected():
    sc = syn.hanging_sheet(6, seed=1)
    ctx = bsc.context_for_scene(sc)
    x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
    opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), warm_start=7)
    st, _ = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(0)), opts, raise_on_error=False)
    assert st == -1
