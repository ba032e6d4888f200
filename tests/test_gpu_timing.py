"""Timing modes of bsc_newton_step: BSC_TIMING_CG (default), BSC_TIMING_PHASES, BSC_TIMING_OFF.

The events are markers on the context's stream and change no result: from the same state on
fresh contexts the three modes give bitwise the same iterate, velocity and counts. PHASES fills
the phase times, CG only the CG kernel time, OFF neither; an unknown mode is rejected.
"""
import pytest

import synthetic as syn

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2506_18867_amd import bsc  # noqa: E402


def _step(sc, timing, precision, warm):
    ctx = bsc.context_for_scene(sc)
    x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
    opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), precision=precision, rtol=1e-6, pcg_rtol=1e-3,
                         max_newton=200, max_pcg=4000, pcg_adaptive=1, warm_start=warm, timing=timing)
    stats = []
    for k in range(2):
        st, s = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(k)), opts)
        assert st == 0
        stats.append(s.as_dict())
    torch.cuda.synchronize()
    return x, v, stats


@pytest.mark.parametrize("precision,warm", [(bsc.BSC_FP32_MIXED, bsc.BSC_WARM_PREVIOUS),
                                            (bsc.BSC_FP64, bsc.BSC_WARM_NONE)])
def test_timing_modes_change_no_result(precision, warm):
    sc = syn.driven_sheet(40, seed=11)
    runs = {m: _step(sc, m, precision, warm) for m in (bsc.BSC_TIMING_CG, bsc.BSC_TIMING_PHASES, bsc.BSC_TIMING_OFF)}
    x0, v0, s0 = runs[bsc.BSC_TIMING_CG]
    counts = ("newton_iters", "pcg_iters_total", "ls_halvings", "warm_start_used", "cg_launches", "cg_active_launches")
    for m, (x, v, s) in runs.items():
        assert torch.equal(x, x0) and torch.equal(v, v0), m
        for a, b in zip(s, s0):
            assert all(a[k] == b[k] for k in counts), (m, a, b)
            assert a["g_norm"] == b["g_norm"] and a["energy"] == b["energy"]
    phase_keys = ("ms_assemble", "ms_pcg", "ms_linesearch")
    for s in runs[bsc.BSC_TIMING_PHASES][2]:
        assert all(s[k] > 0.0 for k in phase_keys) and s["ms_cg_kernels"] > 0.0, s
        assert s["ms_cg_kernels"] <= s["ms_pcg"] * 1.05 + 0.05, s
    for s in runs[bsc.BSC_TIMING_CG][2]:
        assert all(s[k] == 0.0 for k in phase_keys) and s["ms_cg_kernels"] > 0.0, s
    for s in runs[bsc.BSC_TIMING_OFF][2]:
        assert all(s[k] == 0.0 for k in phase_keys + ("ms_cg_kernels",)) and s["ms_total"] > 0.0, s


def test_bad_timing_mode_is_rejected():
    sc = syn.hanging_sheet(6, seed=1)
    ctx = bsc.context_for_scene(sc)
    x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
    opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), timing=3)
    st, _ = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(0)), opts, raise_on_error=False)
    assert st == -1
