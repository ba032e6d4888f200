"""What the trained warm-start network gains over the method without it (GPU).

Uses the committed weights (paper_2506_18867_amd/weights/warmstart_c32.f32, trained by
paper_2506_18867_amd/train_warmstart.py on the method's own 128 x 128 solves, seeds 4000+).
On held-out sheets (seeds 9000+): the trained net's loss on freshly logged (g, p) pairs must be
far below an untrained net's. The warm start itself does not pay: the residual test accepts its
guess in a minority of Newton iterations, the PCG iterations it saves stay within a few
percent, and the network's forward pass costs more time than those iterations, so a
warm-started step is slower than a zero-start step (measured 2.2x slower on the held-out
226 x 226 compressed drape at 1e-6 |g0|). The second test pins that negative result: the
warm-started step meets the same stopping rule, and its PCG iterations stay within 5 % of the
zero start's either way."""
import os

import numpy as np
import pytest

import synthetic as syn

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_2506_18867_amd import bsc  # noqa: E402
from paper_2506_18867_amd.train_warmstart import init_weights  # noqa: E402

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2506_18867_amd", "weights",
                       "warmstart_c32.f32")


def _trained():
    return torch.from_numpy(np.fromfile(WEIGHTS, dtype=np.float32)).cuda()


def test_trained_net_beats_untrained_on_heldout_pairs():
    n = 96
    sc = syn.compressed_sheet(n, seed=9001, material=syn.stvk_material(young=1e5, thickness=1e-3))
    ctx = bsc.context_for_scene(sc)
    cap = 24
    G = torch.zeros(cap, 3 * n * n, dtype=torch.float32, device="cuda")
    P = torch.zeros_like(G)
    ctx.bsc_set_sample_log(G, P, cap)
    x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
    opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), precision=bsc.BSC_FP32_MIXED, stop_mode=bsc.BSC_STOP_STEP,
                         max_newton=25, pcg_rtol=1e-8, max_pcg=6000)
    for step in range(6):
        ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(step)), opts, raise_on_error=False)
        if ctx.bsc_sample_log_count() >= cap:
            break
    k = ctx.bsc_sample_log_count()
    assert k >= 8
    xb = G[:k].view(k, 3, n * n)
    yb = P[:k].view(k, 3, n * n)
    acts = torch.empty(5 * k * 32 * n * n, dtype=torch.float32, device="cuda")
    losses = {}
    for name, w in (("trained", _trained()), ("untrained", torch.from_numpy(init_weights(123)).cuda())):
        out = ctx.bsc_net_forward(w, xb, acts)
        loss, _ = ctx.bsc_net_loss(xb, out, yb)
        losses[name] = loss.item()
    print(f"[warm start] held-out loss trained={losses['trained']:.3f} untrained={losses['untrained']:.3f}")
    assert losses["trained"] < 0.6 * losses["untrained"]


def test_warm_start_gains_no_pcg_iterations_and_keeps_the_stopping_rule():
    sc = syn.driven_sheet(128, seed=9002, cell=7)                 # E = 1e5 Pa, t = 1 mm
    stats = {}
    for ws in (0, 1):
        ctx = bsc.context_for_scene(sc)
        if ws:
            ctx.bsc_warmstart_load(_trained())
        x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
        opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), precision=bsc.BSC_FP32_MIXED, warm_start=ws,
                             stop_mode=bsc.BSC_STOP_STEP, max_newton=60, pcg_rtol=1e-3, max_pcg=6000)
        tot = {"pcg": 0, "newton": 0, "used": 0, "fallbacks": 0, "ms": 0.0}
        for step in range(4):
            st, s = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(step)), opts)
            assert st == 0
            tot["pcg"] += s.pcg_iters_total
            tot["newton"] += s.newton_iters
            tot["used"] += s.warm_start_used
            tot["fallbacks"] += s.warm_start_fallbacks
            tot["ms"] += s.ms_total
        stats[ws] = tot
    print(f"[warm start] zero-start {stats[0]} | warm {stats[1]} | PCG ratio zero/warm = "
          f"{stats[0]['pcg'] / max(1, stats[1]['pcg']):.3f}, time ratio = {stats[0]['ms'] / stats[1]['ms']:.3f}")
    # one warm-start attempt per PCG solve; with the step rule the last solve of a step ends it
    assert stats[1]["newton"] <= stats[1]["used"] + stats[1]["fallbacks"] <= stats[1]["newton"] + 4
    # no gain and no loss beyond 5 % of the PCG iterations (a better network would move this)
    assert 0.95 * stats[0]["pcg"] <= stats[1]["pcg"] <= 1.05 * stats[0]["pcg"]
    # both runs met the same stopping rule at every step (status 0 above); compressed sheets may
    # buckle into different but equally valid states, so the states themselves are not compared
