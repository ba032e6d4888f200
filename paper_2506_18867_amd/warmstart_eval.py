"""Evaluates the learned PCG warm start on a held-out sheet (compression and drape).

From the same state of an FP64 reference trajectory at every step, four solves are run:
(i) FP64 zero-start PCG, (ii) FP32-mixed zero-start PCG, (iii) FP32-mixed PCG warm-started by
the network (falling back to zero start when the prediction does not lower the residual), and
(iv) FP32-mixed PCG warm-started by the previous Newton direction of the same solve (the
recycled start, with the same scaling and fallback). All use the same Newton stopping rule.
The trajectory advances with (i). Reported per variant: ms per step, Newton and PCG
iterations, warm-start use/fallbacks, the final |g|/|g0|.

Usage: python -m paper_2506_18867_amd.warmstart_eval --weights paper_2506_18867_amd/weights/warmstart_c32.f32
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DEFAULT_WEIGHTS = os.path.join(ROOT, "paper_2506_18867_amd", "weights", "warmstart_c32.f32")


def heldout_scene(n: int, seed: int, compression: float):
    import synthetic as syn
    g = syn.rng(seed)
    E, t = syn.MATERIAL_GRID[int(g.integers(0, len(syn.MATERIAL_GRID)))]
    return syn.compressed_sheet(n, seed=seed, material=syn.stvk_material(young=E, thickness=t), compression=compression)


def evaluate(weights_path: str, n: int = 226, seed: int = 5001, steps: int = 20, stop: str = "step", rtol: float = 1e-6,
             atol: float = 1e-2, pcg_rtol: float = 1e-3, max_newton: int = 60, compression: float = 0.1, log=print):
    import torch
    from paper_2506_18867_amd import bsc
    sc = heldout_scene(n, seed, compression)
    ctx = bsc.context_for_scene(sc)
    w = torch.from_numpy(np.fromfile(weights_path, dtype=np.float32)).cuda()
    ctx.bsc_warmstart_load(w)
    x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
    variants = [("fp64", bsc.BSC_FP64, bsc.BSC_WARM_NONE), ("fp32_mixed", bsc.BSC_FP32_MIXED, bsc.BSC_WARM_NONE),
                ("fp32_mixed_warm", bsc.BSC_FP32_MIXED, bsc.BSC_WARM_NET),
                ("fp32_mixed_recycled", bsc.BSC_FP32_MIXED, bsc.BSC_WARM_PREVIOUS)]
    res = {name: {"ms": [], "newton": [], "pcg": [], "used": 0, "fallbacks": 0, "g_rel": [], "status": []}
           for name, _, _ in variants}
    for step in range(steps):
        tgt = bsc.to_soa(sc.pin_targets(step))
        out = {}
        for name, prec, ws in variants:
            xs, vs = x.clone(), v.clone()
            opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), precision=prec, warm_start=ws,
                                 stop_mode=bsc.BSC_STOP_GRAD if stop == "grad" else bsc.BSC_STOP_STEP,
                                 rtol=rtol, atol=atol, pcg_rtol=pcg_rtol, max_newton=max_newton, max_pcg=6000)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, s = ctx.bsc_newton_step(xs, vs, tgt, opts, raise_on_error=False)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0)
            r = res[name]
            r["ms"].append(ms)
            r["newton"].append(s.newton_iters)
            r["pcg"].append(s.pcg_iters_total)
            r["used"] += s.warm_start_used
            r["fallbacks"] += s.warm_start_fallbacks
            r["g_rel"].append(s.g_norm / s.g0_norm if s.g0_norm > 0 else 0.0)
            r["status"].append(st)
            out[name] = (xs, vs)
        x, v = out["fp64"]
        if step % 5 == 0 or step == steps - 1:
            log(f"[eval] step {step}: " + " ".join(f"{k}: {res[k]['ms'][-1]:.1f}ms/{res[k]['pcg'][-1]}it" for k in res))
    summary = {}
    for name in res:
        r = res[name]
        summary[name] = {"ms_per_step": float(np.mean(r["ms"])), "newton_total": int(sum(r["newton"])),
                         "pcg_total": int(sum(r["pcg"])), "warm_used": r["used"], "warm_fallbacks": r["fallbacks"],
                         "g_rel_max": float(np.max(r["g_rel"])), "failed_steps": int(sum(1 for s in r["status"] if s != 0))}
    base = summary["fp32_mixed"]
    summary["gain"] = {"pcg_iters_zero_over_warm": base["pcg_total"] / max(1, summary["fp32_mixed_warm"]["pcg_total"]),
                       "ms_zero_over_warm": base["ms_per_step"] / summary["fp32_mixed_warm"]["ms_per_step"],
                       "ms_fp64_over_warm": summary["fp64"]["ms_per_step"] / summary["fp32_mixed_warm"]["ms_per_step"],
                       "pcg_iters_zero_over_recycled": base["pcg_total"] / max(1, summary["fp32_mixed_recycled"]["pcg_total"]),
                       "ms_zero_over_recycled": base["ms_per_step"] / summary["fp32_mixed_recycled"]["ms_per_step"],
                       "ms_fp64_over_recycled": summary["fp64"]["ms_per_step"] / summary["fp32_mixed_recycled"]["ms_per_step"]}
    summary["config"] = {"n": n, "seed": seed, "steps": steps, "stop": stop, "rtol": rtol, "atol": atol,
                         "pcg_rtol": pcg_rtol, "compression": compression, "material": [sc.material.young, sc.material.thickness]}
    return summary


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--weights", default=DEFAULT_WEIGHTS)
    ap.add_argument("--n", type=int, default=226)
    ap.add_argument("--seed", type=int, default=5001)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--stop", choices=["grad", "step"], default="step")
    ap.add_argument("--rtol", type=float, default=1e-6)
    ap.add_argument("--pcg-rtol", type=float, default=1e-3)
    ap.add_argument("--max-newton", type=int, default=60)
    ap.add_argument("--compression", type=float, default=0.1)
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    s = evaluate(args.weights, args.n, args.seed, args.steps, args.stop, args.rtol, 1e-2, args.pcg_rtol, args.max_newton,
                 args.compression, log=lambda m: print(m, flush=True))
    print(json.dumps(s), flush=True)


if __name__ == "__main__":
    main()
