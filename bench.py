"""Benchmark of the B-spline cloth hot path on one MI355X.

One step = one implicit-Euler step of the 226 x 226-control-point driven sheet (50,176 knot-span
elements; material cell E = 1e4 Pa, t = 1 mm; random held CPs plus a sinusoidally driven corner;
gravity): projected Newton with element evaluation, PSD projection, assembly, block-Jacobi PCG
(Eisenstat-Walker tolerance) and line search, all in the library's HIP kernels, stopped at
|g| <= 1e-6 |g0| (free-DOF gradient, evaluated in double). The headline path is FP32-mixed with
the PCG warm-started from the previous Newton direction (--warm). Every step starts from the
state of the FP32-mixed trajectory, and the same step is also solved from that identical state
to the same residual in plain FP64 (zero-start PCG), which gives the "vs FP64" ratio at equal
final residual, and with the other start in each precision (FP32-mixed zero start, FP64 with the
same warm start), each on a context of its own. The trajectory advances with the FP32-mixed
result.

value = elements advanced per second (n_elem * steps / timed seconds of the FP32-mixed steps) in
Melem/s; ms_per_step is the mean FP32-mixed step time (each step bracketed by device syncs).

The timed steps record HIP events only around the PCG launches (the roofline's kernel time);
phases_ms_per_step_fp32 comes from 5 more steps from the headline's start state with every phase
timed (about 14 events per Newton iteration, each a gap between two kernels).

Further legs (each a field of the one JSON line):
  step_rule         the same steps under the paper's stopping rule |p|_inf / dt <= 1e-2 m/s;
  fp32_vs_fp64_100  the 100 x 100 compressed drape, 200 steps, FP32-mixed and FP64 from the
                    identical FP64-trajectory state every step: per-step error and iteration counts;
  material_sweep    the nine (E, t) cells of the 226 x 226 driven sheet, FP32-mixed at 1e-6 |g0|;
  warm_start        the 226 x 226 held-out compressed drape: FP64, FP32-mixed, FP32-mixed with the
                    learned PCG warm start and with the recycled one, from the same
                    FP64-trajectory state, all at 1e-6 |g0|;
  assembly, spmv    the eval+assembly pass and the plain SpMV timed on their own;
  ceilings          measured copy bandwidth from HBM and from the caches (footprints that stay
                    resident in the L2s and the 256 MB Infinity Cache);
  partial_factorization  the Newton system with a contact Hessian at several contact
                    intensities: the Gershgorin trigger, the series and the merged solve;
  quadrature_ablation, general_rest, contact_conversion, wrinkling_convergence.
The roofline object covers the kernel with the largest share of the step (the fused PCG-iteration
kernel), timed live by the library with HIP events before the first and after the last CG launch of
each burst on its stream (the torch current stream). cpu_baseline is the oracle's eval+assembly on the same 226 x 226 sheet.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 226] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
# Algorithmic FLOPs of eval+assembly per element: about 2.09 membrane points per element x (F 108,
# density and stress ~200, gradient 108, the 45 unique 3x3 blocks of J^T A J at ~80 each) plus
# 1.01 bending evaluations x ~300, before the PSD projection.
ASM_FLOP_PER_ELEM = 8.5e3

# HBM traffic of one active k_cg_fused<float> launch on this workload, from two rocprofv3 --pmc
# passes (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch, mean over the launches that ran an
# iteration), each divided by what the same counter reads for a 1 GiB device copy whose source
# was evicted first (`bench.py --copy-probe 1024`: FETCH_SIZE 0.500, WRITE_SIZE 1.000 of the
# bytes). Summary and commands: profiles/k_cg_fused_226_traffic.md. Valid only for the kernel
# source it was measured on (hash of its text in solve.hip); otherwise reported as null.
CG_TRAFFIC = {"kernel_sha256_16": "0899f3d6f38822e8", "fetch_kib": 16697.6, "write_kib": 5443.2,
              "fetch_factor": 0.500, "write_factor": 1.000}


def cg_kernel_sha():
    import hashlib
    src = open(os.path.join(ROOT, "paper_2506_18867_amd", "csrc", "solve.hip")).read()
    a = src.rindex("template <typename T, bool FIRST>", 0, src.index(" k_cg_fused(DevSheet S"))
    b = src.index("\n}\n", a) + 3
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]


def cg_traffic_bytes():
    """Calibrated HBM bytes per active fused-CG launch, or None if the kernel changed since."""
    t = CG_TRAFFIC
    try:
        if cg_kernel_sha() != t["kernel_sha256_16"]:
            return None
    except (OSError, ValueError):
        return None
    return int(1024 * (t["fetch_kib"] / t["fetch_factor"] + t["write_kib"] / t["write_factor"]))


def parse(argv=None):
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--n", type=int, default=226)
    p.add_argument("--seed", type=int, default=304)
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--kernel-reps", type=int, default=50)
    p.add_argument("--noise", type=float, default=0.0, help="z-noise amplitude of the start state [m]")
    p.add_argument("--rtol", type=float, default=1e-6, help="Newton stop |g| <= rtol |g0| (headline)")
    p.add_argument("--atol", type=float, default=1e-2, help="|p|_inf / dt of the step-rule leg [m/s]")
    p.add_argument("--max-newton", type=int, default=500)
    p.add_argument("--pcg-rtol", type=float, default=1e-3)
    p.add_argument("--adaptive", type=int, default=1, help="Eisenstat-Walker PCG tolerance (1) or fixed (0)")
    p.add_argument("--eta-max", type=float, default=0.0,
                   help="cap of the Eisenstat-Walker PCG tolerance (0: the library's default for the stop rule)")
    p.add_argument("--warm", choices=["previous", "none", "net"], default="previous",
                   help="PCG warm start of the FP32-mixed headline (and of the step-rule, sweep and ablation legs): "
                        "the previous Newton direction, none (zero start) or the learned network")
    p.add_argument("--variants", choices=["all", "headline"], default="all",
                   help="headline steps: FP32-mixed with the warm start beside plain FP64, FP32-mixed zero start and "
                        "FP64 with the same start (all), or FP32-mixed alone (headline: for kernel traces of its launches)")
    p.add_argument("--precond", choices=["jacobi", "mg"], default="jacobi",
                   help="PCG preconditioner: block Jacobi (fused kernel) or the multigrid V-cycle")
    p.add_argument("--start", choices=["predictor", "previous"], default="previous",
                   help="first Newton iterate of the |g| <= rtol |g0| legs (g0 is taken there): x^n, or the "
                        "inertial predictor x^n + dt v^n")
    p.add_argument("--step-rule-start", choices=["predictor", "previous"], default="predictor",
                   help="first Newton iterate of the |p|inf/dt leg")
    p.add_argument("--step-rule-steps", type=int, default=10, help="steps of the |p|inf/dt leg (0: skip)")
    p.add_argument("--c2-steps", type=int, default=200, help="steps of the 100x100 FP32-vs-FP64 leg (0: skip)")
    p.add_argument("--sweep-steps", type=int, default=3, help="timed steps per material cell (0: skip)")
    p.add_argument("--warm-steps", type=int, default=10, help="steps of the warm-start leg (0: skip)")
    p.add_argument("--quad-steps", type=int, default=3,
                   help="steps of the quadrature-ablation leg (reduced vs 2x2 interior rule; 0: skip)")
    p.add_argument("--general-steps", type=int, default=3,
                   help="steps of the general-rest leg (the same driven sheet on a curved domain; 0: skip)")
    p.add_argument("--contact-pairs", type=int, default=100000,
                   help="contact pairs of the contact-Hessian conversion leg (0: skip)")
    p.add_argument("--pf-pairs", type=int, default=20000,
                   help="contact pairs of the partial-factorization leg (0: skip)")
    p.add_argument("--pf-scales", default="1e-6,1e-5,3e-5,1e-4,1e-3,1e-2",
                   help="contact-Hessian scales of the partial-factorization leg, comma-separated")
    p.add_argument("--wrinkle-levels", default="16,32,48,64,80,96,112,128",
                   help="spans across the width of the wrinkling-plate convergence leg, comma-separated "
                        "('': skip)")
    p.add_argument("--cpu-reps", type=int, default=5, help="timed oracle assemblies (after one warm-up)")
    p.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                   help="only run the traffic-counter calibration: one device-to-device copy of MIB MiB whose "
                        "source has been evicted from the caches, then exit")
    return p.parse_args(argv)


def copy_probe(mib, torch):
    """Calibration for the FETCH_SIZE / WRITE_SIZE counters: a plain copy of known size. The source
    is written first, then a second buffer of the same size is written to evict it from the L2s
    and the Infinity Cache, so the copy reads every byte from HBM."""
    n = mib << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    evict = torch.empty(n, dtype=torch.uint8, device="cuda")
    evict.fill_(2)
    dst = torch.empty(n, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n}), flush=True)


def copy_bandwidth(footprint_bytes, reps, torch):
    """GB/s of a device copy whose source plus destination occupy footprint_bytes, repeated reps
    times back to back (HIP events): above the caches' capacity every copy streams from HBM; below
    it the buffers stay resident after the first copy."""
    half = footprint_bytes // 2 // 16 * 16
    src = torch.ones(half // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    return round(2 * half / (ms * 1e-3) / 1e9, 1)


def warm_mode(bsc, name):
    return {"none": bsc.BSC_WARM_NONE, "net": bsc.BSC_WARM_NET, "previous": bsc.BSC_WARM_PREVIOUS}[name]


def step_opts(bsc, sc, precision, args, stop="grad", warm=None):
    """Options of one step; warm None takes --warm."""
    warm = warm_mode(bsc, args.warm) if warm is None else warm
    start = args.start if stop == "grad" else args.step_rule_start
    return bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), precision=precision, rtol=args.rtol, atol=args.atol,
                         stop_mode=bsc.BSC_STOP_GRAD if stop == "grad" else bsc.BSC_STOP_STEP,
                         pcg_rtol=args.pcg_rtol, max_newton=args.max_newton, max_pcg=6000,
                         pcg_adaptive=args.adaptive, warm_start=warm, pcg_eta_max=args.eta_max,
                         preconditioner=bsc.BSC_PRECOND_MULTIGRID if args.precond == "mg" else bsc.BSC_PRECOND_JACOBI,
                         start=bsc.BSC_START_PREVIOUS if start == "previous" else bsc.BSC_START_PREDICTOR)


def phase_opts(bsc, opts):
    """A copy of opts that times every phase of the step (GPU events, about 14 per Newton
    iteration)."""
    o = type(opts).from_buffer_copy(opts)
    o.timing = bsc.BSC_TIMING_PHASES
    return o


def timed_step(ctx, x, v, tgt, opts, torch):
    """One implicit-Euler step in place, bracketed by device syncs; returns (seconds, stats dict).
    The stats carry the step's status: a step that did not converge leaves its last iterate in
    x and v and is counted, not hidden."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, s = ctx.bsc_newton_step(x, v, tgt, opts, raise_on_error=False)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    d = s.as_dict()
    d["status"] = int(st)
    if st not in (0, -5):                 # anything but "not converged within max_newton" is fatal
        raise RuntimeError(f"newton step failed with status {st}")
    return sec, d


def paired_steps(ctx, sc, x, v, step0, steps, variants, advance, torch, bsc, log=None):
    """From the same state every step, runs each (name, opts[, context]) variant (a variant with a
    context of its own keeps its own previous Newton direction for the recycled warm start); the
    trajectory then continues from variant `advance`. Returns {name: [(seconds, stats,
    dx_rel_vs_first_variant)]}."""
    variants = [(vt[0], vt[1], vt[2] if len(vt) > 2 else ctx) for vt in variants]
    out = {name: [] for name, _, _ in variants}
    for k in range(steps):
        tgt = bsc.to_soa(sc.pin_targets(step0 + k))
        res = {}
        for name, opts, vctx in variants:
            xs, vs = x.clone(), v.clone()
            sec, s = timed_step(vctx, xs, vs, tgt, opts, torch)
            res[name] = (xs, vs, sec, s)
        ref = variants[0][0]
        dref = res[ref][0] - x
        nref = float(torch.linalg.vector_norm(dref))
        for name, _, _ in variants:
            err = float(torch.linalg.vector_norm(res[name][0] - res[ref][0])) / max(nref, 1e-300)
            out[name].append((res[name][2], res[name][3], err))
        x.copy_(res[advance][0])
        v.copy_(res[advance][1])
        if log and (k % 50 == 0 or k == steps - 1):
            log(f"[bench] {sc.name} step {step0 + k}: " +
                " ".join(f"{n}: {1e3 * res[n][2]:.2f} ms {res[n][3]['newton_iters']}N/{res[n][3]['pcg_iters_total']}it"
                         for n, _, _ in variants))
    return out


def g_rel(s):
    return s["g_norm"] / s["g0_norm"] if s["g0_norm"] > 0 else 0.0


def summarize(runs, n_elem):
    sec = sum(r[0] for r in runs)
    return {"ms_per_step": round(1e3 * sec / len(runs), 3),
            "melem_s": round(n_elem * len(runs) / sec / 1e6, 3),
            "newton": [r[1]["newton_iters"] for r in runs], "pcg": [r[1]["pcg_iters_total"] for r in runs],
            "g_rel_max": float("%.3g" % max(g_rel(r[1]) for r in runs)),
            "not_converged": int(sum(1 for r in runs if r[1]["status"] != 0))}


def max_deflection(sc, x):
    """Largest |z| of the B-spline surface with CPs x (n_cp, 3) over a 401 x 1001 parameter grid."""
    from scipy.interpolate import BSpline
    ku, kv = sc.knots_u / sc.knots_u[-1], sc.knots_v / sc.knots_v[-1]
    Bu = BSpline.design_matrix(np.linspace(0.0, 1.0, 401), ku, 2).toarray()
    Bv = BSpline.design_matrix(np.linspace(0.0, 1.0, 1001), kv, 2).toarray()
    return float(np.abs(Bv @ x[:, 2].reshape(sc.n_v, sc.n_u) @ Bu.T).max())


def time_kernel(fn, reps, torch):
    """Average duration (ms) of fn() over reps launches, HIP events on the current stream."""
    fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / reps


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(n=226, seed=304, reps=5):
    """The oracle's eval+assembly (plain C, FP64, one thread: element E/g/H with PSD projection,
    lumped-mass inertia, gravity, pins, the Hessian in stencil form) on the same 226 x 226 driven
    sheet as the headline, at a state displaced by a smooth field; median of `reps` timed calls
    after one warm-up. Second field: a sample of the oracle's full Newton step."""
    import oracle
    import synthetic as syn
    sc = syn.driven_sheet(n, seed=seed)
    m = sc.material
    sh = oracle.Sheet(sc.n_u, sc.n_v, sc.knots_u, sc.knots_v, sc.rest, m.membrane, m.young, m.poisson,
                      m.thickness, m.mu_st1, m.mu_st2, m.mu_sh, m.mu_bend, m.rho_area)
    x = sc.x0 + syn.smooth_field(n, n, 3, amp=0.01)
    mask = np.zeros(sc.n_cp, dtype=bool)
    mask[sc.pins] = True
    times = []
    for r in range(reps + 1):
        t0 = time.perf_counter()
        oracle.assemble(sh, x, sc.x0, sc.dt, sc.gravity, mask)
        if r > 0:
            times.append(time.perf_counter() - t0)
    sec = float(np.median(times))
    out = {"value": round(sc.n_elem / sec / 1e6, 5), "unit": "Melem/s", "cores": 1, "kind": "oracle",
           "sample": f"eval+assembly of the {n}x{n} driven sheet ({sc.n_elem} elements), FP64, one thread, "
                     f"median of {reps} after 1 warm-up",
           "ms_per_assembly": round(1e3 * sec, 1), "cpu_model": cpu_model(), "nproc": os.cpu_count(),
           "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}
    # a full Newton step of the oracle (sparse LU directions), at a size it finishes in seconds
    sc2 = syn.driven_sheet(100, seed=seed)
    m2 = sc2.material
    sh2 = oracle.Sheet(sc2.n_u, sc2.n_v, sc2.knots_u, sc2.knots_v, sc2.rest, m2.membrane, m2.young, m2.poisson,
                       m2.thickness, m2.mu_st1, m2.mu_st2, m2.mu_sh, m2.mu_bend, m2.rho_area)
    t0 = time.perf_counter()
    r = oracle.newton_step(sh2, sc2.x0, sc2.v0, sc2.dt, sc2.gravity, sc2.pins, sc2.pin_targets(0), rtol=1e-6,
                           start="predictor")
    s2 = time.perf_counter() - t0
    out["newton_step_sample"] = {"ms_per_step": round(1e3 * s2, 1), "newton": r.iters,
                                 "sample": "one implicit-Euler step of the 100x100 driven sheet from its start "
                                           "state, inertial-predictor start, |g|<=1e-6|g0|, oracle C kernels + "
                                           "scipy sparse LU, one thread"}
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the hot path runs on one GPU; runs on several GPUs are not supported "
              "(a sheet would shard by CP-row strips with a 2-row halo exchange per CG iteration)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_probe > 0:
        copy_probe(args.copy_probe, torch)
        return

    import synthetic as syn
    from paper_2506_18867_amd import bsc

    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    torch.cuda.set_device(0)
    sc = syn.driven_sheet(args.n, seed=args.seed, noise=args.noise)
    ctx = bsc.context_for_scene(sc)
    n, ne = sc.n_cp, sc.n_elem
    x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)

    # ---- headline: FP32-mixed steps at |g| <= rtol |g0| with the warm start, and from the
    #      identical state beside them: plain FP64 (zero start), FP32-mixed with zero start and
    #      FP64 with the same warm start, each on a context of its own ----
    wm = warm_mode(bsc, args.warm)
    lw = bsc.BSC_WARM_PREVIOUS if wm == bsc.BSC_WARM_PREVIOUS else bsc.BSC_WARM_NONE     # the other legs' start
    if wm == bsc.BSC_WARM_NET:
        from paper_2506_18867_amd import warmstart_eval as we
        ctx.bsc_warmstart_load(torch.from_numpy(np.fromfile(we.DEFAULT_WEIGHTS, dtype=np.float32)).cuda())
    o32 = step_opts(bsc, sc, bsc.BSC_FP32_MIXED, args)
    o64 = step_opts(bsc, sc, bsc.BSC_FP64, args, warm=bsc.BSC_WARM_NONE)
    variants = [("fp32_mixed", o32, ctx)]
    if args.variants == "all":
        variants += [("fp64", o64, bsc.context_for_scene(sc))]
    if wm != bsc.BSC_WARM_NONE and args.variants == "all":
        variants += [("fp32_mixed_zero_start", step_opts(bsc, sc, bsc.BSC_FP32_MIXED, args, warm=bsc.BSC_WARM_NONE),
                      bsc.context_for_scene(sc))]
        if wm == bsc.BSC_WARM_PREVIOUS:
            variants += [("fp64_warm", step_opts(bsc, sc, bsc.BSC_FP64, args), bsc.context_for_scene(sc))]
    paired_steps(ctx, sc, x, v, 0, args.warmup, variants, "fp32_mixed", torch, bsc)
    xs, vs = x.clone(), v.clone()
    head = paired_steps(ctx, sc, x, v, args.warmup, args.steps, variants, "fp32_mixed", torch, bsc, log)
    r32, r64 = head["fp32_mixed"], head.get("fp64", [])
    sec32 = sum(r[0] for r in r32)
    sec64 = sum(r[0] for r in r64)
    st32 = [r[1] for r in r32]
    secs = {name: sum(r[0] for r in head[name]) for name in head}
    log("[bench] headline: " + ", ".join(f"{name} {1e3 * secs[name] / args.steps:.3f} ms/step" for name in head))
    # The headline steps record timing events only around the CG launches (the roofline's kernel
    # time); the per-phase breakdown needs about 14 events per Newton iteration, each a gap between
    # two kernels, so it comes from a few more steps of the FP32-mixed legs from the same state.
    phase_legs = [(name, phase_opts(bsc, o), c) for name, o, c in variants
                  if name in ("fp32_mixed", "fp32_mixed_zero_start")]
    n_phase = min(args.steps, 5)
    phases = paired_steps(ctx, sc, xs.clone(), vs.clone(), args.warmup, n_phase, phase_legs, "fp32_mixed", torch, bsc)

    # ---- the same steps under the paper's stopping rule (|p|_inf / dt <= atol) ----
    step_rule = None
    if args.step_rule_steps > 0:
        xr, vr = xs.clone(), vs.clone()
        rv = [("fp32_mixed", step_opts(bsc, sc, bsc.BSC_FP32_MIXED, args, stop="step", warm=lw), bsc.context_for_scene(sc)),
              ("fp64", step_opts(bsc, sc, bsc.BSC_FP64, args, stop="step", warm=lw), bsc.context_for_scene(sc))]
        rr = paired_steps(ctx, sc, xr, vr, args.warmup, args.step_rule_steps, rv, "fp32_mixed", torch, bsc)
        step_rule = {k: summarize(rr[k], ne) for k in rr}
        step_rule["stop"] = f"|p|inf/dt<={args.atol:g} m/s"
        step_rule["newton_start"] = args.step_rule_start
        step_rule["g_rel"] = {k: [float("%.3g" % g_rel(r[1])) for r in rr[k]] for k in rr}
        step_rule["speedup_vs_fp64"] = round(sum(r[0] for r in rr["fp64"]) / sum(r[0] for r in rr["fp32_mixed"]), 3)

    # ---- 100 x 100 compressed drape: FP32-mixed against FP64 from identical states ----
    c2 = None
    if args.c2_steps > 0:
        sc2 = syn.compressed_sheet(100, seed=2)
        ctx2 = bsc.context_for_scene(sc2)
        x2, v2 = bsc.to_soa(sc2.x0), bsc.to_soa(sc2.v0)
        v2s = [("fp64", step_opts(bsc, sc2, bsc.BSC_FP64, args, warm=lw), ctx2),
               ("fp32_mixed", step_opts(bsc, sc2, bsc.BSC_FP32_MIXED, args, warm=lw), bsc.context_for_scene(sc2))]
        rr = paired_steps(ctx2, sc2, x2, v2, 0, args.c2_steps, v2s, "fp64", torch, bsc, log)
        errs = np.array([r[2] for r in rr["fp32_mixed"]])
        c2 = {"workload": "compressed drape 100x100 CPs (9604 elements), 10% compression, E=1e4 Pa, t=1 mm, "
                          f"{args.c2_steps} steps, both precisions from the FP64-trajectory state, |g|<={args.rtol:g}|g0|",
              "dx_rel_err_fp32_vs_fp64": {"max": float("%.3g" % errs.max()), "median": float("%.3g" % np.median(errs))},
              "fp64": {k: v_ for k, v_ in summarize(rr["fp64"], sc2.n_elem).items() if k not in ("newton", "pcg")},
              "fp32_mixed": {k: v_ for k, v_ in summarize(rr["fp32_mixed"], sc2.n_elem).items() if k not in ("newton", "pcg")},
              "newton_total": {k: int(sum(r[1]["newton_iters"] for r in rr[k])) for k in rr},
              "pcg_total": {k: int(sum(r[1]["pcg_iters_total"] for r in rr[k])) for k in rr}}
        del ctx2

    # ---- the nine (E, t) material cells, FP32-mixed at the headline residual ----
    sweep = None
    if args.sweep_steps > 0:
        sweep = []
        for cell in range(len(syn.MATERIAL_GRID)):
            csc = syn.driven_sheet(args.n, seed=300 + cell)
            cctx = bsc.context_for_scene(csc)
            xc, vc = bsc.to_soa(csc.x0), bsc.to_soa(csc.v0)
            oc = step_opts(bsc, csc, bsc.BSC_FP32_MIXED, args, warm=lw)
            timed_step(cctx, xc, vc, bsc.to_soa(csc.pin_targets(0)), oc, torch)          # warm-up step
            runs = [timed_step(cctx, xc, vc, bsc.to_soa(csc.pin_targets(1 + k)), oc, torch) + (0.0,)
                    for k in range(args.sweep_steps)]
            E_, t_ = syn.MATERIAL_GRID[cell]
            sweep.append(dict(E=E_, t_mm=1e3 * t_, seed=300 + cell, **summarize(runs, csc.n_elem)))
            del cctx
        log("[bench] material sweep: " + " ".join(f"{c['E']:g}/{c['t_mm']:g}:{c['ms_per_step']}ms" for c in sweep))

    # ---- learned warm start on the held-out compressed drape ----
    warm = None
    if args.warm_steps > 0:
        from paper_2506_18867_amd import warmstart_eval as we
        warm = we.evaluate(we.DEFAULT_WEIGHTS, args.n, 5001, args.warm_steps, stop="grad", rtol=args.rtol,
                           pcg_rtol=args.pcg_rtol, max_newton=args.max_newton, log=log)

    # ---- quadrature ablation (Sec. 6.5: reduced rule against the standard 2x2 interior rule) ----
    quad_leg = None
    if args.quad_steps > 0:
        quad_leg = {}
        for name, rule in (("reduced", bsc.BSC_QUAD_REDUCED), ("gauss2_interior", bsc.BSC_QUAD_GAUSS2)):
            qctx = bsc.context_for_scene(sc, quadrature=rule)
            xq, vq = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
            oq = step_opts(bsc, sc, bsc.BSC_FP32_MIXED, args, stop="step", warm=lw)
            timed_step(qctx, xq, vq, bsc.to_soa(sc.pin_targets(0)), oq, torch)            # warm-up
            xq, vq = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
            runs = [timed_step(qctx, xq, vq, bsc.to_soa(sc.pin_targets(k)), oq, torch) for k in range(args.quad_steps)]
            nq = sum(r[1]["newton_iters"] for r in runs)
            secq = sum(r[0] for r in runs)
            outq = (torch.zeros(1, dtype=torch.float64, device="cuda"),
                    torch.empty(3, sc.n_cp, dtype=torch.float32, device="cuda"),
                    torch.empty(114, sc.n_cp, dtype=torch.float32, device="cuda"))
            ms_a = time_kernel(lambda: qctx.bsc_assemble(xq, xq, sc.dt, tuple(sc.gravity), bsc.BSC_FP32_MIXED,
                                                         out=outq), 20, torch)
            quad_leg[name] = {"membrane_points": qctx.sizes.n_membrane_pts, "bending_evals": qctx.sizes.n_bending_evals,
                              "ms_per_step": round(1e3 * secq / args.quad_steps, 3),
                              "newton": [r[1]["newton_iters"] for r in runs],
                              "pcg": [r[1]["pcg_iters_total"] for r in runs],
                              "ms_per_newton_iter": round(1e3 * secq / max(1, nq), 4),
                              "assembly_fp32_ms": round(ms_a, 4)}
            del qctx

    # ---- general rest shapes (Sec. 6.2): the driven sheet on domains whose rest map is not affine ----
    general_leg = None
    if args.general_steps > 0:
        general_leg = {}
        for name, dom in (("square", None), ("bend_150deg", ("bend", 150.0)), ("annulus_0.5", ("annulus", 0.5))):
            gsc = syn.driven_sheet(args.n, seed=args.seed, noise=args.noise, domain=dom)
            gctx = bsc.context_for_scene(gsc)
            og = step_opts(bsc, gsc, bsc.BSC_FP32_MIXED, args, stop="step", warm=lw)
            xq, vq = bsc.to_soa(gsc.x0), bsc.to_soa(gsc.v0)
            timed_step(gctx, xq, vq, bsc.to_soa(gsc.pin_targets(0)), og, torch)           # warm-up
            xq, vq = bsc.to_soa(gsc.x0), bsc.to_soa(gsc.v0)
            runs = [timed_step(gctx, xq, vq, bsc.to_soa(gsc.pin_targets(k)), og, torch) for k in range(args.general_steps)]
            outq = (torch.zeros(1, dtype=torch.float64, device="cuda"),
                    torch.empty(3, gsc.n_cp, dtype=torch.float32, device="cuda"),
                    torch.empty(114, gsc.n_cp, dtype=torch.float32, device="cuda"))
            outd = (torch.zeros(1, dtype=torch.float64, device="cuda"),
                    torch.empty(3, gsc.n_cp, dtype=torch.float64, device="cuda"),
                    torch.empty(114, gsc.n_cp, dtype=torch.float64, device="cuda"))
            ms_a32 = time_kernel(lambda: gctx.bsc_assemble(xq, xq, gsc.dt, tuple(gsc.gravity), bsc.BSC_FP32_MIXED,
                                                           out=outq), 20, torch)
            ms_a64 = time_kernel(lambda: gctx.bsc_assemble(xq, xq, gsc.dt, tuple(gsc.gravity), bsc.BSC_FP64,
                                                           out=outd), 20, torch)
            general_leg[name] = {"ms_per_step": round(1e3 * sum(r[0] for r in runs) / args.general_steps, 3),
                                 "newton": [r[1]["newton_iters"] for r in runs],
                                 "pcg": [r[1]["pcg_iters_total"] for r in runs],
                                 "assembly_fp32_ms": round(ms_a32, 4), "assembly_fp64_ms": round(ms_a64, 4)}
            del gctx

    # ---- contact-Hessian conversion (Sec. 5.2, Alg. "Contact Hessian conversion and assembly") ----
    # A contact mesh of twice the sheet's DOFs embedded in it, dense self-contact of the sheet
    # folded onto itself; wall-clock per call (the call synchronises twice), median of 5.
    contact_leg = None
    if args.contact_pairs > 0:
        uvc, tris, cgrid = syn.contact_mesh(sc.n_u, sc.n_v)
        pvc, Hcp, gcp = syn.contact_pairs(uvc, tris, cgrid, args.contact_pairs, seed=args.seed)
        ctx.bsc_contact_setup(uvc, args.contact_pairs)
        dpv = torch.from_numpy(pvc).cuda()
        dH = torch.from_numpy(Hcp).cuda()
        dg = torch.from_numpy(gcp).cuda()
        res = ctx.bsc_contact_hessian(dpv, dH, dg)
        outc = (res[0], torch.empty(res[1].numel(), dtype=torch.int32, device="cuda"),
                torch.empty(res[1].numel(), 9, dtype=torch.float64, device="cuda"), res[3])
        times = []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = ctx.bsc_contact_hessian(dpv, dH, dg, out=outc)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        ms_c = 1e3 * float(np.median(times))
        nblk = int(res[1].numel())
        contact_leg = {"n_vertices": int(uvc.shape[0]), "pairs": args.contact_pairs, "cp_blocks": nblk,
                       "ms_per_call": round(ms_c, 3), "mpairs_per_s": round(args.contact_pairs / ms_c / 1e3, 3),
                       "mblocks_per_s": round(nblk / ms_c / 1e3, 2)}
        del dpv, dH, dg, outc, res

    # ---- partial factorization (Sec. 5.3): the Newton system with a contact Hessian ----
    # At the headline's last state: H (FP32-mixed, as the Newton step forms it) plus a contact
    # Hessian from the folded-sheet pairs at several intensities (the pair Hessians scaled). Per
    # intensity: the Gershgorin bound and the branch it picks, and the time of both branches
    # (the series at the bound's number of terms, the merged PCG), each PCG solve to the Newton
    # step's first forcing term (0.1) and the series truncated at 0.1 likewise.
    pf_leg = None
    if args.pf_pairs > 0:
        uvc, tris, cgrid = syn.contact_mesh(sc.n_u, sc.n_v)
        ctx.bsc_contact_setup(uvc, args.pf_pairs)
        _, _, Hpf = ctx.bsc_assemble(x, x, sc.dt, tuple(sc.gravity), bsc.BSC_FP32_MIXED)
        _, gpf, _ = ctx.bsc_assemble(x, x, sc.dt, tuple(sc.gravity), bsc.BSC_FP64, want_hess=False)
        bpf = (-gpf).contiguous()
        pf_leg = {"pairs": args.pf_pairs, "pcg_rtol": 0.1, "series_tol": 0.1, "rho_max": 0.5, "cases": []}
        for scale in [float(a) for a in args.pf_scales.split(",")]:
            pv, Hp, _ = syn.contact_pairs(uvc, tris, cgrid, args.pf_pairs, seed=args.seed, scale=scale)
            rp, ci, cv, _ = ctx.bsc_contact_hessian(torch.from_numpy(pv).cuda(), torch.from_numpy(Hp).cuda(),
                                                    want_grad=False)
            case = {"scale": scale, "cp_blocks": int(ci.numel())}
            for name, force in (("auto", 0), ("series", 1), ("merged", 2)):
                # the series is timed only where the bound guarantees convergence (rho < 1); above
                # it a forced series would sum max_terms terms of a possibly divergent expansion
                if name == "series" and not case["rho_bound"] < 1.0:
                    case[name] = None
                    continue
                kw = dict(precision=bsc.BSC_FP32_MIXED, rho_max=0.5, series_tol=0.1, pcg_rtol=0.1, max_pcg=6000,
                          force=force, max_terms=64)
                ctx.bsc_contact_solve(Hpf, sc.dt, rp, ci, cv, bpf, **kw)                  # warm-up
                _, stp = ctx.bsc_contact_solve(Hpf, sc.dt, rp, ci, cv, bpf, **kw)
                case[name] = {"ms": round(stp.ms_total, 3), "pcg_iters": stp.pcg_iters, "terms": stp.terms,
                              "triggered": stp.triggered}
                case["rho_bound"] = float("%.4g" % stp.rho_bound)
            pf_leg["cases"].append(case)
        pf_leg["trigger_rate"] = round(sum(c["auto"]["triggered"] for c in pf_leg["cases"]) / len(pf_leg["cases"]), 3)
        log("[bench] partial factorization: " + " ".join(
            f"{c['scale']:g}: rho {c['rho_bound']:.3g} {'S' if c['auto']['triggered'] else 'M'} "
            f"series {c['series']['ms'] if c['series'] else '-'}ms merged {c['merged']['ms']}ms" for c in pf_leg["cases"]))

    # ---- membrane convergence under refinement (Sec. 6.2, the stretched-plate wrinkling benchmark) ----
    # Per resolution one quasi-static FP64 solve (dt = 1e4 s) from the perturbed start to
    # |g| <= 1e-9 |g0|, and the largest out-of-plane deflection of the surface. The paper's
    # reference value is 3.45 mm; it gives no thickness (1 mm here).
    wrinkle_leg = None
    if args.wrinkle_levels:
        wrinkle_leg = {"reference_mm": 3.45, "thickness_m": 1e-3, "levels": []}
        for nw in [int(a) for a in args.wrinkle_levels.split(",")]:
            wsc = syn.wrinkling_sheet(nw)
            wctx = bsc.context_for_scene(wsc)
            xw, vw = bsc.to_soa(wsc.x0), bsc.to_soa(wsc.v0)
            wopts = bsc.make_opts(dt=wsc.dt, gravity=(0.0, 0.0, 0.0), precision=bsc.BSC_FP64,
                                  stop_mode=bsc.BSC_STOP_GRAD, rtol=1e-9, max_newton=4000, max_pcg=5000,
                                  pcg_rtol=1e-3, pcg_adaptive=1)
            secw, wst = timed_step(wctx, xw, vw, bsc.to_soa(wsc.pin_targets(0)), wopts, torch)
            wrinkle_leg["levels"].append({"spans": [nw, wsc.n_v - 2], "n_cp": wsc.n_cp, "newton": wst["newton_iters"],
                                          "pcg": wst["pcg_iters_total"], "seconds": round(secw, 3),
                                          "energy": wst["energy"],
                                          "max_deflection_mm": round(1e3 * max_deflection(wsc, bsc.to_aos(xw)), 4)})
            del wctx

    # ---- per-kernel timings at the current state (same stream as the library) ----
    xhat = x.clone()
    grav = tuple(sc.gravity)
    out32 = (torch.zeros(1, dtype=torch.float64, device="cuda"), torch.empty(3, n, dtype=torch.float32, device="cuda"),
             torch.empty(114, n, dtype=torch.float32, device="cuda"))
    out64 = (torch.zeros(1, dtype=torch.float64, device="cuda"), torch.empty(3, n, dtype=torch.float64, device="cuda"),
             torch.empty(114, n, dtype=torch.float64, device="cuda"))
    ms_asm32 = time_kernel(lambda: ctx.bsc_assemble(x, xhat, sc.dt, grav, bsc.BSC_FP32_MIXED, out=out32), args.kernel_reps, torch)
    ms_asm64 = time_kernel(lambda: ctx.bsc_assemble(x, xhat, sc.dt, grav, bsc.BSC_FP64, out=out64), args.kernel_reps, torch)
    y = torch.empty(3, n, dtype=torch.float64, device="cuda")
    ms_spmv32 = time_kernel(lambda: ctx.bsc_spmv(out32[2], x, bsc.BSC_FP32_MIXED, out=y), args.kernel_reps, torch)
    ms_spmv64 = time_kernel(lambda: ctx.bsc_spmv(out64[2], x, bsc.BSC_FP64, out=y), args.kernel_reps, torch)

    # ---- measured bandwidth ceilings ----
    ceilings = {"hbm_copy_1gib_gb_s": copy_bandwidth(1 << 30, 10, torch),
                "cache_copy_32mb_gb_s": copy_bandwidth(32 << 20, 200, torch),
                "cache_copy_64mb_gb_s": copy_bandwidth(64 << 20, 200, torch),
                "note": "device copies (torch copy_), HIP events; GB/s counts bytes read plus bytes written"}

    # Algorithmic bytes. Assembly: reads x (24 B/CP), writes g and the 114-entry upper-stencil
    # Hessian. SpMV: reads the Hessian and x, writes y. Fused CG iteration (k_cg_fused, FP32
    # Hessian): reads the Hessian (456 B/CP), r, s, p, x (4 x 24 B, double), w (12 B, float: the
    # FP32 SpMV's output) and the block-Jacobi inverse (6 floats, 24 B); writes p, x, s, r
    # (4 x 24 B) and w (12 B): 696 B per CP per iteration.
    asm_bytes32 = n * (24 + 3 * 4 + 114 * 4)
    asm_bytes64 = n * (24 + 3 * 8 + 114 * 8)
    spmv_bytes32 = n * (114 * 4 + 24 + 24)
    spmv_bytes64 = n * (114 * 8 + 24 + 24)
    cg_bytes32 = n * (114 * 4 + 4 * 24 + 12 + 24 + 4 * 24 + 12)
    newton32 = sum(s["newton_iters"] for s in st32)
    pcg32 = sum(s["pcg_iters_total"] for s in st32)
    ms_step32 = 1e3 * sec32 / args.steps
    share_asm = newton32 * ms_asm32 / (1e3 * sec32)
    cg_ms = sum(s["ms_cg_kernels"] for s in st32)
    share_pcg = cg_ms / (1e3 * sec32)                 # the CG launches' GPU time
    cg_launches = sum(s["cg_launches"] for s in st32)
    cg_active = sum(s["cg_active_launches"] for s in st32)
    if share_pcg >= share_asm and cg_ms > 0:
        dom = {"kernel": "k_cg_fused<float> (one PCG iteration: vector updates, block-Jacobi, FP32 upper-stencil SpMV, dots)",
               "bound": "hbm", "achieved": cg_bytes32 * cg_active / (cg_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
               "unit": "GB/s", "avg_ms": cg_ms / cg_launches,
               "launches": cg_launches, "active_launches": cg_active,
               "bytes_per_active_launch": cg_bytes32}
    else:
        dom = {"kernel": "eval+assembly (bsc_assemble FP32-mixed)", "bound": "hbm",
               "achieved": asm_bytes32 / (ms_asm32 * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "avg_ms": ms_asm32}
    roof = {"bound": dom["bound"], "achieved": round(dom["achieved"], 2), "peak": dom["peak"], "unit": dom["unit"],
            "frac": round(dom["achieved"] / dom["peak"], 4), "traffic": None, "kernel": dom["kernel"],
            "avg_ms": round(dom["avg_ms"], 5),
            "share_of_step": {"assembly": round(share_asm, 3), "cg_launches": round(share_pcg, 3)},
            "frac_of_measured_hbm_copy": round(dom["achieved"] / ceilings["hbm_copy_1gib_gb_s"], 4),
            "frac_of_measured_cache_copy_64mb": round(dom["achieved"] / ceilings["cache_copy_64mb_gb_s"], 4)}
    for k in ("launches", "active_launches", "bytes_per_active_launch"):
        if k in dom:
            roof[k] = dom[k]
    if "active_launches" in dom:
        roof["traffic"] = cg_traffic_bytes()          # HBM bytes per active launch (calibrated counters)

    asm_gflop32 = ASM_FLOP_PER_ELEM * ne / (ms_asm32 * 1e-3) / 1e9
    asm_gflop64 = ASM_FLOP_PER_ELEM * ne / (ms_asm64 * 1e-3) / 1e9
    result = {
        "metric": "element E/g/H+assembly Melem/s, HBM GB/s; Newton-step ms at fixed residual vs FP64",
        "value": round(ne * args.steps / sec32 / 1e6, 4),
        "unit": "Melem/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step32, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"driven sheet {args.n}x{args.n} CPs ({ne} elements), E=1e4 Pa, t=1 mm, dt=0.01 s, "
                               f"|g|<={args.rtol:g}|g0| every step, FP32-mixed; plain FP64 (and the other start) "
                               f"from the identical state beside it",
                   "n_cp": n, "n_elem": ne, "seed": args.seed, "noise": args.noise,
                   "pcg": ("multigrid V(1,1)" if args.precond == "mg" else "block-Jacobi") + " PCG, "
                          + ("Eisenstat-Walker tolerance in [%g, 0.1]" % args.pcg_rtol
                             if args.adaptive else "fixed tolerance %g" % args.pcg_rtol),
                   "newton_start": "inertial predictor x^n + dt v^n" if args.start == "predictor" else "x^n",
                   "pcg_warm_start": {"previous": "previous Newton direction (energy-optimal multiple, kept when it "
                                                  "lowers the initial residual)",
                                      "none": "zero start", "net": "learned network prediction"}[args.warm],
                   "parallelism": "single GPU"},
        "newton_step_ms": {name: round(1e3 * secs[name] / args.steps, 3) for name in head},
        "speedup_vs_fp64": round(sec64 / sec32, 3) if r64 else None,
        "speedup_vs_fp64_same_start": round(secs["fp64_warm"] / sec32, 3) if "fp64_warm" in secs else None,
        "speedup_vs_fp32_zero_start": (round(secs["fp32_mixed_zero_start"] / sec32, 3)
                                       if "fp32_mixed_zero_start" in secs else None),
        "per_step": {"newton_fp32": [s["newton_iters"] for s in st32],
                     "newton_fp64": [r[1]["newton_iters"] for r in r64],
                     "pcg_fp32": [s["pcg_iters_total"] for s in st32],
                     "pcg_fp64": [r[1]["pcg_iters_total"] for r in r64],
                     "halvings_fp32": [s["ls_halvings"] for s in st32],
                     "g_rel_fp32": [float("%.3g" % g_rel(s)) for s in st32],
                     "g_rel_fp64": [float("%.3g" % g_rel(r[1])) for r in r64],
                     "dx_rel_fp64_vs_fp32": [float("%.3g" % r[2]) for r in r64],
                     "not_converged": {"fp32_mixed": sum(1 for s in st32 if s["status"] != 0),
                                       "fp64": sum(1 for r in r64 if r[1]["status"] != 0)}},
        "phases_ms_per_step_fp32": dict({k: round(sum(r[1][k] for r in phases["fp32_mixed"]) / n_phase, 3)
                                         for k in ("ms_assemble", "ms_pcg", "ms_linesearch", "ms_warmstart", "ms_total")},
                                        steps=n_phase, note="separate steps from the headline's start state with "
                                                            "every phase timed (events add to ms_total)"),
        "phases_ms_per_step_fp32_zero_start": ({k: round(sum(r[1][k] for r in phases["fp32_mixed_zero_start"]) / n_phase, 3)
                                               for k in ("ms_assemble", "ms_pcg", "ms_linesearch", "ms_total")}
                                               if "fp32_mixed_zero_start" in phases else None),
        "iterations_per_step": {name: {"newton": round(sum(r[1]["newton_iters"] for r in head[name]) / args.steps, 2),
                                       "pcg": round(sum(r[1]["pcg_iters_total"] for r in head[name]) / args.steps, 2),
                                       "warm_used": round(sum(r[1]["warm_start_used"] for r in head[name]) / args.steps, 2),
                                       "cg_launches": round(sum(r[1]["cg_launches"] for r in head[name]) / args.steps, 2),
                                       "g_rel_max": float("%.3g" % max(g_rel(r[1]) for r in head[name])),
                                       "not_converged": sum(1 for r in head[name] if r[1]["status"] != 0)}
                                for name in head},
        "pcg_us_per_iter_fp32": round(1e3 * sum(r[1]["ms_pcg"] for r in phases["fp32_mixed"])
                                      / max(1, sum(r[1]["pcg_iters_total"] for r in phases["fp32_mixed"])), 3),
        "cg_kernel": {"active_us": round(1e3 * cg_ms / max(1, cg_active), 3), "launches": cg_launches,
                      "active_launches": cg_active, "gb_s": round(cg_bytes32 * cg_active / max(cg_ms, 1e-9) / 1e6, 1)},
        "step_rule": step_rule,
        "fp32_vs_fp64_100": c2,
        "material_sweep": sweep,
        "warm_start": warm,
        "assembly": {"fp32_ms": round(ms_asm32, 4), "fp64_ms": round(ms_asm64, 4),
                     "fp32_melem_s": round(ne / ms_asm32 / 1e3, 2), "fp64_melem_s": round(ne / ms_asm64 / 1e3, 2),
                     "fp32_gb_s": round(asm_bytes32 / ms_asm32 / 1e6, 1), "fp64_gb_s": round(asm_bytes64 / ms_asm64 / 1e6, 1),
                     "fp32_hbm_frac": round(asm_bytes32 / ms_asm32 / 1e6 / HBM_PEAK_GBS, 4),
                     "fp64_hbm_frac": round(asm_bytes64 / ms_asm64 / 1e6 / HBM_PEAK_GBS, 4),
                     "fp32_gflop_s": round(asm_gflop32, 1), "fp64_gflop_s": round(asm_gflop64, 1),
                     "fp32_frac_of_fp32_peak": round(asm_gflop32 / 1e3 / FP32_PEAK_TFLOPS, 4),
                     "fp64_frac_of_fp64_peak": round(asm_gflop64 / 1e3 / FP64_PEAK_TFLOPS, 4),
                     "bytes_fp32": asm_bytes32, "bytes_fp64": asm_bytes64, "flop_per_elem": ASM_FLOP_PER_ELEM},
        "spmv": {"fp32_ms": round(ms_spmv32, 5), "fp64_ms": round(ms_spmv64, 5),
                 "fp32_gb_s": round(spmv_bytes32 / ms_spmv32 / 1e6, 1), "fp64_gb_s": round(spmv_bytes64 / ms_spmv64 / 1e6, 1)},
        "ceilings": ceilings,
        "quadrature_ablation": quad_leg,
        "general_rest": general_leg,
        "contact_conversion": contact_leg,
        "partial_factorization": pf_leg,
        "wrinkling_convergence": wrinkle_leg,
        "roofline": roof,
        "cpu_baseline": None,
    }
    if not args.no_cpu:
        try:
            result["cpu_baseline"] = cpu_baseline(args.n, args.seed, args.cpu_reps)
        except Exception as e:  # the baseline is context; never fail the bench on it
            result["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
