"""Trains the learned PCG warm start (a method extension) on the method's own solves.

Data: 128 x 128-control-point sheets with materials drawn from the (E, t) grid; half are driven
sheets with random held CPs and a driven corner, half are compressed-and-draped sheets (10 %
compression between two held columns). Every Newton iteration of their
implicit-Euler steps logs the free gradient g and the PCG direction p solved to a relative
residual of 1e-8 (bsc_set_sample_log). Training: the library's forward, backward, loss and Adam
kernels (bsc_net_*), batch 16, Adam 1e-3 with cosine decay, 10 % of the pairs held out.
Indexing a batch out of the sample tensors is the only PyTorch operation (a device gather).

Usage: python -m paper_2506_18867_amd.train_warmstart --samples 20000 --epochs 12 \
           --out paper_2506_18867_amd/weights/warmstart_c32.f32
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def init_weights(seed: int) -> np.ndarray:
    """He-style initialisation for LeakyReLU(0.1) convolutions, layer by layer."""
    from paper_2506_18867_amd.bsc import BSC_NET_PARAMS
    g = np.random.Generator(np.random.PCG64(seed))
    cin = [3, 32, 32, 32, 32, 32]
    cout = [32, 32, 32, 32, 32, 3]
    parts = []
    for ci, co in zip(cin, cout):
        std = math.sqrt(2.0 / ((1 + 0.1 ** 2) * ci * 9))
        parts.append(g.standard_normal(co * ci * 9) * std)
    w = np.concatenate(parts).astype(np.float32)
    assert w.size == BSC_NET_PARAMS
    return w


def make_scene(seed: int, n: int):
    import synthetic as syn
    g = syn.rng(seed)
    cell = int(g.integers(0, len(syn.MATERIAL_GRID)))
    E, t = syn.MATERIAL_GRID[cell]
    if seed % 2 == 0:
        sc = syn.driven_sheet(n, seed=seed, cell=cell)
    else:
        sc = syn.compressed_sheet(n, seed=seed, material=syn.stvk_material(young=E, thickness=t))
    return sc


def generate(n: int, n_samples: int, seed0: int, steps_per_sheet: int, time_budget: float, log=print):
    """Runs implicit-Euler steps on fresh sheets until n_samples (g, p) pairs are logged."""
    import torch
    from paper_2506_18867_amd import bsc
    n3 = 3 * n * n
    G = torch.zeros(n_samples, n3, dtype=torch.float32, device="cuda")
    P = torch.zeros(n_samples, n3, dtype=torch.float32, device="cuda")
    count, sheets = 0, 0
    t0 = time.perf_counter()
    seed = seed0
    while count < n_samples and time.perf_counter() - t0 < time_budget:
        sc = make_scene(seed, n)
        ctx = bsc.context_for_scene(sc)
        ctx.bsc_set_sample_log(G[count:], P[count:], n_samples - count)
        x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
        opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), precision=bsc.BSC_FP32_MIXED,
                             stop_mode=bsc.BSC_STOP_STEP, atol=1e-2, max_newton=25, pcg_rtol=1e-8, max_pcg=6000)
        for step in range(steps_per_sheet):
            st, _ = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(step)), opts, raise_on_error=False)
            if st not in (0, -5) or ctx.bsc_sample_log_count() >= n_samples - count:
                break
        count += ctx.bsc_sample_log_count()
        sheets += 1
        seed += 1
        if sheets % 5 == 0:
            log(f"[data] sheets={sheets} samples={count} elapsed={time.perf_counter() - t0:.1f}s")
    torch.cuda.synchronize()
    return G[:count], P[:count], {"sheets": sheets, "samples": count, "seconds": time.perf_counter() - t0}


def train(G, P, n: int, epochs: int, batch: int, lr: float, seed: int, val_frac: float = 0.1, log=print,
          time_budget: float = 1e9):
    import torch
    import synthetic as syn
    from paper_2506_18867_amd import bsc
    ku, kv, rest = syn.flat_sheet(n)
    ctx = bsc.Context(n, n, ku, kv, rest, bsc.make_material(0, 1e4, 0.3, 1e-3, mu_bend=1e-6, rho_area=0.2))
    N = G.shape[0]
    g = np.random.Generator(np.random.PCG64(seed))
    perm = g.permutation(N)
    n_val = max(1, int(val_frac * N))
    val_idx = torch.from_numpy(perm[:n_val]).cuda()
    tr_idx = perm[n_val:]
    w = torch.from_numpy(init_weights(seed)).cuda()
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    ncp = n * n
    acts = torch.empty(5 * batch * 32 * ncp, dtype=torch.float32, device="cuda")
    scratch = torch.empty(ctx.bsc_net_scratch_size(batch), dtype=torch.uint8, device="cuda")
    steps_per_epoch = len(tr_idx) // batch
    total = epochs * steps_per_epoch
    history = []
    t = 0
    t0 = time.perf_counter()

    def val_loss():
        losses = []
        for s in range(0, n_val - batch + 1, batch):
            idx = val_idx[s:s + batch]
            xb = G[idx].view(batch, 3, ncp)
            yb = P[idx].view(batch, 3, ncp)
            out = ctx.bsc_net_forward(w, xb, acts)
            loss, _ = ctx.bsc_net_loss(xb, out, yb)
            losses.append(loss.item())
        return float(np.mean(losses)) if losses else float("nan")

    v0 = val_loss()
    log(f"[train] samples={N} train={len(tr_idx)} val={n_val} batch={batch} epochs={epochs} val_loss0={v0:.4f}")
    for ep in range(epochs):
        order = g.permutation(tr_idx)
        ep_losses = []
        for s in range(steps_per_epoch):
            idx = torch.from_numpy(order[s * batch:(s + 1) * batch]).cuda()
            xb = G[idx].view(batch, 3, ncp)
            yb = P[idx].view(batch, 3, ncp)
            out = ctx.bsc_net_forward(w, xb, acts)
            loss, dout = ctx.bsc_net_loss(xb, out, yb)
            dw, _ = ctx.bsc_net_backward(w, xb, acts, dout, scratch=scratch)
            t += 1
            lr_t = lr * 0.5 * (1.0 + math.cos(math.pi * t / total))
            ctx.bsc_adam_step(w, dw, m, v, lr_t, t)
            if s % 50 == 0:
                ep_losses.append(loss.item())
        vl = val_loss()
        history.append({"epoch": ep + 1, "train_loss": float(np.mean(ep_losses)), "val_loss": vl,
                        "seconds": time.perf_counter() - t0})
        log(f"[train] epoch {ep + 1}/{epochs} train_loss={history[-1]['train_loss']:.4f} val_loss={vl:.4f} "
            f"t={time.perf_counter() - t0:.1f}s")
        if time.perf_counter() - t0 > time_budget:
            log("[train] time budget reached")
            break
    torch.cuda.synchronize()
    return w.cpu().numpy(), {"val_loss_init": v0, "history": history, "train_seconds": time.perf_counter() - t0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--samples", type=int, default=20000)
    ap.add_argument("--steps-per-sheet", type=int, default=40)
    ap.add_argument("--data-seconds", type=float, default=420.0)
    ap.add_argument("--train-seconds", type=float, default=300.0)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=4000)
    ap.add_argument("--out", default=os.path.join(ROOT, "paper_2506_18867_amd", "weights", "warmstart_c32.f32"))
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    G, P, dstats = generate(args.n, args.samples, args.seed, args.steps_per_sheet, args.data_seconds,
                            log=lambda s: print(s, flush=True))
    print(f"[data] done: {dstats}", flush=True)
    w, tstats = train(G, P, args.n, args.epochs, args.batch, args.lr, args.seed, log=lambda s: print(s, flush=True),
                      time_budget=args.train_seconds)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    w.astype(np.float32).tofile(args.out)
    meta = {"data": dstats, "train": tstats, "n": args.n, "batch": args.batch, "lr": args.lr, "seed": args.seed}
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps({"weights": args.out, "val_loss_init": tstats["val_loss_init"],
                      "val_loss_final": tstats["history"][-1]["val_loss"] if tstats["history"] else None,
                      "samples": dstats["samples"]}), flush=True)


if __name__ == "__main__":
    main()
