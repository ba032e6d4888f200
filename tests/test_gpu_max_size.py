"""The largest control grid the library accepts: 4096 x 4096 CPs (2^24, about 55 GB of
workspace), through the C ABI.

At that size the 114 Hessian entries per CP fill 1.9 G values, so an offset formed in 32-bit
arithmetic beyond the stated limit would corrupt the rows at the end of the grid. The sheet
carries an affine deformation (F constant), so an interior row of the assembled Hessian depends
only on its neighbourhood, which repeats under shifts (di, dj) with di + dj even (the interior
membrane cells alternate between 1 x 2 and 2 x 1 points in a checkerboard). Each sampled
interior row, including rows in the last CP rows of the grid, must equal the row of the same
checkerboard class at the centre of a 24 x 24 sheet with the same span length, material and
deformation: FP64 within 1e-10 of the row's largest entry (the displacement gradient is a sum
of terms up to |X| / h = 4e3 times larger than itself, so its rounding grows with the distance
from the origin), FP32-mixed within 1e-5. One Newton iteration at full size must lower the
energy."""
import numpy as np
import pytest

import synthetic as syn

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2506_18867_amd import bsc  # noqa: E402

N_MAX = 4096
H_SPAN = 0.01
MAT = bsc.make_material(0, 1e4, 0.3, 1e-3, mu_bend=syn.plate_bending_stiffness(1e4, 0.3, 1e-3), rho_area=0.2)


def _sheet(n):
    ku, kv, rest = syn.flat_sheet(n, L_u=(n - 2) * H_SPAN)
    x = syn.embed(rest)
    x[:, 0] *= 1.05
    x[:, 1] *= 1.02
    return ku, kv, rest, x


def _rows(H, idx):
    return H[:, torch.as_tensor(idx, device=H.device)].double().cpu().numpy().T


@pytest.fixture(scope="module")
def big():
    print(f"[max size] creating the {N_MAX} x {N_MAX} context", flush=True)
    ku, kv, rest, x = _sheet(N_MAX)
    assert N_MAX * N_MAX == 1 << 24
    ctx = bsc.Context(N_MAX, N_MAX, ku, kv, rest, MAT)
    yield ctx, rest, x
    del ctx


def test_max_size_interior_rows_match_a_small_sheet(big):
    ku, kv, rest, x = _sheet(24)
    small = bsc.Context(24, 24, ku, kv, rest, MAT)
    xs = bsc.to_soa(x)
    ref = {}
    for prec in (bsc.BSC_FP64, bsc.BSC_FP32_MIXED):
        _, _, H = small.bsc_assemble(xs, precision=prec)
        ref[prec] = _rows(H, [12 * 24 + 12, 12 * 24 + 13])          # CP (12, 12) and (13, 12)
    del small, xs

    ctx, _, x = big
    xb = bsc.to_soa(x)
    g = np.random.default_rng(11)
    lo, hi = 5, N_MAX - 6                       # rows whose neighbourhood holds inner spans only
    pts = [(lo, lo), (hi, hi), (lo, hi), (hi, lo), (N_MAX // 2, N_MAX // 2), (hi - 1, hi)]
    pts += [tuple(p) for p in g.integers(lo, hi + 1, size=(64, 2))]
    idx = [j * N_MAX + i for i, j in pts]
    cls = np.array([(i + j) % 2 for i, j in pts])
    for prec, tol in ((bsc.BSC_FP64, 1e-10), (bsc.BSC_FP32_MIXED, 1e-5)):
        print(f"[max size] assembling, precision {prec}", flush=True)
        _, _, H = ctx.bsc_assemble(xb, precision=prec)
        rows = _rows(H, idx)
        del H
        scale = np.abs(ref[prec]).max()
        err = np.abs(rows - ref[prec][cls]).max() / scale
        print(f"[max size] precision {prec}: largest row difference {err:.2e} of the row scale", flush=True)
        assert err < tol


def test_max_size_newton_iteration_lowers_the_energy(big):
    ctx, rest, _ = big
    pins = np.array([0, N_MAX - 1], dtype=np.int64)
    ctx.bsc_set_pins(pins)
    x0 = syn.embed(rest)
    x0[:, 2] += 1e-3 * np.sin(np.pi * rest[:, 0] / rest[:, 0].max())
    xb, vb = bsc.to_soa(x0), bsc.to_soa(np.zeros_like(x0))
    xn = xb.clone()
    tgt = bsc.to_soa(x0[pins])
    del x0
    grav = (0.0, 0.0, -9.81)
    E0, _, _ = ctx.bsc_assemble(xb, xn, 0.01, grav, want_hess=False)
    e0 = float(E0.item())
    opts = bsc.make_opts(dt=0.01, gravity=grav, precision=bsc.BSC_FP32_MIXED, fixed_newton_iters=1,
                         pcg_rtol=1e-2, max_pcg=200)
    print("[max size] one Newton iteration", flush=True)
    st, stats = ctx.bsc_newton_step(xb, vb, tgt, opts)
    assert st == 0
    E1, _, _ = ctx.bsc_assemble(xb, xn, 0.01, grav, want_hess=False)
    e1 = float(E1.item())
    print(f"[max size] pcg {stats.pcg_iters_total}, energy {e0:.9e} -> {e1:.9e}", flush=True)
    assert np.isfinite(e1) and e1 < e0


@pytest.mark.parametrize("prec,pcg_rtol,bar", [(bsc.BSC_FP64, 1e-10, 1e-8), (bsc.BSC_FP32_MIXED, 1e-6, 1e-4)])
def test_large_grid_direction_solves_the_newton_system(prec, pcg_rtol, bar):
    """1024 x 1024 CPs: 8192 CG workgroups, so each launch reads the sums of the previous
    launch's partials formed once by a one-block kernel. The first Newton direction must solve
    H p = -g at the start iterate to the PCG tolerance (checked with the library's own assembly
    and SpMV in the step's precision)."""
    n = 1024
    print(f"[large grid] {n} x {n}, precision {prec}", flush=True)
    sc = syn.driven_sheet(n, seed=304)
    ctx = bsc.context_for_scene(sc)
    xs = sc.x0.copy()
    xs[sc.pins] = sc.pin_targets(0)
    x, v = bsc.to_soa(sc.x0), bsc.to_soa(sc.v0)
    opts = bsc.make_opts(dt=sc.dt, gravity=tuple(sc.gravity), precision=prec, fixed_newton_iters=1,
                         pcg_rtol=pcg_rtol, max_pcg=20000)
    st, stats = ctx.bsc_newton_step(x, v, bsc.to_soa(sc.pin_targets(0)), opts)
    assert st == 0
    if stats.ls_halvings:
        pytest.skip("the full step was not taken; the direction is not x1 - x0")
    xsd = bsc.to_soa(xs)
    p = x - xsd
    _, g, H = ctx.bsc_assemble(xsd, bsc.to_soa(sc.x0), sc.dt, tuple(sc.gravity), precision=prec)
    hp = ctx.bsc_spmv(H, p.contiguous(), precision=prec)                  # vectors are double in both precisions
    res = float(torch.linalg.norm(hp.double() + g.double()) / torch.linalg.norm(g.double()))
    print(f"[large grid] pcg {stats.pcg_iters_total}, |H p + g| / |g| = {res:.2e}", flush=True)
    assert res < bar
