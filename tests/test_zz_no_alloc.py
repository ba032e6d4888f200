"""The no-allocation net backward (bsc_net_backward_noalloc, static per-GPU scratch) against the
existing entry point (bsc_net_backward, caller-owned scratch) through the C ABI.

Both run the same deterministic kernels (the weight gradient is reduced over tiles in a fixed
order), so the outputs must agree bit for bit. Two calls in a row, the second with a smaller
input, show that what the first call leaves in the shared array does not leak into the second;
a third request larger than the static array is refused on the host."""
import numpy as np
import pytest

import synthetic as syn

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_2506_18867_amd import bsc  # noqa: E402


def _ctx(n_u, n_v):
    ku, kv, rest = syn.flat_sheet(n_u, n_v)
    return bsc.Context(n_u, n_v, ku, kv, rest, bsc.make_material(0, 1e4, 0.3, 1e-3, mu_bend=1e-6, rho_area=0.2))


def _case(ctx, batch, seed):
    n = ctx.n_cp
    g = torch.Generator(device="cuda").manual_seed(seed)
    w = (0.15 * torch.randn(bsc.BSC_NET_PARAMS, device="cuda", generator=g)).float()
    x = torch.randn(batch, 3, n, device="cuda", generator=g)
    dout = torch.randn(batch, 3, n, device="cuda", generator=g)
    acts = torch.empty(5 * batch * 32 * n, dtype=torch.float32, device="cuda")
    ctx.bsc_net_forward(w, x, acts)
    return w, x, acts, dout


def _compare(ctx, batch, seed):
    w, x, acts, dout = _case(ctx, batch, seed)
    dw_ref, din_ref = ctx.bsc_net_backward(w, x, acts, dout, want_din=True)
    dw = torch.full_like(w, float("nan"))
    din = torch.full_like(x, float("nan"))
    ctx.bsc_net_backward_noalloc(w, x, acts, dout, dw, din)
    torch.cuda.synchronize()
    print(f"[no-alloc] {ctx.n_u}x{ctx.n_v} batch {batch}: scratch {ctx.bsc_net_scratch_size(batch)} B, "
          f"max |dw - dw_ref| {float((dw - dw_ref).abs().max()):.3e}", flush=True)
    assert torch.isfinite(dw_ref).all() and torch.isfinite(din_ref).all()
    assert torch.equal(dw, dw_ref)
    assert torch.equal(din, din_ref)


def test_noalloc_backward_matches_the_workspace_entry_point():
    big = _ctx(61, 47)
    _compare(big, 3, 11)                  # first call: the larger input
    _compare(big, 1, 12)                  # second call, same context: a smaller batch
    _compare(_ctx(37, 16), 2, 13)         # another context, a smaller grid (ragged tiles)


def test_noalloc_backward_refuses_requests_beyond_its_static_scratch():
    ctx = _ctx(226, 226)
    assert ctx.bsc_net_scratch_size(1) <= bsc.BSC_NET_NOALLOC_SCRATCH_BYTES
    assert ctx.bsc_net_scratch_size(2) > bsc.BSC_NET_NOALLOC_SCRATCH_BYTES
    n = ctx.n_cp
    w = torch.zeros(bsc.BSC_NET_PARAMS, device="cuda")
    x = torch.zeros(2, 3, n, device="cuda")
    acts = torch.zeros(5 * 2 * 32 * n, device="cuda")
    dw = torch.zeros_like(w)
    with pytest.raises(bsc.BscError) as e:
        ctx.bsc_net_backward_noalloc(w, x, acts, x, dw)
    assert e.value.status == bsc.BSC_E_INVAL and "scratch" in str(e.value)
    # the refused call enqueued nothing: a valid call afterwards still matches
    _compare(_ctx(20, 23), 2, 14)
