"""CPU-side checks of the C ABI: the library loads, exports every symbol include/bsc.h declares,
and its host-only calls (create, validation, sizes, workspace, BSR pattern) behave as documented.
No kernel is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

import synthetic as syn
from paper_2506_18867_amd import bsc

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "bsc.h")


def declared_symbols():
    text = open(HEADER).read()
    decl = r"^(?:bsc_status|const char \*|void)\s*\*?\s*(bsc_[a-z0-9_]+)\s*\("
    return sorted(set(re.findall(decl, text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    lib = bsc.load()
    names = declared_symbols()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    assert set(bsc.exported_symbols()) == set(names)


def _create(n_u, n_v, ku, kv, rest, mat=None):
    lib = bsc.load()
    mat = mat or bsc.make_material(0, 1e4, 0.3, 1e-3, mu_bend=1e-6, rho_area=0.2)
    h = ctypes.c_void_p()
    ku = np.ascontiguousarray(ku, dtype=np.float64)
    kv = np.ascontiguousarray(kv, dtype=np.float64)
    rest = np.ascontiguousarray(rest, dtype=np.float64).reshape(-1)
    st = lib.bsc_create(ctypes.byref(h), n_u, n_v, bsc._np_ptr(ku), bsc._np_ptr(kv), bsc._np_ptr(rest),
                        ctypes.byref(mat), None)
    return st, h


def test_create_sizes_match_quadrature_counts():
    lib = bsc.load()
    for n_u, n_v in [(5, 5), (7, 7), (20, 20), (9, 6)]:
        ku, kv, rest = syn.flat_sheet(n_u, n_v)
        st, h = _create(n_u, n_v, ku, kv, rest)
        assert st == 0
        s = [ctypes.c_int32() for _ in range(4)]
        assert lib.bsc_sizes(h, *[ctypes.byref(v) for v in s]) == 0
        n_cp, n_elem, n_mp, n_be = [v.value for v in s]
        Nu, Nv = n_u - 2, n_v - 2
        assert n_cp == n_u * n_v and n_elem == Nu * Nv
        if Nu == Nv:
            N = Nu
            assert n_mp == 36 + 24 * (N - 2) + 2 * (N - 3) ** 2 + 8 * (N - 3) + 4
        assert n_be == 4 * (Nu - 1) * (Nv - 1) + (Nu * Nv - (Nu - 2) * (Nv - 2))
        sz = ctypes.c_size_t()
        assert lib.bsc_workspace_size(h, ctypes.byref(sz)) == 0
        assert sz.value > 114 * 8 * n_cp
        lib.bsc_destroy(h)


def test_create_rejects_bad_inputs():
    lib = bsc.load()
    ku, kv, rest = syn.flat_sheet(8)
    bad = ku.copy()
    bad[5] += 0.5
    assert _create(8, 8, bad, kv, rest)[0] == -2                      # BSC_E_KNOTS
    nonopen = np.arange(11, dtype=float)
    assert _create(8, 8, nonopen, kv, rest)[0] == -2
    ku4, kv4, rest4 = syn.flat_sheet(4)
    assert _create(4, 4, ku4, kv4, rest4)[0] == -1                    # too few spans
    folded = rest.copy()
    folded[3 * 8 + 3, 0] += 0.4                                      # crosses two neighbours
    assert _create(8, 8, ku, kv, folded)[0] == -1                     # det J < 0 inside
    flipped = rest.copy()
    flipped[:, 0] *= -1
    assert _create(8, 8, ku, kv, flipped)[0] == -1                    # det < 0
    assert _create(8, 8, ku, kv, rest, bsc.make_material(0, 1e4, 0.6, 1e-3, rho_area=0.2))[0] == -1
    assert _create(8, 8, ku, kv, rest, bsc.make_material(0, 1e4, 0.3, 1e-3, rho_area=0.0))[0] == -1
    assert _create(8, 8, ku, kv, rest, bsc.make_material(7, 1e4, 0.3, 1e-3, rho_area=0.2))[0] == -1
    nan_rest = rest.copy()
    nan_rest[3, 1] = np.nan
    assert _create(8, 8, ku, kv, nan_rest)[0] == -1
    # plane stress is finite at nu = 0.5 (accepted), not beyond
    st, h = _create(8, 8, ku, kv, rest, bsc.make_material(0, 1e6, 0.5, 1e-3, rho_area=0.2))
    assert st == 0
    lib.bsc_destroy(h)
    assert _create(8, 8, ku, kv, rest, bsc.make_material(0, 1e6, 0.5000001, 1e-3, rho_area=0.2))[0] == -1
    # more than 2^24 CPs: offsets into the device tables would leave int32
    n_u, n_v = 4097, 4096
    big = np.zeros((n_u * n_v, 2))
    assert _create(n_u, n_v, syn.open_uniform_knots(n_u), syn.open_uniform_knots(n_v), big)[0] == -1


@pytest.mark.parametrize("kind", syn.MAPPED_KINDS)
def test_create_accepts_general_rest_shapes(kind):
    ku, kv, rest = syn.mapped_sheet(9, 7, kind)
    st, h = _create(9, 7, ku, kv, rest)
    assert st == 0
    bsc.load().bsc_destroy(h)
    nudged = syn.flat_sheet(8)[2].copy()
    nudged[10] += 0.01                                                # a slightly curved rest
    st, h = _create(8, 8, *syn.flat_sheet(8)[:2], nudged)
    assert st == 0
    bsc.load().bsc_destroy(h)


def test_create_accepts_spacing_sheared_and_nonsquare():
    ku, kv, rest = syn.flat_sheet(9, 6, 2.0, 0.7, spacing=3, shear=0.4)
    st, h = _create(9, 6, ku, kv, rest)
    assert st == 0
    bsc.load().bsc_destroy(h)


def test_calls_without_workspace_fail_cleanly():
    lib = bsc.load()
    ku, kv, rest = syn.flat_sheet(6)
    st, h = _create(6, 6, ku, kv, rest)
    assert st == 0
    assert lib.bsc_set_pins(h, None, 0) == -9                          # BSC_E_STATE
    assert lib.bsc_eval_egh(h, 0, None, None, None, None, None) == -9
    assert lib.bsc_assemble(h, 0, None, None, 0.01, None, None, None, None) == -9
    assert lib.bsc_spmv(h, 0, None, None, None) == -9
    opts = bsc.make_opts()
    assert lib.bsc_newton_step(h, ctypes.byref(opts), None, None, None, None) == -9
    assert lib.bsc_net_backward_noalloc(h, 1, None, None, None, None, None, None) == -9
    assert b"workspace" in lib.bsc_last_error(h)
    lib.bsc_destroy(h)
    assert lib.bsc_status_string(-6) == b"line search failed"


def test_bsr_pattern_is_the_5x5_neighbourhood():
    lib = bsc.load()
    n_u, n_v = 7, 6
    ku, kv, rest = syn.flat_sheet(n_u, n_v)
    st, h = _create(n_u, n_v, ku, kv, rest)
    nnzb = ctypes.c_int32()
    assert lib.bsc_bsr_pattern(h, None, None, ctypes.byref(nnzb)) == 0
    rp = np.zeros(n_u * n_v + 1, dtype=np.int32)
    ci = np.zeros(nnzb.value, dtype=np.int32)
    assert lib.bsc_bsr_pattern(h, bsc._np_ptr(rp), bsc._np_ptr(ci), ctypes.byref(nnzb)) == 0
    want = []
    for a in range(n_u * n_v):
        i, j = a % n_u, a // n_u
        row = sorted(jb * n_u + ib for jb in range(n_v) for ib in range(n_u) if abs(ib - i) <= 2 and abs(jb - j) <= 2)
        assert list(ci[rp[a]:rp[a + 1]]) == row
        want += row
    assert nnzb.value == len(want) == (5 * n_u - 6) * (5 * n_v - 6)
    lib.bsc_destroy(h)


def test_binding_refuses_mistyped_or_short_buffers():
    """Before a device pointer crosses the C ABI the binding checks the tensor: type, dtype,
    contiguity, element count and device. Each failure is BSC_E_INVAL, raised on the host, so a
    wrong buffer never reaches a kernel."""
    import torch
    cases = [(np.zeros(6), "torch tensor"),
             (torch.zeros(6, dtype=torch.float32), "must be torch.float64"),
             (torch.zeros(3, 4, dtype=torch.float64).t(), "contiguous"),
             (torch.zeros(5, dtype=torch.float64), "needs 6"),
             (torch.zeros(6, dtype=torch.float64), "device")]
    for t, msg in cases:
        with pytest.raises(bsc.BscError) as e:
            bsc._need(t, torch.float64, 6, "x")
        assert e.value.status == bsc.BSC_E_INVAL and msg in str(e.value)
    bsc._need(None, torch.float64, 6, "x", optional=True)
    with pytest.raises(bsc.BscError) as e:
        bsc._need(None, torch.float64, 6, "x")
    assert e.value.status == bsc.BSC_E_INVAL


def test_binding_structs_match_the_c_layout(tmp_path):
    """Every struct the binding passes by pointer has the C header's size and field offsets:
    a small C program built against include/bsc.h prints them (gcc, host only)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no host C compiler")
    structs = {"bsc_material": bsc.Material, "bsc_step_opts": bsc.StepOpts, "bsc_step_stats": bsc.StepStats,
               "bsc_pf_opts": bsc.PfOpts, "bsc_pf_stats": bsc.PfStats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "bsc.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([gcc, "-std=c11", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(line.split()[:2]): int(line.split()[2]) for line in out if line.strip()}
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)
