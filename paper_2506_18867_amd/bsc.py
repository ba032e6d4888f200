"""Thin ctypes binding of ``include/bsc.h`` (libbsc.so, HIP for gfx950).

Argument marshalling only: every step of the computation runs in the library's kernels.
PyTorch provides device memory (CUDA/HIP tensors passed by ``data_ptr()``) and the stream.
Importing works without a GPU; any call that needs the library raises ``BscError`` when
``libbsc.so`` is missing instead of falling back to anything else.

Tensors: CP vectors are float64 ``(3, n_cp)`` (structure of arrays; CP (i, j) at column
``j * n_u + i``); the Hessian is ``(114, n_cp)`` in the upper-stencil layout of
``bsc_assemble`` (float64 for ``BSC_FP64``, float32 for ``BSC_FP32_MIXED``).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbsc.so")

BSC_OK = 0
BSC_E_INVAL = -1
BSC_E_NOMEM = -3
BSC_FP64 = 0
BSC_FP32_MIXED = 1
BSC_MEMBRANE_STVK = 0
BSC_MEMBRANE_FBW = 1
BSC_STOP_GRAD = 0
BSC_STOP_STEP = 1
BSC_PRECOND_JACOBI = 0
BSC_PRECOND_MULTIGRID = 1
BSC_START_PREVIOUS = 0
BSC_START_PREDICTOR = 1
BSC_WARM_NONE = 0
BSC_WARM_NET = 1
BSC_WARM_PREVIOUS = 2
BSC_TIMING_CG = 0
BSC_TIMING_PHASES = 1
BSC_TIMING_OFF = 2
BSC_HESS_ENTRIES = 114
BSC_NET_PARAMS = 38592
BSC_NET_NOALLOC_SCRATCH_BYTES = 32 << 20   # static scratch of bsc_net_backward_noalloc, per GPU
STATUS = {0: "BSC_OK", -1: "BSC_E_INVAL", -2: "BSC_E_KNOTS", -3: "BSC_E_NOMEM", -4: "BSC_E_HIP",
          -5: "BSC_E_NOT_CONVERGED", -6: "BSC_E_LINESEARCH", -7: "BSC_E_NONFINITE",
          -8: "BSC_E_PCG_BREAKDOWN", -9: "BSC_E_STATE"}
# upper-stencil slot offsets (di, dj); slot 0 is the diagonal
SLOT_OFFSETS = [(0, 0), (1, 0), (2, 0), (-2, 1), (-1, 1), (0, 1), (1, 1), (2, 1), (-2, 2), (-1, 2), (0, 2), (1, 2), (2, 2)]


class BscError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {msg}")


class Material(ctypes.Structure):
    _fields_ = [("membrane", ctypes.c_int32), ("young", ctypes.c_double), ("poisson", ctypes.c_double),
                ("thickness", ctypes.c_double), ("mu_st1", ctypes.c_double), ("mu_st2", ctypes.c_double),
                ("mu_sh", ctypes.c_double), ("mu_bend", ctypes.c_double), ("rho_area", ctypes.c_double),
                ("quadrature", ctypes.c_int32)]


class StepOpts(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("gravity", ctypes.c_double * 3), ("precision", ctypes.c_int32),
                ("stop_mode", ctypes.c_int32), ("rtol", ctypes.c_double), ("atol", ctypes.c_double),
                ("max_newton", ctypes.c_int32), ("max_pcg", ctypes.c_int32), ("pcg_rtol", ctypes.c_double),
                ("warm_start", ctypes.c_int32), ("fixed_newton_iters", ctypes.c_int32),
                ("pcg_adaptive", ctypes.c_int32), ("preconditioner", ctypes.c_int32), ("start", ctypes.c_int32),
                ("pcg_eta_max", ctypes.c_double), ("timing", ctypes.c_int32)]


class PfOpts(ctypes.Structure):
    _fields_ = [("rho_max", ctypes.c_double), ("series_tol", ctypes.c_double), ("max_terms", ctypes.c_int32),
                ("pcg_rtol", ctypes.c_double), ("max_pcg", ctypes.c_int32), ("force", ctypes.c_int32)]


class PfStats(ctypes.Structure):
    _fields_ = [("triggered", ctypes.c_int32), ("terms", ctypes.c_int32), ("pcg_iters", ctypes.c_int32),
                ("rho_bound", ctypes.c_double), ("b_bound", ctypes.c_double), ("d_bound", ctypes.c_double),
                ("ms_total", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class StepStats(ctypes.Structure):
    _fields_ = [("newton_iters", ctypes.c_int32), ("pcg_iters_total", ctypes.c_int32),
                ("ls_halvings", ctypes.c_int32), ("warm_start_used", ctypes.c_int32),
                ("warm_start_fallbacks", ctypes.c_int32), ("g0_norm", ctypes.c_double),
                ("g_norm", ctypes.c_double), ("energy", ctypes.c_double), ("ms_assemble", ctypes.c_double),
                ("ms_pcg", ctypes.c_double), ("ms_linesearch", ctypes.c_double),
                ("ms_warmstart", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("cg_launches", ctypes.c_int32), ("cg_active_launches", ctypes.c_int32),
                ("ms_cg_kernels", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load():
    """Loads libbsc.so (raises BscError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise BscError(-9, f"{LIB_PATH} is missing: build it with `python -m paper_2506_18867_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, D, F, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_float, ctypes.c_size_t
    sig = {
        "bsc_create": [ctypes.POINTER(P), I32, I32, P, P, P, ctypes.POINTER(Material), P],
        "bsc_sizes": [P, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32)],
        "bsc_workspace_size": [P, ctypes.POINTER(SZ)],
        "bsc_bind_workspace": [P, P, SZ],
        "bsc_set_pins": [P, P, I32],
        "bsc_eval_egh": [P, I32, P, P, P, P, P],
        "bsc_assemble": [P, I32, P, P, D, P, P, P, P],
        "bsc_spmv": [P, I32, P, P, P],
        "bsc_bsr_pattern": [P, P, P, ctypes.POINTER(I32)],
        "bsc_export_bsr": [P, I32, P, P],
        "bsc_newton_step": [P, ctypes.POINTER(StepOpts), P, P, P, ctypes.POINTER(StepStats)],
        "bsc_energy_difference": [P, P, P, D, P, P, I32, P, P],
        "bsc_warmstart_load": [P, P, I32],
        "bsc_net_forward": [P, I32, P, P, P, P],
        "bsc_net_backward": [P, I32, P, P, P, P, P, P, P],
        "bsc_net_scratch_size": [P, I32, ctypes.POINTER(SZ)],
        "bsc_net_backward_noalloc": [P, I32, P, P, P, P, P, P],
        "bsc_adam_step": [P, I32, P, P, P, P, F, F, F, F, I32],
        "bsc_net_loss": [P, I32, P, P, P, P, P],
        "bsc_set_sample_log": [P, P, P, I32],
        "bsc_sample_log_count": [P, ctypes.POINTER(I32)],
        "bsc_contact_setup": [P, I32, P, I32, I32],
        "bsc_contact_workspace_size": [P, ctypes.POINTER(SZ)],
        "bsc_contact_bind_workspace": [P, P, SZ],
        "bsc_contact_hessian": [P, I32, P, P, P, I32, P, P, P, ctypes.POINTER(I32), P],
        "bsc_contact_solve": [P, I32, P, D, P, P, P, I32, P, P, ctypes.POINTER(PfOpts), ctypes.POINTER(PfStats)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.bsc_status_string.argtypes = [ctypes.c_int]
    lib.bsc_status_string.restype = ctypes.c_char_p
    lib.bsc_last_error.argtypes = [P]
    lib.bsc_last_error.restype = ctypes.c_char_p
    lib.bsc_destroy.argtypes = [P]
    lib.bsc_destroy.restype = None
    _lib = lib
    return lib


def exported_symbols() -> list[str]:
    return ["bsc_create", "bsc_sizes", "bsc_workspace_size", "bsc_bind_workspace", "bsc_set_pins", "bsc_eval_egh",
            "bsc_assemble", "bsc_spmv", "bsc_bsr_pattern", "bsc_export_bsr", "bsc_newton_step", "bsc_energy_difference",
            "bsc_warmstart_load", "bsc_net_forward", "bsc_net_backward", "bsc_net_scratch_size",
            "bsc_net_backward_noalloc", "bsc_adam_step",
            "bsc_net_loss", "bsc_set_sample_log", "bsc_sample_log_count", "bsc_contact_setup",
            "bsc_contact_workspace_size", "bsc_contact_bind_workspace", "bsc_contact_hessian", "bsc_contact_solve",
            "bsc_status_string",
            "bsc_last_error", "bsc_destroy"]


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _need(t, dtype, numel, name, optional=False):
    """Checks a tensor before its raw pointer crosses the C ABI: a contiguous GPU tensor of
    ``dtype`` holding at least ``numel`` elements, the extent the library reads or writes
    through it. A smaller or mistyped buffer would be accessed out of bounds on the device, so
    it is refused here with BSC_E_INVAL. None passes only where the ABI takes NULL."""
    import torch
    if t is None:
        if optional:
            return
        raise BscError(BSC_E_INVAL, f"{name} is required")
    if not isinstance(t, torch.Tensor):
        raise BscError(BSC_E_INVAL, f"{name} must be a torch tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise BscError(BSC_E_INVAL, f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise BscError(BSC_E_INVAL, f"{name} must be contiguous")
    if t.numel() < numel:
        raise BscError(BSC_E_INVAL, f"{name} holds {t.numel()} elements, needs {numel}")
    if not t.is_cuda:
        raise BscError(BSC_E_INVAL, f"{name} must be a device (GPU) tensor")


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


BSC_QUAD_REDUCED, BSC_QUAD_GAUSS2, BSC_QUAD_INTERIOR1, BSC_QUAD_CORNER2 = 0, 1, 2, 3


def make_material(membrane=0, young=0.0, poisson=0.0, thickness=0.0, mu_st1=0.0, mu_st2=0.0, mu_sh=0.0,
                  mu_bend=0.0, rho_area=0.0, quadrature=BSC_QUAD_REDUCED) -> Material:
    return Material(membrane, young, poisson, thickness, mu_st1, mu_st2, mu_sh, mu_bend, rho_area, quadrature)


def make_opts(dt=0.01, gravity=(0.0, 0.0, -9.81), precision=BSC_FP64, stop_mode=BSC_STOP_GRAD, rtol=1e-6,
              atol=1e-2, max_newton=50, max_pcg=2000, pcg_rtol=1e-4, warm_start=0, fixed_newton_iters=0,
              pcg_adaptive=0, preconditioner=0, start=0, pcg_eta_max=0.0, timing=BSC_TIMING_CG) -> StepOpts:
    return StepOpts(dt, (ctypes.c_double * 3)(*gravity), precision, stop_mode, rtol, atol, max_newton, max_pcg,
                    pcg_rtol, warm_start, fixed_newton_iters, pcg_adaptive, preconditioner, start, pcg_eta_max,
                    timing)


@dataclass
class Sizes:
    n_cp: int
    n_elem: int
    n_membrane_pts: int
    n_bending_evals: int


class Context:
    """One sheet: owns the bsc_ctx handle and its device workspace (a torch uint8 tensor)."""

    def __init__(self, n_u, n_v, knots_u, knots_v, rest, material: Material, device="cuda"):
        import torch
        self.lib = load()
        self.n_u, self.n_v = int(n_u), int(n_v)
        ku = np.ascontiguousarray(knots_u, dtype=np.float64)
        kv = np.ascontiguousarray(knots_v, dtype=np.float64)
        rest = np.ascontiguousarray(rest, dtype=np.float64).reshape(-1)
        h = ctypes.c_void_p()
        self._mat = material
        st = self.lib.bsc_create(ctypes.byref(h), self.n_u, self.n_v, _np_ptr(ku), _np_ptr(kv), _np_ptr(rest),
                                 ctypes.byref(material), _stream())
        if st != BSC_OK:
            raise BscError(st, "bsc_create")
        self.h = h
        sz = ctypes.c_size_t()
        self._check(self.lib.bsc_workspace_size(self.h, ctypes.byref(sz)), "bsc_workspace_size")
        self.ws = torch.empty(int(sz.value) + 256, dtype=torch.uint8, device=device)
        base = self.ws.data_ptr()
        aligned = (base + 255) & ~255
        self._check(self.lib.bsc_bind_workspace(self.h, ctypes.c_void_p(aligned), ctypes.c_size_t(sz.value)),
                    "bsc_bind_workspace")
        s = [ctypes.c_int32() for _ in range(4)]
        self._check(self.lib.bsc_sizes(self.h, *[ctypes.byref(v) for v in s]), "bsc_sizes")
        self.sizes = Sizes(*[v.value for v in s])
        self.pins = np.zeros(0, dtype=np.int32)
        self.device = device

    def _check(self, st, what):
        if st != BSC_OK:
            msg = self.lib.bsc_last_error(self.h).decode() if getattr(self, "h", None) else ""
            raise BscError(st, f"{what}: {msg}")

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and self.lib is not None:
            self.lib.bsc_destroy(h)
            self.h = None

    @property
    def n_cp(self):
        return self.sizes.n_cp

    @property
    def n_elem(self):
        return self.sizes.n_elem

    # ---- calls named after the C ABI -----------------------------------------------------
    def bsc_set_pins(self, idx):
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        self._check(self.lib.bsc_set_pins(self.h, _np_ptr(idx) if idx.size else None, int(idx.size)), "bsc_set_pins")
        self.pins = idx

    def bsc_contact_setup(self, uv, max_pairs, max_vpairs=0):
        """Embeds a contact mesh (vertices at parametric (u, v), knot units) and binds a device
        workspace for conversions of up to max_pairs contact pairs."""
        import torch
        uv = np.ascontiguousarray(uv, dtype=np.float64).reshape(-1, 2)
        self._check(self.lib.bsc_contact_setup(self.h, int(uv.shape[0]), _np_ptr(uv), int(max_pairs), int(max_vpairs)),
                    "bsc_contact_setup")
        sz = ctypes.c_size_t()
        self._check(self.lib.bsc_contact_workspace_size(self.h, ctypes.byref(sz)), "bsc_contact_workspace_size")
        self.ct_ws = torch.empty(int(sz.value) + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.ct_ws.data_ptr() + 255) & ~255
        self._check(self.lib.bsc_contact_bind_workspace(self.h, ctypes.c_void_p(aligned), ctypes.c_size_t(sz.value)),
                    "bsc_contact_bind_workspace")
        self.ct_nvert = int(uv.shape[0])

    def bsc_contact_hessian(self, pair_verts, pair_hess, pair_grad=None, cap_blocks=None, want_grad=True, out=None):
        """pair_verts: (n_pairs, 4) int32, pair_hess: (n_pairs, 12, 12) float64, pair_grad: (n_pairs, 12)
        float64 or None (device tensors). Returns (row_ptr, col_idx, vals (nnzb, 3, 3), grad (3, n_cp) or None),
        the device outputs trimmed to nnzb blocks."""
        import torch
        n_pairs = int(pair_verts.shape[0]) if pair_verts is not None else 0
        if n_pairs:
            _need(pair_verts, torch.int32, 4 * n_pairs, "pair_verts")
            _need(pair_hess, torch.float64, 144 * n_pairs, "pair_hess")
            _need(pair_grad, torch.float64, 12 * n_pairs, "pair_grad", optional=True)
        dev = self.device
        retry = out is None and cap_blocks is None
        if out is None:
            cap = int(cap_blocks) if cap_blocks is not None else 256 * n_pairs + 1024
            row_ptr = torch.empty(self.n_cp + 1, dtype=torch.int32, device=dev)
            col = torch.empty(cap, dtype=torch.int32, device=dev)
            vals = torch.empty(cap, 9, dtype=torch.float64, device=dev)
            grad = torch.empty(3, self.n_cp, dtype=torch.float64, device=dev) if want_grad else None
        else:
            row_ptr, col, vals, grad = out
            cap = int(col.shape[0])
            _need(row_ptr, torch.int32, self.n_cp + 1, "row_ptr")
            _need(col, torch.int32, cap, "col_idx")
            _need(vals, torch.float64, 9 * cap, "vals")
            _need(grad, torch.float64, 3 * self.n_cp, "grad", optional=True)
        nnzb = ctypes.c_int32()

        def call():
            return self.lib.bsc_contact_hessian(self.h, n_pairs, _ptr(pair_verts) if n_pairs else None,
                                                _ptr(pair_hess) if n_pairs else None,
                                                _ptr(pair_grad) if (n_pairs and pair_grad is not None) else None, cap,
                                                _ptr(row_ptr), _ptr(col), _ptr(vals), ctypes.byref(nnzb), _ptr(grad))
        st = call()
        if st == BSC_E_NOMEM and retry and nnzb.value > cap:     # output too small: size it and redo
            cap = nnzb.value
            col = torch.empty(cap, dtype=torch.int32, device=dev)
            vals = torch.empty(cap, 9, dtype=torch.float64, device=dev)
            st = call()
        self._check(st, "bsc_contact_hessian")
        k = nnzb.value
        return row_ptr, col[:k], vals[:k].view(k, 3, 3), grad

    def bsc_eval_egh(self, x, precision=BSC_FP64, want_energy=True, want_grad=True, want_hess=True):
        import torch
        dt = torch.float64 if precision == BSC_FP64 else torch.float32
        _need(x, torch.float64, 3 * self.n_cp, "x")
        E = torch.zeros(1, dtype=torch.float64, device=x.device)
        eE = torch.empty(self.n_elem, dtype=dt, device=x.device) if want_energy else None
        eg = torch.empty(27, self.n_elem, dtype=dt, device=x.device) if want_grad else None
        eH = torch.empty(378, self.n_elem, dtype=dt, device=x.device) if want_hess else None
        self._check(self.lib.bsc_eval_egh(self.h, precision, _ptr(x), _ptr(E), _ptr(eE), _ptr(eg), _ptr(eH)),
                    "bsc_eval_egh")
        return E, eE, eg, eH

    def bsc_contact_solve(self, hess, dt, row_ptr, col_idx, vals, b, precision=BSC_FP64, x=None, rho_max=0.5,
                          series_tol=1e-12, max_terms=64, pcg_rtol=1e-12, max_pcg=20000, force=0):
        """(H + H_c) x = b by partial factorization (Sec. 5.3). hess: (114, n_cp) upper-stencil H in
        the precision's dtype; row_ptr, col_idx, vals: H_c in block CSR as bsc_contact_hessian returns
        it; b: (3, n_cp) float64. Returns (x, PfStats)."""
        import torch
        tdt = torch.float64 if precision == BSC_FP64 else torch.float32
        nnzb = int(col_idx.numel()) if col_idx is not None else 0
        _need(hess, tdt, BSC_HESS_ENTRIES * self.n_cp, "hess")
        _need(row_ptr, torch.int32, self.n_cp + 1, "row_ptr")
        if nnzb:
            _need(col_idx, torch.int32, nnzb, "col_idx")
            _need(vals, torch.float64, 9 * nnzb, "vals")
        _need(b, torch.float64, 3 * self.n_cp, "b")
        x = torch.empty_like(b) if x is None else x
        _need(x, torch.float64, 3 * self.n_cp, "x")
        opts = PfOpts(float(rho_max), float(series_tol), int(max_terms), float(pcg_rtol), int(max_pcg), int(force))
        stats = PfStats()
        self._check(self.lib.bsc_contact_solve(self.h, precision, _ptr(hess), float(dt), _ptr(row_ptr),
                                               _ptr(col_idx) if nnzb else None, _ptr(vals) if nnzb else None, nnzb,
                                               _ptr(b), _ptr(x), ctypes.byref(opts), ctypes.byref(stats)),
                    "bsc_contact_solve")
        return x, stats

    def bsc_assemble(self, x, xhat=None, dt=0.0, gravity=None, precision=BSC_FP64, want_hess=True, out=None):
        import torch
        tdt = torch.float64 if precision == BSC_FP64 else torch.float32
        _need(x, torch.float64, 3 * self.n_cp, "x")
        _need(xhat, torch.float64, 3 * self.n_cp, "xhat", optional=True)
        if out is None:
            E = torch.zeros(1, dtype=torch.float64, device=x.device)
            g = torch.empty(3, self.n_cp, dtype=tdt, device=x.device)
            H = torch.empty(BSC_HESS_ENTRIES, self.n_cp, dtype=tdt, device=x.device) if want_hess else None
        else:
            E, g, H = out
            _need(E, torch.float64, 1, "energy")
            _need(g, tdt, 3 * self.n_cp, "grad")
            _need(H, tdt, BSC_HESS_ENTRIES * self.n_cp, "hess", optional=True)
        grav = (ctypes.c_double * 3)(*gravity) if gravity is not None else None
        self._check(self.lib.bsc_assemble(self.h, precision, _ptr(x), _ptr(xhat), float(dt), grav, _ptr(E), _ptr(g),
                                          _ptr(H)), "bsc_assemble")
        return E, g, H

    def bsc_spmv(self, H, v, precision=BSC_FP64, out=None):
        import torch
        tdt = torch.float64 if precision == BSC_FP64 else torch.float32
        _need(H, tdt, BSC_HESS_ENTRIES * self.n_cp, "hess")
        _need(v, torch.float64, 3 * self.n_cp, "in")       # double vectors in both precisions
        _need(out, torch.float64, 3 * self.n_cp, "out", optional=True)
        y = torch.empty_like(v) if out is None else out
        self._check(self.lib.bsc_spmv(self.h, precision, _ptr(H), _ptr(v), _ptr(y)), "bsc_spmv")
        return y

    def bsc_bsr_pattern(self):
        nnzb = ctypes.c_int32()
        self._check(self.lib.bsc_bsr_pattern(self.h, None, None, ctypes.byref(nnzb)), "bsc_bsr_pattern")
        rp = np.zeros(self.n_cp + 1, dtype=np.int32)
        ci = np.zeros(nnzb.value, dtype=np.int32)
        self._check(self.lib.bsc_bsr_pattern(self.h, _np_ptr(rp), _np_ptr(ci), ctypes.byref(nnzb)), "bsc_bsr_pattern")
        return rp, ci

    def bsc_export_bsr(self, H, precision=BSC_FP64):
        import torch
        _need(H, torch.float64 if precision == BSC_FP64 else torch.float32, BSC_HESS_ENTRIES * self.n_cp, "hess")
        rp, ci = self.bsc_bsr_pattern()
        vals = torch.empty(ci.size, 3, 3, dtype=H.dtype, device=H.device)
        self._check(self.lib.bsc_export_bsr(self.h, precision, _ptr(H), _ptr(vals)), "bsc_export_bsr")
        return rp, ci, vals

    def bsc_newton_step(self, x, v, pin_targets=None, opts: StepOpts | None = None, raise_on_error=True):
        import torch
        opts = opts or make_opts()
        _need(x, torch.float64, 3 * self.n_cp, "x")
        _need(v, torch.float64, 3 * self.n_cp, "v")
        _need(pin_targets, torch.float64, 3 * int(self.pins.size), "pin_targets", optional=True)
        stats = StepStats()
        st = self.lib.bsc_newton_step(self.h, ctypes.byref(opts), _ptr(x), _ptr(v), _ptr(pin_targets),
                                      ctypes.byref(stats))
        if st != BSC_OK and raise_on_error:
            self._check(st, "bsc_newton_step")
        return st, stats

    def bsc_energy_difference(self, x, p, alphas, xhat=None, dt=0.0, gravity=None):
        """E(x + alpha p) - E(x) for each alpha (float64 device tensor of len(alphas))."""
        import torch
        _need(x, torch.float64, 3 * self.n_cp, "x")
        _need(p, torch.float64, 3 * self.n_cp, "p")
        _need(xhat, torch.float64, 3 * self.n_cp, "xhat", optional=True)
        al = np.ascontiguousarray(alphas, dtype=np.float64).reshape(-1)
        out = torch.empty(max(1, al.size), dtype=torch.float64, device=x.device)
        grav = (ctypes.c_double * 3)(*gravity) if gravity is not None else None
        self._check(self.lib.bsc_energy_difference(self.h, _ptr(x), _ptr(xhat), float(dt), grav, _ptr(p), int(al.size),
                                                   _np_ptr(al), _ptr(out)), "bsc_energy_difference")
        return out

    def bsc_set_sample_log(self, g_buf, p_buf, capacity):
        import torch
        if int(capacity) > 0:
            _need(g_buf, torch.float32, 3 * self.n_cp * int(capacity), "g_buf")
            _need(p_buf, torch.float32, 3 * self.n_cp * int(capacity), "p_buf")
        self._check(self.lib.bsc_set_sample_log(self.h, _ptr(g_buf), _ptr(p_buf), int(capacity)), "bsc_set_sample_log")

    def bsc_sample_log_count(self):
        c = ctypes.c_int32()
        self._check(self.lib.bsc_sample_log_count(self.h, ctypes.byref(c)), "bsc_sample_log_count")
        return c.value

    def bsc_warmstart_load(self, weights):
        import torch
        _need(weights, torch.float32, BSC_NET_PARAMS, "weights")
        self._check(self.lib.bsc_warmstart_load(self.h, _ptr(weights), int(weights.numel())), "bsc_warmstart_load")

    def bsc_net_forward(self, weights, inp, acts=None):
        import torch
        batch = inp.shape[0]
        _need(weights, torch.float32, BSC_NET_PARAMS, "weights")
        _need(inp, torch.float32, batch * 3 * self.n_cp, "inp")
        _need(acts, torch.float32, batch * 5 * 32 * self.n_cp, "acts", optional=True)
        out = torch.empty_like(inp)
        self._check(self.lib.bsc_net_forward(self.h, batch, _ptr(weights), _ptr(inp), _ptr(out), _ptr(acts)),
                    "bsc_net_forward")
        return out

    def bsc_net_scratch_size(self, batch):
        sz = ctypes.c_size_t()
        self._check(self.lib.bsc_net_scratch_size(self.h, batch, ctypes.byref(sz)), "bsc_net_scratch_size")
        return sz.value

    def bsc_net_backward(self, weights, inp, acts, dout, want_din=False, scratch=None):
        import torch
        batch = inp.shape[0]
        _need(weights, torch.float32, BSC_NET_PARAMS, "weights")
        _need(inp, torch.float32, batch * 3 * self.n_cp, "inp")
        _need(acts, torch.float32, batch * 5 * 32 * self.n_cp, "acts")
        _need(dout, torch.float32, batch * 3 * self.n_cp, "dout")
        dw = torch.empty_like(weights)
        din = torch.empty_like(inp) if want_din else None
        if scratch is None:
            scratch = torch.empty(max(1, self.bsc_net_scratch_size(batch)), dtype=torch.uint8, device=inp.device)
        _need(scratch, torch.uint8, self.bsc_net_scratch_size(batch), "scratch")
        self._check(self.lib.bsc_net_backward(self.h, batch, _ptr(weights), _ptr(inp), _ptr(acts), _ptr(dout),
                                              _ptr(dw), _ptr(din), _ptr(scratch)), "bsc_net_backward")
        return dw, din

    def bsc_net_backward_noalloc(self, weights, inp, acts, dout, dw, din=None):
        """The no-allocation variant: writes into the caller's dw (and din, if given) and passes
        no scratch (the library's static per-GPU array serves)."""
        import torch
        batch = inp.shape[0]
        _need(weights, torch.float32, BSC_NET_PARAMS, "weights")
        _need(inp, torch.float32, batch * 3 * self.n_cp, "inp")
        _need(acts, torch.float32, batch * 5 * 32 * self.n_cp, "acts")
        _need(dout, torch.float32, batch * 3 * self.n_cp, "dout")
        _need(dw, torch.float32, BSC_NET_PARAMS, "dw")
        _need(din, torch.float32, batch * 3 * self.n_cp, "din", optional=True)
        self._check(self.lib.bsc_net_backward_noalloc(self.h, batch, _ptr(weights), _ptr(inp), _ptr(acts), _ptr(dout),
                                                      _ptr(dw), _ptr(din)), "bsc_net_backward_noalloc")
        return dw, din

    def bsc_adam_step(self, param, grad, m, v, lr, t, beta1=0.9, beta2=0.999, eps=1e-8):
        import torch
        for name, a in (("param", param), ("grad", grad), ("m", m), ("v", v)):
            _need(a, torch.float32, param.numel(), name)
        self._check(self.lib.bsc_adam_step(self.h, int(param.numel()), _ptr(param), _ptr(grad), _ptr(m), _ptr(v),
                                           lr, beta1, beta2, eps, int(t)), "bsc_adam_step")

    def bsc_net_loss(self, inp, pred, target):
        import torch
        n = pred.shape[0] * 3 * self.n_cp
        for name, a in (("inp", inp), ("pred", pred), ("target", target)):
            _need(a, torch.float32, n, name)
        loss = torch.zeros(1, dtype=torch.float32, device=pred.device)
        dpred = torch.empty_like(pred)
        self._check(self.lib.bsc_net_loss(self.h, pred.shape[0], _ptr(inp), _ptr(pred), _ptr(target), _ptr(loss),
                                          _ptr(dpred)), "bsc_net_loss")
        return loss, dpred


def bsc_create(n_u, n_v, knots_u, knots_v, rest, material: Material, device="cuda") -> Context:
    """bsc_create + bsc_workspace_size + bsc_bind_workspace in one call."""
    return Context(n_u, n_v, knots_u, knots_v, rest, material, device)


def context_for_scene(scene, device="cuda", quadrature=BSC_QUAD_REDUCED) -> Context:
    """Context plus pins for a ``synthetic.Scene``."""
    m = scene.material
    mat = make_material(m.membrane, m.young, m.poisson, m.thickness, m.mu_st1, m.mu_st2, m.mu_sh, m.mu_bend,
                        m.rho_area, quadrature)
    ctx = Context(scene.n_u, scene.n_v, scene.knots_u, scene.knots_v, scene.rest, mat, device)
    if len(scene.pins):
        ctx.bsc_set_pins(scene.pins)
    return ctx


def to_soa(x_aos, device="cuda"):
    """(n_cp, 3) numpy -> (3, n_cp) float64 device tensor."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x_aos, dtype=np.float64).T)).to(device)


def to_aos(x_soa) -> np.ndarray:
    return x_soa.detach().cpu().double().numpy().T.copy()


def stencil_to_blocks(H, n_u: int, n_v: int) -> dict:
    """Host-side expansion of an upper-stencil Hessian (numpy (114, n_cp)) into a dict
    (a, b) -> 3x3 block for every CP pair of the 5x5 pattern (both triangles)."""
    Hn = np.asarray(H, dtype=np.float64)
    n = n_u * n_v
    out = {}
    for a in range(n):
        i, j = a % n_u, a // n_u
        d = Hn[0:6, a]
        out[(a, a)] = np.array([[d[0], d[1], d[2]], [d[1], d[3], d[4]], [d[2], d[4], d[5]]])
        for s in range(1, 13):
            di, dj = SLOT_OFFSETS[s]
            ib, jb = i + di, j + dj
            if 0 <= ib < n_u and 0 <= jb < n_v:
                b = jb * n_u + ib
                blk = Hn[6 + 9 * (s - 1): 6 + 9 * s, a].reshape(3, 3)
                out[(a, b)] = blk
                out[(b, a)] = blk.T
    return out
