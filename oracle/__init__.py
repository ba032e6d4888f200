"""CPU FP64 oracle for the quadratic B-spline cloth FEM hot path (arXiv 2506.18867).

TEST INFRASTRUCTURE. Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this package. It is a plain, slow, obviously-correct reference written from the paper:
the arithmetic lives in ``bsc_oracle.c`` (straight loops, FP64) and this module adds ctypes
marshalling plus the projected-Newton loop of Sec. 5.1, whose linear solve is a library
primitive (``scipy.sparse.linalg.spsolve``). It shares no code with the HIP library and
never imports it.

Layouts: world positions are AoS ``(n_cp, 3)`` float64 arrays, control point ``(i, j)`` at row
``j * n_u + i``; the global Hessian is in stencil form ``(n_cp, 25, 3, 3)`` where slot
``s = (dj + 2) * 5 + (di + 2)`` couples CP ``(i, j)`` to CP ``(i + di, j + dj)``.

Parity unpinned: nothing in this module beyond what the tests pin (see ``tests/test_oracle_*``);
the FBW stiffness mapping and the learned warm start have no independent pin.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bsc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None


def build(src: str = _SRC, out: str = _LIB_PATH) -> str:
    """Compiles ``bsc_oracle.c`` (or another copy of it) with gcc into ``oracle/_build/liboracle.so``
    (or ``out``)."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # BSC_ORACLE_LIB names another build of the C source (the pin-strength test loads copies
    # with planted mistakes this way); without it the library is rebuilt when stale.
    path = os.environ.get("BSC_ORACLE_LIB")
    if not path:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        path = _LIB_PATH
    lib = ctypes.CDLL(path)
    d, i, p = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
    lib.or_basis.restype = d
    lib.or_basis.argtypes = [p, i, i, d]
    lib.or_basis_piece.restype = d
    lib.or_basis_piece.argtypes = [p, i, i, i, d, i]
    lib.or_check_knots.restype = i
    lib.or_check_knots.argtypes = [p, i, p]
    lib.or_membrane_rule.restype = i
    lib.or_membrane_rule.argtypes = [i, i, p, i]
    lib.or_bending_rule.restype = i
    lib.or_bending_rule.argtypes = [i, i, p, i]
    lib.or_membrane_rule_q.restype = i
    lib.or_membrane_rule_q.argtypes = [i, i, i, p, i]
    lib.or_bending_rule_q.restype = i
    lib.or_bending_rule_q.argtypes = [i, i, i, p, i]
    lib.or_membrane_density.restype = None
    lib.or_membrane_density.argtypes = [i, p, d, d, d, d, d, d, p, p, p]
    lib.or_project_psd6.restype = None
    lib.or_project_psd6.argtypes = [p]
    for name in ("or_element_egh",):
        getattr(lib, name).restype = i
    lib.or_element_egh.argtypes = [p, p, i, p, p, p]
    lib.or_lumped_mass.restype = i
    lib.or_lumped_mass.argtypes = [p, p]
    lib.or_assemble.restype = i
    lib.or_assemble.argtypes = [p, p, p, d, p, p, i, p, p, p]
    lib.or_energy.restype = i
    lib.or_energy.argtypes = [p, p, p, d, p, p]
    lib.or_surface_point.restype = None
    lib.or_surface_point.argtypes = [p, p, d, d, p]
    lib.or_point_geometry.restype = None
    lib.or_point_geometry.argtypes = [p, i, i, d, d, p]
    _lib = lib
    return lib


class _CSheet(ctypes.Structure):
    _fields_ = [
        ("n_u", ctypes.c_int), ("n_v", ctypes.c_int),
        ("knots_u", ctypes.c_void_p), ("knots_v", ctypes.c_void_p), ("rest", ctypes.c_void_p),
        ("membrane", ctypes.c_int),
        ("young", ctypes.c_double), ("poisson", ctypes.c_double), ("thickness", ctypes.c_double),
        ("mu_st1", ctypes.c_double), ("mu_st2", ctypes.c_double), ("mu_sh", ctypes.c_double),
        ("mu_bend", ctypes.c_double), ("rho_area", ctypes.c_double),
        ("quadrature", ctypes.c_int),
    ]


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


@dataclass
class Sheet:
    """A B-spline sheet: knots, rest control points (AoS (n_cp, 2)) and material.

    ``membrane``: 0 = StVK (young, poisson, thickness), 1 = FBW (mu_st1, mu_st2, mu_sh).
    ``mu_bend`` is the bending stiffness of Eq. "general bending energy"; ``rho_area`` the rest
    mass per unit area R^0."""
    n_u: int
    n_v: int
    knots_u: np.ndarray
    knots_v: np.ndarray
    rest: np.ndarray
    membrane: int = 0
    young: float = 0.0
    poisson: float = 0.0
    thickness: float = 0.0
    mu_st1: float = 0.0
    mu_st2: float = 0.0
    mu_sh: float = 0.0
    mu_bend: float = 0.0
    rho_area: float = 0.0
    quadrature: int = 0
    _keep: list = field(default_factory=list, repr=False)

    def c(self) -> _CSheet:
        ku, kv, rest = _f64(self.knots_u), _f64(self.knots_v), _f64(self.rest).reshape(-1)
        assert ku.size == self.n_u + 3 and kv.size == self.n_v + 3 and rest.size == 2 * self.n_u * self.n_v
        self._keep = [ku, kv, rest]
        return _CSheet(self.n_u, self.n_v, ku.ctypes.data, kv.ctypes.data, rest.ctypes.data,
                       int(self.membrane), self.young, self.poisson, self.thickness,
                       self.mu_st1, self.mu_st2, self.mu_sh, self.mu_bend, self.rho_area,
                       _quad(self.quadrature))

    @property
    def n_cp(self) -> int:
        return self.n_u * self.n_v

    @property
    def spans(self) -> tuple[int, int]:
        return self.n_u - 2, self.n_v - 2


# ---- basis and rules --------------------------------------------------------------------

def basis(knots, i: int, u: float, p: int = 2) -> float:
    """N_{i,p}(u) by the literal Cox-de Boor recursion (Eq. "B-spline basis")."""
    k = _f64(knots)
    return _load().or_basis(_ptr(k), i, p, float(u))


def basis_piece(knots, i: int, interval: int, u: float, deriv: int = 0, p: int = 2) -> float:
    """d-th derivative of the polynomial piece of N_{i,p} on knot interval ``interval``."""
    k = _f64(knots)
    return _load().or_basis_piece(_ptr(k), i, p, interval, float(u), deriv)


def check_knots(knots, n: int):
    k = _f64(knots)
    h = ctypes.c_double(0.0)
    N = _load().or_check_knots(_ptr(k), n, ctypes.byref(h))
    return (N, h.value) if N > 0 else (None, None)


QUAD_REDUCED, QUAD_GAUSS2, QUAD_INTERIOR1, QUAD_CORNER2 = 0, 1, 2, 3
QUADRATURES = {"reduced": QUAD_REDUCED, "gauss2": QUAD_GAUSS2, "interior1": QUAD_INTERIOR1, "corner2": QUAD_CORNER2}


def _quad(q) -> int:
    q = QUADRATURES.get(q, q) if isinstance(q, str) else int(q)
    if q not in (0, 1, 2, 3):
        raise ValueError(f"unknown quadrature {q}")
    return q


def membrane_rule(Nu: int, Nv: int, quadrature=QUAD_REDUCED) -> np.ndarray:
    """(M, 5) array of (u, v, wbar, k, l) in span units. QUAD_REDUCED is the paper's rule
    (Sec. 4.1, Reduced Integration); the others are the comparison rules of Sec. 6.5 (standard
    2x2 Gauss on interior spans, 1x1 interior, 2x2 corners)."""
    lib = _load()
    q = _quad(quadrature)
    n = lib.or_membrane_rule_q(Nu, Nv, q, None, 0)
    out = np.zeros((n, 5))
    lib.or_membrane_rule_q(Nu, Nv, q, _ptr(out), n)
    return out


def bending_rule(Nu: int, Nv: int, quadrature=QUAD_REDUCED) -> np.ndarray:
    """(B', 5) array of bending evaluations (u, v, wbar, k, l) (Sec. 4.2; reading R2). With
    QUAD_GAUSS2 the interior spans take 2x2 Gauss points (Sec. 6.5, configuration (A))."""
    lib = _load()
    q = _quad(quadrature)
    n = lib.or_bending_rule_q(Nu, Nv, q, None, 0)
    out = np.zeros((n, 5))
    lib.or_bending_rule_q(Nu, Nv, q, _ptr(out), n)
    return out


# ---- densities and projection -------------------------------------------------------------

def membrane_density(F, model=0, young=0.0, poisson=0.0, thickness=0.0, mu_st1=0.0, mu_st2=0.0, mu_sh=0.0):
    """Psi, P (3x2) and the 6x6 Hessian (vec(F) column-major) of the membrane density."""
    Fa = _f64(F).reshape(3, 2).copy()
    P = np.zeros((3, 2))
    A = np.zeros((6, 6))
    psi = ctypes.c_double(0.0)
    _load().or_membrane_density(int(model), _ptr(Fa), young, poisson, thickness, mu_st1, mu_st2, mu_sh,
                                ctypes.byref(psi), _ptr(P), _ptr(A))
    return psi.value, P, A


def project_psd6(A) -> np.ndarray:
    out = _f64(A).reshape(6, 6).copy()
    _load().or_project_psd6(_ptr(out))
    return out


# ---- element and global quantities --------------------------------------------------------

def element_egh(sheet: Sheet, x, project: bool = True, want_hessian: bool = True):
    """Per-element elastic energy (Ne,), gradient (Ne, 27), Hessian (Ne, 27, 27)."""
    Nu, Nv = sheet.spans
    ne = Nu * Nv
    xs = _f64(x).reshape(-1)
    E = np.zeros(ne)
    g = np.zeros((ne, 27))
    H = np.zeros((ne, 27, 27)) if want_hessian else None
    cs = sheet.c()
    st = _load().or_element_egh(ctypes.byref(cs), _ptr(xs), int(project), _ptr(E), _ptr(g),
                                _ptr(H) if H is not None else None)
    if st != 0:
        raise ValueError("oracle: invalid sheet")
    return E, g, H


def lumped_mass(sheet: Sheet) -> np.ndarray:
    M = np.zeros(sheet.n_cp)
    cs = sheet.c()
    if _load().or_lumped_mass(ctypes.byref(cs), _ptr(M)) != 0:
        raise ValueError("oracle: invalid sheet")
    return M


def assemble(sheet: Sheet, x, xhat=None, dt=None, gravity=None, pinned=None, project=True,
             want_hessian=True):
    """Incremental potential E, gradient (n_cp, 3) and Hessian in stencil form (n_cp, 25, 3, 3).

    ``dt=None`` drops the inertia term; ``pinned`` is a boolean mask over CPs (Dirichlet
    elimination: zero gradient, identity rows and columns)."""
    n = sheet.n_cp
    xs = _f64(x).reshape(-1)
    inv_dt2 = 0.0 if dt is None else 1.0 / (dt * dt)
    xh = _f64(xhat).reshape(-1) if xhat is not None else None
    gr = _f64(gravity) if gravity is not None else None
    pm = np.ascontiguousarray(np.asarray(pinned, dtype=np.int32)) if pinned is not None else None
    E = ctypes.c_double(0.0)
    g = np.zeros((n, 3))
    H = np.zeros((n, 25, 3, 3)) if want_hessian else None
    cs = sheet.c()
    st = _load().or_assemble(ctypes.byref(cs), _ptr(xs), _ptr(xh) if xh is not None else None, inv_dt2,
                             _ptr(gr) if gr is not None else None, _ptr(pm) if pm is not None else None,
                             int(project), ctypes.byref(E), _ptr(g), _ptr(H) if H is not None else None)
    if st != 0:
        raise ValueError("oracle: invalid sheet")
    return E.value, g, H


def energy(sheet: Sheet, x, xhat=None, dt=None, gravity=None) -> float:
    xs = _f64(x).reshape(-1)
    inv_dt2 = 0.0 if dt is None else 1.0 / (dt * dt)
    xh = _f64(xhat).reshape(-1) if xhat is not None else None
    gr = _f64(gravity) if gravity is not None else None
    E = ctypes.c_double(0.0)
    cs = sheet.c()
    _load().or_energy(ctypes.byref(cs), _ptr(xs), _ptr(xh) if xh is not None else None, inv_dt2,
                      _ptr(gr) if gr is not None else None, ctypes.byref(E))
    return E.value


def surface_point(sheet: Sheet, x, u: float, v: float) -> np.ndarray:
    """S(u, v) (Eq. "general B-spline patch") at knot coordinates (u, v)."""
    xs = _f64(x).reshape(-1)
    out = np.zeros(3)
    cs = sheet.c()
    _load().or_surface_point(ctypes.byref(cs), _ptr(xs), float(u), float(v), _ptr(out))
    return out


def point_geometry(sheet: Sheet, k: int, l: int, u: float, v: float):
    """Rest-map data at (u, v) (span units) evaluated in span (k, l): K = d(u,v)/dX (2x2),
    det J, and the five Laplacian coefficients of Eq. "Laplacian in parametric space"."""
    out = np.zeros(10)
    cs = sheet.c()
    _load().or_point_geometry(ctypes.byref(cs), k, l, float(u), float(v), _ptr(out))
    return out[:4].reshape(2, 2), out[4], out[5:]


def stencil_to_csr(sheet: Sheet, H):
    """Global (3 n_cp) x (3 n_cp) scipy CSR matrix from the stencil form."""
    import scipy.sparse as sp
    nu, nv = sheet.n_u, sheet.n_v
    rows, cols, vals = [], [], []
    a = np.arange(sheet.n_cp)
    ia, ja = a % nu, a // nu
    for s in range(25):
        di, dj = s % 5 - 2, s // 5 - 2
        ib, jb = ia + di, ja + dj
        ok = (ib >= 0) & (ib < nu) & (jb >= 0) & (jb < nv)
        A, B = a[ok], (jb * nu + ib)[ok]
        for r in range(3):
            for c in range(3):
                rows.append(3 * A + r)
                cols.append(3 * B + c)
                vals.append(H[ok, s, r, c])
    rows = np.concatenate(rows); cols = np.concatenate(cols); vals = np.concatenate(vals)
    return sp.csr_matrix((vals, (rows, cols)), shape=(3 * sheet.n_cp, 3 * sheet.n_cp))


# ---- projected Newton on the incremental potential (Sec. 3.2, Sec. 5.1) ------------------

@dataclass
class NewtonResult:
    x: np.ndarray
    v: np.ndarray
    iters: int
    g0_norm: float
    g_norm: float
    energy: float
    alphas: list


def newton_step(sheet: Sheet, x_n, v_n, dt: float, gravity, pins=None, pin_targets=None,
                rtol: float = 1e-6, atol: float | None = None, max_newton: int = 100,
                fixed_iters: int | None = None, max_halvings: int = 20,
                start: str = "previous") -> NewtonResult:
    """One implicit-Euler step: minimise E(x) = |x - xhat|_M^2/(2 dt^2) + V(x) from
    x0 = x_n (``start="previous"``) or x0 = xhat (``start="predictor"``), with pinned CPs at
    their targets, xhat = x_n + dt v_n. The paper leaves the first iterate open (Sec. 5.1 refers
    to IPC, whose x_n start serves a contact barrier); both are the same minimisation.

    Each iteration: gradient and projected Hessian; stop when |g_free| <= rtol |g0_free|
    (or, with ``atol``, when |p|_inf / dt <= atol); exact direction by sparse LU;
    backtracking from alpha = 1, halving until E(x + alpha p) <= E(x).
    ``fixed_iters`` runs exactly that many iterations (used to compare iterates)."""
    import scipy.sparse.linalg as spla
    x_n = _f64(x_n).reshape(-1, 3)
    v_n = _f64(v_n).reshape(-1, 3)
    xhat = x_n + dt * v_n
    if start not in ("previous", "predictor"):
        raise ValueError("start must be 'previous' or 'predictor'")
    x = (xhat if start == "predictor" else x_n).copy()
    mask = np.zeros(sheet.n_cp, dtype=bool)
    if pins is not None and len(pins):
        pins = np.asarray(pins, dtype=np.int64)
        mask[pins] = True
        x[pins] = _f64(pin_targets).reshape(-1, 3)
    g0 = None
    alphas = []
    it = 0
    E = None
    gn = 0.0
    while True:
        E, g, H = assemble(sheet, x, xhat, dt, gravity, mask, project=True)
        gn = float(np.linalg.norm(g))
        if g0 is None:
            g0 = gn
        if fixed_iters is not None:
            if it >= fixed_iters:
                break
        elif (atol is None and gn <= rtol * g0) or it >= max_newton:
            break
        A = stencil_to_csr(sheet, H)
        p = spla.spsolve(A.tocsc(), -g.reshape(-1)).reshape(-1, 3)
        if fixed_iters is None and atol is not None and np.abs(p).max() / dt <= atol:
            break
        alpha = 1.0
        for _ in range(max_halvings + 1):
            if energy(sheet, x + alpha * p, xhat, dt, gravity) <= E:
                break
            alpha *= 0.5
        else:
            raise RuntimeError("oracle line search failed")
        alphas.append(alpha)
        x = x + alpha * p
        it += 1
    return NewtonResult(x=x, v=(x - x_n) / dt, iters=it, g0_norm=g0, g_norm=gn, energy=E, alphas=alphas)
