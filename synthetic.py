"""Seeded synthetic inputs for the B-spline cloth hot path: sheets, states, pins and drives.

This module holds none of the method's arithmetic (no basis, quadrature, energy or solver
code); it only builds inputs. Both the oracle-based tests and the HIP path take their inputs
from here, so that the two sides see identical data.

Every sheet is a flat rectangle in the plane z = 0 on open uniform quadratic knots
(0,0,0,1,...,N,N,N). Its rest control points sit at the Greville abscissae of the knots
(x_i = L (xi_{i+1} + xi_{i+2}) / (2N), 0-based knots), the placement at which the B-spline
rest map is exactly affine, matching the control-point drawing of the paper's quadrature
figure. Random numbers come from ``numpy.random.Generator(PCG64(seed))``.

These sheets stand in for the paper's square-sheet benchmarks (upright hanging, drape,
compression); no benchmark assets are used.

``mapped_sheet`` builds the non-rectangular domains of the paper's robustness study of its
reduced quadrature on distorted patches (varying aspect ratio, skewed corners, sharp turns
within an edge) plus a curved quarter annulus: the Greville grid of the unit square pushed
through a closed-form map. The rest map is then no longer affine.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def open_uniform_knots(n: int, spacing: int = 1) -> np.ndarray:
    """Open uniform quadratic knot vector for n control points (n + 3 entries)."""
    N = n - 2
    return spacing * np.concatenate([[0.0, 0.0], np.arange(N + 1, dtype=np.float64), [N, N]])


def greville(knots: np.ndarray, n: int) -> np.ndarray:
    """Greville abscissae (xi_{i+1} + xi_{i+2}) / 2, 0-based knots, i = 0..n-1."""
    return 0.5 * (knots[1:n + 1] + knots[2:n + 2])


@dataclass
class Material:
    """membrane: 0 = StVK (young [Pa], poisson, thickness [m]); 1 = FBW (mu_* [N/m]).
    mu_bend [N m] is the bending stiffness; rho_area [kg/m^2] the rest mass per area."""
    membrane: int = 0
    young: float = 1e4
    poisson: float = 0.3
    thickness: float = 1e-3
    mu_st1: float = 0.0
    mu_st2: float = 0.0
    mu_sh: float = 0.0
    mu_bend: float = 0.0
    rho_area: float = 0.2


def plate_bending_stiffness(young: float, poisson: float, thickness: float) -> float:
    """Kirchhoff plate stiffness D = E t^3 / (12 (1 - nu^2)), used as the bending stiffness."""
    return young * thickness ** 3 / (12.0 * (1.0 - poisson ** 2))


def stvk_material(young=1e4, poisson=0.3, thickness=1e-3, rho_area=0.2, mu_bend=None) -> Material:
    if mu_bend is None:
        mu_bend = plate_bending_stiffness(young, poisson, thickness)
    return Material(0, young, poisson, thickness, 0.0, 0.0, 0.0, mu_bend, rho_area)


@dataclass
class Scene:
    """Everything one implicit-Euler step needs. Positions are AoS (n_cp, 3) float64 with
    control point (i, j) at row j * n_u + i; ``rest`` is (n_cp, 2)."""
    name: str
    n_u: int
    n_v: int
    knots_u: np.ndarray
    knots_v: np.ndarray
    rest: np.ndarray
    material: Material
    x0: np.ndarray
    v0: np.ndarray
    pins: np.ndarray                     # int64 CP indices
    pin_rest: np.ndarray                 # (n_pins, 3) pin positions at t = 0
    dt: float = 0.01
    gravity: np.ndarray = field(default_factory=lambda: np.array([0.0, 0.0, -9.81]))
    drive_cp: int = -1                   # CP whose z is driven sinusoidally (-1: none)
    drive_amp: float = 0.0
    drive_hz: float = 0.0

    @property
    def n_cp(self) -> int:
        return self.n_u * self.n_v

    @property
    def n_elem(self) -> int:
        return (self.n_u - 2) * (self.n_v - 2)

    def pin_targets(self, step: int) -> np.ndarray:
        """Pin positions at the end of step ``step`` (0-based): the driven CP moves in z as
        amp * sin(2 pi f t) with t = (step + 1) dt; every other pin holds its start position."""
        tgt = self.pin_rest.copy()
        if self.drive_cp >= 0:
            t = (step + 1) * self.dt
            k = int(np.nonzero(self.pins == self.drive_cp)[0][0])
            tgt[k, 2] += self.drive_amp * np.sin(2.0 * np.pi * self.drive_hz * t)
        return tgt


def flat_sheet(n_u: int, n_v: int | None = None, L_u: float = 1.0, L_v: float | None = None,
               spacing: int = 1, shear: float = 0.0):
    """Knots and Greville rest CPs of a flat L_u x L_v sheet; ``shear`` skews it affinely."""
    n_v = n_u if n_v is None else n_v
    L_v = L_u if L_v is None else L_v
    ku, kv = open_uniform_knots(n_u, spacing), open_uniform_knots(n_v, spacing)
    gu = greville(ku, n_u) / ku[-1] * L_u
    gv = greville(kv, n_v) / kv[-1] * L_v
    X1, X2 = np.meshgrid(gu, gv)                     # [j, i]
    rest = np.stack([X1.ravel() + shear * X2.ravel(), X2.ravel()], axis=1)
    return ku, kv, rest


MAPPED_KINDS = ("aspect", "skew", "bend", "annulus")


def mapped_sheet(n_u: int, n_v: int | None = None, kind: str = "skew", param: float | None = None,
                 L_u: float = 1.0, L_v: float | None = None):
    """Knots and rest CPs (n_cp, 2) of a non-rectangular sheet: CP (i, j) sits at the image of
    its Greville point (s, t) in [0, 1]^2 under

    - "aspect": the rectangle L_u x (L_u / param), param the aspect ratio (affine map);
    - "skew": the bilinear map onto the quadrilateral (0, 0), (L_u, 0), P01 + (1.25 L_u, 0),
      P01 = L_v (cos param, sin param): its corner at the origin has the angle param (degrees),
      and its top edge is 25% longer than its bottom edge;
    - "bend": X = (L_u s, L_v t + (1 - t) k L_u (1/2 - |s - 1/2|)) with k = tan((180 - param)/2):
      the edge t = 0 turns at its midpoint with the interior angle param (degrees);
    - "annulus": the quarter annulus r = r_in + (r_out - r_in) s, angle (pi / 2) t, with
      r_out = L_u and r_in = param L_u.
    """
    n_v = n_u if n_v is None else n_v
    L_v = L_u if L_v is None else L_v
    ku, kv = open_uniform_knots(n_u), open_uniform_knots(n_v)
    su = greville(ku, n_u) / ku[-1]
    tv = greville(kv, n_v) / kv[-1]
    S, T = np.meshgrid(su, tv)                       # [j, i]
    if kind == "aspect":
        ratio = 4.0 if param is None else param
        X, Y = L_u * S, (L_u / ratio) * T
    elif kind == "skew":
        ang = np.deg2rad(60.0 if param is None else param)
        P01 = np.array([L_v * np.cos(ang), L_v * np.sin(ang)])
        P = np.array([[0.0, 0.0], [L_u, 0.0], P01, [L_u + 0.25 * L_u + P01[0], P01[1]]])
        w = [(1 - S) * (1 - T), S * (1 - T), (1 - S) * T, S * T]
        X = sum(wk * P[k, 0] for k, wk in enumerate(w))
        Y = sum(wk * P[k, 1] for k, wk in enumerate(w))
    elif kind == "bend":
        k = np.tan(np.deg2rad(180.0 - (150.0 if param is None else param)) / 2.0)
        X = L_u * S
        Y = L_v * T + (1.0 - T) * k * L_u * (0.5 - np.abs(S - 0.5))
    elif kind == "annulus":
        r_in = (0.5 if param is None else param) * L_u
        r = r_in + (L_u - r_in) * S
        th = 0.5 * np.pi * T
        X, Y = r * np.cos(th), r * np.sin(th)
    else:
        raise ValueError(f"unknown mapped sheet kind {kind!r}")
    rest = np.stack([X.ravel(), Y.ravel()], axis=1)
    return ku, kv, rest


def mapped_hanging_sheet(n: int, kind: str, param: float | None = None, seed: int = 1,
                         material: Material | None = None, noise: float = 1e-3) -> Scene:
    """A mapped sheet hanging from the two corner CPs of its last row (j = n - 1), z-noise
    U(+-noise), gravity along -y, dt = 0.01 s."""
    g = rng(seed)
    ku, kv, rest = mapped_sheet(n, n, kind, param)
    x0 = embed(rest)
    x0[:, 2] += g.uniform(-noise, noise, size=x0.shape[0])
    pins = np.array([cp_index(n, 0, n - 1), cp_index(n, n - 1, n - 1)], dtype=np.int64)
    mat = material or stvk_material()
    return Scene(f"hanging-{kind}", n, n, ku, kv, rest, mat, x0, np.zeros_like(x0), pins, x0[pins].copy(),
                 0.01, np.array([0.0, -9.81, 0.0]))


def embed(rest: np.ndarray) -> np.ndarray:
    return np.concatenate([rest, np.zeros((rest.shape[0], 1))], axis=1)


def cp_index(n_u: int, i: int, j: int) -> int:
    return j * n_u + i


def hanging_sheet(n: int = 20, seed: int = 1, material: Material | None = None, noise: float = 1e-3) -> Scene:
    """Upright hanging sheet: side 1 m, flat rest, x0 = rest + U(+-noise) in z, the two top
    corners pinned, gravity along -y (in the sheet's plane), dt = 0.01 s."""
    g = rng(seed)
    ku, kv, rest = flat_sheet(n)
    x0 = embed(rest)
    x0[:, 2] += g.uniform(-noise, noise, size=x0.shape[0])
    pins = np.array([cp_index(n, 0, n - 1), cp_index(n, n - 1, n - 1)], dtype=np.int64)
    mat = material or stvk_material()
    return Scene("hanging", n, n, ku, kv, rest, mat, x0, np.zeros_like(x0), pins, x0[pins].copy(),
                 0.01, np.array([0.0, -9.81, 0.0]))


def compressed_sheet(n: int = 100, seed: int = 2, material: Material | None = None,
                     compression: float = 0.1, noise: float = 2e-3) -> Scene:
    """Drape with in-plane compression: X1 -> (1 - compression) X1, z-noise U(+-noise), the
    first and last CP columns held at their compressed positions, gravity along -z."""
    g = rng(seed)
    ku, kv, rest = flat_sheet(n)
    x0 = embed(rest)
    x0[:, 0] *= (1.0 - compression)
    x0[:, 2] += g.uniform(-noise, noise, size=x0.shape[0])
    j = np.arange(n)
    pins = np.concatenate([j * n + 0, j * n + (n - 1)]).astype(np.int64)
    mat = material or stvk_material()
    return Scene("compressed", n, n, ku, kv, rest, mat, x0, np.zeros_like(x0), pins, x0[pins].copy(),
                 0.01, np.array([0.0, 0.0, -9.81]))


MATERIAL_GRID = [(E, t) for E in (1e3, 1e4, 1e5) for t in (0.5e-3, 1e-3, 2e-3)]


def driven_sheet(n: int = 226, seed: int = 300, cell: int | None = None, noise: float = 0.0,
                 domain: tuple | None = None) -> Scene:
    """Large sheet with a material cell from the (E, t) grid, K ~ U{4..16} random held CPs plus
    the corner CP (0,0) driven in z with amplitude 5 cm at 1 Hz; gravity along -z. Starts flat
    (optional z-noise U(+-noise)). ``domain`` = (kind, param) places the rest CPs with
    ``mapped_sheet`` instead of on the unit square (same pins and drive)."""
    g = rng(seed)
    if cell is None:
        cell = (seed - 300) % len(MATERIAL_GRID)
    E, t = MATERIAL_GRID[cell]
    ku, kv, rest = flat_sheet(n) if domain is None else mapped_sheet(n, n, domain[0], domain[1])
    x0 = embed(rest)
    x0[:, 2] += g.uniform(-noise, noise, size=x0.shape[0])
    K = int(g.integers(4, 17))
    others = g.choice(np.arange(1, n * n), size=K, replace=False)
    pins = np.concatenate([[0], np.sort(others)]).astype(np.int64)
    mat = stvk_material(young=E, thickness=t)
    return Scene("driven", n, n, ku, kv, rest, mat, x0, np.zeros_like(x0), pins, x0[pins].copy(),
                 0.01, np.array([0.0, 0.0, -9.81]), drive_cp=0, drive_amp=0.05, drive_hz=1.0)


def wrinkling_sheet(n_width: int, thickness: float = 1e-3, stretch: float = 1.1, amp: float = 0.02,
                    mode: int = 1) -> Scene:
    """The stretched-plate wrinkling benchmark (Sec. 6.2, convergence under refinement of the
    membrane): a flat W x L = 1.0 m x 2.5 m plate, n_width spans across the width and
    2.5 n_width along the length, both short edges clamped (their two CP rows held) and pulled
    apart so that the length grows by ``stretch`` about the middle, no gravity. StVK with E = 1e6 Pa, nu = 0.5 and the given
    thickness (the paper gives none; 1 mm here), bending stiffness D. The start state is the
    uniform stretch plus the perturbation amp sin(pi Y / L) sin(mode pi X / W) in z (zero on
    the clamped rows); dt = 1e4 s, so one implicit-Euler step is the quasi-static solve."""
    W, L = 1.0, 2.5
    n_len = int(round(2.5 * n_width))
    n_u, n_v = n_width + 2, n_len + 2
    ku, kv, rest = flat_sheet(n_u, n_v, L_u=W, L_v=L)
    x0 = embed(rest)
    x0[:, 1] = stretch * (rest[:, 1] - 0.5 * L) + 0.5 * L
    x0[:, 2] = amp * np.sin(np.pi * rest[:, 1] / L) * np.sin(mode * np.pi * rest[:, 0] / W)
    rows = (0, 1, n_v - 2, n_v - 1)
    pins = np.array([cp_index(n_u, i, j) for j in rows for i in range(n_u)], dtype=np.int64)
    x0[pins, 2] = 0.0
    mat = stvk_material(young=1e6, poisson=0.5, thickness=thickness, rho_area=0.2)
    return Scene("wrinkling", n_u, n_v, ku, kv, rest, mat, x0, np.zeros_like(x0), pins, x0[pins].copy(),
                 1e4, np.array([0.0, 0.0, 0.0]))


def smooth_field(n_u: int, n_v: int, seed: int, amp: float = 0.05, modes: int = 3) -> np.ndarray:
    """A smooth random displacement field on the CP grid (sum of low sine modes), (n_cp, 3)."""
    g = rng(seed)
    s = np.linspace(0.0, 1.0, n_u)[None, :]
    t = np.linspace(0.0, 1.0, n_v)[:, None]
    out = np.zeros((n_v, n_u, 3))
    for c in range(3):
        for _ in range(modes):
            a, b = g.integers(1, 4, size=2)
            ph = g.uniform(0, 2 * np.pi, size=2)
            out[:, :, c] += amp * g.uniform(-1, 1) * np.sin(a * np.pi * s + ph[0]) * np.sin(b * np.pi * t + ph[1])
    return out.reshape(-1, 3)


# ---- contact mesh and contact pairs (input data for the contact-Hessian conversion) ----------

def contact_mesh(n_u: int, n_v: int | None = None, dof_ratio: float = 2.0, spacing: int = 1):
    """A triangle contact mesh embedded in the surface: an m_u x m_v grid of vertices at uniform
    parametric coordinates covering the whole parameter rectangle (knot units), with about
    dof_ratio times the control points' count (the paper uses twice the surface's DOFs), and the
    two triangles of every grid cell. Returns (uv (n_vert, 2), triangles (n_tri, 3), (m_u, m_v))."""
    n_v = n_u if n_v is None else n_v
    m_u = max(2, int(round(np.sqrt(dof_ratio) * (n_u - 1))) + 1)
    m_v = max(2, int(round(np.sqrt(dof_ratio) * (n_v - 1))) + 1)
    U = np.linspace(0.0, spacing * (n_u - 2), m_u)
    V = np.linspace(0.0, spacing * (n_v - 2), m_v)
    uu, vv = np.meshgrid(U, V)                     # vertex (p, q) at row q * m_u + p
    uv = np.stack([uu.ravel(), vv.ravel()], axis=1)
    p, q = np.meshgrid(np.arange(m_u - 1), np.arange(m_v - 1))
    a = (q * m_u + p).ravel()
    tris = np.concatenate([np.stack([a, a + 1, a + m_u + 1], 1), np.stack([a, a + m_u + 1, a + m_u], 1)])
    return uv, tris.astype(np.int64), (m_u, m_v)


def contact_pairs(uv: np.ndarray, tris: np.ndarray, grid: tuple, n_pairs: int, seed: int = 7,
                  fold: float = 0.5, scale: float = 1.0):
    """Synthetic contact pairs of a sheet folded onto itself across the line u = fold * u_max,
    the dense self-contact of a folded cloth: each pair couples a vertex (or an edge) of one
    layer with the nearest triangle (or edge) of the mirrored layer. The mix is 70% point-
    triangle (4 vertices), 20% edge-edge (4), 7% point-edge (3) and 3% point-point (2); unused
    slots hold -1. Each pair gets a Hessian D^T Q D with Q a random symmetric positive
    semi-definite 9x9 matrix and D the map from the pair's vertex positions to the positions of
    vertices 1..k-1 relative to vertex 0, so it only depends on relative positions, like a
    barrier; its gradient is D^T q for a random q. Returns (verts (n_pairs, 4) int32,
    hess (n_pairs, 12, 12), grad (n_pairs, 12))."""
    g = rng(seed)
    m_u, m_v = grid
    umax = uv[:, 0].max()
    cols = np.rint(uv[:, 0] / umax * (m_u - 1)).astype(np.int64)
    rows_ = np.arange(uv.shape[0]) // m_u
    left = np.nonzero(cols < fold * (m_u - 1))[0]
    verts = -np.ones((n_pairs, 4), dtype=np.int32)
    kinds = g.choice(4, size=n_pairs, p=[0.7, 0.2, 0.07, 0.03])

    def mirror(a):
        c = int(round(2 * fold * (m_u - 1))) - cols[a]
        c = min(max(c, 0), m_u - 1)
        return rows_[a] * m_u + c

    for t in range(n_pairs):
        a = int(g.choice(left))
        b = mirror(a)
        bi, bj = b % m_u, b // m_u
        bi, bj = min(bi, m_u - 2), min(bj, m_v - 2)
        cell = bj * (m_u - 1) + bi
        tri = tris[cell + (g.integers(2) * (m_u - 1) * (m_v - 1))]
        ai, aj = min(a % m_u, m_u - 2), min(a // m_u, m_v - 2)
        if kinds[t] == 0:
            verts[t] = [a, tri[0], tri[1], tri[2]]
        elif kinds[t] == 1:
            verts[t] = [a, aj * m_u + ai + 1, tri[0], tri[1]]
        elif kinds[t] == 2:
            verts[t, :3] = [a, tri[0], tri[2]]
        else:
            verts[t, :2] = [a, b]
    hess = np.zeros((n_pairs, 12, 12))
    grad = np.zeros((n_pairs, 12))
    for t in range(n_pairs):
        k = int((verts[t] >= 0).sum())
        D = np.zeros((3 * (k - 1), 12))
        for s in range(1, k):
            D[3 * (s - 1):3 * s, 3 * s:3 * s + 3] = np.eye(3)
            D[3 * (s - 1):3 * s, 0:3] = -np.eye(3)
        R = g.standard_normal((3 * (k - 1), 2))
        Q = scale * (R @ R.T + 0.1 * np.eye(3 * (k - 1)))
        hess[t] = D.T @ Q @ D
        grad[t] = D.T @ (scale * g.standard_normal(3 * (k - 1)))
    return verts, hess, grad
