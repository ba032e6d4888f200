"""Partial factorization of the Newton system with a contact Hessian, the plain definition (TEST
INFRASTRUCTURE: only tests, the smoke check and the benchmark's CPU-baseline leg may use it).

Sec. 5.3 (Eq. "per iteration solve"): a projected-Newton direction solves
(H_inertia + H_elasticity + H_barrier) dC = -g. The barrier Hessian is split into its diagonal
and off-diagonal parts, D = H_inertia + H_elasticity + H_barrier,d and B = H_barrier,od, and
(D + B)^-1 is expanded by the Woodbury identity with U = V = I into the Neumann series
(Eq. "Neumann expansion"): (D + B)^-1 = sum_k (-D^-1 B)^k D^-1, which needs solves with D only.
The series is used when a cheap upper bound on |D^-1 B|_op, |B|_op / lambda_min(D) with the
spectrum of B bounded by Gershgorin discs, says that it converges fast; otherwise the merged
system D + B is solved.

Readings (the paper is silent on them; the HIP path takes the same ones):
  - "diagonal part" of the barrier Hessian: its 3x3 control-point self-blocks H_c[a, a] (the
    blocks on the diagonal of the block matrix the conversion of Sec. 5.2 produces); every other
    block is B. D then keeps the elasticity Hessian's block pattern.
  - lambda_min(D) is bounded from below by one pass over diagonal blocks: the elastic Hessian is
    positive semi-definite after the per-point projection (Sec. 5.1) and so is the barrier
    Hessian, hence lambda_min(D) >= min_a lambda_min(M_a / dt^2 I + H_c[a, a]) >= min_a (M_a / dt^2
    + max(0, Gershgorin lower bound of H_c[a, a])), the minimum over free control points: a
    pinned control point's rows and columns are identity rows in D and zero in B, so D^-1 B
    vanishes on them and they do not enter |D^-1 B|_op.
  - lambda_max(B) <= max_i R_i, R_i = sum_{j != i} |B_ij| (Gershgorin; B has a zero diagonal).
  - trigger: rho = max_i R_i / lambda_min bound <= rho_max; the series keeps K + 1 terms with K
    the smallest integer for which rho^(K + 1) / (1 - rho) <= series_tol (at most max_terms
    terms); the paper fixes neither constant.
  - Dirichlet control points (Sec. 5.1's eliminated DOFs): their rows and columns of the barrier
    Hessian are dropped, as for the elastic Hessian, whose pinned rows are identity rows.

Each step below is written out with scipy sparse matrices and LU solves (library primitives)."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def dof_mask(n_cp: int, pinned) -> np.ndarray:
    """1 on free DOFs, 0 on the 3 DOFs of each pinned control point."""
    m = np.ones(3 * n_cp)
    if pinned is not None:
        p = np.nonzero(np.asarray(pinned, dtype=bool))[0]
        for c in range(3):
            m[3 * p + c] = 0.0
    return m


def split_barrier(Hc, n_cp: int, pinned=None):
    """(H_c,d, H_c,od): the 3x3 self-blocks of each control point and the rest, after dropping the
    rows and columns of pinned control points. DOF order 3 a + c."""
    P = sp.diags(dof_mask(n_cp, pinned))
    Hc = (P @ sp.csr_matrix(Hc) @ P).tocoo()
    same = (Hc.row // 3) == (Hc.col // 3)
    shape = (3 * n_cp, 3 * n_cp)
    Hd = sp.csr_matrix((Hc.data[same], (Hc.row[same], Hc.col[same])), shape=shape)
    Ho = sp.csr_matrix((Hc.data[~same], (Hc.row[~same], Hc.col[~same])), shape=shape)
    return Hd, Ho


def gershgorin_radius_max(B) -> float:
    """max_i sum_{j != i} |B_ij| (B with a zero diagonal): the Gershgorin bound of |lambda(B)|."""
    B = sp.csr_matrix(B)
    if B.nnz == 0:
        return 0.0
    A = abs(B).tolil()
    A.setdiag(0.0)
    return float(np.asarray(A.tocsr().sum(axis=1)).max())


def lambda_min_lower(mass, dt: float, Hd, pinned=None) -> float:
    """Lower bound of lambda_min(D) on the free control points from the diagonal blocks: min over
    them of M_a / dt^2 + max(0, min_r (h_rr - sum_{c != r} |h_rc|)) of the barrier self-block
    h = H_c[a, a]; inf when every control point is pinned."""
    n = len(mass)
    Hd = sp.csr_matrix(Hd)
    pin = np.zeros(n, dtype=bool) if pinned is None else np.asarray(pinned, dtype=bool)
    best = np.inf
    for a in range(n):
        if pin[a]:
            continue
        h = Hd[3 * a:3 * a + 3, 3 * a:3 * a + 3].toarray()
        g = min(h[r, r] - sum(abs(h[r, c]) for c in range(3) if c != r) for r in range(3))
        best = min(best, mass[a] / (dt * dt) + max(0.0, g))
    return float(best)


def series_terms(rho: float, series_tol: float, max_terms: int) -> int:
    """K + 1, the number of kept terms: K the smallest integer with rho^(K+1) / (1 - rho) <= tol."""
    if rho <= 0.0:
        return 1
    K = 0
    while rho ** (K + 1) / (1.0 - rho) > series_tol and K + 1 < max_terms:
        K += 1
    return K + 1


@dataclass
class PartialResult:
    x: np.ndarray          # (n_cp, 3)
    triggered: bool
    terms: int             # terms of the series (0 when the merged system was solved)
    rho_bound: float
    b_bound: float
    d_bound: float


def solve(A_el, Hc, mass, dt: float, b, pinned=None, rho_max: float = 0.5, series_tol: float = 1e-12,
          max_terms: int = 64, force: str | None = None) -> PartialResult:
    """The Newton system (A_el + H_c) x = b of Sec. 5.3. A_el: inertia plus elasticity, 3 n_cp
    square (pins already applied: identity rows and columns); H_c: the barrier (contact) Hessian
    on the control points; b: (n_cp, 3). force: None (the Gershgorin trigger decides), "series" or
    "merged"."""
    n = len(mass)
    Hd, Ho = split_barrier(Hc, n, pinned)
    D = (sp.csr_matrix(A_el) + Hd).tocsc()
    B = Ho.tocsr()
    bb = np.asarray(b, dtype=np.float64).reshape(-1)
    r_b = gershgorin_radius_max(B)
    d_lo = lambda_min_lower(mass, dt, Hd, pinned)
    rho = r_b / d_lo
    use_series = (rho <= rho_max and rho < 1.0) if force is None else (force == "series")
    if use_series:
        # Eq. "Neumann expansion": x = sum_k t_k with t_0 = D^-1 b and t_k = -D^-1 B t_{k-1}
        K1 = series_terms(rho, series_tol, max_terms) if rho < 1.0 else max_terms
        lu = spla.splu(D)
        t = lu.solve(bb)
        x = t.copy()
        for _ in range(1, K1):
            t = -lu.solve(B @ t)
            x += t
        return PartialResult(x.reshape(-1, 3), True, K1, rho, r_b, d_lo)
    x = spla.spsolve((D + B).tocsc(), bb)
    return PartialResult(np.asarray(x).reshape(-1, 3), False, 0, rho, r_b, d_lo)
