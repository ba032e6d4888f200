"""Contact Hessian conversion to the control points, the plain definition (TEST INFRASTRUCTURE:
only tests, the smoke check and the benchmark's CPU-baseline leg may use it).

Sec. 4.3 (contact barrier): a vertex a of the triangle contact mesh sits at fixed parametric
coordinates (u_a, v_a), so its position is x_a = sum_ij N_ij(u_a, v_a) C^{ij} (Eq. "trig mesh node
from control points"). The chain rule (Eq. "gradient and hessian of contact barrier", whose
second-derivative term vanishes because x_a is linear in the CPs) gives

    dB/dC = J^T dB/dx,    d2B/dC2 = J^T (d2B/dx2) J,    J = W kron I_3,

with W[a, cp] = N_cp(u_a, v_a). Here W is built from the oracle's Cox-de Boor basis (the piece
of the span holding the vertex: span min(floor(u), N - 1), so the right end belongs to the last
span), the vertex-level Hessian d2B/dx2 is the sum of the per-pair Hessians placed at their
vertices, and the products are sparse library products. No blocking or reordering beyond that.
Sec. 5.2's hash maps and spatial blocks are an implementation strategy for the same sums and
are not reproduced here."""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import Sheet, basis_piece


def vertex_weights(sheet: Sheet, uv) -> sp.csr_matrix:
    """W (n_vert x n_cp): the B-spline basis values of each vertex, nonzero entries only."""
    uv = np.asarray(uv, dtype=np.float64).reshape(-1, 2)
    ku, kv = sheet.knots_u, sheet.knots_v
    Nu, Nv = sheet.n_u - 2, sheet.n_v - 2
    hu, hv = ku[3] - ku[2], kv[3] - kv[2]
    rows, cols, vals = [], [], []
    for a, (u, v) in enumerate(uv):
        k = min(int(math.floor(u / hu)), Nu - 1)
        l = min(int(math.floor(v / hv)), Nv - 1)
        wu = [basis_piece(ku, i, 2 + k, u) for i in range(k, k + 3)]
        wv = [basis_piece(kv, j, 2 + l, v) for j in range(l, l + 3)]
        for b in range(3):
            for c in range(3):
                w = wu[c] * wv[b]
                if w != 0.0:
                    rows.append(a)
                    cols.append((l + b) * sheet.n_u + (k + c))
                    vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(uv.shape[0], sheet.n_cp))


def vertex_hessian(n_vert: int, pair_verts, pair_hess, pair_grad=None):
    """Vertex-level Hessian (3 n_vert square, sparse) and gradient (n_vert, 3): the per-pair
    blocks summed at their vertices; slots holding -1 are unused."""
    pv = np.asarray(pair_verts)
    H = np.asarray(pair_hess, dtype=np.float64).reshape(-1, 12, 12)
    rows, cols, vals = [], [], []
    g = np.zeros((n_vert, 3))
    for c in range(pv.shape[0]):
        for s in range(4):
            a = pv[c, s]
            if a < 0:
                continue
            if pair_grad is not None:
                g[a] += pair_grad[c, 3 * s:3 * s + 3]
            for s2 in range(4):
                b = pv[c, s2]
                if b < 0:
                    continue
                for r in range(3):
                    for k in range(3):
                        rows.append(3 * a + r)
                        cols.append(3 * b + k)
                        vals.append(H[c, 3 * s + r, 3 * s2 + k])
    Hv = sp.coo_matrix((vals, (rows, cols)), shape=(3 * n_vert, 3 * n_vert)).tocsr()
    return Hv, g


def contact_to_cp(sheet: Sheet, uv, pair_verts, pair_hess, pair_grad=None):
    """CP Hessian (3 n_cp square, sparse CSR) and CP gradient (n_cp, 3)."""
    W = vertex_weights(sheet, uv)
    Hv, gv = vertex_hessian(W.shape[0], pair_verts, pair_hess, pair_grad)
    J = sp.kron(W, sp.identity(3), format="csr")
    Hc = (J.T @ Hv @ J).tocsr()
    gc = (W.T @ gv)
    return Hc, np.asarray(gc)


def cp_block_pattern(sheet: Sheet, uv, pair_verts):
    """The set of CP pairs (i, j) reached by some vertex pair of some contact pair with nonzero
    weights on both sides (the blocks the conversion produces)."""
    W = vertex_weights(sheet, uv).tolil()
    supp = [set(r) for r in W.rows]
    out = set()
    for row in np.asarray(pair_verts):
        vs = [a for a in row if a >= 0]
        for a in vs:
            for b in vs:
                for i in supp[a]:
                    for j in supp[b]:
                        out.add((i, j))
    return out
