"""Independent brute-force energy evaluator for tiny B-spline sheets (a pin for the oracle).

Written separately from ``oracle/``: its own Cox-de Boor recursion (pure Python), its own
quadrature lists built from the wording of Sec. 4.1/4.2, and derivatives taken from the exact
quadratic interpolant of each basis piece (three samples inside the span) instead of the
derivative recursion. Affine rest maps only: d(u,v)/dX is the inverse of the constant
Jacobian, obtained by differencing the rest surface. Energy only; tests take finite
differences of it. Slow by design (N <= 8).
"""
from __future__ import annotations

import math

import numpy as np


def cox_de_boor(xi, i, p, u):
    if p == 0:
        return 1.0 if xi[i] <= u < xi[i + 1] else 0.0
    a = 0.0
    if xi[i + p] != xi[i]:
        a = (u - xi[i]) / (xi[i + p] - xi[i]) * cox_de_boor(xi, i, p - 1, u)
    b = 0.0
    if xi[i + p + 1] != xi[i + 1]:
        b = (xi[i + p + 1] - u) / (xi[i + p + 1] - xi[i + 1]) * cox_de_boor(xi, i + 1, p - 1, u)
    return a + b


def piece_poly(xi, i, k):
    """Coefficients (c0, c1, c2) of basis i on span [k, k+1] in t = u - k (unit knots)."""
    ts = np.array([0.2, 0.5, 0.8])
    vals = [cox_de_boor(xi, i, 2, k + t) for t in ts]
    V = np.vander(ts, 3, increasing=True)
    return np.linalg.solve(V, vals)


def piece_eval(c, t, d):
    if d == 0:
        return c[0] + c[1] * t + c[2] * t * t
    if d == 1:
        return c[1] + 2 * c[2] * t
    return 2 * c[2]


class Tiny:
    def __init__(self, n_u, n_v, rest, membrane_params, mu_bend, rho_area):
        self.n_u, self.n_v = n_u, n_v
        self.Nu, self.Nv = n_u - 2, n_v - 2
        self.xu = [0.0, 0.0] + list(range(self.Nu + 1)) + [self.Nu, self.Nu]
        self.xv = [0.0, 0.0] + list(range(self.Nv + 1)) + [self.Nv, self.Nv]
        self.rest = np.asarray(rest, dtype=float)
        self.E, self.nu, self.t = membrane_params
        self.mu_bend = mu_bend
        self.rho = rho_area
        self.cu = {(i, k): piece_poly(self.xu, i, k) for k in range(self.Nu) for i in range(k, k + 3)}
        self.cv = {(j, l): piece_poly(self.xv, j, l) for l in range(self.Nv) for j in range(l, l + 3)}
        # constant Jacobian of the affine rest map from differences of the rest surface
        X00 = self.surface(self.rest, 0.5, 0.5)
        J = np.stack([self.surface(self.rest, 1.5, 0.5) - X00, self.surface(self.rest, 0.5, 1.5) - X00], axis=1)
        self.K = np.linalg.inv(J)
        self.detJ = abs(np.linalg.det(J))

    def surface(self, C, u, v):
        out = 0.0
        for j in range(self.n_v):
            for i in range(self.n_u):
                w = cox_de_boor(self.xu, i, 2, u) * cox_de_boor(self.xv, j, 2, v)
                if w:
                    out = out + w * np.asarray(C[j * self.n_u + i])
        return out

    def derivs(self, C, k, l, u, v):
        """Parametric derivatives of phi on span (k, l): value, u, v, uu, vv, uv."""
        tu, tv = u - k, v - l
        out = {key: 0.0 for key in ("d0", "u", "v", "uu", "vv", "uv")}
        for b in range(3):
            j = l + b
            cv = self.cv[(j, l)]
            for a in range(3):
                i = k + a
                cu = self.cu[(i, k)]
                P = np.asarray(C[j * self.n_u + i])
                out["u"] = out["u"] + piece_eval(cu, tu, 1) * piece_eval(cv, tv, 0) * P
                out["v"] = out["v"] + piece_eval(cu, tu, 0) * piece_eval(cv, tv, 1) * P
                out["uu"] = out["uu"] + piece_eval(cu, tu, 2) * piece_eval(cv, tv, 0) * P
                out["vv"] = out["vv"] + piece_eval(cu, tu, 0) * piece_eval(cv, tv, 2) * P
                out["uv"] = out["uv"] + piece_eval(cu, tu, 1) * piece_eval(cv, tv, 1) * P
        return out

    # quadrature, rebuilt from the wording of the paper (span units)
    def membrane_points(self, full_gauss=False, rule="reduced"):
        """rule: "reduced" (Sec. 4.1), or the comparison rules of Sec. 6.5: "gauss2" (2x2 on the
        interior spans), "interior1" (one midpoint per interior span), "corner2" (2x2 on the
        corner spans instead of 3x3)."""
        g2 = 0.5 / math.sqrt(3.0)
        g3 = 0.5 * math.sqrt(0.6)
        G = {1: [(0.0, 1.0)], 2: [(-g2, 0.5), (g2, 0.5)], 3: [(-g3, 5 / 18), (0.0, 8 / 18), (g3, 5 / 18)]}
        pts = []
        Nu, Nv = self.Nu, self.Nv
        for l in range(Nv):
            for k in range(Nu):
                on_u = k in (0, Nu - 1)
                on_v = l in (0, Nv - 1)
                if full_gauss:
                    nu_, nv_ = 3, 3
                elif on_u and on_v and rule == "corner2":
                    nu_, nv_ = 2, 2
                elif on_u or on_v:
                    nu_, nv_ = (3 if on_u else 2), (3 if on_v else 2)
                elif rule == "gauss2":
                    nu_, nv_ = 2, 2
                elif rule == "interior1":
                    nu_, nv_ = 1, 1
                else:
                    continue
                for ou, wu in G[nu_]:
                    for ov, wv in G[nv_]:
                        pts.append((k + 0.5 + ou, l + 0.5 + ov, wu * wv, k, l))
        if full_gauss or rule in ("gauss2", "interior1"):
            return pts
        for b in range(1, Nv):
            for a in range(1, Nu):
                hu = a in (1, Nu - 1)
                hv = b in (1, Nv - 1)
                if hu and hv:
                    cand = [(a, b, 0.25)]
                elif hu:
                    cand = [(a, b - g2, 0.25), (a, b + g2, 0.25)]
                elif hv:
                    cand = [(a - g2, b, 0.25), (a + g2, b, 0.25)]
                elif (a + b) % 2 == 0:
                    cand = [(a, b - g2, 0.5), (a, b + g2, 0.5)]
                else:
                    cand = [(a - g2, b, 0.5), (a + g2, b, 0.5)]
                for u, v, w in cand:
                    pts.append((u, v, w, min(int(math.floor(u)), Nu - 1), min(int(math.floor(v)), Nv - 1)))
        return pts

    def bending_points(self, full_gauss=False, rule="reduced"):
        pts = []
        Nu, Nv = self.Nu, self.Nv
        if rule == "gauss2":                   # span centres on the boundary ring, 2x2 inside
            g2 = 0.5 / math.sqrt(3.0)
            for l in range(Nv):
                for k in range(Nu):
                    if k in (0, Nu - 1) or l in (0, Nv - 1):
                        pts.append((k + 0.5, l + 0.5, 1.0, k, l))
                    else:
                        for ou in (-g2, g2):
                            for ov in (-g2, g2):
                                pts.append((k + 0.5 + ou, l + 0.5 + ov, 0.25, k, l))
            return pts
        if full_gauss:
            g3 = 0.5 * math.sqrt(0.6)
            G = [(-g3, 5 / 18), (0.0, 8 / 18), (g3, 5 / 18)]
            for l in range(Nv):
                for k in range(Nu):
                    for ou, wu in G:
                        for ov, wv in G:
                            pts.append((k + 0.5 + ou, l + 0.5 + ov, wu * wv, k, l))
            return pts
        for l in range(Nv):
            for k in range(Nu):
                if k in (0, Nu - 1) or l in (0, Nv - 1):
                    pts.append((k + 0.5, l + 0.5, 1.0, k, l))
        for b in range(1, Nv):
            for a in range(1, Nu):
                w = (0.5 if a in (1, Nu - 1) else 1.0) * (0.5 if b in (1, Nv - 1) else 1.0)
                for k, l in ((a - 1, b - 1), (a, b - 1), (a - 1, b), (a, b)):
                    pts.append((a, b, w / 4, k, l))
        return pts

    def stvk(self, F):
        mu = self.E * self.t / (2 * (1 + self.nu))
        lam = self.E * self.t * self.nu / (1 - self.nu ** 2)
        Eg = 0.5 * (F.T @ F - np.eye(2))
        return mu * np.sum(Eg * Eg) + 0.5 * lam * np.trace(Eg) ** 2

    def elastic_energy(self, x, full_gauss=False, rule="reduced"):
        x = np.asarray(x, dtype=float)
        K = self.K
        total = 0.0
        for u, v, w, k, l in self.membrane_points(full_gauss, rule):
            d = self.derivs(x, k, l, u, v)
            F = np.stack([d["u"] * K[0, 0] + d["v"] * K[1, 0], d["u"] * K[0, 1] + d["v"] * K[1, 1]], axis=1)
            total += w * self.detJ * self.stvk(F)
        c_uu = K[0, 0] ** 2 + K[0, 1] ** 2
        c_vv = K[1, 0] ** 2 + K[1, 1] ** 2
        c_uv = 2 * (K[0, 0] * K[1, 0] + K[0, 1] * K[1, 1])
        for u, v, w, k, l in self.bending_points(full_gauss, rule):
            d = self.derivs(x, k, l, u, v)
            lap = c_uu * d["uu"] + c_vv * d["vv"] + c_uv * d["uv"]
            total += w * self.detJ * 0.5 * self.mu_bend * float(np.dot(lap, lap))
        return total
