// geom.h -- device-side basis pieces and rest-map geometry, shared by the evaluation and the
// solver kernels. Included inside namespace bsc::{anonymous} of each .hip file.
//
// Quadratic B-splines on open uniform knots (Eq. "B-spline basis"): on span k of N spans the
// three nonzero basis functions are one of three pieces (first span, inner, last span), in the
// local coordinate t in [0, 1] (span units).
//
// Rest geometry (Sec. 4.1 inverse function theorem, Sec. 4.2 Laplacian in parametric space):
// for an affine rest map X = A (u, v) + b the inverse Jacobian K = A^{-1} and the Laplacian
// coefficients are sheet constants. For a general rest map they are tabulated per quadrature
// point at create: K for membrane points, (c_uu, c_vv, c_uv, l_u, l_v) for bending
// evaluations, where Lap_X f = c_uu f_uu + c_vv f_vv + c_uv f_uv + l_u f_u + l_v f_v.
#pragma once

enum { kFirst = 0, kInner = 1, kLast = 2 };

__device__ __forceinline__ int span_type(int k, int N) { return k == 0 ? kFirst : (k == N - 1 ? kLast : kInner); }

// Values and first derivatives of the three quadratic pieces on a span (local t in [0,1]).
template <typename T>
__device__ __forceinline__ void pieces(int type, T t, T N[3], T D[3]) {
    const T s = T(1) - t;
    if (type == kInner) {
        N[0] = T(0.5) * s * s; N[1] = T(0.5) + t * s; N[2] = T(0.5) * t * t;
        D[0] = -s; D[1] = s - t; D[2] = t;
    } else if (type == kFirst) {
        N[0] = s * s; N[1] = t * (T(2) - T(1.5) * t); N[2] = T(0.5) * t * t;
        D[0] = T(-2) * s; D[1] = T(2) - T(3) * t; D[2] = t;
    } else {
        N[0] = T(0.5) * s * s; N[1] = s * (T(2) - T(1.5) * s); N[2] = t * t;
        D[0] = -s; D[1] = T(1) - T(3) * t; D[2] = T(2) * t;
    }
}

// Second derivatives of the three pieces (constant on a span).
__device__ __forceinline__ void second(int type, double D2[3]) {
    if (type == kInner) { D2[0] = 1.0; D2[1] = -2.0; D2[2] = 1.0; }
    else if (type == kFirst) { D2[0] = 2.0; D2[1] = -3.0; D2[2] = 1.0; }
    else { D2[0] = 1.0; D2[1] = -3.0; D2[2] = 2.0; }
}

// Value, first and second derivative of local piece a (0..2) alone, selected without indexing
// a local array (a runtime index into one would place it in scratch memory).
template <typename T>
__device__ __forceinline__ void piece_at(int type, int a, T t, T &n, T &d, T &d2) {
    const T s = T(1) - t;
    T n0, n1, n2, e0, e1, e2, f0, f1, f2;
    if (type == kInner) {
        n0 = T(0.5) * s * s; n1 = T(0.5) + t * s; n2 = T(0.5) * t * t;
        e0 = -s; e1 = s - t; e2 = t;
        f0 = T(1); f1 = T(-2); f2 = T(1);
    } else if (type == kFirst) {
        n0 = s * s; n1 = t * (T(2) - T(1.5) * t); n2 = T(0.5) * t * t;
        e0 = T(-2) * s; e1 = T(2) - T(3) * t; e2 = t;
        f0 = T(2); f1 = T(-3); f2 = T(1);
    } else {
        n0 = T(0.5) * s * s; n1 = s * (T(2) - T(1.5) * s); n2 = t * t;
        e0 = -s; e1 = T(1) - T(3) * t; e2 = T(2) * t;
        f0 = T(1); f1 = T(-3); f2 = T(2);
    }
    n = a == 0 ? n0 : (a == 1 ? n1 : n2);
    d = a == 0 ? e0 : (a == 1 ? e1 : e2);
    d2 = a == 0 ? f0 : (a == 1 ? f1 : f2);
}

// Inverse Jacobian K[m][b] = d xi_m / d X_b at membrane point q.
struct PtK { double k00, k01, k10, k11; };

template <bool CURVED>
__device__ __forceinline__ PtK mp_geo_t(const DevSheet &S, int q) {
    if (CURVED) {
        const size_t n = S.n_mp;
        return {S.mp_K[q], S.mp_K[n + q], S.mp_K[2 * n + q], S.mp_K[3 * n + q]};
    }
    return {S.K00, S.K01, S.K10, S.K11};
}

__device__ __forceinline__ PtK mp_geo(const DevSheet &S, int q) {
    return S.curved ? mp_geo_t<true>(S, q) : mp_geo_t<false>(S, q);
}

// Laplacian coefficients at bending evaluation q.
struct PtL { double cuu, cvv, cuv, lu, lv; };

template <bool CURVED>
__device__ __forceinline__ PtL be_geo_t(const DevSheet &S, int q) {
    if (CURVED) {
        const size_t n = S.n_be;
        return {S.be_L[q], S.be_L[n + q], S.be_L[2 * n + q], S.be_L[3 * n + q], S.be_L[4 * n + q]};
    }
    return {S.c_uu, S.c_vv, S.c_uv, 0.0, 0.0};
}

__device__ __forceinline__ PtL be_geo(const DevSheet &S, int q) {
    return S.curved ? be_geo_t<true>(S, q) : be_geo_t<false>(S, q);
}

// Gradient w.r.t. X of local basis function (a, b) of span (k, l) at (tu, tv).
template <typename T>
__device__ __forceinline__ void grad_at(const DevSheet &S, const PtK &K, int k, int l, int a, int b, T tu, T tv, T g[2]) {
    T nu, du, d2u, nv, dv, d2v;
    piece_at<T>(span_type(k, S.Nu), a, tu, nu, du, d2u);
    piece_at<T>(span_type(l, S.Nv), b, tv, nv, dv, d2v);
    const T xu = du * nv, xv = nu * dv;
    g[0] = xu * T(K.k00) + xv * T(K.k10);
    g[1] = xu * T(K.k01) + xv * T(K.k11);
}

// Gradient w.r.t. X of the 9 local basis functions at span coordinates (tu, tv).
template <typename T>
__device__ __forceinline__ void local_grads(const DevSheet &S, const PtK &K, int k, int l, T tu, T tv, T dN[9][2]) {
    T Nu[3], Du[3], Nv[3], Dv[3];
    pieces<T>(span_type(k, S.Nu), tu, Nu, Du);
    pieces<T>(span_type(l, S.Nv), tv, Nv, Dv);
    const T K00 = T(K.k00), K01 = T(K.k01), K10 = T(K.k10), K11 = T(K.k11);
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const T du = Du[a] * Nv[b], dv = Nu[a] * Dv[b];
            dN[3 * b + a][0] = du * K00 + dv * K10;
            dN[3 * b + a][1] = du * K01 + dv * K11;
        }
}

template <typename T>
__device__ __forceinline__ void one_grad(const DevSheet &S, const PtK &K, int k, int l, int a, int b, T tu, T tv, T g[2]) {
    T Nu[3], Du[3], Nv[3], Dv[3];
    pieces<T>(span_type(k, S.Nu), tu, Nu, Du);
    pieces<T>(span_type(l, S.Nv), tv, Nv, Dv);
    const T du = Du[a] * Nv[b], dv = Nu[a] * Dv[b];
    g[0] = du * T(K.k00) + dv * T(K.k10);
    g[1] = du * T(K.k01) + dv * T(K.k11);
}

// Laplacian coefficients L of the 9 local CPs for a bending evaluation (FIRST: with the
// first-derivative terms of a general rest map; they vanish for an affine rest).
template <bool FIRST>
__device__ __forceinline__ void bend_L_t(const DevSheet &S, const PtL &G, int k, int l, double tu, double tv, double L[9]) {
    double Nu[3], Du[3], D2u[3], Nv[3], Dv[3], D2v[3];
    const int tyu = span_type(k, S.Nu), tyv = span_type(l, S.Nv);
    pieces<double>(tyu, tu, Nu, Du);
    pieces<double>(tyv, tv, Nv, Dv);
    second(tyu, D2u);
    second(tyv, D2v);
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            L[3 * b + a] = G.cuu * D2u[a] * Nv[b] + G.cvv * Nu[a] * D2v[b] + G.cuv * Du[a] * Dv[b];
            if (FIRST) L[3 * b + a] += G.lu * Du[a] * Nv[b] + G.lv * Nu[a] * Dv[b];
        }
}

__device__ __forceinline__ void bend_L(const DevSheet &S, const PtL &G, int k, int l, double tu, double tv, double L[9]) {
    if (S.curved) bend_L_t<true>(S, G, k, l, tu, tv, L);
    else bend_L_t<false>(S, G, k, l, tu, tv, L);
}

__device__ __forceinline__ double greville(int i, int n) {
    return i == 0 ? 0.0 : (i == n - 1 ? double(n - 2) : double(i) - 0.5);
}

// Displacement of CP (i,j) from its rest position embedded in the plane z = 0.
template <bool CURVED>
__device__ __forceinline__ void displacement_t(const DevSheet &S, const double *x, int i, int j, double d[3]) {
    const int a = j * S.n_u + i;
    double X0, X1;
    if (CURVED) {
        X0 = S.rest[a];
        X1 = S.rest[S.n_cp + a];
    } else {
        const double gu = greville(i, S.n_u), gv = greville(j, S.n_v);
        X0 = S.A00 * gu + S.A01 * gv + S.b0;
        X1 = S.A10 * gu + S.A11 * gv + S.b1;
    }
    d[0] = x[a] - X0;
    d[1] = x[S.n_cp + a] - X1;
    d[2] = x[2 * S.n_cp + a];
}

__device__ __forceinline__ void displacement(const DevSheet &S, const double *x, int i, int j, double d[3]) {
    if (S.curved) displacement_t<true>(S, x, i, j, d);
    else displacement_t<false>(S, x, i, j, d);
}
