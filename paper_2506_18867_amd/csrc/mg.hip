// mg.hip -- multigrid preconditioner for the Newton systems, built on the B-spline hierarchy.
//
// Halving the knot spans of a quadratic B-spline patch (knot insertion at every span midpoint)
// represents each coarse basis function exactly by at most four fine ones per direction, with
// weights (1/4, 3/4, 3/4, 1/4) inside and (1, 1/2) / (1/2, 3/4, 1/4) at the open ends. With this
// exact prolongation P (tensor product, rows of pinned CPs zeroed), the Galerkin operators
// P^T A P of the Newton Hessian are again 5x5-stencil block matrices, stored in the same
// symmetric upper-stencil layout as the fine Hessian. They are formed every Newton iteration by
// two one-dimensional passes (u, then v). The preconditioner is one symmetric V(1,1) cycle:
// damped block-Jacobi smoothing (weight 1/3: lambda_max(D^-1 A) stays between 2.2 and 3.6 on
// the sheets of this library, so the smoother contracts with a margin), down to a grid whose span
// count is odd, where one smoothing sweep stands for the coarse solve. The outer solver is the
// standard preconditioned CG, its scalars reduced in every block in a fixed order (no atomics);
// the stop test, the iteration count and a breakdown flag live on the device as for the
// block-Jacobi solver, so the same burst loop drives both.
//
// The paper solves its Newton systems with a sparse Cholesky factorisation (Sec. 5.3); this
// preconditioner is part of the GPU design, not of the paper's method.
#include "bsc_internal.h"

namespace bsc {
namespace {

constexpr int kMgBlock = 256;
constexpr double kMgOmega = 1.0 / 3.0;


inline unsigned grid(size_t n) { return unsigned((n + kMgBlock - 1) / kMgBlock); }

__device__ __forceinline__ double mg_block_sum(double v, double *sh) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    const int nw = (blockDim.x + 63) >> 6;
    v = (int(threadIdx.x) < nw) ? sh[threadIdx.x] : 0.0;
    if (wid == 0) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
    }
    return v;                                   // valid in thread 0
}

// Sum of n partials, the same in every block (fixed assignment and order), broadcast.
__device__ double mg_all_sum(const double *__restrict__ part, int n, double *sh, double *bc) {
    double v = 0.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) v += part[t];
    v = mg_block_sum(v, sh);
    if (threadIdx.x == 0) *bc = v;
    __syncthreads();
    const double out = *bc;
    __syncthreads();
    return out;
}

// Prolongation weight P(f, J) of the midpoint refinement: fine CP f (nf = 2 nc - 2 CPs) and
// coarse CP J (nc CPs), one direction.
__device__ __forceinline__ double pw(int f, int J, int nc) {
    const int nf = 2 * nc - 2;
    if (f == 0) return J == 0 ? 1.0 : 0.0;
    if (f == 1) return (J == 0 || J == 1) ? 0.5 : 0.0;
    if (f == nf - 1) return J == nc - 1 ? 1.0 : 0.0;
    if (f == nf - 2) return (J == nc - 2 || J == nc - 1) ? 0.5 : 0.0;
    const int k = f >> 1;
    if (J == k) return (f & 1) ? 0.25 : 0.75;
    if (J == k + 1) return (f & 1) ? 0.75 : 0.25;
    return 0.0;
}

// 3x3 block A(a, a + d) of a symmetric upper-stencil matrix on an nu x nv grid, row-major;
// |d| <= 2 per direction and a + d inside the grid.
template <typename T>
__device__ __forceinline__ void hget(const T *__restrict__ H, int nu, int nv, int ai, int aj, int di, int dj, double out[9]) {
    const size_t n = size_t(nu) * nv;
    if (di == 0 && dj == 0) {
        const size_t a = size_t(aj) * nu + ai;
        const double e0 = H[a], e1 = H[n + a], e2 = H[2 * n + a], e3 = H[3 * n + a], e4 = H[4 * n + a], e5 = H[5 * n + a];
        out[0] = e0; out[1] = e1; out[2] = e2; out[3] = e1; out[4] = e3; out[5] = e4; out[6] = e2; out[7] = e4; out[8] = e5;
        return;
    }
    const int s = upper_slot(di, dj);
    if (s > 0) {
        const size_t a = size_t(aj) * nu + ai, e = slot_entry(s);
#pragma unroll
        for (int k = 0; k < 9; ++k) out[k] = H[(e + k) * n + a];
    } else {
        const int s2 = upper_slot(-di, -dj);
        const size_t b = size_t(aj + dj) * nu + (ai + di), e = slot_entry(s2);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) out[3 * r + c] = H[(e + 3 * c + r) * n + b];
    }
}

template <typename T>
__device__ __forceinline__ void hput(T *__restrict__ H, size_t n, size_t a, int s, const double v[9]) {
    if (s == 0) {
        H[a] = T(v[0]); H[n + a] = T(v[1]); H[2 * n + a] = T(v[2]);
        H[3 * n + a] = T(v[4]); H[4 * n + a] = T(v[5]); H[5 * n + a] = T(v[8]);
    } else {
        const size_t e = slot_entry(s);
#pragma unroll
        for (int k = 0; k < 9; ++k) H[(e + k) * n + a] = T(v[k]);
    }
}

// Galerkin pass along u: the fine grid nuf x nv to the intermediate grid nuc x nv. One thread
// per (row, upper slot). Pinned fine CPs (level 0) are left out (their prolongation rows are 0).
template <typename T>
__global__ void __launch_bounds__(kMgBlock) k_mg_pass_u(int nuf, int nv, int nuc, const T *__restrict__ Hf, T *__restrict__ Hm,
                                                        const int32_t *__restrict__ pinmask) {
    const size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const size_t nm = size_t(nuc) * nv;
    if (t >= nm * kSlots) return;
    const int s = int(t / nm);
    const size_t row = t % nm;
    const int I = int(row % nuc), j = int(row / nuc);
    const int du = slot_di(s), dv = slot_dj(s), I2 = I + du, j2 = j + dv;
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (I2 >= 0 && I2 < nuc && j2 < nv) {
        for (int f = max(0, 2 * I - 2); f <= min(nuf - 1, 2 * I + 1); ++f) {
            const double w1 = pw(f, I, nuc);
            if (w1 == 0.0 || (pinmask && pinmask[size_t(j) * nuf + f])) continue;
            for (int g = max(max(0, 2 * I2 - 2), f - 2); g <= min(min(nuf - 1, 2 * I2 + 1), f + 2); ++g) {
                const double w2 = pw(g, I2, nuc);
                if (w2 == 0.0 || (pinmask && pinmask[size_t(j2) * nuf + g])) continue;
                double b[9];
                hget<T>(Hf, nuf, nv, f, j, g - f, dv, b);
                const double w = w1 * w2;
#pragma unroll
                for (int k = 0; k < 9; ++k) acc[k] += w * b[k];
            }
        }
    }
    hput<T>(Hm, nm, row, s, acc);
}

// Galerkin pass along v: the intermediate grid nuc x nvf to the coarse grid nuc x nvc.
template <typename T>
__global__ void __launch_bounds__(kMgBlock) k_mg_pass_v(int nuc, int nvf, int nvc, const T *__restrict__ Hm, T *__restrict__ Hc) {
    const size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const size_t nc = size_t(nuc) * nvc;
    if (t >= nc * kSlots) return;
    const int s = int(t / nc);
    const size_t row = t % nc;
    const int I = int(row % nuc), J = int(row / nuc);
    const int du = slot_di(s), dv = slot_dj(s), I2 = I + du, J2 = J + dv;
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (I2 >= 0 && I2 < nuc && J2 < nvc) {
        for (int c = max(0, 2 * J - 2); c <= min(nvf - 1, 2 * J + 1); ++c) {
            const double w1 = pw(c, J, nvc);
            if (w1 == 0.0) continue;
            for (int d = max(max(0, 2 * J2 - 2), c - 2); d <= min(min(nvf - 1, 2 * J2 + 1), c + 2); ++d) {
                const double w2 = pw(d, J2, nvc);
                if (w2 == 0.0) continue;
                double b[9];
                hget<T>(Hm, nuc, nvf, I, c, du, d - c, b);
                const double w = w1 * w2;
#pragma unroll
                for (int k = 0; k < 9; ++k) acc[k] += w * b[k];
            }
        }
    }
    hput<T>(Hc, nc, row, s, acc);
}

// Inverse diagonal blocks (symmetric, 6 entries); a block that is not positive definite (a coarse
// CP whose fine children are all pinned has a zero block) falls back to the inverse diagonal or
// the identity.
template <typename T>
__global__ void k_mg_pinv(int n, const T *__restrict__ H, T *__restrict__ pinv) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    const size_t N = n;
    const double a00 = H[a], a01 = H[N + a], a02 = H[2 * N + a], a11 = H[3 * N + a], a12 = H[4 * N + a], a22 = H[5 * N + a];
    const double c00 = a11 * a22 - a12 * a12, c01 = a02 * a12 - a01 * a22, c02 = a01 * a12 - a02 * a11;
    const double det = a00 * c00 + a01 * c01 + a02 * c02;
    double inv[6];
    if (det > 0.0 && a00 > 0.0) {
        const double id = 1.0 / det;
        inv[0] = c00 * id; inv[1] = c01 * id; inv[2] = c02 * id;
        inv[3] = (a00 * a22 - a02 * a02) * id; inv[4] = (a02 * a01 - a00 * a12) * id; inv[5] = (a00 * a11 - a01 * a01) * id;
    } else {
        inv[0] = a00 > 0.0 ? 1.0 / a00 : 1.0; inv[1] = inv[2] = 0.0;
        inv[3] = a11 > 0.0 ? 1.0 / a11 : 1.0; inv[4] = 0.0; inv[5] = a22 > 0.0 ? 1.0 / a22 : 1.0;
    }
    for (int k = 0; k < 6; ++k) pinv[k * N + a] = T(inv[k]);
}

// y = D^-1 v at CP a (symmetric 3x3 inverse, 6 entries).
template <typename T>
__device__ __forceinline__ void dinv(const T *__restrict__ pinv, size_t n, size_t a, const double v[3], double y[3]) {
    const double i0 = pinv[a], i1 = pinv[n + a], i2 = pinv[2 * n + a], i3 = pinv[3 * n + a], i4 = pinv[4 * n + a],
                 i5 = pinv[5 * n + a];
    y[0] = i0 * v[0] + i1 * v[1] + i2 * v[2];
    y[1] = i1 * v[0] + i3 * v[1] + i4 * v[2];
    y[2] = i2 * v[0] + i4 * v[1] + i5 * v[2];
}


// Tiled stencil products: 64 rows per workgroup, 8 waves, wave g forms the block products
// g, g + 8, g + 16, g + 24 (0: diagonal, 1..12 upper, 13..24 lower) and the partial sums meet in
// LDS, as in the library's plain SpMV. The epilogue (wave 0) depends on the mode.
constexpr int kTileRows = 64, kTileWaves = 8;
enum { MG_RESID = 0, MG_POST = 1, MG_Q = 2 };

template <typename T>
__device__ __forceinline__ void mg_block_product(int nu, int nv, const T *__restrict__ H, const double *__restrict__ u, int a,
                                                 int i, int j, int pid, T acc[3]) {
    const size_t n = size_t(nu) * nv;
    if (pid == 0) {
        const T u0 = T(u[a]), u1 = T(u[n + a]), u2 = T(u[2 * n + a]);
        const T d0 = H[a], d1 = H[n + a], d2 = H[2 * n + a], d3 = H[3 * n + a], d4 = H[4 * n + a], d5 = H[5 * n + a];
        acc[0] += d0 * u0 + d1 * u1 + d2 * u2;
        acc[1] += d1 * u0 + d3 * u1 + d4 * u2;
        acc[2] += d2 * u0 + d4 * u1 + d5 * u2;
        return;
    }
    const bool upper = pid <= 12;
    const int s = upper ? pid : pid - 12;
    const int di = slot_di(s), dj = slot_dj(s), e0 = slot_entry(s);
    if (upper) {
        const int ib = i + di, jb = j + dj;
        if (ib < 0 || ib >= nu || jb >= nv) return;
        const int b = jb * nu + ib;
        const T u0 = T(u[b]), u1 = T(u[n + b]), u2 = T(u[2 * n + b]);
#pragma unroll
        for (int r = 0; r < 3; ++r)
            acc[r] += H[(e0 + 3 * r) * n + a] * u0 + H[(e0 + 3 * r + 1) * n + a] * u1 + H[(e0 + 3 * r + 2) * n + a] * u2;
    } else {
        const int ic = i - di, jc = j - dj;
        if (ic < 0 || ic >= nu || jc < 0) return;
        const int b = jc * nu + ic;
        const T u0 = T(u[b]), u1 = T(u[n + b]), u2 = T(u[2 * n + b]);
#pragma unroll
        for (int c = 0; c < 3; ++c)
            acc[c] += H[(e0 + c) * n + b] * u0 + H[(e0 + 3 + c) * n + b] * u1 + H[(e0 + 6 + c) * n + b] * u2;
    }
}

// RESID: out = r - A u.  POST: out = u + omega D^-1 (r - A u), partials of r . out.
// Q: out = A u, partials of u . out.
template <typename T, int MODE>
__global__ void __launch_bounds__(kTileRows * kTileWaves) k_mg_apply(int nu, int nv, const T *__restrict__ H,
                                                                     const T *__restrict__ pinv, const double *__restrict__ u,
                                                                     const double *__restrict__ r, double *__restrict__ out,
                                                                     double *__restrict__ part, const int32_t *__restrict__ isc) {
    __shared__ T ys[kTileWaves][3][kTileRows];
    if (isc[I_DONE]) return;
    const int n = nu * nv;
    const int g = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int a = blockIdx.x * kTileRows + lane;
    T acc[3] = {T(0), T(0), T(0)};
    if (a < n) {
        const int i = a % nu, j = a / nu;
        for (int m = 0; m < 4; ++m) {
            const int pid = g + kTileWaves * m;
            if (pid < 25) mg_block_product<T>(nu, nv, H, u, a, i, j, pid, acc);
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) ys[g][c][lane] = acc[c];
    __syncthreads();
    if (g != 0) return;
    double dot = 0.0;
    if (a < n) {
        double y[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T v = ys[0][c][lane];
#pragma unroll
            for (int q = 1; q < kTileWaves; ++q) v += ys[q][c][lane];
            y[c] = double(v);
        }
        const size_t N = n;
        if (MODE == MG_RESID) {
#pragma unroll
            for (int c = 0; c < 3; ++c) out[c * N + a] = r[c * N + a] - y[c];
        } else if (MODE == MG_POST) {
            double v[3], d[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) v[c] = r[c * N + a] - y[c];
            dinv<T>(pinv, N, a, v, d);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double o = u[c * N + a] + kMgOmega * d[c];
                out[c * N + a] = o;
                dot += r[c * N + a] * o;
            }
        } else {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                out[c * N + a] = y[c];
                dot += u[c * N + a] * y[c];
            }
        }
    }
    if (MODE != MG_RESID && part) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) dot += __shfl_down(dot, off);
        if (lane == 0) part[blockIdx.x] = dot;
    }
}

inline unsigned tiles(size_t n) { return unsigned((n + kTileRows - 1) / kTileRows); }

// x = omega D^-1 r
template <typename T>
__global__ void __launch_bounds__(kMgBlock) k_mg_smooth0(int n, const T *__restrict__ pinv, const double *__restrict__ r,
                                                         double *__restrict__ x, const int32_t *__restrict__ isc) {
    if (isc[I_DONE]) return;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    const double v[3] = {r[a], r[size_t(n) + a], r[2 * size_t(n) + a]};
    double y[3];
    dinv<T>(pinv, n, a, v, y);
    for (int c = 0; c < 3; ++c) x[c * size_t(n) + a] = kMgOmega * y[c];
}


// rc = P^T t (coarse grid nuc x nvc from the fine grid nuf x nvf)
__global__ void __launch_bounds__(kMgBlock) k_mg_restrict(int nuf, int nvf, int nuc, int nvc, const double *__restrict__ t,
                                                          double *__restrict__ rc, const int32_t *__restrict__ isc) {
    if (isc[I_DONE]) return;
    const int J = blockIdx.x * blockDim.x + threadIdx.x;
    const int nc = nuc * nvc;
    if (J >= nc) return;
    const int I = J % nuc, K = J / nuc;
    const size_t nf = size_t(nuf) * nvf;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int fv = max(0, 2 * K - 2); fv <= min(nvf - 1, 2 * K + 1); ++fv) {
        const double wv = pw(fv, K, nvc);
        if (wv == 0.0) continue;
        for (int fu = max(0, 2 * I - 2); fu <= min(nuf - 1, 2 * I + 1); ++fu) {
            const double w = wv * pw(fu, I, nuc);
            if (w == 0.0) continue;
            const size_t f = size_t(fv) * nuf + fu;
            for (int c = 0; c < 3; ++c) acc[c] += w * t[c * nf + f];
        }
    }
    for (int c = 0; c < 3; ++c) rc[c * size_t(nc) + J] = acc[c];
}

// x += P e (fine grid), except at pinned CPs (level 0)
__global__ void __launch_bounds__(kMgBlock) k_mg_prolong(int nuf, int nvf, int nuc, int nvc, const double *__restrict__ e,
                                                         double *__restrict__ x, const int32_t *__restrict__ pinmask,
                                                         const int32_t *__restrict__ isc) {
    if (isc[I_DONE]) return;
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    const int nf = nuf * nvf;
    if (f >= nf || (pinmask && pinmask[f])) return;
    const int fu = f % nuf, fv = f / nuf;
    const size_t nc = size_t(nuc) * nvc;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int K = max(0, (fv - 1) >> 1); K <= min(nvc - 1, (fv >> 1) + 1); ++K) {
        const double wv = pw(fv, K, nvc);
        if (wv == 0.0) continue;
        for (int I = max(0, (fu - 1) >> 1); I <= min(nuc - 1, (fu >> 1) + 1); ++I) {
            const double w = wv * pw(fu, I, nuc);
            if (w == 0.0) continue;
            const size_t J = size_t(K) * nuc + I;
            for (int c = 0; c < 3; ++c) acc[c] += w * e[c * nc + J];
        }
    }
    for (int c = 0; c < 3; ++c) x[c * size_t(nf) + f] += acc[c];
}


// ---- preconditioned CG (the standard form, one preconditioner application per iteration) ----

// Stop test on |r|^2 (per-block partials; at the first iteration |b|^2, which also sets the
// tolerance), iteration count, done flag.
__global__ void __launch_bounds__(kMgBlock) k_mgcg_stop(int nb, const double *__restrict__ rr_part, double *scal, int32_t *isc) {
    __shared__ double sh[kMgBlock / 64];
    __shared__ double bc;
    if (isc[I_DONE]) return;
    const double rr = mg_all_sum(rr_part, nb, sh, &bc);
    if (threadIdx.x == 0) {
        const int it = isc[I_ITA];
        if (it == 0) scal[S_TOL2] = scal[S_RTOL] * scal[S_RTOL] * rr;
        scal[S_RHO] = rr;
        if (rr <= scal[S_TOL2] || it >= isc[I_MAXIT] || !(rr == rr)) {
            isc[I_ITERS] = it;
            isc[I_DONE] = 1;
        } else {
            isc[I_ITA] = it + 1;
        }
    }
}

// rho_i = r . z (partials from the last smoothing kernel); beta = rho_i / rho_{i-1}; p = z + beta p.
// rho is double-buffered by iteration parity so that no block reads what another writes.
__global__ void __launch_bounds__(kMgBlock) k_mgcg_p(int n3, int nb, const double *__restrict__ rz_part, double *scal,
                                                     const int32_t *__restrict__ isc, const double *__restrict__ z,
                                                     double *__restrict__ p) {
    __shared__ double sh[kMgBlock / 64];
    __shared__ double bc;
    if (isc[I_DONE]) return;
    const double rho = mg_all_sum(rz_part, nb, sh, &bc);
    const int it = isc[I_ITA];                    // 1 at the first iteration
    const double beta = it == 1 ? 0.0 : rho / scal[S_MGRHO0 + ((it - 1) & 1)];
    if (blockIdx.x == 0 && threadIdx.x == 0) scal[S_MGRHO0 + (it & 1)] = rho;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n3) p[t] = z[t] + beta * p[t];
}


// alpha = rho / p.q; x += alpha p; r -= alpha q; per-block partials of |r|^2. A non-positive p.q
// stops the solve with the breakdown flag.
__global__ void __launch_bounds__(kMgBlock) k_mgcg_x(int n, int nb, const double *__restrict__ pq_part,
                                                     const double *__restrict__ rz_part, int32_t *isc, const double *__restrict__ p,
                                                     const double *__restrict__ q, double *__restrict__ x, double *__restrict__ r,
                                                     double *__restrict__ rr_part) {
    __shared__ double sh[kMgBlock / 64];
    __shared__ double bc;
    if (isc[I_DONE]) return;
    const double pq = mg_all_sum(pq_part, nb, sh, &bc);
    const double rho = mg_all_sum(rz_part, nb, sh, &bc);
    if (!(pq > 0.0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            isc[I_ITERS] = isc[I_ITA];
            isc[I_BREAK] = 1;
            isc[I_DONE] = 1;
        }
        return;
    }
    const double alpha = rho / pq;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    double rr = 0.0;
    if (a < n) {
        for (int c = 0; c < 3; ++c) {
            const size_t k = c * size_t(n) + a;
            x[k] += alpha * p[k];
            const double rn = r[k] - alpha * q[k];
            r[k] = rn;
            rr += rn * rn;
        }
    }
    rr = mg_block_sum(rr, sh);
    if (threadIdx.x == 0) rr_part[blockIdx.x] = rr;
}

template <typename T>
void mg_setup_t(const DevSheet &S, const DevBufs &B, hipStream_t st) {
    const T *Hf = (const T *)B.hess;
    int nuf = S.n_u, nvf = S.n_v;
    for (int l = 0; l < B.mg_levels; ++l) {
        const MgLevel &L = B.mg[l];
        k_mg_pass_u<T><<<grid(size_t(L.n_u) * nvf * kSlots), kMgBlock, 0, st>>>(nuf, nvf, L.n_u, Hf, (T *)L.Hmid,
                                                                                 l == 0 ? S.pinmask : nullptr);
        k_mg_pass_v<T><<<grid(size_t(L.n_u) * L.n_v * kSlots), kMgBlock, 0, st>>>(L.n_u, nvf, L.n_v, (const T *)L.Hmid, (T *)L.H);
        k_mg_pinv<T><<<grid(size_t(L.n_u) * L.n_v), kMgBlock, 0, st>>>(L.n_u * L.n_v, (const T *)L.H, (T *)L.pinv);
        Hf = (const T *)L.H;
        nuf = L.n_u;
        nvf = L.n_v;
    }
}

// One V(1,1) cycle from level l: input r, output out (level 0: the fine grid and its vectors).
template <typename T>
void vcycle_t(const DevSheet &S, const DevBufs &B, int l, const double *r, double *out, double *rz_part, hipStream_t st) {
    const int32_t *isc = B.iscalars;
    const int nu = l == 0 ? S.n_u : B.mg[l - 1].n_u, nv = l == 0 ? S.n_v : B.mg[l - 1].n_v, n = nu * nv;
    const T *H = l == 0 ? (const T *)B.hess : (const T *)B.mg[l - 1].H;
    const T *pinv = l == 0 ? (const T *)B.pinv : (const T *)B.mg[l - 1].pinv;
    double *xa = l == 0 ? B.mg_x0 : B.mg[l - 1].xa;
    double *t = l == 0 ? B.mg_t0 : B.mg[l - 1].t;
    if (l == B.mg_levels) {                          // coarsest: one smoothing sweep
        k_mg_smooth0<T><<<grid(n), kMgBlock, 0, st>>>(n, pinv, r, out, isc);
        return;
    }
    const MgLevel &C = B.mg[l];
    k_mg_smooth0<T><<<grid(n), kMgBlock, 0, st>>>(n, pinv, r, xa, isc);
    k_mg_apply<T, MG_RESID><<<tiles(n), kTileRows * kTileWaves, 0, st>>>(nu, nv, H, pinv, xa, r, t, nullptr, isc);
    k_mg_restrict<<<grid(size_t(C.n_u) * C.n_v), kMgBlock, 0, st>>>(nu, nv, C.n_u, C.n_v, t, C.r, isc);
    vcycle_t<T>(S, B, l + 1, C.r, C.xb, nullptr, st);
    k_mg_prolong<<<grid(n), kMgBlock, 0, st>>>(nu, nv, C.n_u, C.n_v, C.xb, xa, l == 0 ? S.pinmask : nullptr, isc);
    k_mg_apply<T, MG_POST><<<tiles(n), kTileRows * kTileWaves, 0, st>>>(nu, nv, H, pinv, xa, r, out, rz_part, isc);
}

}  // namespace

int mg_level_count(int n_u, int n_v) {
    int L = 0;
    while (L < kMgMaxLevels && (n_u - 2) % 2 == 0 && (n_v - 2) % 2 == 0 && n_u >= 10 && n_v >= 10) {
        n_u = (n_u - 2) / 2 + 2;
        n_v = (n_v - 2) / 2 + 2;
        ++L;
    }
    return L;
}

hipError_t mg_setup(const DevSheet &S, const DevBufs &B, int prec, hipStream_t st) {
    if (prec == BSC_FP64) mg_setup_t<double>(S, B, st);
    else mg_setup_t<float>(S, B, st);
    return hipGetLastError();
}

// One preconditioned CG iteration with the V-cycle as the preconditioner. Vectors: b is not
// needed (r starts as b); x = B.dir; the partials of |r|^2 are in rr_part (k_cg_init writes
// those of |b|^2 there).
hipError_t mg_cg_iteration(const DevSheet &S, const DevBufs &B, int prec, double *r, double *z, double *p, double *q,
                           double *rz_part, double *pq_part, double *rr_part, hipStream_t st) {
    const int n = S.n_cp, nb = int(grid(n)), nt = int(tiles(n));
    k_mgcg_stop<<<1, kMgBlock, 0, st>>>(nb, rr_part, B.scalars, B.iscalars);
    if (prec == BSC_FP64) vcycle_t<double>(S, B, 0, r, z, rz_part, st);
    else vcycle_t<float>(S, B, 0, r, z, rz_part, st);
    k_mgcg_p<<<grid(3 * size_t(n)), kMgBlock, 0, st>>>(3 * n, nt, rz_part, B.scalars, B.iscalars, z, p);
    if (prec == BSC_FP64)
        k_mg_apply<double, MG_Q><<<nt, kTileRows * kTileWaves, 0, st>>>(S.n_u, S.n_v, (const double *)B.hess, nullptr, p, nullptr,
                                                                        q, pq_part, B.iscalars);
    else
        k_mg_apply<float, MG_Q><<<nt, kTileRows * kTileWaves, 0, st>>>(S.n_u, S.n_v, (const float *)B.hess, nullptr, p, nullptr,
                                                                       q, pq_part, B.iscalars);
    k_mgcg_x<<<nb, kMgBlock, 0, st>>>(n, nt, pq_part, rz_part, B.iscalars, p, q, B.dir, r, rr_part);
    return hipGetLastError();
}

}  // namespace bsc
