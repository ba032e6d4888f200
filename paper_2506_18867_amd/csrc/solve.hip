// solve.hip -- projected-Newton minimisation of the incremental potential (Sec. 3.2, Sec. 5.1)
// with a hand-written block-Jacobi PCG on the upper-stencil Hessian.
//
// SpMV: one thread per CP row; the 13 stored blocks of the row (diagonal + upper offsets) are
// read at the row's own index in 114 coalesced planes, and the 12 lower blocks are the
// transposes of the upper blocks stored at the neighbour rows a - d_s (also coalesced).
// PCG: two kernels per iteration. Scalars (alpha, beta, r.z, ...) live in device memory; the
// last block of each kernel (a device-scope counter) finishes the dot products from per-block
// partial sums in a fixed order, so results are deterministic and the host only polls a
// convergence flag every few iterations.
// Line search: the energy difference E(x + alpha p) - E(x) is evaluated in double without
// forming the two energies: the inertia, gravity and bending terms are exact quadratics in
// alpha (coefficients computed once), and each membrane point evaluates Psi(F + alpha dF) -
// Psi(F) from the strain increment.
#include <chrono>
#include <cmath>

#include "bsc_internal.h"

namespace bsc {
namespace {

inline int blocks(int n) { return (n + kBlock - 1) / kBlock; }

enum { S_RZ = 0, S_PQ, S_ALPHA, S_BETA, S_RR, S_TOL2, S_BB, S_E, S_GG, S_C1, S_C2, S_DEM, S_PMAX, S_WS_NUM, S_WS_DEN, S_WS_RR };
enum { I_DONE = 0, I_ITERS, I_BREAK, I_CNT_A, I_CNT_B, I_CNT_C, I_MAXIT };

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
    return v;
}

__device__ double block_sum(double v, double *sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    const int nw = (blockDim.x + 63) >> 6;
    v = (int(threadIdx.x) < nw) ? sh[threadIdx.x] : 0.0;
    if (wid == 0) v = wave_sum(v);
    return v;
}

// Publishes this block's partial sums and reports whether it is the last block to finish.
// The release/acquire pair at agent scope orders the partial stores before the counter.
__device__ bool publish_last(double *partials, int stride, const double *vals, int nvals, int32_t *counter) {
    __shared__ bool last;
    if (threadIdx.x == 0) {
        for (int t = 0; t < nvals; ++t) partials[t * stride + blockIdx.x] = vals[t];
        const int prev = __hip_atomic_fetch_add(counter, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        last = (prev == int(gridDim.x) - 1);
    }
    __syncthreads();
    return last;
}

// In the last block: ordered sum of one partial array (coherent loads).
__device__ double gather_sum(const double *partials, int n, double *sh) {
    double v = 0.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x)
        v += __hip_atomic_load(partials + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return block_sum(v, sh);
}

// ---- SpMV ------------------------------------------------------------------------------------

// y_a = sum_b H_ab p_b with p given by a functor (so PCG can form p = z + beta p_old on the fly).
template <typename T, typename PF>
__device__ __forceinline__ void row_product(const DevSheet &S, const T *__restrict__ H, int a, PF pf, double y[3]) {
    const size_t n = S.n_cp;
    const int i = a % S.n_u, j = a / S.n_u;
    T pa[3];
    pf(a, pa);
    const T d0 = H[0 * n + a], d1 = H[1 * n + a], d2 = H[2 * n + a], d3 = H[3 * n + a], d4 = H[4 * n + a], d5 = H[5 * n + a];
    T acc0 = d0 * pa[0] + d1 * pa[1] + d2 * pa[2];
    T acc1 = d1 * pa[0] + d3 * pa[1] + d4 * pa[2];
    T acc2 = d2 * pa[0] + d4 * pa[1] + d5 * pa[2];
#pragma unroll
    for (int s = 1; s < kSlots; ++s) {
        const int di = kSlotDi[s], dj = kSlotDj[s], e0 = slot_entry(s);
        const int ib = i + di, jb = j + dj;
        if (ib >= 0 && ib < S.n_u && jb < S.n_v) {          // upper block (a, a + d)
            const int b = jb * S.n_u + ib;
            T pb[3];
            pf(b, pb);
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const T v = H[(e0 + 3 * r) * n + a] * pb[0] + H[(e0 + 3 * r + 1) * n + a] * pb[1] + H[(e0 + 3 * r + 2) * n + a] * pb[2];
                if (r == 0) acc0 += v; else if (r == 1) acc1 += v; else acc2 += v;
            }
        }
        const int ic = i - di, jc = j - dj;
        if (ic >= 0 && ic < S.n_u && jc >= 0) {             // lower block = (block (a - d, a))^T
            const int b = jc * S.n_u + ic;
            T pb[3];
            pf(b, pb);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T v = H[(e0 + c) * n + b] * pb[0] + H[(e0 + 3 + c) * n + b] * pb[1] + H[(e0 + 6 + c) * n + b] * pb[2];
                if (c == 0) acc0 += v; else if (c == 1) acc1 += v; else acc2 += v;
            }
        }
    }
    y[0] = double(acc0); y[1] = double(acc1); y[2] = double(acc2);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_spmv(DevSheet S, const T *__restrict__ H, const double *__restrict__ in,
                                                 double *__restrict__ out) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= S.n_cp) return;
    const size_t n = S.n_cp;
    double y[3];
    row_product<T>(S, H, a, [&](int b, T p[3]) { p[0] = T(in[b]); p[1] = T(in[n + b]); p[2] = T(in[2 * n + b]); }, y);
    out[a] = y[0]; out[n + a] = y[1]; out[2 * n + a] = y[2];
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_export_bsr(DevSheet S, const T *__restrict__ H, const int32_t *__restrict__ rowptr,
                                                       T *__restrict__ vals) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= S.n_cp) return;
    const size_t n = S.n_cp;
    const int i = a % S.n_u, j = a / S.n_u;
    int k = rowptr[a];
    for (int jb = max(0, j - 2); jb <= min(S.n_v - 1, j + 2); ++jb) {
        for (int ib = max(0, i - 2); ib <= min(S.n_u - 1, i + 2); ++ib, ++k) {
            T blk[9];
            const int di = ib - i, dj = jb - j;
            if (di == 0 && dj == 0) {
                const T d[6] = {H[a], H[n + a], H[2 * n + a], H[3 * n + a], H[4 * n + a], H[5 * n + a]};
                blk[0] = d[0]; blk[1] = d[1]; blk[2] = d[2];
                blk[3] = d[1]; blk[4] = d[3]; blk[5] = d[4];
                blk[6] = d[2]; blk[7] = d[4]; blk[8] = d[5];
            } else {
                int s = upper_slot(di, dj);
                if (s >= 0) {
                    for (int t = 0; t < 9; ++t) blk[t] = H[(slot_entry(s) + t) * n + a];
                } else {
                    s = upper_slot(-di, -dj);
                    const int b = jb * S.n_u + ib;
                    for (int r = 0; r < 3; ++r)
                        for (int c = 0; c < 3; ++c) blk[3 * r + c] = H[(slot_entry(s) + 3 * c + r) * n + b];
                }
            }
            for (int t = 0; t < 9; ++t) vals[size_t(k) * 9 + t] = blk[t];
        }
    }
}

// ---- small vector kernels ------------------------------------------------------------------

__global__ void k_axpby(int n, double a, const double *__restrict__ x, double b, const double *__restrict__ y,
                        double *__restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[t] = a * x[t] + b * y[t];
}

__global__ void k_apply_pins(int n_cp, int npins, const int32_t *__restrict__ idx, const double *__restrict__ tgt,
                             double *__restrict__ x) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npins) return;
    const int a = idx[t];
    for (int c = 0; c < 3; ++c) x[c * n_cp + a] = tgt[c * npins + t];
}

// Dot product of two vectors of length n into scalars[slot] (single kernel, last-block finish).
__global__ void __launch_bounds__(kBlock) k_dot(int n, const double *__restrict__ x, const double *__restrict__ y,
                                                double *partials, double *scal, int slot, int32_t *cnt) {
    __shared__ double sh[kBlock / 64];
    double v = 0.0;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) v += x[t] * y[t];
    const double s = block_sum(v, sh);
    if (publish_last(partials, 0, &s, 1, cnt)) {
        const double tot = gather_sum(partials, gridDim.x, sh);
        if (threadIdx.x == 0) { scal[slot] = tot; *cnt = 0; }
    }
}

__global__ void __launch_bounds__(kBlock) k_absmax(int n, const double *__restrict__ x, double *partials, double *scal,
                                                   int slot, int32_t *cnt) {
    __shared__ double sh[kBlock / 64];
    double v = 0.0;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) v = fmax(v, fabs(x[t]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) for (int w = 1; w < int(blockDim.x >> 6); ++w) v = fmax(v, sh[w]);
    if (publish_last(partials, 0, &v, 1, cnt)) {
        if (threadIdx.x == 0) {
            double m = 0.0;
            for (int t = 0; t < int(gridDim.x); ++t)
                m = fmax(m, __hip_atomic_load(partials + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            scal[slot] = m;
            *cnt = 0;
        }
    }
}

// ---- PCG -----------------------------------------------------------------------------------

// Block-Jacobi preconditioner: inverse of each CP's 3x3 diagonal block, in double.
template <typename T>
__global__ void k_block_jacobi(DevSheet S, const T *__restrict__ H, double *__restrict__ pinv) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= S.n_cp) return;
    const size_t n = S.n_cp;
    const double a00 = H[a], a01 = H[n + a], a02 = H[2 * n + a], a11 = H[3 * n + a], a12 = H[4 * n + a], a22 = H[5 * n + a];
    const double c00 = a11 * a22 - a12 * a12, c01 = a02 * a12 - a01 * a22, c02 = a01 * a12 - a02 * a11;
    const double det = a00 * c00 + a01 * c01 + a02 * c02;
    double inv[6];
    if (det > 0.0 && a00 > 0.0) {
        const double id = 1.0 / det;
        inv[0] = c00 * id; inv[1] = c01 * id; inv[2] = c02 * id;
        inv[3] = (a00 * a22 - a02 * a02) * id; inv[4] = (a02 * a01 - a00 * a12) * id; inv[5] = (a00 * a11 - a01 * a01) * id;
    } else {   // not positive definite: fall back to the inverse diagonal
        inv[0] = a00 > 0.0 ? 1.0 / a00 : 1.0; inv[1] = inv[2] = 0.0;
        inv[3] = a11 > 0.0 ? 1.0 / a11 : 1.0; inv[4] = 0.0; inv[5] = a22 > 0.0 ? 1.0 / a22 : 1.0;
    }
    for (int t = 0; t < 6; ++t) pinv[t * n + a] = inv[t];
}

__device__ __forceinline__ void apply_pinv(const double *__restrict__ P, size_t n, int a, const double r[3], double z[3]) {
    const double i0 = P[a], i1 = P[n + a], i2 = P[2 * n + a], i3 = P[3 * n + a], i4 = P[4 * n + a], i5 = P[5 * n + a];
    z[0] = i0 * r[0] + i1 * r[1] + i2 * r[2];
    z[1] = i1 * r[0] + i3 * r[1] + i4 * r[2];
    z[2] = i2 * r[0] + i4 * r[1] + i5 * r[2];
}

// r = b - q (q = A x0, or zero), z = M^-1 r, p_old = 0; finishes r.z, r.r, b.b and the tolerance.
__global__ void __launch_bounds__(kBlock) k_pcg_init(DevSheet S, const double *__restrict__ b, const double *__restrict__ q,
                                                     const double *__restrict__ pinv, double *__restrict__ r,
                                                     double *__restrict__ z, double *__restrict__ p0, double *__restrict__ p1,
                                                     double *partials, int stride, double *scal, int32_t *isc,
                                                     double rtol, int maxit) {
    __shared__ double sh[kBlock / 64];
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n = S.n_cp;
    double rz = 0.0, rr = 0.0, bb = 0.0;
    if (a < S.n_cp) {
        double rv[3], zv[3];
        for (int c = 0; c < 3; ++c) {
            const double bc = b[c * n + a];
            rv[c] = q ? bc - q[c * n + a] : bc;
            bb += bc * bc;
        }
        apply_pinv(pinv, n, a, rv, zv);
        for (int c = 0; c < 3; ++c) {
            r[c * n + a] = rv[c]; z[c * n + a] = zv[c];
            p0[c * n + a] = 0.0; p1[c * n + a] = 0.0;
            rz += rv[c] * zv[c]; rr += rv[c] * rv[c];
        }
    }
    double v[3];
    v[0] = block_sum(rz, sh); v[1] = block_sum(rr, sh); v[2] = block_sum(bb, sh);
    if (publish_last(partials, stride, v, 3, isc + I_CNT_A)) {
        const double trz = gather_sum(partials, gridDim.x, sh);
        const double trr = gather_sum(partials + stride, gridDim.x, sh);
        const double tbb = gather_sum(partials + 2 * stride, gridDim.x, sh);
        if (threadIdx.x == 0) {
            scal[S_RZ] = trz; scal[S_RR] = trr; scal[S_BB] = tbb; scal[S_BETA] = 0.0;
            scal[S_TOL2] = rtol * rtol * tbb;
            isc[I_ITERS] = 0; isc[I_BREAK] = 0; isc[I_MAXIT] = maxit;
            isc[I_DONE] = (trr <= rtol * rtol * tbb || trr == 0.0) ? 1 : 0;
            isc[I_CNT_A] = 0;
        }
    }
}

// p_new = z + beta p_old (formed on the fly for neighbours), q = A p_new, alpha = r.z / p.q.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_pcg_a(DevSheet S, const T *__restrict__ H, const double *__restrict__ z,
                                                  const double *__restrict__ pold, double *__restrict__ pnew,
                                                  double *__restrict__ q, double *partials, double *scal, int32_t *isc) {
    __shared__ double sh[kBlock / 64];
    if (isc[I_DONE]) return;
    const double beta = scal[S_BETA];
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n = S.n_cp;
    double pq = 0.0;
    if (a < S.n_cp) {
        auto pf = [&](int b, T p[3]) {
            p[0] = T(z[b] + beta * pold[b]);
            p[1] = T(z[n + b] + beta * pold[n + b]);
            p[2] = T(z[2 * n + b] + beta * pold[2 * n + b]);
        };
        double y[3];
        row_product<T>(S, H, a, pf, y);
        for (int c = 0; c < 3; ++c) {
            const double pc = z[c * n + a] + beta * pold[c * n + a];
            pnew[c * n + a] = pc;
            q[c * n + a] = y[c];
            pq += pc * y[c];
        }
    }
    const double s = block_sum(pq, sh);
    if (publish_last(partials, 0, &s, 1, isc + I_CNT_A)) {
        const double tot = gather_sum(partials, gridDim.x, sh);
        if (threadIdx.x == 0) {
            scal[S_PQ] = tot;
            if (!(tot > 0.0)) { isc[I_BREAK] = 1; isc[I_DONE] = 1; scal[S_ALPHA] = 0.0; }
            else scal[S_ALPHA] = scal[S_RZ] / tot;
            isc[I_CNT_A] = 0;
        }
    }
}

// x += alpha p, r -= alpha q, z = M^-1 r; beta = r.z_new / r.z; convergence on |r|.
__global__ void __launch_bounds__(kBlock) k_pcg_b(DevSheet S, double *__restrict__ x, double *__restrict__ r,
                                                  double *__restrict__ z, const double *__restrict__ pinv,
                                                  const double *__restrict__ p, const double *__restrict__ q,
                                                  double *partials, int stride, double *scal, int32_t *isc) {
    __shared__ double sh[kBlock / 64];
    if (isc[I_DONE]) return;
    const double alpha = scal[S_ALPHA];
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n = S.n_cp;
    double rz = 0.0, rr = 0.0;
    if (a < S.n_cp) {
        double rv[3], zv[3];
        for (int c = 0; c < 3; ++c) {
            x[c * n + a] += alpha * p[c * n + a];
            rv[c] = r[c * n + a] - alpha * q[c * n + a];
            r[c * n + a] = rv[c];
        }
        apply_pinv(pinv, n, a, rv, zv);
        for (int c = 0; c < 3; ++c) {
            z[c * n + a] = zv[c];
            rz += rv[c] * zv[c];
            rr += rv[c] * rv[c];
        }
    }
    double v[2];
    v[0] = block_sum(rz, sh);
    v[1] = block_sum(rr, sh);
    if (publish_last(partials, stride, v, 2, isc + I_CNT_B)) {
        const double trz = gather_sum(partials, gridDim.x, sh);
        const double trr = gather_sum(partials + stride, gridDim.x, sh);
        if (threadIdx.x == 0) {
            scal[S_BETA] = trz / scal[S_RZ];
            scal[S_RZ] = trz;
            scal[S_RR] = trr;
            const int it = isc[I_ITERS] + 1;
            isc[I_ITERS] = it;
            if (trr <= scal[S_TOL2] || it >= isc[I_MAXIT] || !(trr == trr)) isc[I_DONE] = 1;
            isc[I_CNT_B] = 0;
        }
    }
}

// ---- line search -------------------------------------------------------------------------

// Quadratic coefficients of the inertia + gravity + bending energy along p:
// dE(alpha) = alpha c1 + alpha^2 c2 / 2.
__global__ void __launch_bounds__(kBlock) k_ls_quad_cp(DevSheet S, const double *__restrict__ x, const double *__restrict__ xhat,
                                                       const double *__restrict__ p, double inv_dt2, double gx, double gy,
                                                       double gz, double *partials, int stride) {
    __shared__ double sh[kBlock / 64];
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n = S.n_cp;
    double c1 = 0.0, c2 = 0.0;
    if (a < S.n_cp) {
        const double M = S.mass[a], g[3] = {gx, gy, gz};
        for (int c = 0; c < 3; ++c) {
            const double pc = p[c * n + a];
            c1 += M * inv_dt2 * pc * (x[c * n + a] - xhat[c * n + a]) - M * g[c] * pc;
            c2 += M * inv_dt2 * pc * pc;
        }
    }
    c1 = block_sum(c1, sh);
    c2 = block_sum(c2, sh);
    if (threadIdx.x == 0) { partials[blockIdx.x] = c1; partials[stride + blockIdx.x] = c2; }
}

__global__ void __launch_bounds__(kBlock) k_ls_quad_bend(DevSheet S, const double *__restrict__ beD, const double *__restrict__ p,
                                                         double *partials, int stride) {
    __shared__ double sh[kBlock / 64];
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n = S.n_cp;
    double c1 = 0.0, c2 = 0.0;
    if (q < S.n_be) {
        const int e = S.be_elem[q], k = e % S.Nu, l = e / S.Nu;
        // Laplacian weights of the 9 local CPs (same pieces as the bending kernel)
        const double tu = S.be_tu[q], tv = S.be_tv[q];
        const int tyu = k == 0 ? 0 : (k == S.Nu - 1 ? 2 : 1), tyv = l == 0 ? 0 : (l == S.Nv - 1 ? 2 : 1);
        double Nu[3], Du[3], D2u[3], Nv[3], Dv[3], D2v[3];
        auto pc = [](int ty, double t, double N[3], double D[3], double D2[3]) {
            const double s = 1.0 - t;
            if (ty == 1) { N[0] = 0.5 * s * s; N[1] = 0.5 + t * s; N[2] = 0.5 * t * t; D[0] = -s; D[1] = s - t; D[2] = t; D2[0] = 1; D2[1] = -2; D2[2] = 1; }
            else if (ty == 0) { N[0] = s * s; N[1] = t * (2.0 - 1.5 * t); N[2] = 0.5 * t * t; D[0] = -2 * s; D[1] = 2 - 3 * t; D[2] = t; D2[0] = 2; D2[1] = -3; D2[2] = 1; }
            else { N[0] = 0.5 * s * s; N[1] = s * (2.0 - 1.5 * s); N[2] = t * t; D[0] = -s; D[1] = 1 - 3 * t; D[2] = 2 * t; D2[0] = 1; D2[1] = -3; D2[2] = 2; }
        };
        pc(tyu, tu, Nu, Du, D2u);
        pc(tyv, tv, Nv, Dv, D2v);
        double lp[3] = {0.0, 0.0, 0.0};
        for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a) {
                const double L = S.c_uu * D2u[a] * Nv[b] + S.c_vv * Nu[a] * D2v[b] + S.c_uv * Du[a] * Dv[b];
                const int cp = (l + b) * S.n_u + (k + a);
                for (int c = 0; c < 3; ++c) lp[c] += L * p[c * n + cp];
            }
        const double wm = S.be_w[q] * S.mu_bend;
        for (int c = 0; c < 3; ++c) {
            c1 += beD[c * S.n_be + q] * lp[c];     // beD = w mu Laplacian(phi(x))
            c2 += wm * lp[c] * lp[c];
        }
    }
    c1 = block_sum(c1, sh);
    c2 = block_sum(c2, sh);
    if (threadIdx.x == 0) { partials[blockIdx.x] = c1; partials[stride + blockIdx.x] = c2; }
}

// Membrane energy difference sum_q w (Psi(F + alpha dF) - Psi(F)) in double.
__global__ void __launch_bounds__(kBlock) k_ls_membrane(DevSheet S, const double *__restrict__ x, const double *__restrict__ p,
                                                        double alpha, double *partials) {
    __shared__ double sh[kBlock / 64];
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n = S.n_cp;
    double de = 0.0;
    if (q < S.n_mp) {
        const int e = S.mp_elem[q], k = e % S.Nu, l = e / S.Nu;
        const double tu = S.mp_tu[q], tv = S.mp_tv[q];
        const int tyu = k == 0 ? 0 : (k == S.Nu - 1 ? 2 : 1), tyv = l == 0 ? 0 : (l == S.Nv - 1 ? 2 : 1);
        double Nu[3], Du[3], Nv[3], Dv[3];
        auto pc = [](int ty, double t, double N[3], double D[3]) {
            const double s = 1.0 - t;
            if (ty == 1) { N[0] = 0.5 * s * s; N[1] = 0.5 + t * s; N[2] = 0.5 * t * t; D[0] = -s; D[1] = s - t; D[2] = t; }
            else if (ty == 0) { N[0] = s * s; N[1] = t * (2.0 - 1.5 * t); N[2] = 0.5 * t * t; D[0] = -2 * s; D[1] = 2 - 3 * t; D[2] = t; }
            else { N[0] = 0.5 * s * s; N[1] = s * (2.0 - 1.5 * s); N[2] = t * t; D[0] = -s; D[1] = 1 - 3 * t; D[2] = 2 * t; }
        };
        pc(tyu, tu, Nu, Du);
        pc(tyv, tv, Nv, Dv);
        double G[3][2] = {{0, 0}, {0, 0}, {0, 0}}, dG[3][2] = {{0, 0}, {0, 0}, {0, 0}};
        for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a) {
                const double du = Du[a] * Nv[b], dv = Nu[a] * Dv[b];
                const double g0 = du * S.K00 + dv * S.K10, g1 = du * S.K01 + dv * S.K11;
                const int i = k + a, j = l + b, cp = j * S.n_u + i;
                const double gu = i == 0 ? 0.0 : (i == S.n_u - 1 ? double(S.n_u - 2) : i - 0.5);
                const double gv = j == 0 ? 0.0 : (j == S.n_v - 1 ? double(S.n_v - 2) : j - 0.5);
                const double d[3] = {x[cp] - (S.A00 * gu + S.A01 * gv + S.b0), x[n + cp] - (S.A10 * gu + S.A11 * gv + S.b1), x[2 * n + cp]};
                for (int c = 0; c < 3; ++c) {
                    G[c][0] += d[c] * g0; G[c][1] += d[c] * g1;
                    const double pcv = p[c * n + cp];
                    dG[c][0] += pcv * g0; dG[c][1] += pcv * g1;
                }
            }
        double F[3][2];
        for (int c = 0; c < 3; ++c)
            for (int g = 0; g < 2; ++g) F[c][g] = G[c][g] + (c == g ? 1.0 : 0.0);
        double dPsi;
        if (S.membrane == BSC_MEMBRANE_STVK) {
            double E[2][2], D[2][2];
            for (int g = 0; g < 2; ++g)
                for (int h = 0; h < 2; ++h) {
                    E[g][h] = 0.5 * (G[g][h] + G[h][g] + G[0][g] * G[0][h] + G[1][g] * G[1][h] + G[2][g] * G[2][h]);
                    const double fd = F[0][g] * dG[0][h] + F[1][g] * dG[1][h] + F[2][g] * dG[2][h];
                    const double df = F[0][h] * dG[0][g] + F[1][h] * dG[1][g] + F[2][h] * dG[2][g];
                    const double dd = dG[0][g] * dG[0][h] + dG[1][g] * dG[1][h] + dG[2][g] * dG[2][h];
                    D[g][h] = alpha * 0.5 * (fd + df) + 0.5 * alpha * alpha * dd;
                }
            const double trE = E[0][0] + E[1][1], trD = D[0][0] + D[1][1];
            double dot_DE = 0.0, dot_DD = 0.0;
            for (int g = 0; g < 2; ++g)
                for (int h = 0; h < 2; ++h) { dot_DE += D[g][h] * E[g][h]; dot_DD += D[g][h] * D[g][h]; }
            dPsi = S.mu * (dot_DD + 2.0 * dot_DE) + 0.5 * S.lam * trD * (trD + 2.0 * trE);
        } else {
            double dI5[2], I5m1[2];
            const double mus[2] = {S.mu1, S.mu2};
            dPsi = 0.0;
            for (int g = 0; g < 2; ++g) {
                double fdf = 0.0, dfdf = 0.0;
                for (int c = 0; c < 3; ++c) { fdf += F[c][g] * dG[c][g]; dfdf += dG[c][g] * dG[c][g]; }
                I5m1[g] = 2.0 * G[g][g] + G[0][g] * G[0][g] + G[1][g] * G[1][g] + G[2][g] * G[2][g];
                dI5[g] = 2.0 * alpha * fdf + alpha * alpha * dfdf;
                const double len = sqrt(1.0 + I5m1[g]), len2 = sqrt(1.0 + I5m1[g] + dI5[g]);
                const double dlen = dI5[g] / (len + len2);
                const double lm1 = I5m1[g] / (len + 1.0);
                dPsi += mus[g] * dlen * (2.0 * lm1 + dlen);
            }
            double I6 = 0.0, dI6 = 0.0;
            for (int c = 0; c < 3; ++c) {
                I6 += F[c][0] * F[c][1];
                dI6 += alpha * (F[c][0] * dG[c][1] + F[c][1] * dG[c][0]) + alpha * alpha * dG[c][0] * dG[c][1];
            }
            dPsi += S.msh * dI6 * (2.0 * I6 + dI6);
        }
        de = S.mp_w[q] * dPsi;
    }
    const double s = block_sum(de, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void k_sum_into(const double *__restrict__ p, int n, double *scal, int slot) {
    __shared__ double sh[kBlock / 64];
    double v = 0.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) v += p[t];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) scal[slot] = v;
}

__global__ void k_sum2_into(const double *__restrict__ p, int n0, const double *__restrict__ p1, int n1, double *scal, int slot) {
    __shared__ double sh[kBlock / 64];
    double v = 0.0;
    for (int t = threadIdx.x; t < n0; t += blockDim.x) v += p[t];
    for (int t = threadIdx.x; t < n1; t += blockDim.x) v += p1[t];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) scal[slot] = v;
}

__global__ void k_update(int n, double alpha, const double *__restrict__ p, double *__restrict__ x) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) x[t] += alpha * p[t];
}

}  // namespace

hipError_t launch_spmv(const DevSheet &S, int precision, const void *hess, const double *in, double *out, hipStream_t st) {
    if (precision == BSC_FP64) k_spmv<double><<<blocks(S.n_cp), kBlock, 0, st>>>(S, (const double *)hess, in, out);
    else k_spmv<float><<<blocks(S.n_cp), kBlock, 0, st>>>(S, (const float *)hess, in, out);
    return hipGetLastError();
}

hipError_t launch_export_bsr(const DevSheet &S, int precision, const void *hess, const int32_t *row_ptr,
                             const int32_t *, void *vals, hipStream_t st) {
    if (precision == BSC_FP64) k_export_bsr<double><<<blocks(S.n_cp), kBlock, 0, st>>>(S, (const double *)hess, row_ptr, (double *)vals);
    else k_export_bsr<float><<<blocks(S.n_cp), kBlock, 0, st>>>(S, (const float *)hess, row_ptr, (float *)vals);
    return hipGetLastError();
}

namespace {

struct Timer {
    hipStream_t st;
    hipEvent_t a, b;
    bool ok;
    explicit Timer(hipStream_t s) : st(s) {
        ok = hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess;
        if (ok) hipEventRecord(a, st);
    }
    double stop() {
        if (!ok) return 0.0;
        float ms = 0.f;
        hipEventRecord(b, st);
        hipEventSynchronize(b);
        hipEventElapsedTime(&ms, a, b);
        return ms;
    }
    ~Timer() {
        if (ok) { hipEventDestroy(a); hipEventDestroy(b); }
    }
};

#define HIPX(expr, what)                                            \
    do {                                                            \
        hipError_t e_ = (expr);                                     \
        if (e_ != hipSuccess) return hip_check(ctx, e_, what);      \
    } while (0)

// Assembles E, g (double) and H (working precision) at x for one Newton iteration.
bsc_status assemble_iter(bsc_ctx *ctx, int prec, const double *x, const double *xhat, double inv_dt2, const double *grav) {
    const DevSheet &S = ctx->dev;
    const DevBufs &B = ctx->buf;
    hipStream_t st = ctx->stream;
    if (prec == BSC_FP64) {
        HIPX(launch_points(S, B, BSC_FP64, true, false, x, st), "points");
        HIPX(launch_grad(S, B, BSC_FP64, x, xhat, inv_dt2, grav, B.g, false, st), "gradient");
        HIPX(launch_hess(S, B, BSC_FP64, inv_dt2, B.hess, st), "hessian");
    } else {
        HIPX(launch_points(S, B, BSC_FP32_MIXED, true, false, x, st), "points32");
        HIPX(launch_hess(S, B, BSC_FP32_MIXED, inv_dt2, B.hess, st), "hessian32");
        HIPX(launch_points(S, B, BSC_FP64, false, true, x, st), "points64");
        HIPX(launch_grad(S, B, BSC_FP64, x, xhat, inv_dt2, grav, B.g, true, st), "gradient64");
    }
    HIPX(launch_energy_reduce(S, B, true, B.scalars + S_E, st), "energy");
    return BSC_OK;
}

}  // namespace

bsc_status newton_step(bsc_ctx *ctx, const bsc_step_opts *o, double *x, double *v, const double *pin_tgt,
                       bsc_step_stats *stats) {
    const DevSheet &S = ctx->dev;
    const DevBufs &B = ctx->buf;
    hipStream_t st = ctx->stream;
    const int n3 = 3 * S.n_cp;
    const int npins = int(ctx->pins.size());
    const int prec = o->precision;
    const double dt = o->dt, inv_dt2 = 1.0 / (dt * dt);
    const double *grav = o->gravity;
    const int stride = B.max_blocks;
    bsc_step_stats s{};
    auto t_start = std::chrono::steady_clock::now();

    HIPX(hipMemcpyAsync(B.xn, x, 8 * size_t(n3), hipMemcpyDeviceToDevice, st), "copy x");
    k_axpby<<<blocks(n3), kBlock, 0, st>>>(n3, 1.0, x, dt, v, B.xhat);
    if (npins > 0) k_apply_pins<<<blocks(npins), kBlock, 0, st>>>(S.n_cp, npins, B.pin_idx, pin_tgt, x);
    HIPX(hipGetLastError(), "step setup");

    bsc_status result = BSC_OK;
    double g0 = -1.0;
    double host[4];
    int it = 0;
    for (;; ++it) {
        {
            Timer t(st);
            bsc_status as = assemble_iter(ctx, prec, x, B.xhat, inv_dt2, grav);
            if (as != BSC_OK) return as;
            k_dot<<<256, kBlock, 0, st>>>(n3, B.g, B.g, B.partials + 7 * stride, B.scalars, S_GG, B.iscalars + I_CNT_C);
            HIPX(hipMemcpyAsync(host, B.scalars + S_E, 2 * sizeof(double), hipMemcpyDeviceToHost, st), "read norms");
            HIPX(hipStreamSynchronize(st), "sync");
            s.ms_assemble += t.stop();
        }
        const double E = host[0], gn = std::sqrt(host[1]);
        if (!std::isfinite(E) || !std::isfinite(gn)) { result = BSC_E_NONFINITE; break; }
        if (g0 < 0.0) g0 = gn;
        s.energy = E;
        s.g_norm = gn;
        if (o->fixed_newton_iters > 0) {
            if (it >= o->fixed_newton_iters) break;
        } else if (o->stop_mode == BSC_STOP_GRAD && gn <= o->rtol * g0) {
            break;
        } else if (gn == 0.0) {
            break;
        }
        if (it >= o->max_newton) { result = BSC_E_NOT_CONVERGED; break; }

        // ---- direction: PCG on H p = -g -----------------------------------------------
        {
            Timer t(st);
            if (prec == BSC_FP64) k_block_jacobi<double><<<blocks(S.n_cp), kBlock, 0, st>>>(S, (const double *)B.hess, B.pinv);
            else k_block_jacobi<float><<<blocks(S.n_cp), kBlock, 0, st>>>(S, (const float *)B.hess, B.pinv);
            k_axpby<<<blocks(n3), kBlock, 0, st>>>(n3, -1.0, B.g, 0.0, B.g, B.tmp);          // b = -g
            HIPX(hipMemsetAsync(B.dir, 0, 8 * size_t(n3), st), "zero dir");
            k_pcg_init<<<blocks(S.n_cp), kBlock, 0, st>>>(S, B.tmp, nullptr, B.pinv, B.r, B.z, B.p0, B.p1,
                                                           B.partials, stride, B.scalars, B.iscalars, o->pcg_rtol, o->max_pcg);
            HIPX(hipGetLastError(), "pcg init");
            int32_t flags[2] = {0, 0};
            int k = 0;
            const int chunk = 16;
            while (true) {
                for (int c = 0; c < chunk; ++c, ++k) {
                    double *pold = (k & 1) ? B.p1 : B.p0, *pnew = (k & 1) ? B.p0 : B.p1;
                    if (prec == BSC_FP64)
                        k_pcg_a<double><<<blocks(S.n_cp), kBlock, 0, st>>>(S, (const double *)B.hess, B.z, pold, pnew, B.q, B.partials, B.scalars, B.iscalars);
                    else
                        k_pcg_a<float><<<blocks(S.n_cp), kBlock, 0, st>>>(S, (const float *)B.hess, B.z, pold, pnew, B.q, B.partials, B.scalars, B.iscalars);
                    k_pcg_b<<<blocks(S.n_cp), kBlock, 0, st>>>(S, B.dir, B.r, B.z, B.pinv, pnew, B.q, B.partials + 2 * stride, stride, B.scalars, B.iscalars);
                }
                HIPX(hipGetLastError(), "pcg");
                HIPX(hipMemcpyAsync(flags, B.iscalars + I_DONE, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st), "read pcg flags");
                HIPX(hipStreamSynchronize(st), "sync pcg");
                if (flags[0]) break;
            }
            int32_t brk = 0;
            HIPX(hipMemcpyAsync(&brk, B.iscalars + I_BREAK, sizeof(int32_t), hipMemcpyDeviceToHost, st), "read pcg break");
            HIPX(hipStreamSynchronize(st), "sync");
            s.pcg_iters_total += flags[1];
            s.ms_pcg += t.stop();
            if (brk) { result = BSC_E_PCG_BREAKDOWN; break; }
        }
        if (o->fixed_newton_iters <= 0 && o->stop_mode == BSC_STOP_STEP) {
            k_absmax<<<256, kBlock, 0, st>>>(n3, B.dir, B.partials + 7 * stride, B.scalars, S_PMAX, B.iscalars + I_CNT_C);
            double pmax = 0.0;
            HIPX(hipMemcpyAsync(&pmax, B.scalars + S_PMAX, sizeof(double), hipMemcpyDeviceToHost, st), "read pmax");
            HIPX(hipStreamSynchronize(st), "sync");
            if (pmax / dt <= o->atol) break;
        }

        // ---- backtracking line search on the energy difference ---------------------------
        {
            Timer t(st);
            const double gx = grav ? grav[0] : 0.0, gy = grav ? grav[1] : 0.0, gz = grav ? grav[2] : 0.0;
            double *pa = B.partials + 3 * stride, *pb = B.partials + 5 * stride;
            k_ls_quad_cp<<<blocks(S.n_cp), kBlock, 0, st>>>(S, x, B.xhat, B.dir, inv_dt2, gx, gy, gz, pa, stride);
            k_ls_quad_bend<<<blocks(S.n_be), kBlock, 0, st>>>(S, B.beD, B.dir, pb, stride);
            k_sum2_into<<<1, kBlock, 0, st>>>(pa, blocks(S.n_cp), pb, blocks(S.n_be), B.scalars, S_C1);
            k_sum2_into<<<1, kBlock, 0, st>>>(pa + stride, blocks(S.n_cp), pb + stride, blocks(S.n_be), B.scalars, S_C2);
            HIPX(hipGetLastError(), "line search setup");
            double c12[2];
            HIPX(hipMemcpyAsync(c12, B.scalars + S_C1, 2 * sizeof(double), hipMemcpyDeviceToHost, st), "read c1 c2");
            double alpha = 1.0;
            bool ok = false;
            for (int h = 0; h <= 20; ++h) {
                k_ls_membrane<<<blocks(S.n_mp), kBlock, 0, st>>>(S, x, B.dir, alpha, B.partials + 6 * stride);
                k_sum_into<<<1, kBlock, 0, st>>>(B.partials + 6 * stride, blocks(S.n_mp), B.scalars, S_DEM);
                double dem = 0.0;
                HIPX(hipMemcpyAsync(&dem, B.scalars + S_DEM, sizeof(double), hipMemcpyDeviceToHost, st), "read dE");
                HIPX(hipStreamSynchronize(st), "sync ls");
                const double dE = alpha * c12[0] + 0.5 * alpha * alpha * c12[1] + dem;
                if (!std::isfinite(dE)) { alpha *= 0.5; s.ls_halvings++; continue; }
                if (dE <= 0.0) { ok = true; break; }
                alpha *= 0.5;
                s.ls_halvings++;
            }
            s.ms_linesearch += t.stop();
            if (!ok) { result = BSC_E_LINESEARCH; break; }
            k_update<<<blocks(n3), kBlock, 0, st>>>(n3, alpha, B.dir, x);
            HIPX(hipGetLastError(), "update");
        }
    }
    s.newton_iters = it;
    s.g0_norm = g0;
    k_axpby<<<blocks(n3), kBlock, 0, st>>>(n3, 1.0 / dt, x, -1.0 / dt, B.xn, v);
    HIPX(hipGetLastError(), "velocity");
    HIPX(hipStreamSynchronize(st), "sync end");
    s.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (stats) *stats = s;
    return result;
}

}  // namespace bsc

using namespace bsc;

extern "C" {

bsc_status bsc_spmv(bsc_ctx *c, int32_t precision, const void *d_hess, const double *d_in, double *d_out) {
    if (!c) return BSC_E_INVAL;
    if (!c->ws) return fail(c, BSC_E_STATE, "no workspace bound");
    if (!d_hess || !d_in || !d_out || d_in == d_out) return fail(c, BSC_E_INVAL, "bad pointers");
    if (precision != BSC_FP64 && precision != BSC_FP32_MIXED) return fail(c, BSC_E_INVAL, "bad precision");
    return hip_check(c, launch_spmv(c->dev, precision, d_hess, d_in, d_out, c->stream), "spmv");
}

bsc_status bsc_export_bsr(bsc_ctx *c, int32_t precision, const void *d_hess, void *d_bsr_vals) {
    if (!c) return BSC_E_INVAL;
    if (!c->ws) return fail(c, BSC_E_STATE, "no workspace bound");
    if (!d_hess || !d_bsr_vals) return fail(c, BSC_E_INVAL, "null pointer");
    if (precision != BSC_FP64 && precision != BSC_FP32_MIXED) return fail(c, BSC_E_INVAL, "bad precision");
    return hip_check(c, launch_export_bsr(c->dev, precision, d_hess, c->buf.bsr_rowptr, nullptr, d_bsr_vals, c->stream), "export bsr");
}

bsc_status bsc_newton_step(bsc_ctx *c, const bsc_step_opts *o, double *d_x, double *d_v, const double *d_pin_targets,
                           bsc_step_stats *stats) {
    if (!c || !o) return BSC_E_INVAL;
    if (!c->ws) return fail(c, BSC_E_STATE, "no workspace bound");
    if (!d_x || !d_v) return fail(c, BSC_E_INVAL, "null state");
    if (!(o->dt > 0.0) || !std::isfinite(o->dt)) return fail(c, BSC_E_INVAL, "dt must be positive");
    if (o->precision != BSC_FP64 && o->precision != BSC_FP32_MIXED) return fail(c, BSC_E_INVAL, "bad precision");
    if (o->stop_mode != BSC_STOP_GRAD && o->stop_mode != BSC_STOP_STEP) return fail(c, BSC_E_INVAL, "bad stop mode");
    if (o->max_newton < 1 || o->max_pcg < 1 || !(o->pcg_rtol > 0.0)) return fail(c, BSC_E_INVAL, "bad iteration limits");
    if (!c->pins.empty() && !d_pin_targets) return fail(c, BSC_E_INVAL, "pins set but no targets");
    if (o->warm_start && !c->net_loaded) return fail(c, BSC_E_STATE, "warm start requested but no network loaded");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(o->gravity[k])) return fail(c, BSC_E_INVAL, "gravity must be finite");
    bsc_status st = newton_step(c, o, d_x, d_v, d_pin_targets, stats);
    if (st != BSC_OK && c->err.empty()) c->err = bsc_status_string(st);
    return st;
}

}  // extern "C"
