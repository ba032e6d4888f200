// partial.hip -- the Newton system with a contact Hessian by partial factorization (Sec. 5.3,
// Eq. "per iteration solve", Eq. "Woodbury", Eq. "Neumann expansion", the Gershgorin bound).
//
// (H + H_c) x = b with H the elastic-plus-inertia Hessian in upper-stencil form and H_c a contact
// Hessian in block CSR (both triangles). H_c is split into its 3x3 control-point self-blocks and
// the rest: D = H + diag-blocks(H_c) keeps the stencil pattern, B = off-diagonal blocks of H_c.
//   One pass over the rows (k_pf_form_d) writes D into the workspace's Hessian buffer and forms
//   the two Gershgorin quantities: max_i sum_j |B_ij| (bounds |lambda(B)|, B has a zero
//   diagonal) and min over free control points of M_a / dt^2 + max(0, the Gershgorin lower bound
//   of H_c[a, a]) (bounds lambda_min(D) from below, since the elastic part and H_c are PSD).
//   Their ratio bounds |D^-1 B|_op. Below rho_max the series sum_k (-D^-1 B)^k D^-1 b is summed
//   term by term, each D^-1 by the fused stencil PCG (the structured kernel plays the part of the
//   reused symbolic factorization); otherwise PCG runs on D + B with the contact blocks applied
//   by a block-CSR product next to the stencil SpMV.
// Pinned control points: rows and columns of H_c are dropped there (H has identity rows).
#include <chrono>
#include <cmath>
#include <vector>

#include "bsc_internal.h"

namespace bsc {
namespace {

inline int nblocks(int n) { return (n + kBlock - 1) / kBlock; }

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
    return v;
}
__device__ __forceinline__ double wmax(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off));
    return v;
}
__device__ __forceinline__ double wmin(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_down(v, off));
    return v;
}

// Block reductions (kBlock threads); the result is valid in thread 0.
template <int OP>   // 0 sum, 1 max, 2 min
__device__ double block_reduce(double v, double *sh) {
    v = OP == 0 ? wsum(v) : (OP == 1 ? wmax(v) : wmin(v));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < int(blockDim.x >> 6); ++w) v = OP == 0 ? v + sh[w] : (OP == 1 ? fmax(v, sh[w]) : fmin(v, sh[w]));
    }
    return v;
}

// Scalars of the partial-factorization solve (doubles) and its flags (int32), in the workspace's
// partials area past the arrays the stencil PCG uses.
enum { P_RB = 0, P_DLO, P_RZ, P_PQ, P_RR, P_ALPHA, P_BETA, P_TOL2, P_COUNT };
enum { F_DONE = 0, F_ITERS, F_BREAK, F_BADCOL, F_COUNT };

// D = H + the contact self-blocks (symmetrised) on free control points; per-block partials of
// max_i R_i over the scalar rows of B and of the lambda_min(D) lower bound.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_pf_form_d(DevSheet S, const T *__restrict__ H, T *__restrict__ D,
                                                      const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                      const double *__restrict__ cv, double inv_dt2,
                                                      double *__restrict__ part_rb, double *__restrict__ part_dlo,
                                                      int32_t *__restrict__ flags) {
    __shared__ double sh[kBlock / 64];
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n = S.n_cp;
    double rb = 0.0, dlo = INFINITY;
    if (a < S.n_cp) {
        for (int e = 0; e < kHessEntries; ++e) D[e * n + a] = H[e * n + a];
        if (!S.pinmask[a]) {
            double h[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
            double R[3] = {0.0, 0.0, 0.0};
            for (int k = rp[a]; k < rp[a + 1]; ++k) {
                const int c = ci[k];
                if (c < 0 || c >= S.n_cp) {
                    flags[F_BADCOL] = 1;
                    continue;
                }
                const double *v = cv + 9 * size_t(k);
                if (c == a) {
#pragma unroll
                    for (int q = 0; q < 9; ++q) h[q / 3][q % 3] += v[q];
                } else if (!S.pinmask[c]) {
#pragma unroll
                    for (int r = 0; r < 3; ++r) R[r] += fabs(v[3 * r]) + fabs(v[3 * r + 1]) + fabs(v[3 * r + 2]);
                }
            }
            rb = fmax(R[0], fmax(R[1], R[2]));
            double g = INFINITY;
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                double off = 0.0;
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    if (c != r) off += fabs(h[r][c]);
                g = fmin(g, h[r][r] - off);
            }
            dlo = S.mass[a] * inv_dt2 + fmax(0.0, g);
            // the six stored entries of the diagonal block (xx, xy, xz, yy, yz, zz)
            const double d6[6] = {h[0][0], 0.5 * (h[0][1] + h[1][0]), 0.5 * (h[0][2] + h[2][0]), h[1][1],
                                  0.5 * (h[1][2] + h[2][1]), h[2][2]};
#pragma unroll
            for (int e = 0; e < 6; ++e) D[e * n + a] = T(double(H[e * n + a]) + d6[e]);
        }
    }
    const double m1 = block_reduce<1>(rb, sh);
    if (threadIdx.x == 0) part_rb[blockIdx.x] = m1;
    const double m2 = block_reduce<2>(dlo, sh);
    if (threadIdx.x == 0) part_dlo[blockIdx.x] = m2;
}

__global__ void __launch_bounds__(kBlock) k_pf_bounds(const double *__restrict__ part_rb, const double *__restrict__ part_dlo,
                                                      int nb, double *__restrict__ scal) {
    __shared__ double sh[kBlock / 64];
    double a = 0.0, b = INFINITY;
    for (int t = threadIdx.x; t < nb; t += blockDim.x) {
        a = fmax(a, part_rb[t]);
        b = fmin(b, part_dlo[t]);
    }
    a = block_reduce<1>(a, sh);
    if (threadIdx.x == 0) scal[P_RB] = a;
    b = block_reduce<2>(b, sh);
    if (threadIdx.x == 0) scal[P_DLO] = b;
}

// y = B x (accumulate: y += B x when acc), B the off-diagonal contact blocks between free
// control points; one thread per block row.
__global__ void __launch_bounds__(kBlock) k_pf_offdiag(DevSheet S, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                       const double *__restrict__ cv, const double *__restrict__ x,
                                                       double *__restrict__ y, int acc, const int32_t *__restrict__ flags) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= S.n_cp || (flags && flags[F_DONE])) return;
    const size_t n = S.n_cp;
    double s[3] = {0.0, 0.0, 0.0};
    if (!S.pinmask[a]) {
        for (int k = rp[a]; k < rp[a + 1]; ++k) {
            const int c = ci[k];
            if (c == a || c < 0 || c >= S.n_cp || S.pinmask[c]) continue;
            const double *v = cv + 9 * size_t(k);
            const double x0 = x[c], x1 = x[n + c], x2 = x[2 * n + c];
#pragma unroll
            for (int r = 0; r < 3; ++r) s[r] += v[3 * r] * x0 + v[3 * r + 1] * x1 + v[3 * r + 2] * x2;
        }
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) y[r * n + a] = acc ? y[r * n + a] + s[r] : s[r];
}

// The next term of the series from w = D^-1 (B t): t = -w, x += t.
__global__ void k_pf_term(int n3, const double *__restrict__ w, double *__restrict__ t, double *__restrict__ x) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n3) return;
    const double v = -w[i];
    t[i] = v;
    x[i] += v;
}

// ---- PCG on the merged system D + B (block Jacobi on D's diagonal blocks) --------------------
// Scalars stay on the device; every kernel after the stop exits at once, so the host reads the
// flags only every few iterations.

template <typename T>
__global__ void __launch_bounds__(kBlock) k_pf_pinv(DevSheet S, const T *__restrict__ D, double *__restrict__ pinv) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= S.n_cp) return;
    const size_t n = S.n_cp;
    const double a00 = D[a], a01 = D[n + a], a02 = D[2 * n + a], a11 = D[3 * n + a], a12 = D[4 * n + a], a22 = D[5 * n + a];
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
#pragma unroll
    for (int t = 0; t < 6; ++t) pinv[t * n + a] = inv[t];
}

__device__ __forceinline__ void apply_pinv(const double *__restrict__ pinv, size_t n, int a, const double r[3], double z[3]) {
    const double p0 = pinv[a], p1 = pinv[n + a], p2 = pinv[2 * n + a], p3 = pinv[3 * n + a], p4 = pinv[4 * n + a],
                 p5 = pinv[5 * n + a];
    z[0] = p0 * r[0] + p1 * r[1] + p2 * r[2];
    z[1] = p1 * r[0] + p3 * r[1] + p4 * r[2];
    z[2] = p2 * r[0] + p4 * r[1] + p5 * r[2];
}

// x = 0, r = b, z = M^-1 r, p = z; partials of r.z and b.b.
__global__ void __launch_bounds__(kBlock) k_pf_cg_init(DevSheet S, const double *__restrict__ b, const double *__restrict__ pinv,
                                                       double *__restrict__ x, double *__restrict__ r, double *__restrict__ p,
                                                       double *__restrict__ part_rz, double *__restrict__ part_bb) {
    __shared__ double sh[kBlock / 64];
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n = S.n_cp;
    double rz = 0.0, bb = 0.0;
    if (a < S.n_cp) {
        double rv[3], z[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) { rv[c] = b[c * n + a]; x[c * n + a] = 0.0; r[c * n + a] = rv[c]; }
        apply_pinv(pinv, n, a, rv, z);
#pragma unroll
        for (int c = 0; c < 3; ++c) { p[c * n + a] = z[c]; rz += rv[c] * z[c]; bb += rv[c] * rv[c]; }
    }
    const double s1 = block_reduce<0>(rz, sh);
    if (threadIdx.x == 0) part_rz[blockIdx.x] = s1;
    const double s2 = block_reduce<0>(bb, sh);
    if (threadIdx.x == 0) part_bb[blockIdx.x] = s2;
}

__global__ void __launch_bounds__(kBlock) k_pf_cg_start(const double *__restrict__ part_rz, const double *__restrict__ part_bb,
                                                        int nb, double rtol, int maxit, double *__restrict__ scal,
                                                        int32_t *__restrict__ flags) {
    __shared__ double sh[kBlock / 64];
    double a = 0.0, b = 0.0;
    for (int t = threadIdx.x; t < nb; t += blockDim.x) { a += part_rz[t]; b += part_bb[t]; }
    a = block_reduce<0>(a, sh);
    const double bb = block_reduce<0>(b, sh);
    if (threadIdx.x == 0) {
        scal[P_RZ] = a;
        scal[P_RR] = bb;
        scal[P_TOL2] = rtol * rtol * bb;
        flags[F_ITERS] = 0;
        flags[F_BREAK] = 0;
        flags[F_DONE] = (bb == 0.0 || maxit <= 0) ? 1 : 0;
    }
}

// partials of p.q (q = (D + B) p)
__global__ void __launch_bounds__(kBlock) k_pf_dot(int n3, const double *__restrict__ p, const double *__restrict__ q,
                                                   double *__restrict__ part, const int32_t *__restrict__ flags) {
    __shared__ double sh[kBlock / 64];
    if (flags[F_DONE]) return;
    double s = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += gridDim.x * blockDim.x) s += p[i] * q[i];
    s = block_reduce<0>(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kBlock) k_pf_alpha(const double *__restrict__ part, int nb, double *__restrict__ scal,
                                                     int32_t *__restrict__ flags) {
    __shared__ double sh[kBlock / 64];
    if (flags[F_DONE]) return;
    double s = 0.0;
    for (int t = threadIdx.x; t < nb; t += blockDim.x) s += part[t];
    s = block_reduce<0>(s, sh);
    if (threadIdx.x == 0) {
        scal[P_PQ] = s;
        if (!(s > 0.0)) {
            flags[F_BREAK] = 1;
            flags[F_DONE] = 1;
        } else {
            scal[P_ALPHA] = scal[P_RZ] / s;
        }
    }
}

// x += alpha p, r -= alpha q, z = M^-1 r (kept in q's place is not possible: q is needed; z goes
// to zbuf); partials of r.z and r.r.
__global__ void __launch_bounds__(kBlock) k_pf_update(DevSheet S, const double *__restrict__ pinv, const double *__restrict__ scal,
                                                      double *__restrict__ x, double *__restrict__ r, const double *__restrict__ p,
                                                      const double *__restrict__ q, double *__restrict__ z,
                                                      double *__restrict__ part_rz, double *__restrict__ part_rr,
                                                      const int32_t *__restrict__ flags) {
    __shared__ double sh[kBlock / 64];
    if (flags[F_DONE]) return;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n = S.n_cp;
    const double alpha = scal[P_ALPHA];
    double rz = 0.0, rr = 0.0;
    if (a < S.n_cp) {
        double rv[3], zv[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const size_t k = c * n + a;
            x[k] += alpha * p[k];
            rv[c] = r[k] - alpha * q[k];
            r[k] = rv[c];
        }
        apply_pinv(pinv, n, a, rv, zv);
#pragma unroll
        for (int c = 0; c < 3; ++c) { z[c * n + a] = zv[c]; rz += rv[c] * zv[c]; rr += rv[c] * rv[c]; }
    }
    const double s1 = block_reduce<0>(rz, sh);
    if (threadIdx.x == 0) part_rz[blockIdx.x] = s1;
    const double s2 = block_reduce<0>(rr, sh);
    if (threadIdx.x == 0) part_rr[blockIdx.x] = s2;
}

__global__ void __launch_bounds__(kBlock) k_pf_beta(const double *__restrict__ part_rz, const double *__restrict__ part_rr, int nb,
                                                    int maxit, double *__restrict__ scal, int32_t *__restrict__ flags) {
    __shared__ double sh[kBlock / 64];
    if (flags[F_DONE]) return;
    double a = 0.0, b = 0.0;
    for (int t = threadIdx.x; t < nb; t += blockDim.x) { a += part_rz[t]; b += part_rr[t]; }
    a = block_reduce<0>(a, sh);
    const double rr = block_reduce<0>(b, sh);
    if (threadIdx.x == 0) {
        const int it = flags[F_ITERS] + 1;
        flags[F_ITERS] = it;
        scal[P_RR] = rr;
        scal[P_BETA] = a / scal[P_RZ];
        scal[P_RZ] = a;
        if (rr <= scal[P_TOL2] || it >= maxit || !(rr == rr)) flags[F_DONE] = 1;
    }
}

// p = z + beta p
__global__ void k_pf_pupdate(int n3, const double *__restrict__ z, const double *__restrict__ scal, double *__restrict__ p,
                             const int32_t *__restrict__ flags) {
    if (flags[F_DONE]) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n3) p[i] = z[i] + scal[P_BETA] * p[i];
}

#define PFX(expr, what)                                             \
    do {                                                            \
        hipError_t e_ = (expr);                                     \
        if (e_ != hipSuccess) return hip_check(ctx, e_, what);      \
    } while (0)

}  // namespace

// PCG on (D + B) x = b, D in the workspace's Hessian buffer. Vectors: x (caller), r, z, p, q from
// the workspace.
bsc_status merged_pcg(bsc_ctx *ctx, int prec, const int32_t *rp, const int32_t *ci, const double *cv, const double *b,
                      double *x, double rtol, int maxit, double *scal, int32_t *flags, int *iters) {
    const DevSheet &S = ctx->dev;
    const DevBufs &B = ctx->buf;
    hipStream_t st = ctx->stream;
    const int n3 = 3 * S.n_cp, nb = nblocks(S.n_cp), nbd = std::min(nblocks(n3), 1024);
    const int stride = B.max_blocks;
    double *r = B.r, *z = B.r2, *p = B.p0, *q = B.p1, *pinv = B.pinv;
    double *pa = B.partials, *pb = B.partials + stride;
    if (prec == BSC_FP64) k_pf_pinv<double><<<nb, kBlock, 0, st>>>(S, (const double *)B.hess, pinv);
    else k_pf_pinv<float><<<nb, kBlock, 0, st>>>(S, (const float *)B.hess, pinv);
    k_pf_cg_init<<<nb, kBlock, 0, st>>>(S, b, pinv, x, r, p, pa, pb);
    k_pf_cg_start<<<1, kBlock, 0, st>>>(pa, pb, nb, rtol, maxit, scal, flags);
    PFX(hipGetLastError(), "merged pcg init");
    int32_t hf[F_COUNT] = {};
    for (int launched = 0;;) {
        for (int k = 0; k < 8; ++k, ++launched) {
            PFX(launch_spmv(S, prec, B.hess, p, q, st), "merged pcg spmv");
            k_pf_offdiag<<<nb, kBlock, 0, st>>>(S, rp, ci, cv, p, q, 1, flags);
            k_pf_dot<<<nbd, kBlock, 0, st>>>(n3, p, q, pa, flags);
            k_pf_alpha<<<1, kBlock, 0, st>>>(pa, nbd, scal, flags);
            k_pf_update<<<nb, kBlock, 0, st>>>(S, pinv, scal, x, r, p, q, z, pa, pb, flags);
            k_pf_beta<<<1, kBlock, 0, st>>>(pa, pb, nb, maxit, scal, flags);
            k_pf_pupdate<<<nblocks(n3), kBlock, 0, st>>>(n3, z, scal, p, flags);
        }
        PFX(hipGetLastError(), "merged pcg");
        PFX(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, st), "merged pcg flags");
        PFX(hipStreamSynchronize(st), "merged pcg");
        if (hf[F_DONE]) break;
        if (launched > maxit + 8) return fail(ctx, BSC_E_STATE, "merged pcg did not finish");
    }
    if (iters) *iters = hf[F_ITERS];
    if (hf[F_BREAK]) return fail(ctx, BSC_E_PCG_BREAKDOWN, "merged pcg: p^T A p <= 0");
    return BSC_OK;
}

}  // namespace bsc

using namespace bsc;

extern "C" {

bsc_status bsc_contact_solve(bsc_ctx *c, int32_t precision, const void *d_hess, double dt, const int32_t *d_row_ptr,
                             const int32_t *d_col_idx, const double *d_vals, int32_t nnzb, const double *d_b,
                             double *d_x, const bsc_pf_opts *o, bsc_pf_stats *stats) {
    if (!c) return BSC_E_INVAL;
    bsc_ctx *ctx = c;
    if (!c->ws) return fail(c, BSC_E_STATE, "no workspace bound");
    if (precision != BSC_FP64 && precision != BSC_FP32_MIXED) return fail(c, BSC_E_INVAL, "bad precision");
    if (!o || !d_hess || !d_row_ptr || !d_b || !d_x || nnzb < 0 || (nnzb > 0 && (!d_col_idx || !d_vals)))
        return fail(c, BSC_E_INVAL, "bad arguments");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, BSC_E_INVAL, "dt must be positive");
    if (!(o->rho_max >= 0.0) || !(o->series_tol >= 0.0) || o->max_terms < 1 || o->max_terms > 1000 ||
        !(o->pcg_rtol > 0.0) || o->max_pcg < 1 || o->force < 0 || o->force > 2)
        return fail(c, BSC_E_INVAL, "bad options");
    const DevSheet &S = c->dev;
    const DevBufs &B = c->buf;
    hipStream_t st = c->stream;
    const int n = S.n_cp, n3 = 3 * n, nb = nblocks(n);
    if (d_hess == B.hess || d_b == d_x) return fail(c, BSC_E_INVAL, "d_hess may not be the workspace's Hessian; d_b and d_x may not alias");
    const auto t0 = std::chrono::steady_clock::now();
    bsc_pf_stats s{};
    // the row pointer bounds every access to the blocks: it must start at 0, never decrease and
    // end at nnzb (the block count the caller owns)
    std::vector<int32_t> rp(n + 1);
    PFX(hipMemcpyAsync(rp.data(), d_row_ptr, 4 * size_t(n + 1), hipMemcpyDeviceToHost, st), "row_ptr");
    PFX(hipStreamSynchronize(st), "row_ptr");
    if (rp[0] != 0 || rp[n] != nnzb) return fail(c, BSC_E_INVAL, "row_ptr must start at 0 and end at nnzb");
    for (int a = 0; a < n; ++a)
        if (rp[a + 1] < rp[a]) return fail(c, BSC_E_INVAL, "row_ptr decreases");
    // scalars and flags past the stencil PCG's partial arrays
    const int stride = B.max_blocks;
    double *scal = B.partials + 7 * stride;
    int32_t *flags = (int32_t *)(scal + P_COUNT);
    static_assert(P_COUNT + (F_COUNT + 1) / 2 <= 64, "partial-factorization scalars fit");
    PFX(hipMemsetAsync(flags, 0, 4 * F_COUNT, st), "flags");
    double *part_a = B.partials + 2 * stride, *part_b = B.partials + 5 * stride;
    if (precision == BSC_FP64)
        k_pf_form_d<double><<<nb, kBlock, 0, st>>>(S, (const double *)d_hess, (double *)B.hess, d_row_ptr, d_col_idx, d_vals,
                                                   1.0 / (dt * dt), part_a, part_b, flags);
    else
        k_pf_form_d<float><<<nb, kBlock, 0, st>>>(S, (const float *)d_hess, (float *)B.hess, d_row_ptr, d_col_idx, d_vals,
                                                  1.0 / (dt * dt), part_a, part_b, flags);
    k_pf_bounds<<<1, kBlock, 0, st>>>(part_a, part_b, nb, scal);
    PFX(hipGetLastError(), "form D");
    double hs[2] = {0.0, 0.0};
    int32_t hf[F_COUNT] = {};
    PFX(hipMemcpyAsync(hs, scal, sizeof(hs), hipMemcpyDeviceToHost, st), "bounds");
    PFX(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, st), "bounds");
    PFX(hipStreamSynchronize(st), "bounds");
    if (hf[F_BADCOL]) return fail(c, BSC_E_INVAL, "contact column index outside [0, n_cp)");
    s.b_bound = hs[0];
    s.d_bound = hs[1];
    s.rho_bound = hs[0] == 0.0 ? 0.0 : hs[0] / hs[1];      // d_bound = inf when every CP is pinned
    const bool series = o->force == 0 ? (s.rho_bound <= o->rho_max && s.rho_bound < 1.0) : o->force == 1;
    bsc_status res = BSC_OK;
    if (series) {
        // number of terms: K + 1 with K the smallest integer such that rho^(K+1) / (1 - rho) <= tol
        int terms = o->max_terms;
        if (s.rho_bound <= 0.0) {
            terms = 1;
        } else if (s.rho_bound < 1.0) {
            int K = 0;
            while (std::pow(s.rho_bound, K + 1) / (1.0 - s.rho_bound) > o->series_tol && K + 1 < o->max_terms) ++K;
            terms = K + 1;
        }
        s.triggered = 1;
        s.terms = terms;
        double *t = B.xn, *u = B.xhat, *w = B.phat;
        int it = 0;
        res = stencil_pcg(c, precision, d_b, t, o->pcg_rtol, o->max_pcg, &it);          // t_0 = D^-1 b
        s.pcg_iters += it;
        if (res == BSC_OK) PFX(hipMemcpyAsync(d_x, t, 8 * size_t(n3), hipMemcpyDeviceToDevice, st), "x = t0");
        for (int k = 1; k < terms && res == BSC_OK; ++k) {
            k_pf_offdiag<<<nb, kBlock, 0, st>>>(S, d_row_ptr, d_col_idx, d_vals, t, u, 0, nullptr);  // u = B t
            PFX(hipGetLastError(), "B t");
            res = stencil_pcg(c, precision, u, w, o->pcg_rtol, o->max_pcg, &it);              // w = D^-1 B t
            s.pcg_iters += it;
            if (res == BSC_OK) {
                k_pf_term<<<nblocks(n3), kBlock, 0, st>>>(n3, w, t, d_x);                        // t = -w, x += t
                PFX(hipGetLastError(), "series term");
            }
        }
    } else {
        int it = 0;
        res = merged_pcg(c, precision, d_row_ptr, d_col_idx, d_vals, d_b, d_x, o->pcg_rtol, o->max_pcg, scal, flags, &it);
        s.pcg_iters = it;
    }
    if (res == BSC_OK) PFX(hipStreamSynchronize(st), "contact solve");
    s.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = s;
    return res;
}

}  // extern "C"
