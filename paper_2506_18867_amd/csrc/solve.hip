// solve.hip -- projected-Newton minimisation of the incremental potential (Sec. 3.2, Sec. 5.1)
// with a hand-written block-Jacobi PCG on the upper-stencil Hessian.
//
// SpMV: tiles of 64 rows, 8 waves per tile, each wave one group of the row's 25 block
// products; the 13 stored blocks of a row (diagonal + upper offsets) are read at the row's own
// index in 114 coalesced planes, the 12 lower blocks are the transposes of the upper blocks
// stored at the neighbour rows a - d_s (also coalesced, usually from the same XCD's L2).
// PCG (Chronopoulos-Gear form): one fused kernel per iteration (k_cg_fused: the previous
// iteration's scalars from the partial dot products, the vector updates, the block-Jacobi
// preconditioner, the SpMV and the new partials); every block re-sums the partials in the same
// fixed order (large grids: a one-block kernel sums them once per launch). Scalars live in
// device memory, nothing uses atomics or in-kernel fences, results are deterministic, and the
// host reads the solver state once per burst of launches.
// Line search: the energy difference E(x + alpha p) - E(x) is evaluated in double without
// forming the two energies: the inertia, gravity and bending terms are exact quadratics in
// alpha (coefficients computed once), and each membrane point evaluates Psi(F + alpha dF) -
// Psi(F) from the strain increment.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "bsc_internal.h"

namespace bsc {
namespace {

#include "geom.h"

inline int blocks(int n) { return (n + kBlock - 1) / kBlock; }


constexpr int kRowsPerTile = 64;     // one wave of rows per SpMV block
constexpr int kGroups = 8;           // waves per SpMV block, one group of block products each
constexpr int kReduceBlocks = 256;   // grid of the fixed-grid reductions

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
    return v;          // valid in thread 0
}

// Block-wide sums of three values at once (one LDS round trip); valid in every thread.
__device__ void block_sum3(double v[3], double *sh /* 3 * 16 */) {
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = wave_sum(v[k]);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) sh[16 * k + wid] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double t = 0.0;
        for (int q = 0; q < nw; ++q) t += sh[16 * k + q];
        v[k] = t;
    }
}

// Butterfly sum over a wave: every lane ends with the same, bitwise identical total (each
// step adds the same two numbers in both lanes of a pair).
__device__ __forceinline__ double wave_sum_all(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Block totals of three values whose per-wave totals are already in every lane (one LDS round
// trip); valid in every thread, summed over the waves in a fixed order.
__device__ void wave_totals3(double v[3], double *sh /* 3 * 16 */) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) sh[16 * k + wid] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double t = 0.0;
        for (int q = 0; q < nw; ++q) t += sh[16 * k + q];
        v[k] = t;
    }
}

// ---- SpMV ------------------------------------------------------------------------------------

// One of the 25 block products of row a: 0 = diagonal, 1..12 = upper slot s (block stored at
// row a), 13..24 = lower slot s - 12 (transpose of the block stored at row a - d_s).
template <typename T>
__device__ __forceinline__ void block_product(const DevSheet &S, const T *__restrict__ H, const double *__restrict__ u,
                                              int a, int i, int j, int pid, T acc[3]) {
    const size_t n = S.n_cp;
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
        if (ib < 0 || ib >= S.n_u || jb >= S.n_v) return;
        const int b = jb * S.n_u + ib;
        const T u0 = T(u[b]), u1 = T(u[n + b]), u2 = T(u[2 * n + b]);
#pragma unroll
        for (int r = 0; r < 3; ++r)
            acc[r] += H[(e0 + 3 * r) * n + a] * u0 + H[(e0 + 3 * r + 1) * n + a] * u1 + H[(e0 + 3 * r + 2) * n + a] * u2;
    } else {
        const int ic = i - di, jc = j - dj;
        if (ic < 0 || ic >= S.n_u || jc < 0) return;
        const int b = jc * S.n_u + ic;
        const T u0 = T(u[b]), u1 = T(u[n + b]), u2 = T(u[2 * n + b]);
#pragma unroll
        for (int c = 0; c < 3; ++c)
            acc[c] += H[(e0 + c) * n + b] * u0 + H[(e0 + 3 + c) * n + b] * u1 + H[(e0 + 6 + c) * n + b] * u2;
    }
}

// Per-CP set-up of a block-Jacobi PCG solve: b = -g and the inverse of the diagonal block
// (the inverse diagonal where the block is not positive definite).
template <typename T>
__device__ __forceinline__ void prep_row(const DevSheet &S, const T *__restrict__ H, T *__restrict__ pinv,
                                         const double *__restrict__ g, double *__restrict__ b, int a) {
    const size_t n = S.n_cp;
#pragma unroll
    for (int c = 0; c < 3; ++c) b[c * n + a] = 0.0 - g[c * n + a];
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
#pragma unroll
    for (int t = 0; t < 6; ++t) pinv[t * n + a] = T(inv[t]);
}

// The energy and |g|^2 of an assembly from its partial sums, formed by one block of the first
// kernel after it (so that no launch of its own separates the assembly from the solve): the
// points pass's energy partials p0, p1, p2 and the tiles' |g|^2 partials pg, each summed in a
// fixed order, then with do_pub the read-back of the solver scalars and flags. out == nullptr:
// nothing to do.
struct EnergyRed {
    const double *p0, *p1, *p2, *pg;
    int n0, n1, n2, ng;
    double *out, *out_g;
    PubPtrs pub;
    int do_pub;
};

__device__ void energy_reduce_block(const EnergyRed &R, const double *scal, int32_t *flags, double *sh) {
    double v = 0.0, u = 0.0;
    for (int t = threadIdx.x; t < R.n0; t += blockDim.x) v += R.p0[t];
    for (int t = threadIdx.x; t < R.n1; t += blockDim.x) v += R.p1[t];
    for (int t = threadIdx.x; t < R.n2; t += blockDim.x) v += R.p2[t];
    for (int t = threadIdx.x; t < R.ng; t += blockDim.x) u += R.pg[t];
    const double se = block_sum(v, sh);
    const double sg = block_sum(u, sh);
    if (threadIdx.x == 0) {
        R.out[0] = se;
        R.out_g[0] = sg;
    }
    if (R.do_pub) {
        __syncthreads();
        publish_block(scal, flags, R.pub);
    }
}

// w = H u for a tile of 64 rows; wave g computes block products g, g+8, g+16, g+24 and the
// eight partial results are summed through LDS. DOTS (the warm start): the tile's partials of
// g.u, u.w, g.w and w.w go to part[k * stride + block] (a fixed-order wave sum per tile).
template <typename T, bool DOTS = false>
__global__ void __launch_bounds__(kRowsPerTile * kGroups) k_spmv_tile(DevSheet S, const T *__restrict__ H,
                                                                     const double *__restrict__ u, double *__restrict__ w,
                                                                     const double *__restrict__ gv = nullptr,
                                                                     double *__restrict__ part = nullptr, int stride = 0,
                                                                     T *__restrict__ pinv = nullptr,
                                                                     double *__restrict__ bvec = nullptr,
                                                                     EnergyRed red = EnergyRed{}, const double *scal = nullptr,
                                                                     int32_t *flags = nullptr) {
    __shared__ T ys[kGroups][3][kRowsPerTile];
    __shared__ double shr[kRowsPerTile * kGroups / 64];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int g = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int a = tile * kRowsPerTile + lane;
    T acc[3] = {T(0), T(0), T(0)};
    if (a < S.n_cp) {
        const int i = a % S.n_u, j = a / S.n_u;
        for (int m = 0; m < 4; ++m) {
            const int pid = g + kGroups * m;
            if (pid < 25) block_product<T>(S, H, u, a, i, j, pid, acc);
        }
        // with pinv: the PCG set-up of the tile's rows, by the last wave (one product fewer)
        if (pinv && g == kGroups - 1) prep_row<T>(S, H, pinv, gv, bvec, a);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) ys[g][c][lane] = acc[c];
    __syncthreads();
    if (g == 0) {
        double d[4] = {0.0, 0.0, 0.0, 0.0};
        if (a < S.n_cp) {
            const size_t n = S.n_cp;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                T y = ys[0][c][lane];
#pragma unroll
                for (int q = 1; q < kGroups; ++q) y += ys[q][c][lane];
                const double wy = double(y);
                w[c * n + a] = wy;
                if (DOTS) {
                    const double gc = gv[c * n + a], uc = u[c * n + a];
                    d[0] += gc * uc; d[1] += uc * wy; d[2] += gc * wy; d[3] += wy * wy;
                }
            }
        }
        if (DOTS) {
#pragma unroll
            for (int k = 0; k < 4; ++k) d[k] = wave_sum_all(d[k]);
            if (lane == 0) {
#pragma unroll
                for (int k = 0; k < 4; ++k) part[k * stride + blockIdx.x] = d[k];
            }
        }
    }
    if (red.out && blockIdx.x == 0) energy_reduce_block(red, scal, flags, shr);
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

__global__ void k_zero(int n, double *__restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[t] = 0.0;
}

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

// Per-block partials of max |x| (grid of kReduceBlocks); k_finish reduces them into scal[slot].
__global__ void __launch_bounds__(kBlock) k_absmax_part(int n, const double *__restrict__ x, double *__restrict__ partials) {
    __shared__ double sh[kBlock / 64];
    double v = 0.0;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) v = fmax(v, fabs(x[t]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < int(blockDim.x >> 6); ++w) v = fmax(v, sh[w]);
        partials[blockIdx.x] = v;
    }
}

__global__ void __launch_bounds__(kBlock) k_finish(const double *__restrict__ partials, int n, int is_max, double *scal, int slot) {
    __shared__ double sh[kBlock / 64];
    if (is_max) {                       // max is exact in any order
        double m = 0.0;
        for (int t = threadIdx.x; t < n; t += blockDim.x) m = fmax(m, partials[t]);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off));
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
        if (lane == 0) sh[wid] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int q = 1; q < int(blockDim.x + 63) / 64; ++q) m = fmax(m, sh[q]);
            scal[slot] = m;
        }
        return;
    }
    double v = 0.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) v += partials[t];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) scal[slot] = v;
}

// ---- preconditioned CG (Chronopoulos-Gear form: one reduction phase per iteration) --------
//
//   r0 = b - A x0, u0 = M^-1 r0; per iteration i:
//     w_i = A u_i;  gamma_i = r_i.u_i, delta_i = w_i.u_i
//     stop if |r_i| <= tol; beta_i = gamma_i / gamma_{i-1};
//     alpha_i = gamma_i / (delta_i - beta_i gamma_i / alpha_{i-1})  (alpha_0 = gamma_0/delta_0)
//     p_i = u_i + beta_i p_{i-1}, s_i = w_i + beta_i s_{i-1}
//     x_{i+1} = x_i + alpha_i p_i, r_{i+1} = r_i - alpha_i s_i, u_{i+1} = M^-1 r_{i+1}
// M is the block-Jacobi preconditioner (inverse 3x3 diagonal blocks, in double). One launch of
// k_cg_fused per iteration (below).

// The PCG set-up of a Newton iteration in one pass over the CPs: the block-Jacobi inverse (the
// inverse of the 3x3 diagonal block, or its inverse diagonal where that block is not positive
// definite), the right-hand side b = -g (written 0 - g, so that a zero gradient gives +0) and
// the initial direction x0 = 0. With keep, the direction that x0 held (the previous Newton
// direction of the step; zero at the step's first iteration) is saved there first, zero on
// pinned CPs.
// The set-up without a warm start: prep_row and x0 = 0.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_cg_prep(DevSheet S, const T *__restrict__ H, T *__restrict__ pinv,
                                                    const double *__restrict__ g, double *__restrict__ b,
                                                    double *__restrict__ x0, EnergyRed red = EnergyRed{},
                                                    const double *scal = nullptr, int32_t *flags = nullptr) {
    __shared__ double sh[kBlock / 64];
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a < S.n_cp) {
        const size_t n = S.n_cp;
#pragma unroll
        for (int c = 0; c < 3; ++c) x0[c * n + a] = 0.0;
        prep_row<T>(S, H, pinv, g, b, a);
    }
    if (red.out && blockIdx.x == 0) energy_reduce_block(red, scal, flags, sh);
}

// PCG tolerance of a Newton iteration. EXPLICIT: given by the host. FIXED / TIGHT: pcg_rtol.
// ADAPTIVE: Eisenstat-Walker forcing term (choice 2, gamma = 0.9, exponent 2) with the
// safeguard, clamped to [pcg_rtol, 0.1], from |g| of this and the previous Newton iteration
// (0.1 at the first); computed on the device so that no host round trip separates the
// assembly from the solve.
enum { ETA_EXPLICIT = 0, ETA_FIXED = 1, ETA_ADAPTIVE = 2, ETA_TIGHT = 3 };

__device__ double forcing_term(int mode, int first, double eta_host, double rtol_min, double eta_max, double gn, double g_prev,
                               double eta_prev) {
    if (mode == ETA_EXPLICIT) return eta_host;
    if (mode != ETA_ADAPTIVE) return rtol_min;
    if (first) return fmax(rtol_min, eta_max);
    const double ratio = gn / g_prev;
    double e = 0.9 * ratio * ratio;
    const double guard = 0.9 * eta_prev * eta_prev;
    if (guard > 0.1) e = fmax(e, guard);
    return fmin(eta_max, fmax(rtol_min, e));
}

// The warm start's decision, made by every block of the CG initialisation alike: the sums of
// the four partial arrays of the SpMV with the prediction p (one wave per array: lane l sums
// entries l, l + 64, ... in order, then the butterfly sum) give gp = g.p, pw = p.Hp, gw = g.Hp,
// ww = |Hp|^2; with bb = |g|^2 the energy-optimal multiple a = -gp / pw (either sign) gives the
// initial residual |b - a Hp|^2 = bb + 2 a gw + a^2 ww with b = -g. The start x0 = a p is kept
// only when that is below bb (the zero start's residual), else a = 0. Needs at least 256
// threads (waves after the fourth add nothing).
static_assert(kBlock >= 256, "the warm start's decision takes one wave per partial array");
__device__ double ws_decide(const double *__restrict__ part, int stride, int nb, double bb, double tot[4]) {
    __shared__ double sm[4];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // the lane's elements t = lane, lane + 64, ... added in that order; loaded eight at a time so
    // that their latencies overlap
    const double *pw_ = part + size_t(w < 4 ? w : 0) * stride;
    double s = 0.0;
    int t = w < 4 ? lane : nb;                    // one wave per array; further waves add nothing
    for (; t + 7 * 64 < nb; t += 8 * 64) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = pw_[t + 64 * k];
#pragma unroll
        for (int k = 0; k < 8; ++k) s += v[k];
    }
    for (; t < nb; t += 64) s += pw_[t];
    s = wave_sum_all(s);
    if (lane == 0 && w < 4) sm[w] = s;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) tot[k] = sm[k];
    const double gp = tot[0], pw = tot[1], gw = tot[2], ww = tot[3];
    double a = 0.0;
    if (pw > 0.0 && std::isfinite(gp) && std::isfinite(pw) && std::isfinite(gw) && std::isfinite(ww)) {
        const double as = -gp / pw;
        const double rr = bb + 2.0 * as * gw + as * as * ww;
        if (as != 0.0 && rr < bb) a = as;
    }
    return a;
}

// r = b - A x0, p = s = 0; per-block partials of b.b; the solve's tolerance. Without a warm
// start (ph null) x0 = 0 (set by the prep kernel) and r = b. With one, x0 = a ph and A x0 = a hq
// for the multiple a that every block decides from the partials wpart of the product hq = H ph
// (a = 0: x0 = 0 and r = b exactly); block 0 stores the dots at S_WS0..3, a at S_WSA and the
// flag I_WS.
__global__ void __launch_bounds__(kBlock) k_cg_init(DevSheet S, const double *__restrict__ b, const double *ph,
                                                    const double *__restrict__ hq, const double *__restrict__ wpart,
                                                    int wstride, int wnb, double *x0,
                                                    double *__restrict__ r, double *__restrict__ p, double *__restrict__ sv,
                                                    double *__restrict__ pbb, int32_t *isc, double *scal, int maxit,
                                                    int eta_mode, int first, double eta_host, double rtol_min,
                                                    double eta_max, double grad_rtol) {
    __shared__ double sh[kBlock / 64];
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n = S.n_cp;
    // the gradient stop (below) is known to every thread: a solve that will not run keeps x0 = 0
    const double gn0 = sqrt(scal[S_GG]);
    const bool gstop = grad_rtol > 0.0 && (gn0 == 0.0 || (!first && gn0 <= grad_rtol * scal[S_G0]));
    double ws = 0.0;
    if (ph && !gstop) {                          // uniform over the block
        double tot[4];
        ws = ws_decide(wpart, wstride, wnb, scal[S_GG], tot);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) scal[S_WS0 + k] = tot[k];
        }
    }
    if (ph && blockIdx.x == 0 && threadIdx.x == 0) {
        scal[S_WSA] = ws;
        isc[I_WS] = ws != 0.0 ? 1 : 0;
    }
    double bb = 0.0;
    if (a < S.n_cp) {
        for (int c = 0; c < 3; ++c) {
            const size_t k = c * n + a;
            const double bc = b[k];
            if (ws != 0.0) {
                const double aq = ws * hq[k];
                x0[k] = ws * ph[k];
                r[k] = bc - aq;
            } else {
                if (ph) x0[k] = 0.0;
                r[k] = bc;
            }
            p[k] = 0.0;
            sv[k] = 0.0;
            bb += bc * bc;
        }
    }
    bb = block_sum(bb, sh);
    if (threadIdx.x == 0) pbb[blockIdx.x] = bb;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        isc[I_DONE] = 0; isc[I_ITA] = 0; isc[I_ITB] = 0; isc[I_BREAK] = 0; isc[I_MAXIT] = maxit; isc[I_ITERS] = 0;
        const double gn = sqrt(scal[S_GG]);
        const double eta = forcing_term(eta_mode, first, eta_host, rtol_min, eta_max, gn, scal[S_GPREV], scal[S_ETA]);
        scal[S_RTOL] = eta;
        scal[S_ETA] = eta;
        scal[S_GPREV] = gn;
        // gradient rule with the solve enqueued before the host has read |g|: a Newton iterate
        // that already meets |g| <= grad_rtol |g0| (or |g| = 0) solves nothing (the host stops)
        if (first) scal[S_G0] = gn;
        if (gstop) isc[I_DONE] = 1;
    }
}

// ---- fused CG iteration ---------------------------------------------------------------------
//
// Launch K_j (j >= 1) finishes CG iteration j-1 and starts iteration j in one kernel, on a tile
// of kCgTileU x kCgTileV control points:
//   prologue  gamma, delta, rho of iteration j-1 re-summed from the partials of K_{j-1} in
//             every block (fixed order); stop test; alpha_{j-1}, beta_{j-1}.
//   footprint for every CP of the tile and its 2-CP stencil halo:
//               s_{j-1} = w_{j-1} + beta s_{j-2},  r_j = r_{j-1} - alpha s_{j-1},  u_j = M^-1 r_j
//             into LDS (one expression everywhere, so all blocks agree bitwise on u_j); on the
//             tile's own CPs also p_{j-1} = M^-1 r_{j-1} + beta p_{j-2}, x += alpha p_{j-1}, and
//             the stores of s_{j-1}, r_j, p_{j-1}, x.
//   SpMV      w_j = A u_j with u from LDS (8 waves; each wave one group of block products of a
//             64-row set).
//   partials  r_j.u_j, w_j.u_j, r_j.r_j per block.
// u is never stored: M^-1 r is recomputed from r. r, w, s and the partials are double-buffered by
// the parity of j, so no block reads a value another block of the same launch writes. K_0
// (FIRST) forms u_0, w_0 = A u_0, its partials and the threshold rtol^2 b.b.

struct CgBufs {
    double *x, *p;
    const double *r_in, *s_in;                    // r_{j-1}, s_{j-2}
    double *r_out, *s_out;                        // r_j, s_{j-1}
    const void *w_in;                             // w_{j-1}, working precision (SpMV output)
    void *w_out;                                  // w_j
    const void *pinv;                             // block-Jacobi inverse, working precision
    const double *part_in;                        // 3 arrays (stride) from K_{j-1}
    double *part_out;                             // 3 arrays (stride) for K_{j+1}
    const double *pbb;                            // b.b partials of the init kernel (FIRST)
    const double *pre;                            // the sums of part_in (large grids), or null
    int stride, nb_init;
    int slot_in, slot_out;                        // iteration-counter slots (alternate)
    // K_0 with the set-up folded in (fold != 0; otherwise k_cg_init ran before it): r_0 = b - a hq
    // formed on every footprint and x_0 = a ph, with the multiple a decided in every block from
    // the warm start's dot-product partials (wpart; ph null: a = 0), then the gradient stop, the
    // forcing term, the tolerance rtol^2 |g|^2 (b = -g) and the flags by block 0
    const double *b, *hq, *ph, *wpart;
    int fold, wstride, wnb, maxit, eta_mode, first;
    double eta_host, rtol_min, eta_max, grad_rtol;
};

template <typename T, bool FIRST>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) k_cg_fused(DevSheet S, const T *__restrict__ H, CgBufs B, double *scal,
                                                  int32_t *isc) {
    constexpr int TX = kCgTileU, TY = kCgTileV, HX = TX + 4, HY = TY + 4, R = TX * TY;
    constexpr int RS = R / 64, PG = 8 / RS;      // 64-row sets, product groups per set
    constexpr int NP = (25 + PG - 1) / PG;       // block products per wave
    static_assert(R % 64 == 0 && 8 % RS == 0 && HX * HY <= 512, "tile shape");
    __shared__ T us[3][HY][HX];
    __shared__ double u64[3][R];
    __shared__ T ys[8][3][64];
    __shared__ double sh[48];
    const bool fold = FIRST && B.fold;
    if (!fold && isc[I_DONE]) return;
    const T *__restrict__ w_in = (const T *)B.w_in;
    const T *__restrict__ pinv = (const T *)B.pinv;
    T *__restrict__ w_out = (T *)B.w_out;
    const int nb = gridDim.x;
    const int ntx = (S.n_u + TX - 1) / TX;
    const int tile = xcd_tile(blockIdx.x, nb);
    const int tx0 = (tile % ntx) * TX, ty0 = (tile / ntx) * TY;
    const size_t n = S.n_cp;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;

    // (1) loads that do not depend on this launch's scalars: first the partials and scalars of
    //     the previous launch (waited for at once), then the footprint vectors (in flight during
    //     the cross-wave half of the reduction)
    double v[3] = {0.0, 0.0, 0.0};
    int it = 0, maxit = 0;
    double tol2 = 0.0, gam01[2] = {0.0, 0.0}, alp01[2] = {0.0, 0.0};
    if (!FIRST) {
        it = isc[B.slot_in];                      // CG updates done before this launch (j - 1)
        maxit = isc[I_MAXIT];
        tol2 = scal[S_TOL2];
        gam01[0] = scal[S_GAMMA0]; gam01[1] = scal[S_GAMMA1];
        alp01[0] = scal[S_ALPHA0]; alp01[1] = scal[S_ALPHA1];
        if (!B.pre) {
            if (int(threadIdx.x) < nb) {
                v[0] = B.part_in[threadIdx.x];
                v[1] = B.part_in[B.stride + threadIdx.x];
                v[2] = B.part_in[2 * B.stride + threadIdx.x];
            }
            for (int t = threadIdx.x + blockDim.x; t < nb; t += blockDim.x) {
                v[0] += B.part_in[t];
                v[1] += B.part_in[B.stride + t];
                v[2] += B.part_in[2 * B.stride + t];
            }
        }
    } else if (blockIdx.x == 0 && !fold) {
        for (int t = threadIdx.x; t < B.nb_init; t += blockDim.x) v[0] += B.pbb[t];
    }
    // wave sums now, so that only the partials are waited for; the cross-wave half of the
    // reduction runs after the loads below are issued (a barrier does not wait for loads)
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = wave_sum_all(v[k]);
    const int g = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rs = g / PG, pg = g % PG;
    const int rrow = rs * 64 + lane;
    const int lx = rrow % TX, ly = rrow / TX;
    const int ri_ = tx0 + lx, rj_ = ty0 + ly;
    const bool row_ok = ri_ < S.n_u && rj_ < S.n_v;
    const int ra = row_ok ? rj_ * S.n_u + ri_ : 0;
    // the footprint CP of this thread (the tile and its 2-CP halo)
    const int t = threadIdx.x;
    const int hx = t % HX, hy = t / HX;
    const int fi = tx0 - 2 + hx, fj = ty0 - 2 + hy;
    const bool fp = t < HX * HY && fi >= 0 && fi < S.n_u && fj >= 0 && fj < S.n_v;
    const bool own = fp && hx >= 2 && hx < 2 + TX && hy >= 2 && hy < 2 + TY;
    const int fa = fp ? fj * S.n_u + fi : 0;
    // (w and M^-1 stay in the working precision until phase 3: a conversion here would wait for
    // the loads before the prologue)
    double rin[3] = {0.0, 0.0, 0.0}, sin_[3] = {0.0, 0.0, 0.0};
    double po[3] = {0.0, 0.0, 0.0}, xo[3] = {0.0, 0.0, 0.0};
    T win_t[3] = {T(0), T(0), T(0)}, pv_t[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    double hqf[3] = {0.0, 0.0, 0.0}, phf[3] = {0.0, 0.0, 0.0};
    if (fp) {
        if (fold) {
            // r_0 = b - a hq once a is known (below); b into rin for now
#pragma unroll
            for (int c = 0; c < 3; ++c) rin[c] = B.b[c * n + fa];
            if (B.ph) {
#pragma unroll
                for (int c = 0; c < 3; ++c) hqf[c] = B.hq[c * n + fa];
                if (own) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) phf[c] = B.ph[c * n + fa];
                }
            }
        } else {
#pragma unroll
            for (int c = 0; c < 3; ++c) rin[c] = B.r_in[c * n + fa];
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) pv_t[k] = pinv[k * n + fa];
        if (!FIRST) {
#pragma unroll
            for (int c = 0; c < 3; ++c) { win_t[c] = w_in[c * n + fa]; sin_[c] = B.s_in[c * n + fa]; }
            if (own) {
#pragma unroll
                for (int c = 0; c < 3; ++c) { po[c] = B.p[c * n + fa]; xo[c] = B.x[c * n + fa]; }
            }
        }
    }
    // the wave's first NPRE Hessian blocks (FP32: they depend on nothing computed below), issued
    // now so that their latency overlaps the prologue; at most 63 loads are outstanding per wave.
    // The scheduling fence keeps them behind the footprint loads, which phase 3 waits for.
    __builtin_amdgcn_sched_barrier(0);
    constexpr bool BRANCH_FREE = sizeof(T) == 4;
    constexpr int NPRE = BRANCH_FREE ? (kCgPrefetch < NP ? kCgPrefetch : NP) : 0;
    // One straight-line sequence of 9 loads per block on every path (the diagonal block's 6
    // planes padded with repeats), so that the wait for the footprint loads in phase 3 does not
    // have to cover these.
    static_assert(NPRE == 0 || PG * NPRE <= 25, "prefetched products are all real");
    T hpre[NPRE > 0 ? NPRE : 1][9];
#pragma unroll
    for (int m = 0; m < NPRE; ++m) {
        const int pid = pg + PG * m;
        const bool diag = pid == 0, upper = pid <= 12;
        const int sl = diag ? 1 : (upper ? pid : pid - 12);
        const int di = slot_di(sl), dj = slot_dj(sl), e0 = slot_entry(sl);
        const int ib = upper ? ri_ + di : ri_ - di, jb = upper ? rj_ + dj : rj_ - dj;
        const bool ok = row_ok && ib >= 0 && ib < S.n_u && jb >= 0 && jb < S.n_v;
        const int src = (upper || !ok) ? ra : jb * S.n_u + ib;
#pragma unroll
        for (int k = 0; k < 9; ++k) hpre[m][k] = H[size_t(diag ? (k < 6 ? k : 5) : e0 + k) * n + src];
    }

    // (2) prologue: the scalars of iteration j-1 (bitwise the same in every block)
    double alpha = 0.0, beta = 0.0;
    if (!FIRST) {
        wave_totals3(v, sh);
        if (B.pre) {
            v[0] = B.pre[0];
            v[1] = B.pre[1];
            v[2] = B.pre[2];
        }
        const double gam = v[0], del = v[1], rho = v[2];
        if (rho <= tol2 || it >= maxit || !(rho == rho)) {
            if (lead) { isc[I_ITERS] = it; isc[I_DONE] = 1; }
            return;
        }
        if (it == 0) {
            alpha = del > 0.0 ? gam / del : -1.0;
        } else {
            const double gprev = gam01[(it + 1) & 1], aprev = alp01[(it + 1) & 1];
            beta = gam / gprev;
            const double den = del - beta * gam / aprev;
            alpha = den > 0.0 ? gam / den : -1.0;
        }
        if (!(alpha > 0.0)) {                     // p^T A p <= 0: breakdown
            if (lead) { isc[I_ITERS] = it; isc[I_BREAK] = 1; isc[I_DONE] = 1; }
            return;
        }
        if (lead) {
            scal[S_GAMMA0 + (it & 1)] = gam;
            scal[S_ALPHA0 + (it & 1)] = alpha;
            scal[S_RHO] = rho;                    // |r|^2 of iteration j-1: read by the host between bursts
            isc[B.slot_out] = it + 1;
        }
    } else if (!fold) {
        if (blockIdx.x == 0) {                    // uniform per block
            wave_totals3(v, sh);
            if (threadIdx.x == 0) {
                scal[S_TOL2] = scal[S_RTOL] * scal[S_RTOL] * v[0];
                isc[B.slot_out] = 0;
            }
        }
    }
    // the folded set-up (the same decisions as k_cg_init, made by every block alike)
    double ws = 0.0;
    bool gstop = false;
    if (fold) {
        const double gg = scal[S_GG], gn0 = sqrt(gg);
        gstop = B.grad_rtol > 0.0 && (gn0 == 0.0 || (!B.first && gn0 <= B.grad_rtol * scal[S_G0]));
        double tot[4] = {0.0, 0.0, 0.0, 0.0};
        if (B.ph && !gstop) ws = ws_decide(B.wpart, B.wstride, B.wnb, gg, tot);
        if (lead) {
            if (B.ph) {
                if (!gstop) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) scal[S_WS0 + k] = tot[k];
                }
                scal[S_WSA] = ws;
                isc[I_WS] = ws != 0.0 ? 1 : 0;
            }
            isc[I_ITA] = 0; isc[I_ITB] = 0; isc[I_BREAK] = 0; isc[I_MAXIT] = B.maxit; isc[I_ITERS] = 0;
            const double eta = forcing_term(B.eta_mode, B.first, B.eta_host, B.rtol_min, B.eta_max, gn0, scal[S_GPREV],
                                            scal[S_ETA]);
            scal[S_RTOL] = eta;
            scal[S_ETA] = eta;
            scal[S_GPREV] = gn0;
            scal[S_TOL2] = eta * eta * gg;        // b = -g: |b|^2 = |g|^2
            if (B.first) scal[S_G0] = gn0;
            isc[I_DONE] = gstop ? 1 : 0;
        }
        if (ws != 0.0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) rin[c] = rin[c] - ws * hqf[c];
        }
    }

    // (3) footprint: s, r, u = M^-1 r; own CPs also p, x and the stores
    double gam = 0.0, rho = 0.0, del = 0.0;
    if (t < HX * HY) {
        double uv[3] = {0.0, 0.0, 0.0};
        if (fp) {
            double rv[3], sc[3], win[3], pv[6];
#pragma unroll
            for (int c = 0; c < 3; ++c) win[c] = double(win_t[c]);
#pragma unroll
            for (int k = 0; k < 6; ++k) pv[k] = double(pv_t[k]);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                sc[c] = win[c] + beta * sin_[c];
                rv[c] = FIRST ? rin[c] : rin[c] - alpha * sc[c];
            }
            uv[0] = pv[0] * rv[0] + pv[1] * rv[1] + pv[2] * rv[2];
            uv[1] = pv[1] * rv[0] + pv[3] * rv[1] + pv[4] * rv[2];
            uv[2] = pv[2] * rv[0] + pv[4] * rv[1] + pv[5] * rv[2];
            if (own) {
                if (fold) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const size_t k = c * n + fa;
                        B.x[k] = ws * phf[c];
                        B.r_out[k] = rv[c];
                        B.p[k] = 0.0;
                        B.s_out[k] = 0.0;
                    }
                }
                if (!FIRST) {
                    double uo[3];
                    uo[0] = pv[0] * rin[0] + pv[1] * rin[1] + pv[2] * rin[2];
                    uo[1] = pv[1] * rin[0] + pv[3] * rin[1] + pv[4] * rin[2];
                    uo[2] = pv[2] * rin[0] + pv[4] * rin[1] + pv[5] * rin[2];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const size_t k = c * n + fa;
                        const double pc = uo[c] + beta * po[c];
                        B.p[k] = pc;
                        B.x[k] = xo[c] + alpha * pc;
                        B.s_out[k] = sc[c];
                        B.r_out[k] = rv[c];
                    }
                }
                const int o = (hy - 2) * TX + (hx - 2);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    u64[c][o] = uv[c];
                    gam += rv[c] * uv[c];
                    rho += rv[c] * rv[c];
                }
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) us[c][hy][hx] = T(uv[c]);
    }
    __syncthreads();
    if (gstop) return;                            // uniform: the iterate already meets the stop

    // (4) w = A u for the wave's block products, u from LDS. In FP32, out-of-grid neighbours read
    //     a valid row and take u = 0, so the body has no data-dependent branch and the compiler
    //     keeps several products' loads in flight; FP64 blocks take twice the registers, so there
    //     they are skipped by a branch (higher occupancy).
    {
        T acc[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int m = 0; m < NP; ++m) {
            const int pid = pg + PG * m;                 // wave-uniform
            if (pid >= 25) break;
            if (pid == 0) {
                T h[6];
#pragma unroll
                for (int k = 0; k < 6; ++k) h[k] = m < NPRE ? hpre[m < NPRE ? m : 0][k] : H[k * n + ra];
                const T u0 = us[0][ly + 2][lx + 2], u1 = us[1][ly + 2][lx + 2], u2 = us[2][ly + 2][lx + 2];
                acc[0] += h[0] * u0 + h[1] * u1 + h[2] * u2;
                acc[1] += h[1] * u0 + h[3] * u1 + h[4] * u2;
                acc[2] += h[2] * u0 + h[4] * u1 + h[5] * u2;
                continue;
            }
            const bool upper = pid <= 12;
            const int sl = upper ? pid : pid - 12;
            const int di = slot_di(sl), dj = slot_dj(sl), e0 = slot_entry(sl);
            const int sgn = upper ? 1 : -1;
            const int ib = ri_ + sgn * di, jb = rj_ + sgn * dj;
            const bool ok = row_ok && ib >= 0 && ib < S.n_u && jb >= 0 && jb < S.n_v;
            if constexpr (!BRANCH_FREE) {
                if (!ok) continue;
            }
            const int src = (upper || !ok) ? ra : jb * S.n_u + ib;
            T h[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) h[k] = m < NPRE ? hpre[m < NPRE ? m : 0][k] : H[(e0 + k) * n + src];
            const int yy = ly + 2 + sgn * dj, xx = lx + 2 + sgn * di;
            const T u0 = ok ? us[0][yy][xx] : T(0), u1 = ok ? us[1][yy][xx] : T(0), u2 = ok ? us[2][yy][xx] : T(0);
            if (upper) {
#pragma unroll
                for (int q = 0; q < 3; ++q) acc[q] += h[3 * q] * u0 + h[3 * q + 1] * u1 + h[3 * q + 2] * u2;
            } else {
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[c] += h[c] * u0 + h[3 + c] * u1 + h[6 + c] * u2;
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) ys[g][c][lane] = acc[c];
    }
    __syncthreads();

    // (5) w_j, the partials r.u, w.u, r.r
    if (threadIdx.x < R) {
        const int rr = threadIdx.x, rset = rr >> 6, l = rr & 63;
        const int gi = tx0 + rr % TX, gj = ty0 + rr / TX;
        if (gi < S.n_u && gj < S.n_v) {
            const int a = gj * S.n_u + gi;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                T y = ys[rset * PG][c][l];
#pragma unroll
                for (int q = 1; q < PG; ++q) y += ys[rset * PG + q][c][l];
                w_out[c * n + a] = y;
                del += double(y) * u64[c][rr];
            }
        }
    }
    double w3[3] = {gam, del, rho};
    block_sum3(w3, sh);
    if (threadIdx.x == 0) {
        B.part_out[blockIdx.x] = w3[0];
        B.part_out[B.stride + blockIdx.x] = w3[1];
        B.part_out[2 * B.stride + blockIdx.x] = w3[2];
    }
}

// Large grids: the sums of one fused launch's partials (r.u, w.u, r.r) in a fixed order, formed
// once for the next launch to read.
__global__ void __launch_bounds__(1024) k_cg_sum(const double *__restrict__ part, int stride, int nb,
                                                 const int32_t *__restrict__ isc, double *__restrict__ out) {
    __shared__ double sh[48];
    if (isc[I_DONE]) return;
    double v[3] = {0.0, 0.0, 0.0};
    for (int t = threadIdx.x; t < nb; t += blockDim.x) {
        v[0] += part[t];
        v[1] += part[stride + t];
        v[2] += part[2 * stride + t];
    }
    block_sum3(v, sh);
    if (threadIdx.x == 0) {
        out[0] = v[0];
        out[1] = v[1];
        out[2] = v[2];
    }
}

// ---- warm start and sample log ------------------------------------------------------------

__global__ void k_to_float(int n, const double *__restrict__ x, float *__restrict__ y) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] = float(x[t]);
}

// p_hat (double) from the net output, zero on pinned CPs.
__global__ void k_phat(int n_cp, const float *__restrict__ out, const int32_t *__restrict__ pinmask, double *__restrict__ ph) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n_cp) return;
    const bool pinned = pinmask[a] != 0;
    for (int c = 0; c < 3; ++c) ph[c * n_cp + a] = pinned ? 0.0 : double(out[c * n_cp + a]);
}

// ---- line search -------------------------------------------------------------------------

// The energy difference along p is dE(alpha) = alpha c1 + alpha^2 c2 / 2 for the inertia,
// gravity and bending terms (quadratics in alpha) plus the membrane term, summed point by point.
// Per CP, in one pass over p: partials of c1 = gpre . p over the quadratic terms (gpre: the
// assembly's per-CP gradient terms at x, bending included), of the inertia's part of c2,
// M p . p / dt^2, and of max |p| (the stop tests). The bending part of c2 comes from the
// bending evaluations (ls_bend_block).
__device__ __forceinline__ void ls_cp_block(const DevSheet &S, const double *__restrict__ gpre, const double *__restrict__ p,
                                            double inv_dt2, double *partials, int stride, double *__restrict__ pmax_part,
                                            int blk) {
    __shared__ double sh[kBlock / 64];
    const int a = blk * blockDim.x + threadIdx.x;
    const size_t n = S.n_cp;
    double c1 = 0.0, c2 = 0.0, m = 0.0;
    if (a < S.n_cp) {
        const double M = S.mass[a];
        for (int c = 0; c < 3; ++c) {
            const double pc = p[c * n + a];
            c1 += gpre[c * n + a] * pc;
            c2 += M * inv_dt2 * pc * pc;
            m = fmax(m, fabs(pc));
        }
    }
    c1 = block_sum(c1, sh);
    c2 = block_sum(c2, sh);
    if (threadIdx.x == 0) { partials[blk] = c1; partials[stride + blk] = c2; }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < int(blockDim.x >> 6); ++w) m = fmax(m, sh[w]);
        pmax_part[blk] = m;
    }
}

__global__ void __launch_bounds__(kBlock) k_ls_cp(DevSheet S, const double *__restrict__ gpre, const double *__restrict__ p,
                                                  double inv_dt2, double *partials, int stride, double *__restrict__ pmax_part) {
    ls_cp_block(S, gpre, p, inv_dt2, partials, stride, pmax_part, blockIdx.x);
}

// The line-search scalars in one block, each in a fixed order: max |p| (exact in any order),
// c1 and c2 over the CP and bending partials, the membrane energy difference at alpha = 1;
// out[0..3] = max |p|, c1, c2, dE_membrane, valid in every thread of the block. Each thread
// reads its elements of all the partial arrays in one loop (the loads issue together), then
// the four values are reduced across the block at once.
__device__ void ls_sums(const double *__restrict__ pm, int n_cpb, const double *__restrict__ pa, const double *__restrict__ pb,
                        int n_beb, int stride, const double *__restrict__ pd, int n_mpb, double *sh, double out[4]) {
    __shared__ double res[4][kBlock / 64];
    double m = 0.0, c1 = 0.0, c2 = 0.0, dm = 0.0;
    const int n = max(max(n_cpb, n_beb), n_mpb);
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        if (t < n_cpb) {
            m = fmax(m, pm[t]);
            c1 += pa[t];
            c2 += pa[stride + t];
        }
        if (t < n_beb) {
            c1 += pb[t];
            c2 += pb[stride + t];
        }
        if (t < n_mpb) dm += pd[t];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        m = fmax(m, __shfl_down(m, off));
        c1 += __shfl_down(c1, off);
        c2 += __shfl_down(c2, off);
        dm += __shfl_down(dm, off);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        res[0][wid] = m;
        res[1][wid] = c1;
        res[2][wid] = c2;
        res[3][wid] = dm;
    }
    __syncthreads();
    double r[4] = {res[0][0], res[1][0], res[2][0], res[3][0]};
    for (int w = 1; w < int(blockDim.x >> 6); ++w) {
        r[0] = fmax(r[0], res[0][w]);
        r[1] += res[1][w];
        r[2] += res[2][w];
        r[3] += res[3][w];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = r[k];
    (void)sh;
}

__global__ void __launch_bounds__(kBlock) k_ls_finish(const double *__restrict__ pm, int n_cpb, const double *__restrict__ pa,
                                                      const double *__restrict__ pb, int n_beb, int stride,
                                                      const double *__restrict__ pd, int n_mpb, double *scal) {
    __shared__ double sh[kBlock / 64];
    double r[4];
    ls_sums(pm, n_cpb, pa, pb, n_beb, stride, pd, n_mpb, sh, r);
    if (threadIdx.x == 0) { scal[S_PMAX] = r[0]; scal[S_C1] = r[1]; scal[S_C2] = r[2]; scal[S_DEM] = r[3]; }
}

// Per bending evaluation: partials of the bending term's c2 = sum_q w mu |Laplacian(p)|^2 (its
// Laplacian is linear in the CPs); its c1 is part of gpre . p. The c1 partial is zero.
__device__ __forceinline__ void ls_bend_block(const DevSheet &S, const double *__restrict__ p, double *partials, int stride,
                                              int blk) {
    __shared__ double sh[kBlock / 64];
    const int q = blk * blockDim.x + threadIdx.x;
    const size_t n = S.n_cp;
    double c2 = 0.0;
    if (q < S.n_be) {
        const int e = S.be_elem[q], k = e % S.Nu, l = e / S.Nu;
        // Laplacian weights of the 9 local CPs (the same as the bending kernel's)
        double L[9];
        bend_L(S, be_geo(S, q), k, l, S.be_tu[q], S.be_tv[q], L);
        double lp[3] = {0.0, 0.0, 0.0};
        for (int m = 0; m < 9; ++m) {
            const int cp = (l + m / 3) * S.n_u + (k + m % 3);
            for (int c = 0; c < 3; ++c) lp[c] += L[m] * p[c * n + cp];
        }
        const double wm = S.be_w[q] * S.mu_bend;
        for (int c = 0; c < 3; ++c) c2 += wm * lp[c] * lp[c];
    }
    c2 = block_sum(c2, sh);
    if (threadIdx.x == 0) { partials[blk] = 0.0; partials[stride + blk] = c2; }
}

__global__ void __launch_bounds__(kBlock) k_ls_quad_bend(DevSheet S, const double *__restrict__ p, double *partials, int stride) {
    ls_bend_block(S, p, partials, stride, blockIdx.x);
}

// Membrane energy difference sum_q w (Psi(F + alpha dF) - Psi(F)) in double.
__device__ __forceinline__ void ls_membrane_block(const DevSheet &S, const double *__restrict__ x, const double *__restrict__ p,
                                                  double alpha, double *partials, int blk) {
    __shared__ double sh[kBlock / 64];
    const int q = blk * blockDim.x + threadIdx.x;
    const size_t n = S.n_cp;
    double de = 0.0;
    if (q < S.n_mp) {
        const int e = S.mp_elem[q], k = e % S.Nu, l = e / S.Nu;
        double dN[9][2];
        local_grads<double>(S, mp_geo(S, q), k, l, S.mp_tu[q], S.mp_tv[q], dN);
        double G[3][2] = {{0, 0}, {0, 0}, {0, 0}}, dG[3][2] = {{0, 0}, {0, 0}, {0, 0}};
        for (int m = 0; m < 9; ++m) {
            const int cp = (l + m / 3) * S.n_u + (k + m % 3);
            double d[3];
            displacement(S, x, k + m % 3, l + m / 3, d);
            for (int c = 0; c < 3; ++c) {
                G[c][0] += d[c] * dN[m][0]; G[c][1] += d[c] * dN[m][1];
                const double pcv = p[c * n + cp];
                dG[c][0] += pcv * dN[m][0]; dG[c][1] += pcv * dN[m][1];
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
    if (threadIdx.x == 0) partials[blk] = s;
}

__global__ void __launch_bounds__(kBlock) k_ls_membrane(DevSheet S, const double *__restrict__ x, const double *__restrict__ p,
                                                        double alpha, double *partials) {
    ls_membrane_block(S, x, p, alpha, partials, blockIdx.x);
}

// The line-search set-up in one launch, gated by the solve's done flag (the end of a PCG burst):
// blocks [0, nbc) the CP terms, [nbc, nbc + nbb) the bending terms, the rest the membrane
// energy difference at alpha = 1; each block writes the partial slot its own launch would.
__global__ void __launch_bounds__(kBlock) k_ls_setup(DevSheet S, const double *__restrict__ x, const double *__restrict__ gpre,
                                                     const double *__restrict__ p, double inv_dt2, double *pa, int stride,
                                                     double *__restrict__ pmax_part, double *pbend, double *pmem, int nbc, int nbb,
                                                     const int32_t *__restrict__ gate) {
    if (!gate[I_DONE]) return;
    const int b = blockIdx.x;
    if (b < nbc) ls_cp_block(S, gpre, p, inv_dt2, pa, stride, pmax_part, b);
    else if (b < nbc + nbb) ls_bend_block(S, p, pbend, stride, b - nbc);
    else ls_membrane_block(S, x, p, 1.0, pmem, b - nbc - nbb);
}

__global__ void k_sum_into(const double *__restrict__ p, int n, double *scal, int slot) {
    __shared__ double sh[kBlock / 64];
    double v = 0.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) v += p[t];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) scal[slot] = v;
}


// Copies the solver scalars and flags into host-mapped coherent pinned memory, then publishes the
// next sequence number (kept in the device flags, so that the kernel can sit in a replayed
// graph) behind a system-scope fence. The host polls that number instead of waiting for a
// stream synchronisation, which wakes it sooner.
__global__ void __launch_bounds__(64) k_publish(const double *__restrict__ scal, int32_t *__restrict__ flags, PubPtrs P) {
    publish_block(scal, flags, P);
}

__global__ void k_update(int n, double alpha, const double *__restrict__ p, double *__restrict__ x) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) x[t] += alpha * p[t];
}

// The line search's first trial on the device, at the end of the burst in which the solve
// finished (gated by its done flag; not after a breakdown). Every block re-sums the line-search
// partials in k_ls_finish's order (block 0 stores the scalars), so every thread takes the same
// decision: dE(1) = (c1 + c2 / 2) + dE_membrane in the host's order and rounding. A direction
// below the stagnation scale (|p|_inf <= stag |x0|_inf, when stag > 0) leaves x untouched (flag
// 2); dE(1) finite and <= 0 applies x += p, the same update as k_update with alpha = 1 (flag 1);
// otherwise x is untouched (flag 0) and the host halves alpha. With do_pub, block 0 then
// publishes the scalars and flags to the host (gate open or not): the burst's read-back.
__global__ void __launch_bounds__(kBlock) k_ls_accept(int n, int32_t *isc, double *scal, const double *__restrict__ pm,
                                                      int n_cpb, const double *__restrict__ pa, const double *__restrict__ pb,
                                                      int n_beb, int stride, const double *__restrict__ pd, int n_mpb,
                                                      const double *__restrict__ p, double *__restrict__ x, double stag,
                                                      PubPtrs pub, int do_pub) {
    __shared__ double sh[kBlock / 64];
    if (isc[I_DONE] && !isc[I_BREAK]) {
        double r[4];
        ls_sums(pm, n_cpb, pa, pb, n_beb, stride, pd, n_mpb, sh, r);
        const double dE = __dadd_rn(__dadd_rn(r[1], __dmul_rn(0.5, r[2])), r[3]);
        int d = (std::isfinite(dE) && dE <= 0.0) ? 1 : 0;
        if (stag > 0.0 && r[0] <= stag * scal[S_XMAX]) d = 2;
        const int t = blockIdx.x * blockDim.x + threadIdx.x;
        if (d == 1 && t < n) x[t] += 1.0 * p[t];
        if (t == 0) {
            scal[S_PMAX] = r[0]; scal[S_C1] = r[1]; scal[S_C2] = r[2]; scal[S_DEM] = r[3];
            isc[I_LSACC] = d;
        }
    }
    if (do_pub && blockIdx.x == 0) {
        __syncthreads();
        publish_block(scal, isc, pub);
    }
}

// dE(alpha) = alpha c1 + alpha^2 c2 / 2 + (membrane difference at alpha), the line search's
// energy difference, written to device memory (bsc_energy_difference).
__global__ void k_de_combine(const double *__restrict__ scal, double alpha, double *__restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *out = alpha * scal[S_C1] + 0.5 * alpha * alpha * scal[S_C2] + scal[S_DEM];
}

}  // namespace

inline int spmv_blocks(int n_cp) { return (n_cp + kRowsPerTile - 1) / kRowsPerTile; }
inline int cg_blocks(int n_u, int n_v) { return ((n_u + kCgTileU - 1) / kCgTileU) * ((n_v + kCgTileV - 1) / kCgTileV); }

hipError_t launch_spmv(const DevSheet &S, int precision, const void *hess, const double *in, double *out, hipStream_t st) {
    const int nb = spmv_blocks(S.n_cp);
    if (precision == BSC_FP64)
        k_spmv_tile<double><<<nb, kRowsPerTile * kGroups, 0, st>>>(S, (const double *)hess, in, out);
    else
        k_spmv_tile<float><<<nb, kRowsPerTile * kGroups, 0, st>>>(S, (const float *)hess, in, out);
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
    explicit Timer(hipStream_t s, bool on = true) : st(s), a(nullptr), b(nullptr), ok(false) {
        if (!on) return;
        if (hipEventCreate(&a) != hipSuccess) a = nullptr;
        if (hipEventCreate(&b) != hipSuccess) b = nullptr;
        ok = a && b;
        if (ok) (void)hipEventRecord(a, st);
        else (void)hipGetLastError();
    }
    double stop() {
        if (!ok) return 0.0;
        float ms = 0.f;
        (void)hipEventRecord(b, st);
        (void)hipEventSynchronize(b);
        (void)hipEventElapsedTime(&ms, a, b);
        return ms;
    }
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

#define HIPX(expr, what)                                            \
    do {                                                            \
        hipError_t e_ = (expr);                                     \
        if (e_ != hipSuccess) return hip_check(ctx, e_, what);      \
    } while (0)

// Assembles E, g (double), |g|^2 and H (working precision) at x for one Newton iteration. With
// red, E and |g|^2 are left to the next kernel (energy_reduce_block), whose arguments go to red.
bsc_status assemble_iter(bsc_ctx *ctx, int prec, const double *x, const double *xhat, double inv_dt2, const double *grav,
                         hipStream_t st, const PubPtrs *pub, EnergyRed *red = nullptr) {
    const DevSheet &S = ctx->dev;
    const DevBufs &B = ctx->buf;
    // FP32-mixed: the points in FP64 arithmetic, the Hessian stored in FP32 and the stresses (for
    // the FP64 gradient and energy) in FP64
    const CpTerms cpt{xhat, inv_dt2, grav ? grav[0] : 0.0, grav ? grav[1] : 0.0, grav ? grav[2] : 0.0, B.gpre};
    if (prec == BSC_FP64) HIPX(launch_points(S, B, BSC_FP64, true, false, x, st, false, &cpt), "points");
    else HIPX(launch_points_mixed(S, B, x, st, &cpt), "points");
    const int kind = prec == BSC_FP64 ? kAsmF64 : kAsmMixed;
    HIPX(launch_assemble(S, B, kind, inv_dt2, B.g, B.hess, st, true), "assemble");
    if (red) {
        // the same arrays and counts as launch_energy_reduce
        const int mb = B.max_blocks;
        *red = EnergyRed{B.partials, B.partials + mb, B.partials + 2 * mb, B.partials + 3 * mb, blocks(S.n_mp), 0,
                         cp_blocks(S), assemble_tiles(S, kind), B.scalars + S_E, B.scalars + S_GG,
                         pub ? *pub : PubPtrs{nullptr, nullptr, nullptr}, pub ? 1 : 0};
        return BSC_OK;
    }
    HIPX(launch_energy_reduce(S, B, cp_blocks(S), assemble_tiles(S, kind), B.scalars + S_E, st, B.scalars + S_GG, pub),
         "energy");
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
    const bool step_rule = o->fixed_newton_iters <= 0 && o->stop_mode == BSC_STOP_STEP;
    // With the step rule nothing the host decides before the solve depends on the assembly: the
    // PCG tolerance is formed on the device and E, |g| are read back with |p| and the line
    // search's first trial after the solve, in one synchronisation. Both warm starts run on the
    // device without a host decision.
    const int warm = o->warm_start;
    const bool deferred = step_rule;
    const bool use_mg = o->preconditioner == BSC_PRECOND_MULTIGRID && B.mg_levels > 0 && !warm;
    // gradient rule (no multigrid): the PCG set-up follows the assembly without a host decision
    // (below), and the assembly's reduction publishes E and |g| in the same launch
    const bool early = !deferred && !use_mg;
    bsc_step_stats s{};
    double ls_in_bursts = 0.0;   // line-search kernels timed inside the PCG bursts (moved from ms_pcg)
    auto t_start = std::chrono::steady_clock::now();
    // Timing: events from a pool, recorded as the step goes and read once at its end (a read in
    // the middle of the step would wait for the event and delay the next launch). Each event sits
    // between two kernels and delays the second by a few microseconds (without the system-scope
    // fence, which a timestamp read after the stream's synchronisation does not need, by less), so
    // rec_cg() (the CG spans) records unless timing is off and rec() (the phases) only on request.
    size_t ev_used = 0;
    auto rec_any = [&](bool on) -> hipEvent_t {
        if (!on || ctx->ev_failed) return nullptr;
        if (ev_used == ctx->ev_pool.size()) {
            hipEvent_t e = nullptr;
            if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
                (void)hipGetLastError();
                ctx->ev_failed = true;
                return nullptr;
            }
            ctx->ev_pool.push_back(e);
        }
        hipEvent_t e = ctx->ev_pool[ev_used++];
        if (hipEventRecord(e, st) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return e;
    };
    const bool time_phases = o->timing == BSC_TIMING_PHASES, time_cg = o->timing != BSC_TIMING_OFF;
    auto rec = [&]() { return rec_any(time_phases); };
    auto rec_cg = [&]() { return rec_any(time_cg); };
    struct Span {
        hipEvent_t a, b;
        double *acc;
    };
    std::vector<Span> spans;
    auto span = [&](hipEvent_t a, hipEvent_t b, double *acc) {
        if (a && b) spans.push_back({a, b, acc});
    };
    // read-backs: the scalars and, right after them in the workspace, the int flags, in one copy
    // into pinned host memory
    if (!ctx->pinned) {
        HIPX(hipHostMalloc((void **)&ctx->pinned, 1024, hipHostMallocMapped | hipHostMallocCoherent), "pinned host buffer");
        std::memset(ctx->pinned, 0, 1024);
        if (hipHostGetDevicePointer((void **)&ctx->pinned_dev, ctx->pinned, 0) != hipSuccess) {
            ctx->pinned_dev = nullptr;
            (void)hipGetLastError();
        }
    }
    if ((const char *)B.iscalars != (const char *)B.scalars + 8 * kScalars) return fail(ctx, BSC_E_STATE, "workspace layout");
    const double *hs = (const double *)ctx->pinned;
    const int32_t *hf = (const int32_t *)(ctx->pinned + 8 * kScalars);
    // The sequence number sits after the flags. The host records it, enqueues work that ends in
    // k_publish, and spins until it moves on; every 1024 spins it asks the runtime whether the
    // stream has failed or gone idle (then the number must have moved; if it has not, the
    // read-back falls back to a copy and a synchronisation).
    int32_t *hseq = (int32_t *)(ctx->pinned + 8 * kScalars + 64);
    const bool pub = ctx->pinned_dev != nullptr;
    auto seen = [&]() { return __atomic_load_n(hseq, __ATOMIC_ACQUIRE); };
    const PubPtrs pubp{(double *)ctx->pinned_dev, (int32_t *)(ctx->pinned_dev + 8 * kScalars),
                       (int32_t *)(ctx->pinned_dev + 8 * kScalars + 64)};
    auto publish = [&](hipStream_t cs) {
        k_publish<<<1, 64, 0, cs>>>(B.scalars, B.iscalars, pubp);
    };
    auto copy_sync = [&]() -> hipError_t {
        hipError_t e = hipMemcpyAsync(ctx->pinned, B.scalars, 8 * kScalars + 4 * 8, hipMemcpyDeviceToHost, st);
        return e == hipSuccess ? hipStreamSynchronize(st) : e;
    };
    auto wait_pub = [&](int32_t last) -> hipError_t {
        for (long spin = 1;; ++spin) {
            if (seen() != last) return hipSuccess;
            if ((spin & 1023) == 0) {
                const hipError_t e = hipStreamQuery(st);
                if (e == hipSuccess) return seen() != last ? hipSuccess : copy_sync();
                if (e != hipErrorNotReady) return e;
            }
#if !defined(__HIP_DEVICE_COMPILE__)
            __builtin_ia32_pause();
#endif
        }
    };
    auto pull = [&]() -> hipError_t {
        if (!pub) return copy_sync();
        const int32_t last = seen();
        publish(st);
        const hipError_t e = hipGetLastError();
        return e == hipSuccess ? wait_pub(last) : e;
    };

    HIPX(hipMemcpyAsync(B.xn, x, 8 * size_t(n3), hipMemcpyDeviceToDevice, st), "copy x");
    k_axpby<<<blocks(n3), kBlock, 0, st>>>(n3, 1.0, x, dt, v, B.xhat);
    if (o->start == BSC_START_PREDICTOR)
        HIPX(hipMemcpyAsync(x, B.xhat, 8 * size_t(n3), hipMemcpyDeviceToDevice, st), "predictor start");
    if (npins > 0) k_apply_pins<<<blocks(npins), kBlock, 0, st>>>(S.n_cp, npins, B.pin_idx, pin_tgt, x);
    // the recycled warm start draws on the directions of this step only: its first Newton
    // iteration sees p = 0 and starts from zero (a new step solves for a new inertia term)
    if (o->warm_start == BSC_WARM_PREVIOUS) k_zero<<<blocks(n3), kBlock, 0, st>>>(n3, B.dir);
    // |x0|_inf: the scale below which a Newton update only moves x by rounding
    k_absmax_part<<<kReduceBlocks, kBlock, 0, st>>>(n3, x, B.partials + 7 * stride);
    k_finish<<<1, kBlock, 0, st>>>(B.partials + 7 * stride, kReduceBlocks, 1, B.scalars, S_XMAX);
    HIPX(hipGetLastError(), "step setup");

    bsc_status result = BSC_OK;
    double g0 = -1.0, g_prev = -1.0;
    const double eta_max = o->pcg_eta_max > 0.0 ? o->pcg_eta_max : (step_rule ? kEtaMaxStep : kEtaMaxGrad);
    double eta = o->pcg_adaptive ? std::max(o->pcg_rtol, eta_max) : o->pcg_rtol;   // PCG tolerance (host-side modes)
    bool force_tight = false;
    double host[2];
    int it = 0;
    for (;; ++it) {
        // ---- assembly: E, g, H at x ---------------------------------------------------------
        hipEvent_t e0 = rec();
        // (plain launches: the sequences of a Newton iteration measured faster enqueued directly
        // than replayed as captured graphs, whose switches with plain launches on the stream each
        // cost a gap)
        const int32_t last_asm = seen();
        // Under the gradient stop the first burst follows the set-up at once (speculative, below)
        // and its read-back carries E and |g| too, so the set-up publishes nothing of its own.
        const bool speculate = early && o->stop_mode == BSC_STOP_GRAD && o->fixed_newton_iters <= 0 && it < o->max_newton;
        EnergyRed red{};                 // early: E and |g|^2 summed (and published) by the PCG set-up's first kernel
        {
            const bsc_status sa = assemble_iter(ctx, prec, x, B.xhat, inv_dt2, grav, st,
                                                early && pub && !speculate ? &pubp : nullptr, early ? &red : nullptr);
            if (sa != BSC_OK) return sa;
        }
        hipEvent_t e1 = rec();
        int eta_mode = ETA_EXPLICIT;
        // CG vectors: p; r, w (= A M^-1 r) and s double-buffered by iteration parity (u = M^-1 r
        // is recomputed where it is needed)
        double *rb[2] = {B.r, B.r2}, *wb[2] = {B.q, B.q2}, *sb[2] = {B.p1, B.p2};
        double *p = B.p0;
        double *hq = rb[1];                      // H p_hat of the warm start (free until the CG's first odd launch)
        const int nbi = blocks(S.n_cp), nbc = cg_blocks(S.n_u, S.n_v);
        double *part[2] = {B.partials, B.partials + 3 * stride}, *pbb = B.partials + 6 * stride;
        const bool presum = nbc > kCgPreSumBlocks;
        auto bufs = [&](int j) {
            CgBufs c{};
            c.x = B.dir; c.p = p; c.pinv = B.pinv;
            c.pbb = pbb; c.stride = stride; c.nb_init = nbi;
            c.pre = presum ? B.scalars + S_CGSUM : nullptr;
            const int cur = j & 1, prev = (j + 1) & 1;
            c.r_in = rb[j == 0 ? 0 : prev]; c.r_out = rb[cur];
            c.w_in = wb[prev]; c.w_out = wb[cur];
            c.s_in = sb[prev]; c.s_out = sb[cur];
            c.part_in = part[prev]; c.part_out = part[cur];
            c.slot_in = prev ? I_ITB : I_ITA; c.slot_out = cur ? I_ITB : I_ITA;
            return c;
        };
        const int first = it == 0 ? 1 : 0;
        double eta_arg = 0.0;                    // the explicit mode's tolerance (set before the solve)
        double grad_rtol = 0.0;                  // the device-side gradient stop of the speculative solve
        // block-Jacobi inverse, b = -g, x0 = 0
        auto enqueue_prep = [&](hipStream_t cs) {
            if (prec == BSC_FP64)
                k_cg_prep<double><<<blocks(S.n_cp), kBlock, 0, cs>>>(S, (const double *)B.hess, (double *)B.pinv, B.g, B.tmp, B.dir,
                                                                      red, B.scalars, B.iscalars);
            else
                k_cg_prep<float><<<blocks(S.n_cp), kBlock, 0, cs>>>(S, (const float *)B.hess, (float *)B.pinv, B.g, B.tmp, B.dir,
                                                                     red, B.scalars, B.iscalars);
            red.out = nullptr;
        };
        // warm start from the prediction ph: H ph into hq with the partials of its four dot
        // products (k_cg_init sums them, decides and applies the start, all on the device), and
        // the set-up of enqueue_prep except x0 = 0 (k_cg_init writes every entry of x0)
        auto enqueue_warm = [&](hipStream_t cs, const double *ph) {
            const int nb = spmv_blocks(S.n_cp);
            if (prec == BSC_FP64)
                k_spmv_tile<double, true><<<nb, kRowsPerTile * kGroups, 0, cs>>>(S, (const double *)B.hess, ph, hq, B.g,
                                                                                B.partials + 4 * stride, stride,
                                                                                (double *)B.pinv, B.tmp, red, B.scalars,
                                                                                B.iscalars);
            else
                k_spmv_tile<float, true><<<nb, kRowsPerTile * kGroups, 0, cs>>>(S, (const float *)B.hess, ph, hq, B.g,
                                                                               B.partials + 4 * stride, stride,
                                                                               (float *)B.pinv, B.tmp, red, B.scalars,
                                                                               B.iscalars);
            red.out = nullptr;
        };
        // the first CG launch (it forms w_0) with the set-up folded in: r_0 = b - A x_0 (x_0 = a ph
        // with the decided multiple, when ph is given), the gradient stop, the tolerance and the flags
        auto enqueue_init = [&](hipStream_t cs, const double *ph) {
            CgBufs c0 = bufs(0);
            c0.fold = 1;
            c0.b = B.tmp; c0.hq = hq; c0.ph = ph;
            c0.wpart = B.partials + 4 * stride; c0.wstride = stride; c0.wnb = spmv_blocks(S.n_cp);
            c0.maxit = o->max_pcg; c0.eta_mode = eta_mode; c0.first = first; c0.eta_host = eta_arg;
            c0.rtol_min = o->pcg_rtol; c0.eta_max = eta_max; c0.grad_rtol = grad_rtol;
            if (prec == BSC_FP64)
                k_cg_fused<double, true><<<nbc, 512, 0, cs>>>(S, (const double *)B.hess, c0, B.scalars, B.iscalars);
            else
                k_cg_fused<float, true><<<nbc, 512, 0, cs>>>(S, (const float *)B.hess, c0, B.scalars, B.iscalars);
            if (presum) k_cg_sum<<<1, 1024, 0, cs>>>(part[0], stride, nbc, B.iscalars, B.scalars + S_CGSUM);
        };
        // the block-Jacobi solve's set-up (prep, the recycled warm start, init and the first
        // launch), enqueued as plain launches: as a captured sequence it measured slower (each
        // switch between a graph and plain launches on the stream costs a gap)
        // The recycled start reads the previous direction in place (k_cg_init scales it into x0
        // elementwise); it is zero at pinned CPs, whose rows of H are the identity with a zero
        // right-hand side, so PCG never moves them.
        const double *ph = warm == BSC_WARM_PREVIOUS ? B.dir : (warm == BSC_WARM_NET ? B.phat : nullptr);
        auto cg_setup = [&]() -> hipError_t {
            if (!ph) enqueue_prep(st);
            if (warm == BSC_WARM_NET) {
                // the learned prediction p_hat = net(g), zero on pinned CPs
                hipEvent_t w0 = rec();
                k_to_float<<<blocks(n3), kBlock, 0, st>>>(n3, B.g, B.net_in);
                const hipError_t e = net_forward_impl(S.n_u, S.n_v, 1, B.net_w, B.net_in, B.net_out, nullptr, B.net_act0,
                                                      B.net_act1, B.net_scale, B.net_w_fwd, true, st);
                if (e != hipSuccess) return e;
                k_phat<<<blocks(S.n_cp), kBlock, 0, st>>>(S.n_cp, B.net_out, S.pinmask, B.phat);
                span(w0, rec(), &s.ms_warmstart);
            }
            if (ph) enqueue_warm(st, ph);
            enqueue_init(st, ph);
            return hipGetLastError();
        };
        int32_t flags[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        // a chunk: 8 fused block-Jacobi CG launches (even: every chunk starts on an odd launch),
        // or one multigrid-preconditioned CG iteration
        const int chunk = use_mg ? 1 : 8;
        auto enqueue_chunk = [&](hipStream_t cs) {
            if (use_mg) {
                (void)mg_cg_iteration(S, B, prec, rb[0], sb[0], p, wb[0], B.partials, B.partials + stride, pbb, cs);
                return;
            }
            for (int c = 1; c <= chunk; ++c) {
                if (prec == BSC_FP64)
                    k_cg_fused<double, false><<<nbc, 512, 0, cs>>>(S, (const double *)B.hess, bufs(c), B.scalars, B.iscalars);
                else
                    k_cg_fused<float, false><<<nbc, 512, 0, cs>>>(S, (const float *)B.hess, bufs(c), B.scalars, B.iscalars);
                if (presum) k_cg_sum<<<1, 1024, 0, cs>>>(part[c & 1], stride, nbc, B.iscalars, B.scalars + S_CGSUM);
            }
        };
        // A burst of K chunks (K = 1..8) is enqueued as plain launches (the host keeps ahead of
        // the GPU). With BSC_GRAPHS=1 at create it is one graph of 8K launches instead, captured
        // the first time it is needed (on a private stream) and replayed on the context's stream
        // (the kernel arguments depend only on the bound workspace); at 226^2 the graphs measured
        // slower (a start-up gap per burst and gaps between their launches).
        auto graph_for = [&](int K) -> hipGraphExec_t {
            hipGraphExec_t &gxe = (use_mg ? ctx->mg_graph : ctx->cg_graph)[prec == BSC_FP64 ? 0 : 1][K];
            if (!gxe && ctx->use_graphs) {
                hipStream_t cs = nullptr;
                hipGraph_t graph = nullptr;
                bool ok = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess;
                ok = ok && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
                if (ok) {
                    for (int k = 0; k < K; ++k) enqueue_chunk(cs);
                    if (pub) publish(cs);
                    ok = hipStreamEndCapture(cs, &graph) == hipSuccess;
                }
                ok = ok && hipGraphInstantiate(&gxe, graph, nullptr, nullptr, 0) == hipSuccess;
                if (graph) (void)hipGraphDestroy(graph);
                if (cs) (void)hipStreamDestroy(cs);
                if (!ok) {
                    if (gxe) { (void)hipGraphExecDestroy(gxe); gxe = nullptr; }
                    (void)hipGetLastError();
                }
            }
            return gxe;
        };
        // Gradient rule, plain launches: every burst ends with the line-search set-up and the
        // trial at alpha = 1, gated by the solve's done flag (they exit at once while the solve
        // runs), so that the burst that finishes the solve also returns |p|_inf, the energy
        // difference and the decision, and x is updated without a host round trip.
        const bool ls_dev = !deferred && !use_mg && !ctx->use_graphs;
        double *pa = B.partials + 3 * stride, *pbend = B.partials + 5 * stride;
        // (partial arrays: c1, c2 of the CPs at 3, 4; of the bending at 5, 6; max |p| at 7; the
        // membrane difference at 0, free once PCG has finished)
        auto enqueue_ls = [&](hipStream_t cs) {
            k_ls_cp<<<blocks(S.n_cp), kBlock, 0, cs>>>(S, B.gpre, B.dir, inv_dt2, pa, stride, B.partials + 7 * stride);
            k_ls_quad_bend<<<blocks(S.n_be), kBlock, 0, cs>>>(S, B.dir, pbend, stride);
            k_ls_membrane<<<blocks(S.n_mp), kBlock, 0, cs>>>(S, x, B.dir, 1.0, B.partials);
            k_ls_finish<<<1, kBlock, 0, cs>>>(B.partials + 7 * stride, blocks(S.n_cp), pa, pbend, blocks(S.n_be), stride,
                                               B.partials, blocks(S.n_mp), B.scalars);
        };
        // cg_end: an event right behind the burst's CG launches (the line-search kernels follow it)
        auto launch_burst = [&](int K, hipEvent_t *cg_end) -> hipError_t {
            hipGraphExec_t ge = graph_for(K);
            if (ge) {
                const hipError_t e = hipGraphLaunch(ge, st);
                *cg_end = rec_cg();
                return e;
            }
            for (int bi = 0; bi < K; ++bi) enqueue_chunk(st);
            *cg_end = rec_cg();
            if (ls_dev) {
                hipEvent_t la = time_phases ? *cg_end : nullptr;
                const int nbc_ = blocks(S.n_cp), nbb_ = blocks(S.n_be), nbm_ = blocks(S.n_mp);
                k_ls_setup<<<nbc_ + nbb_ + nbm_, kBlock, 0, st>>>(S, x, B.gpre, B.dir, inv_dt2, pa, stride,
                                                                  B.partials + 7 * stride, pbend, B.partials, nbc_, nbb_,
                                                                  B.iscalars);
                k_ls_accept<<<blocks(n3), kBlock, 0, st>>>(n3, B.iscalars, B.scalars, B.partials + 7 * stride, nbc_, pa, pbend,
                                                           nbb_, stride, B.partials, nbm_, B.dir, x,
                                                           o->fixed_newton_iters <= 0 ? kStagnation : 0.0, pubp, pub ? 1 : 0);
                hipEvent_t lb = rec();
                span(la, lb, &s.ms_linesearch);
                span(la, lb, &ls_in_bursts);     // inside the span of ms_pcg
            } else if (pub) {
                publish(st);
            }
            return hipGetLastError();
        };
        // Chunks are enqueued in bursts with one flag read per burst (launches after convergence
        // exit at once, in about 3 us, while a burst boundary costs a host round trip). The first
        // burst covers the iterations that the same Newton iteration of the previous step needed
        // plus four (two chunks without such a record); after each burst the host extrapolates the
        // residual's geometric decay to the stopping threshold and sizes the next burst to cover
        // the iterations that remain plus half a chunk.
        int burst = 2, done_prev = 0;
        if (!use_mg && it < 64 && ctx->pcg_hist[it] > 0)
            burst = std::max(1, std::min(8, (ctx->pcg_hist[it] + 4 + chunk) / chunk));
        // Gradient rule (no multigrid): the set-up is enqueued right behind
        // the assembly with the forcing term formed on the device (the same formula as the
        // host's). Under the gradient stop the first burst follows at once (speculative): the
        // set-up marks the solve done on the device when |g| already meets the stop, so a
        // converged iterate costs only the set-up and a burst of launches that exit (x is not
        // touched), and the host reads E and |g| with the burst's read-back. Otherwise the set-up
        // publishes them and the host reads them while the GPU runs it.
        hipEvent_t e2 = nullptr, burst_c0 = nullptr, burst_c1 = nullptr;
        bool burst_pending = false;
        int32_t burst_last = 0;
        if (early) {
            eta_mode = o->pcg_adaptive ? ETA_ADAPTIVE : ETA_FIXED;
            grad_rtol = speculate ? o->rtol : 0.0;
            const int32_t last = last_asm;           // E and |g| come with the next read-back
            e2 = rec();
            HIPX(cg_setup(), "cg init");
            if (speculate) {
                burst_c0 = rec_cg();
                HIPX(launch_burst(burst, &burst_c1), "cg graph");
                burst_last = last;                 // the burst's read-back is the first after the assembly
                burst_pending = true;
            }
            HIPX(pub ? wait_pub(last) : copy_sync(), "read norms");
        }
        if (!deferred) {
            if (!early) HIPX(pull(), "read norms");
            host[0] = hs[S_E];
            host[1] = hs[S_GG];
            span(e0, e1, &s.ms_assemble);
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
            if (force_tight) {
                eta = o->pcg_rtol;
                force_tight = false;
            } else if (o->pcg_adaptive && g_prev > 0.0) {
                // Eisenstat-Walker forcing term (choice 2, gamma = 0.9, exponent 2) with safeguard
                const double ratio = gn / g_prev;
                double e = 0.9 * ratio * ratio;
                const double guard = 0.9 * eta * eta;
                if (guard > 0.1) e = std::max(e, guard);
                eta = std::min(eta_max, std::max(o->pcg_rtol, e));
            }
            g_prev = gn;
        } else {
            if (it >= o->max_newton) {
                HIPX(pull(), "read norms");
                host[0] = hs[S_E];
                host[1] = hs[S_GG];
                s.energy = host[0];
                s.g_norm = std::sqrt(host[1]);
                span(e0, e1, &s.ms_assemble);
                result = std::isfinite(host[0]) && std::isfinite(host[1]) ? BSC_E_NOT_CONVERGED : BSC_E_NONFINITE;
                break;
            }
            eta_mode = force_tight ? ETA_TIGHT : (o->pcg_adaptive ? ETA_ADAPTIVE : ETA_FIXED);
            force_tight = false;
        }

        // ---- direction: PCG on H p = -g -----------------------------------------------------
        if (!early) e2 = rec();
        eta_arg = eta_mode == ETA_EXPLICIT ? eta : 0.0;
        if (early) {
            // set-up already enqueued behind the assembly
        } else if (use_mg) {
            // multigrid: Galerkin hierarchy and block-Jacobi inverses of every level, then r = b,
            // p = 0, the flags and the tolerance (the first iteration's stop test sets |b|-relative
            // tolerance from the partials of |b|^2)
            enqueue_prep(st);
            HIPX(mg_setup(S, B, prec, st), "mg setup");
            k_cg_init<<<nbi, kBlock, 0, st>>>(S, B.tmp, nullptr, nullptr, nullptr, 0, 0, nullptr, rb[0], p, sb[0], pbb, B.iscalars, B.scalars,
                                               o->max_pcg, eta_mode, first, eta_arg, o->pcg_rtol, eta_max, 0.0);
            HIPX(hipGetLastError(), "mg init");
        } else {
            HIPX(cg_setup(), "cg init");
        }
        double lrho_prev = 0.0;
        bool have_prev = false;
        while (true) {
            hipEvent_t c0 = burst_c0, c1 = burst_c1;
            int32_t last = burst_last;
            if (!burst_pending) {
                c0 = rec_cg();
                last = seen();
                HIPX(launch_burst(burst, &c1), "cg graph");
            }
            burst_pending = false;
            span(c0, c1, &s.ms_cg_kernels);
            HIPX(pub ? wait_pub(last) : copy_sync(), "read cg state");
            for (int k = 0; k < 8; ++k) flags[k] = hf[k];
            const double *cgs = hs;
            s.cg_launches += chunk * burst;
            if (flags[I_DONE]) break;
            // iterations done so far: the launches of the bursts minus the first (which forms w_0)
            const int done = std::max(1, (flags[I_ITA] > flags[I_ITB] ? flags[I_ITA] : flags[I_ITB]) - 1);
            const double tol2 = cgs[S_TOL2], rho = cgs[S_RHO];
            if (!have_prev) {
                const double eta_now = cgs[S_RTOL];
                lrho_prev = eta_now > 0.0 ? std::log(tol2 / (eta_now * eta_now)) : std::log(rho);   // |b|^2
                done_prev = 0;
                have_prev = true;
            }
            burst = 1;
            if (rho > 0.0 && tol2 > 0.0 && done > done_prev) {
                const double rate = (std::log(rho) - lrho_prev) / double(done - done_prev);
                if (rate < 0.0) {
                    const double remaining = (std::log(tol2) - std::log(rho)) / rate;
                    burst = std::max(1, std::min(8, int(std::ceil((remaining + 0.5 * chunk) / chunk))));
                }
                lrho_prev = std::log(rho);
                done_prev = done;
            }
        }
        hipEvent_t e3 = rec();
        if (warm) {
            if (flags[I_WS]) s.warm_start_used++;
            else s.warm_start_fallbacks++;
        }
        s.cg_active_launches += flags[I_ITERS];
        if (it < 64) ctx->pcg_hist[it] = flags[I_ITERS];
        s.pcg_iters_total += flags[I_ITERS];
        if (flags[I_BREAK]) { result = BSC_E_PCG_BREAKDOWN; break; }
        if (ctx->log_count < ctx->log_cap) {
            const size_t off = size_t(ctx->log_count) * n3;
            k_to_float<<<blocks(n3), kBlock, 0, st>>>(n3, B.g, ctx->log_g + off);
            k_to_float<<<blocks(n3), kBlock, 0, st>>>(n3, B.dir, ctx->log_p + off);
            HIPX(hipGetLastError(), "sample log");
            ctx->log_count++;
        }

        // ---- |p|_inf for the stop tests, line-search coefficients and the trial at alpha = 1 ---
        // The energy difference along p: the inertia, gravity and bending terms are quadratics in
        // alpha (coefficients c1, c2), the membrane term is summed point by point. With ls_dev they
        // ran at the end of the last burst and the scalars are already here.
        if (!ls_dev) {
            hipEvent_t e4 = rec();
            const int32_t last = seen();
            enqueue_ls(st);
            if (pub) publish(st);
            HIPX(hipGetLastError(), "line search setup");
            span(e4, rec(), &s.ms_linesearch);
            HIPX(pub ? wait_pub(last) : copy_sync(), "read scalars");
        }
        double sc[S_GPREV - S_E + 1];
        for (int k = S_E; k <= S_GPREV; ++k) sc[k - S_E] = hs[k];
        if (deferred) span(e0, e1, &s.ms_assemble);
        span(e2, e3, &s.ms_pcg);
        auto scal = [&](int i) { return sc[i - S_E]; };
        if (deferred) {
            const double E = scal(S_E), gn = std::sqrt(scal(S_GG));
            if (!std::isfinite(E) || !std::isfinite(gn)) { result = BSC_E_NONFINITE; break; }
            if (g0 < 0.0) g0 = gn;
            s.energy = E;
            s.g_norm = gn;
            eta = scal(S_ETA);
        }
        if (step_rule && scal(S_PMAX) / dt <= o->atol) {
            if (eta <= o->pcg_rtol) break;
            force_tight = true;        // confirm the stop on a direction solved to pcg_rtol
        }
        // gradient rule: a direction that moves no coordinate by more than a few ulps of |x0|_inf
        // cannot improve x any further (e.g. a sheet at rest without forces, whose gradient is
        // rounding alone); the step has converged
        if (!step_rule && o->fixed_newton_iters <= 0 && scal(S_PMAX) <= kStagnation * hs[S_XMAX]) break;
        // the device's trial at alpha = 1 was accepted and applied (else x is untouched and the
        // host halves alpha below, from the same scalars)
        if (ls_dev && flags[I_LSACC] == 1) continue;

        // ---- backtracking line search on the energy difference ------------------------------
        {
            Timer t(st, time_phases);
            const double c1 = scal(S_C1), c2 = scal(S_C2);
            double dem = scal(S_DEM);
            double alpha = 1.0;
            bool ok = false;
            int h = 0;
            for (; h <= 20; ++h) {
                if (h > 0) {
                    k_ls_membrane<<<blocks(S.n_mp), kBlock, 0, st>>>(S, x, B.dir, alpha, B.partials + 6 * stride);
                    k_sum_into<<<1, kBlock, 0, st>>>(B.partials + 6 * stride, blocks(S.n_mp), B.scalars, S_DEM);
                    HIPX(pull(), "read dE");
                    dem = hs[S_DEM];
                }
                const double dE = alpha * c1 + 0.5 * alpha * alpha * c2 + dem;
                if (std::isfinite(dE) && dE <= 0.0) { ok = true; break; }
                alpha *= 0.5;
                s.ls_halvings++;
            }
            if (h > 0) s.ms_linesearch += t.stop();
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
    for (const Span &sp : spans) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, sp.a, sp.b) == hipSuccess) *sp.acc += ms;
        else (void)hipGetLastError();
    }
    s.ms_pcg -= ls_in_bursts;
    s.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (stats) *stats = s;
    return result;
}

// Solves H x = b for the upper-stencil matrix in the workspace (B.hess, working precision prec)
// with the fused block-Jacobi PCG from x0 = 0 until |r|_2 <= rtol |b|_2 or max_iter iterations.
// The launches are enqueued in bursts of 16 with one flag read per burst. Uses the workspace's
// CG vectors, partials and scalars and B.g, B.tmp, B.dir (overwritten). b and x may not alias
// those buffers.
bsc_status stencil_pcg(bsc_ctx *ctx, int prec, const double *b, double *x, double rtol, int max_iter, int *iters) {
    const DevSheet &S = ctx->dev;
    const DevBufs &B = ctx->buf;
    hipStream_t st = ctx->stream;
    const int n3 = 3 * S.n_cp, stride = B.max_blocks;
    const int nbi = blocks(S.n_cp), nbc = cg_blocks(S.n_u, S.n_v);
    const bool presum = nbc > kCgPreSumBlocks;
    double *rb[2] = {B.r, B.r2}, *wb[2] = {B.q, B.q2}, *sb[2] = {B.p1, B.p2};
    double *part[2] = {B.partials, B.partials + 3 * stride}, *pbb = B.partials + 6 * stride;
    auto bufs = [&](int j) {
        CgBufs c{};
        c.x = B.dir; c.p = B.p0; c.pinv = B.pinv;
        c.pbb = pbb; c.stride = stride; c.nb_init = nbi;
        c.pre = presum ? B.scalars + S_CGSUM : nullptr;
        const int cur = j & 1, prev = (j + 1) & 1;
        c.r_in = rb[j == 0 ? 0 : prev]; c.r_out = rb[cur];
        c.w_in = wb[prev]; c.w_out = wb[cur];
        c.s_in = sb[prev]; c.s_out = sb[cur];
        c.part_in = part[prev]; c.part_out = part[cur];
        c.slot_in = prev ? I_ITB : I_ITA; c.slot_out = cur ? I_ITB : I_ITA;
        return c;
    };
    auto fused = [&](int j) {
        if (prec == BSC_FP64) {
            if (j == 0) k_cg_fused<double, true><<<nbc, 512, 0, st>>>(S, (const double *)B.hess, bufs(0), B.scalars, B.iscalars);
            else k_cg_fused<double, false><<<nbc, 512, 0, st>>>(S, (const double *)B.hess, bufs(j), B.scalars, B.iscalars);
        } else {
            if (j == 0) k_cg_fused<float, true><<<nbc, 512, 0, st>>>(S, (const float *)B.hess, bufs(0), B.scalars, B.iscalars);
            else k_cg_fused<float, false><<<nbc, 512, 0, st>>>(S, (const float *)B.hess, bufs(j), B.scalars, B.iscalars);
        }
        if (presum) k_cg_sum<<<1, 1024, 0, st>>>(part[j & 1], stride, nbc, B.iscalars, B.scalars + S_CGSUM);
    };
    // block-Jacobi inverse of the matrix, b (as 0 - (-b)) into B.tmp, x0 = 0 into B.dir
    k_axpby<<<blocks(n3), kBlock, 0, st>>>(n3, -1.0, b, 0.0, b, B.g);
    if (prec == BSC_FP64)
        k_cg_prep<double><<<nbi, kBlock, 0, st>>>(S, (const double *)B.hess, (double *)B.pinv, B.g, B.tmp, B.dir);
    else
        k_cg_prep<float><<<nbi, kBlock, 0, st>>>(S, (const float *)B.hess, (float *)B.pinv, B.g, B.tmp, B.dir);
    k_cg_init<<<nbi, kBlock, 0, st>>>(S, B.tmp, nullptr, nullptr, nullptr, 0, 0, nullptr, rb[0], B.p0, sb[0], pbb, B.iscalars, B.scalars, max_iter,
                                       ETA_EXPLICIT, 1, rtol, rtol, rtol, 0.0);
    fused(0);
    HIPX(hipGetLastError(), "stencil pcg");
    int32_t flags[8] = {};
    for (int launched = 1;;) {
        for (int k = 0; k < 16; ++k) fused(launched++);
        HIPX(hipGetLastError(), "stencil pcg");
        HIPX(hipMemcpyAsync(flags, B.iscalars, sizeof(flags), hipMemcpyDeviceToHost, st), "stencil pcg flags");
        HIPX(hipStreamSynchronize(st), "stencil pcg");
        if (flags[I_DONE]) break;
        if (launched > max_iter + 2) return fail(ctx, BSC_E_STATE, "stencil pcg: solver did not finish");
    }
    if (iters) *iters = flags[I_ITERS];
    if (flags[I_BREAK])
        return fail(ctx, BSC_E_PCG_BREAKDOWN, "stencil pcg: p^T H p <= 0 at iteration " + std::to_string(flags[I_ITERS]));
    HIPX(hipMemcpyAsync(x, B.dir, 8 * size_t(n3), hipMemcpyDeviceToDevice, st), "stencil pcg result");
    return BSC_OK;
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
    if (o->start != BSC_START_PREVIOUS && o->start != BSC_START_PREDICTOR) return fail(c, BSC_E_INVAL, "bad start");
    if (o->max_newton < 1 || o->max_pcg < 1 || !(o->pcg_rtol > 0.0)) return fail(c, BSC_E_INVAL, "bad iteration limits");
    if (!(o->pcg_eta_max == 0.0 || (o->pcg_eta_max >= o->pcg_rtol && o->pcg_eta_max <= 0.9)))
        return fail(c, BSC_E_INVAL, "pcg_eta_max must be 0 or in [pcg_rtol, 0.9]");
    if (!c->pins.empty() && !d_pin_targets) return fail(c, BSC_E_INVAL, "pins set but no targets");
    if (o->warm_start < BSC_WARM_NONE || o->warm_start > BSC_WARM_PREVIOUS) return fail(c, BSC_E_INVAL, "bad warm start");
    if (o->warm_start == BSC_WARM_NET && !c->net_loaded) return fail(c, BSC_E_STATE, "warm start requested but no network loaded");
    if (o->timing < BSC_TIMING_CG || o->timing > BSC_TIMING_OFF) return fail(c, BSC_E_INVAL, "bad timing mode");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(o->gravity[k])) return fail(c, BSC_E_INVAL, "gravity must be finite");
    bsc_status st = newton_step(c, o, d_x, d_v, d_pin_targets, stats);
    if (st != BSC_OK && c->err.empty()) c->err = bsc_status_string(st);
    return st;
}

bsc_status bsc_energy_difference(bsc_ctx *c, const double *d_x, const double *d_xhat, double dt, const double *gravity,
                                 const double *d_p, int32_t n_alpha, const double *alphas, double *d_de) {
    if (!c) return BSC_E_INVAL;
    if (!c->ws) return fail(c, BSC_E_STATE, "no workspace bound");
    if (!d_x || !d_p || !d_de || !alphas) return fail(c, BSC_E_INVAL, "null pointer");
    if (n_alpha < 1 || n_alpha > 64) return fail(c, BSC_E_INVAL, "n_alpha must be in 1..64");
    for (int k = 0; k < n_alpha; ++k)
        if (!std::isfinite(alphas[k])) return fail(c, BSC_E_INVAL, "step lengths must be finite");
    double inv_dt2 = 0.0;
    if (d_xhat) {
        if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, BSC_E_INVAL, "dt must be positive");
        inv_dt2 = 1.0 / (dt * dt);
    }
    const double gx = gravity ? gravity[0] : 0.0, gy = gravity ? gravity[1] : 0.0, gz = gravity ? gravity[2] : 0.0;
    if (!std::isfinite(gx) || !std::isfinite(gy) || !std::isfinite(gz)) return fail(c, BSC_E_INVAL, "gravity must be finite");
    const DevSheet &S = c->dev;
    const DevBufs &B = c->buf;
    hipStream_t st = c->stream;
    const int stride = B.max_blocks;
    // c1 of the quadratic terms needs their gradient at x: the per-CP terms of the points pass
    // (without xhat the inertia term is dropped: inv_dt2 = 0)
    const CpTerms cpt{d_xhat, inv_dt2, gx, gy, gz, B.gpre};
    bsc_status r = hip_check(c, launch_points(S, B, BSC_FP64, false, false, d_x, st, false, &cpt), "energy difference points");
    if (r != BSC_OK) return r;
    double *pa = B.partials + 3 * stride, *pb = B.partials + 5 * stride;
    k_ls_cp<<<blocks(S.n_cp), kBlock, 0, st>>>(S, B.gpre, d_p, inv_dt2, pa, stride, B.partials + 7 * stride);
    k_ls_quad_bend<<<blocks(S.n_be), kBlock, 0, st>>>(S, d_p, pb, stride);
    k_ls_finish<<<1, kBlock, 0, st>>>(B.partials + 7 * stride, blocks(S.n_cp), pa, pb, blocks(S.n_be), stride,
                                      B.partials, 0, B.scalars);
    for (int k = 0; k < n_alpha; ++k) {
        k_ls_membrane<<<blocks(S.n_mp), kBlock, 0, st>>>(S, d_x, d_p, alphas[k], B.partials + 6 * stride);
        k_sum_into<<<1, kBlock, 0, st>>>(B.partials + 6 * stride, blocks(S.n_mp), B.scalars, S_DEM);
        k_de_combine<<<1, 64, 0, st>>>(B.scalars, alphas[k], d_de + k);
    }
    return hip_check(c, hipGetLastError(), "energy difference");
}

}  // extern "C"
