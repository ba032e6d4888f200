// eval.hip -- element evaluation and spline-structured assembly for gfx950.
//
// Stage 1 (one thread per quadrature point, coalesced SoA tables):
//   membrane point: deformation gradient from the 3x3 CP stencil of its span (Eq. "deformation
//   gradient"), energy density, first Piola stress and the 6x6 density Hessian (Sec. 4.1),
//   projected to PSD in double (Sec. 5.1); stored pre-multiplied by the point weight.
//   bending evaluation: Laplacian of phi (Eq. "Laplacian in parametric space"), stored as
//   w mu_bend Laplacian(phi) (Sec. 4.2).
// Stage 2 (gathers, no atomics, deterministic): per CP gradient and per (CP, upper-stencil
//   slot) 3x3 Hessian block summing the weighted contributions of the quadrature points shared
//   by the two CPs (Sec. 5.2, "Elasticity Hessian Assembly"), one workgroup per tile of CPs with
//   the tile's points staged in LDS; per element outputs.
// Energies are reduced per block into partial sums and summed in a fixed order.
#include "bsc_internal.h"

namespace bsc {
namespace {

#include "geom.h"

// Index of (r, c), r <= c, in the row-major upper triangle of a 6x6 matrix.
__host__ __device__ constexpr int u6(int r, int c) { return r <= c ? r * 6 - r * (r - 1) / 2 + (c - r) : c * 6 - c * (c - 1) / 2 + (r - c); }

__device__ __forceinline__ double block_sum(double v, double *sh) {
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
    return v;
}

// ---- membrane densities (T precision) -------------------------------------------------------
// G = dd/dX (3x2) is the displacement gradient; F = [I; 0] + G. Green strain is formed from G
// (E = sym(G_top) + G^T G / 2) so that no O(1) cancellation against I occurs.

template <typename T>
__device__ void stvk(const T G[3][2], T mu, T lam, T &psi, T P[3][2], T A[6][6], bool hess) {
    T F[3][2];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int g = 0; g < 2; ++g) F[i][g] = G[i][g] + ((i == g) ? T(1) : T(0));
    T E[2][2];
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int d = 0; d < 2; ++d)
            E[g][d] = T(0.5) * (G[g][d] + G[d][g] + G[0][g] * G[0][d] + G[1][g] * G[1][d] + G[2][g] * G[2][d]);
    const T tr = E[0][0] + E[1][1];
    psi = mu * (E[0][0] * E[0][0] + T(2) * E[0][1] * E[0][1] + E[1][1] * E[1][1]) + T(0.5) * lam * tr * tr;
    T Sm[2][2] = {{T(2) * mu * E[0][0] + lam * tr, T(2) * mu * E[0][1]}, {T(2) * mu * E[1][0], T(2) * mu * E[1][1] + lam * tr}};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int g = 0; g < 2; ++g) P[i][g] = F[i][0] * Sm[0][g] + F[i][1] * Sm[1][g];
    if (!hess) return;
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int d = 0; d < 2; ++d)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const T ffij = F[i][0] * F[j][0] + F[i][1] * F[j][1];
                    A[3 * g + i][3 * d + j] = (i == j ? Sm[g][d] : T(0)) + mu * F[i][d] * F[j][g] +
                                              (g == d ? mu * ffij : T(0)) + lam * F[i][g] * F[j][d];
                }
}

template <typename T>
__device__ void fbw(const T G[3][2], T mu1, T mu2, T msh, T &psi, T P[3][2], T A[6][6], bool hess) {
    T f[2][3];
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int i = 0; i < 3; ++i) f[g][i] = G[i][g] + ((i == g) ? T(1) : T(0));
    const T mus[2] = {mu1, mu2};
    T len[2], lm1[2];
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        // I5 - 1 = 2 G_gg + |G_:g|^2 without cancellation; sqrt(I5) - 1 = (I5 - 1)/(sqrt(I5) + 1)
        const T i5m1 = T(2) * G[g][g] + G[0][g] * G[0][g] + G[1][g] * G[1][g] + G[2][g] * G[2][g];
        len[g] = sqrt(T(1) + i5m1);
        lm1[g] = i5m1 / (len[g] + T(1));
    }
    const T I6 = f[0][0] * f[1][0] + f[0][1] * f[1][1] + f[0][2] * f[1][2];
    psi = msh * I6 * I6 + mu1 * lm1[0] * lm1[0] + mu2 * lm1[1] * lm1[1];
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int i = 0; i < 3; ++i)
            P[i][g] = T(2) * msh * I6 * f[1 - g][i] + T(2) * mus[g] * (lm1[g] / len[g]) * f[g][i];
    if (!hess) return;
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int d = 0; d < 2; ++d)
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    T a;
                    if (g == d) {
                        a = T(2) * msh * f[1 - g][i] * f[1 - g][j] +
                            T(2) * mus[g] * ((i == j ? lm1[g] / len[g] : T(0)) + f[g][i] * f[g][j] / (len[g] * len[g] * len[g]));
                    } else {
                        a = T(2) * msh * (f[d][i] * f[g][j] + (i == j ? I6 : T(0)));
                    }
                    A[3 * g + i][3 * d + j] = a;
                }
}

// ---- PSD projection in double -------------------------------------------------------------
// A positive-definite matrix (Cholesky succeeds) is its own projection; otherwise a cyclic
// Jacobi eigen-decomposition (symmetric Schur rotations) is run to convergence and the
// negative eigenvalues are clamped to zero.

__device__ bool cholesky_pd(const double A[6][6]) {
    double L[6][6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double d = A[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
        if (!(d > 0.0)) return false;
        const double ljj = sqrt(d), inv = 1.0 / ljj;
        L[j][j] = ljj;
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
            double s = A[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
            L[i][j] = s * inv;
        }
    }
    return true;
}

__device__ void project_psd(double A[6][6]) {
    if (cholesky_pd(A)) return;
    double V[6][6];
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = 0; c < 6; ++c) V[r][c] = (r == c) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 16; ++sweep) {
        double off = 0.0, tot = 0.0;
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const double a2 = A[r][c] * A[r][c];
                tot += a2;
                if (r != c) off += a2;
            }
        if (off <= 1e-32 * tot) break;
#pragma unroll
        for (int p = 0; p < 5; ++p) {
#pragma unroll
            for (int q = p + 1; q < 6; ++q) {
                const double apq = A[p][q];
                if (apq != 0.0) {
                    const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
                    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
#pragma unroll
                    for (int k = 0; k < 6; ++k) {
                        const double akp = A[k][p], akq = A[k][q];
                        A[k][p] = c * akp - s * akq;
                        A[k][q] = s * akp + c * akq;
                    }
#pragma unroll
                    for (int k = 0; k < 6; ++k) {
                        const double apk = A[p][k], aqk = A[q][k];
                        A[p][k] = c * apk - s * aqk;
                        A[q][k] = s * apk + c * aqk;
                    }
#pragma unroll
                    for (int k = 0; k < 6; ++k) {
                        const double vkp = V[k][p], vkq = V[k][q];
                        V[k][p] = c * vkp - s * vkq;
                        V[k][q] = s * vkp + c * vkq;
                    }
                }
            }
        }
    }
    double lam[6];
#pragma unroll
    for (int r = 0; r < 6; ++r) lam[r] = A[r][r] > 0.0 ? A[r][r] : 0.0;
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = r; c < 6; ++c) {
            double s = 0.0;
#pragma unroll
            for (int m = 0; m < 6; ++m) s += V[r][m] * lam[m] * V[c][m];
            A[r][c] = s;
            A[c][r] = s;
        }
}

// Structured projection. Both membrane models depend on F only through f1, f2, so in the
// orthonormal frame (e1 = f1/|f1|, e3 = f1 x f2 / |f1 x f2|, e2 = e3 x e1) the 6x6 density
// Hessian splits into a 4x4 in-plane block and a 2x2 block acting on the normal components
// (for StVK the latter is exactly the second Piola stress S). Each block is projected on its
// own (Cholesky test, then Jacobi for the 4x4, closed form for the 2x2) and rotated back. This
// equals the projection of the full matrix; degenerate F (parallel columns) returns false.

__device__ bool cholesky_pd4(const double A[4][4]) {
    double L[4][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        double d = A[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
        if (!(d > 0.0)) return false;
        const double ljj = sqrt(d), inv = 1.0 / ljj;
        L[j][j] = ljj;
#pragma unroll
        for (int i = j + 1; i < 4; ++i) {
            double sm = A[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) sm -= L[i][k] * L[j][k];
            L[i][j] = sm * inv;
        }
    }
    return true;
}

__device__ void project_psd4(double A[4][4]) {
    if (cholesky_pd4(A)) return;
    double V[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) V[r][c] = (r == c) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 16; ++sweep) {
        double off = 0.0, tot = 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double a2 = A[r][c] * A[r][c];
                tot += a2;
                if (r != c) off += a2;
            }
        if (off <= 1e-32 * tot) break;
#pragma unroll
        for (int p = 0; p < 3; ++p) {
#pragma unroll
            for (int q = p + 1; q < 4; ++q) {
                const double apq = A[p][q];
                if (apq != 0.0) {
                    const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
                    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const double akp = A[k][p], akq = A[k][q];
                        A[k][p] = c * akp - s * akq;
                        A[k][q] = s * akp + c * akq;
                    }
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const double apk = A[p][k], aqk = A[q][k];
                        A[p][k] = c * apk - s * aqk;
                        A[q][k] = s * apk + c * aqk;
                    }
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const double vkp = V[k][p], vkq = V[k][q];
                        V[k][p] = c * vkp - s * vkq;
                        V[k][q] = s * vkp + c * vkq;
                    }
                }
            }
        }
    }
    double lam[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) lam[r] = A[r][r] > 0.0 ? A[r][r] : 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = r; c < 4; ++c) {
            double sm = 0.0;
#pragma unroll
            for (int m = 0; m < 4; ++m) sm += V[r][m] * lam[m] * V[c][m];
            A[r][c] = sm;
            A[c][r] = sm;
        }
}

// Symmetric 2x2 [[a, b], [b, c]] projected to PSD in closed form (R: the arithmetic).
template <typename R>
__device__ void project_psd2(R &a, R &b, R &c) {
    const R h = R(0.5) * (a - c), m = R(0.5) * (a + c);
    const R r = sqrt(h * h + b * b);
    const R l1 = m + r, l2 = m - r;               // l1 >= l2
    if (l2 >= R(0)) return;
    if (l1 <= R(0)) { a = b = c = R(0); return; }
    // keep l1 v v^T, v the unit eigenvector of l1
    R vx, vy;
    if (h >= R(0)) { vx = h + r; vy = b; } else { vx = b; vy = r - h; }
    const R nn = vx * vx + vy * vy;
    if (nn == R(0)) { a = fmax(a, R(0)); c = fmax(c, R(0)); b = R(0); return; }
    const R k = l1 / nn;
    a = k * vx * vx; b = k * vx * vy; c = k * vy * vy;
}

// PSD projection of the in-plane StVK block d^2 Psi / dF^2 (4x4, index 2 gamma + i) at the
// in-plane deformation gradient F = [[a, b], [0, d]] (a, d > 0), in closed form. Psi depends on
// F only through its singular values s1 >= s2 > 0; with F = U diag(s1, s2) V^T (U, V rotations)
// the block's eigenvectors are the scaling directions u1 v1^T, u2 v2^T (mixed by the 2x2
// Hessian of psi(s1, s2)), the twist (u2 v1^T - u1 v2^T)/sqrt2 and the flip
// (u1 v2^T + u2 v1^T)/sqrt2, with eigenvalues (psi_1 + psi_2)/(s1 + s2) and
// (psi_1 - psi_2)/(s1 - s2) (Smith, de Goes and Kim 2019, analytic eigensystems of isotropic
// energies). For StVK, psi = mu/4 sum (s_i^2 - 1)^2 + lam/8 (s1^2 + s2^2 - 2)^2, both
// quotients are polynomials, so equal singular values need no special case.
template <typename R>
__device__ void stvk_inplane_projected(R a, R b, R d, R mu, R lam, R P[4][4]) {
    const R p = a * a, q = a * b, r = b * b + d * d;                // C = F^T F
    const R h = R(0.5) * (p - r), m = R(0.5) * (p + r), rad = sqrt(h * h + q * q);
    const R s1 = sqrt(m + rad), s2 = a * d / s1;
    R vx, vy;                                                       // eigenvector of C for s1^2
    if (h >= R(0)) { vx = h + rad; vy = q; } else { vx = q; vy = rad - h; }
    const R nn = sqrt(vx * vx + vy * vy);
    if (nn > R(0)) { vx /= nn; vy /= nn; } else { vx = R(1); vy = R(0); }
    const R v1[2] = {vx, vy}, v2[2] = {-vy, vx};
    const R u1[2] = {(a * vx + b * vy) / s1, (d * vy) / s1}, u2[2] = {-u1[1], u1[0]};
    const R I = s1 * s1 + s2 * s2;
    R b11 = mu * (R(3) * s1 * s1 - R(1)) + R(0.5) * lam * (I - R(2)) + lam * s1 * s1;
    R b22 = mu * (R(3) * s2 * s2 - R(1)) + R(0.5) * lam * (I - R(2)) + lam * s2 * s2;
    R b12 = lam * s1 * s2;
    project_psd2<R>(b11, b12, b22);
    const R lt = fmax(mu * (s1 * s1 - s1 * s2 + s2 * s2 - R(1)) + R(0.5) * lam * (I - R(2)), R(0));
    const R ll = fmax(mu * (s1 * s1 + s1 * s2 + s2 * s2 - R(1)) + R(0.5) * lam * (I - R(2)), R(0));
    R D1[4], D2[4], T[4], L[4];                                     // vec index 2 gamma + i
    const R k = R(0.70710678118654752440);
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            D1[2 * g + i] = u1[i] * v1[g];
            D2[2 * g + i] = u2[i] * v2[g];
            T[2 * g + i] = k * (u2[i] * v1[g] - u1[i] * v2[g]);
            L[2 * g + i] = k * (u1[i] * v2[g] + u2[i] * v1[g]);
        }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
            P[x][y] = b11 * D1[x] * D1[y] + b22 * D2[x] * D2[y] + b12 * (D1[x] * D2[y] + D2[x] * D1[y]) +
                      lt * T[x] * T[y] + ll * L[x] * L[y];
}

// Builds the projected 6x6 density Hessian of the membrane model at displacement gradient G
// into A, in the arithmetic R. The rounding of n = f1 x f2 tilts the frame by about 2 eps / r,
// r = |f1 x f2| / (|f1| |f2|), so the projection declines (returns false) below r = 1e-5 in FP64
// (tilt <= 4e-11) and r = 0.1 in FP32 (StVK only, whose Hessian is then stored in FP32; tilt
// <= 2.4e-6); the caller then projects the full 6x6 matrix.
template <typename R>
__device__ bool project_structured(const DevSheet &S, const R G[3][2], R A[6][6]) {
    R f[2][3];
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int i = 0; i < 3; ++i) f[g][i] = G[i][g] + ((i == g) ? R(1) : R(0));
    const R l1 = sqrt(f[0][0] * f[0][0] + f[0][1] * f[0][1] + f[0][2] * f[0][2]);
    R n[3] = {f[0][1] * f[1][2] - f[0][2] * f[1][1], f[0][2] * f[1][0] - f[0][0] * f[1][2], f[0][0] * f[1][1] - f[0][1] * f[1][0]};
    const R ln = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    const R l2 = sqrt(f[1][0] * f[1][0] + f[1][1] * f[1][1] + f[1][2] * f[1][2]);
    const R par = sizeof(R) == 8 ? R(1e-5) : R(0.1);
    if (!(l1 > R(0)) || !(ln > par * l1 * l2)) return false;
    R e[3][3];                                      // e[0] = e1, e[1] = e2, e[2] = e3
#pragma unroll
    for (int i = 0; i < 3; ++i) { e[0][i] = f[0][i] / l1; e[2][i] = n[i] / ln; }
    e[1][0] = e[2][1] * e[0][2] - e[2][2] * e[0][1];
    e[1][1] = e[2][2] * e[0][0] - e[2][0] * e[0][2];
    e[1][2] = e[2][0] * e[0][1] - e[2][1] * e[0][0];
    // in-plane components: F2[i][g] = f_g . e_i (i, g in {0,1}); f1 . e2 = 0
    R F2[2][2];
    F2[0][0] = l1; F2[1][0] = R(0);
    F2[0][1] = f[1][0] * e[0][0] + f[1][1] * e[0][1] + f[1][2] * e[0][2];
    F2[1][1] = ln / l1;
    R P4[4][4], Na, Nb, Nc;                         // P4 index 2*gamma + i
    if (S.membrane == BSC_MEMBRANE_STVK) {
        const R mu = R(S.mu), lam = R(S.lam);
        R E[2][2];
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int d = 0; d < 2; ++d)
                E[g][d] = R(0.5) * (G[g][d] + G[d][g] + G[0][g] * G[0][d] + G[1][g] * G[1][d] + G[2][g] * G[2][d]);
        const R tr = E[0][0] + E[1][1];
        Na = R(2) * mu * E[0][0] + lam * tr;        // normal block: the second Piola-Kirchhoff stress
        Nb = R(2) * mu * E[0][1];
        Nc = R(2) * mu * E[1][1] + lam * tr;
        stvk_inplane_projected<R>(F2[0][0], F2[0][1], F2[1][1], mu, lam, P4);
    } else if constexpr (sizeof(R) == 8) {
        const double mus[2] = {S.mu1, S.mu2};
        double len[2], q[2];
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            const double i5m1 = 2.0 * G[g][g] + G[0][g] * G[0][g] + G[1][g] * G[1][g] + G[2][g] * G[2][g];
            len[g] = sqrt(1.0 + i5m1);
            q[g] = (i5m1 / (len[g] + 1.0)) / len[g];          // 1 - 1/|f_g|
        }
        const double I6 = F2[0][0] * F2[0][1] + F2[1][0] * F2[1][1];
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int d = 0; d < 2; ++d)
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        double a;
                        if (g == d) {
                            a = 2.0 * S.msh * F2[i][1 - g] * F2[j][1 - g] +
                                2.0 * mus[g] * ((i == j ? q[g] : 0.0) + F2[i][g] * F2[j][g] / (len[g] * len[g] * len[g]));
                        } else {
                            a = 2.0 * S.msh * (F2[i][d] * F2[j][g] + (i == j ? I6 : 0.0));
                        }
                        P4[2 * g + i][2 * d + j] = a;
                    }
        Na = 2.0 * mus[0] * q[0]; Nb = 2.0 * S.msh * I6; Nc = 2.0 * mus[1] * q[1];
        project_psd4(P4);
    } else {
        return false;                               // FBW is projected in FP64 only
    }
    project_psd2<R>(Na, Nb, Nc);
    const R N2[2][2] = {{Na, Nb}, {Nb, Nc}};
    // rotate back: A[(g,i),(d,j)] = sum_{a,b<2} e_a[i] P4[(g,a),(d,b)] e_b[j] + N[g][d] e3[i] e3[j]
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int d = 0; d < 2; ++d)
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    R v = N2[g][d] * e[2][i] * e[2][j];
#pragma unroll
                    for (int aa = 0; aa < 2; ++aa)
#pragma unroll
                        for (int bb = 0; bb < 2; ++bb) v += e[aa][i] * P4[2 * g + aa][2 * d + bb] * e[bb][j];
                    A[3 * g + i][3 * d + j] = v;
                }
    return true;
}

// ---- stage 1 kernels ------------------------------------------------------------------------

// T: arithmetic; TA, TP: stored precision of the weighted density Hessian and stress.
template <typename T, bool HESS, bool CURVED, typename TA, typename TP>
__device__ __forceinline__ double membrane_point(const DevSheet &S, const double *__restrict__ x, TA *__restrict__ ptA,
                                                 TP *__restrict__ ptP, double *__restrict__ ptE, int q) {
    double e_loc = 0.0;
    if (q < S.n_mp) {
        const int e = S.mp_elem[q], k = e % S.Nu, l = e / S.Nu;
        const T tu = T(S.mp_tu[q]), tv = T(S.mp_tv[q]);
        const double w = S.mp_w[q];
        T dN[9][2];
        local_grads<T>(S, mp_geo_t<CURVED>(S, q), k, l, tu, tv, dN);
        // G from the displacements relative to the span's centre CP, formed in FP64: the basis
        // gradients sum to zero, so this is the same G, and in FP32 its rounding follows the local
        // variation of the displacement, not its size (which grows with the sheet)
        T G[3][2] = {{T(0), T(0)}, {T(0), T(0)}, {T(0), T(0)}};
        double dref[3];
        displacement_t<CURVED>(S, x, k + 1, l + 1, dref);
#pragma unroll
        for (int m = 0; m < 9; ++m) {
            double d[3];
            displacement_t<CURVED>(S, x, k + m % 3, l + m / 3, d);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T dc = T(d[c] - dref[c]);
                G[c][0] += dc * dN[m][0];
                G[c][1] += dc * dN[m][1];
            }
        }
        T psi, P[3][2], A[6][6];
        // StVK: the projected density Hessian comes in closed form from the structured projection
        // (exact for definite and indefinite points alike), so the full 6x6 and its Cholesky test
        // are only formed for a degenerate F (parallel columns), where that projection declines
        const bool direct = HESS && S.membrane == BSC_MEMBRANE_STVK;
        if (S.membrane == BSC_MEMBRANE_STVK) stvk<T>(G, T(S.mu), T(S.lam), psi, P, A, HESS && !direct);
        else fbw<T>(G, T(S.mu1), T(S.mu2), T(S.msh), psi, P, A, HESS);
        e_loc = w * double(psi);
        ptE[q] = e_loc;
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int i = 0; i < 3; ++i) ptP[(2 * i + g) * S.n_mp + q] = TP(w * double(P[i][g]));
        if (HESS) {
            double Ad[6][6], Gd[3][2];
#pragma unroll
            for (int c = 0; c < 3; ++c) { Gd[c][0] = double(G[c][0]); Gd[c][1] = double(G[c][1]); }
            if constexpr (sizeof(TA) == 4) {
                // stored in FP32: the StVK projection in FP32 arithmetic; columns of F within
                // r = 0.1 of parallel take the FP64 path below
                if (direct) {
                    float Gf[3][2], Af[6][6];
#pragma unroll
                    for (int c = 0; c < 3; ++c) { Gf[c][0] = float(G[c][0]); Gf[c][1] = float(G[c][1]); }
                    if (project_structured<float>(S, Gf, Af)) {
#pragma unroll
                        for (int r = 0; r < 6; ++r)
#pragma unroll
                            for (int c = r; c < 6; ++c) ptA[u6(r, c) * S.n_mp + q] = TA(w * double(Af[r][c]));
                        return e_loc;
                    }
                }
            }
            if (!direct || !project_structured<double>(S, Gd, Ad)) {
                if (direct) {
                    T psi2, P2[3][2];
                    stvk<T>(G, T(S.mu), T(S.lam), psi2, P2, A, true);
                }
#pragma unroll
                for (int r = 0; r < 6; ++r)
#pragma unroll
                    for (int c = 0; c < 6; ++c) Ad[r][c] = 0.5 * (double(A[r][c]) + double(A[c][r]));
                if (!cholesky_pd(Ad) && (direct || !project_structured<double>(S, Gd, Ad))) project_psd(Ad);
            }
#pragma unroll
            for (int r = 0; r < 6; ++r)
#pragma unroll
                for (int c = r; c < 6; ++c) ptA[u6(r, c) * S.n_mp + q] = TA(w * Ad[r][c]);
        }
    }
    return e_loc;
}

template <bool CURVED>
__device__ __forceinline__ double bending_point(const DevSheet &S, const double *__restrict__ x, double *__restrict__ beD,
                                                double *__restrict__ beE, int q) {
    double e_loc = 0.0;
    if (q < S.n_be) {
        const int e = S.be_elem[q], k = e % S.Nu, l = e / S.Nu;
        double L[9];
        bend_L_t<CURVED>(S, be_geo_t<CURVED>(S, q), k, l, S.be_tu[q], S.be_tv[q], L);
        double lap[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int m = 0; m < 9; ++m) {
            double d[3];
            displacement_t<CURVED>(S, x, k + m % 3, l + m / 3, d);
#pragma unroll
            for (int c = 0; c < 3; ++c) lap[c] += L[m] * d[c];
        }
        const double wm = S.be_w[q] * S.mu_bend;
        e_loc = 0.5 * wm * (lap[0] * lap[0] + lap[1] * lap[1] + lap[2] * lap[2]);
        beE[q] = e_loc;
#pragma unroll
        for (int c = 0; c < 3; ++c) beD[c * S.n_be + q] = wm * lap[c];
    }
    return e_loc;
}

// Displacement component c of CP (i, j) from its rest position (the component of
// displacement_t, in the same arithmetic).
template <bool CURVED>
__device__ __forceinline__ double displacement_c(const DevSheet &S, const double *__restrict__ x, int i, int j, int c) {
    const int a = j * S.n_u + i;
    double X = 0.0;
    if (c < 2) {
        if (CURVED) {
            X = S.rest[c * S.n_cp + a];
        } else {
            const double gu = greville(i, S.n_u), gv = greville(j, S.n_v);
            X = c == 0 ? S.A00 * gu + S.A01 * gv + S.b0 : S.A10 * gu + S.A11 * gv + S.b1;
        }
    }
    return x[size_t(c) * S.n_cp + a] - X;
}

// The per-CP gradient terms that need no quadrature point, for CP a: the bending energy is
// quadratic in the displacement d = x - X and zero at rest, so its gradient is exactly K_b d, the
// constant bending stencil (a scalar times I3 per block, built at create from the same bending
// evaluations) over the 25 neighbours; then the inertia M (x - xhat) / dt^2 and the gravity load
// -M g (Sec. 3.2, the incremental potential). Returns the CP's share of the energy of these terms:
// inertia, gravity and d_a . (K_b d)_a / 2, so that the CPs' shares sum to the bending energy
// (the bending evaluations are then not needed in an assembly). Every neighbour is read (an
// absent one reads CP a and its term is discarded by a select), so the loads carry no branches
// and issue in a few batches.
template <bool CURVED>
__device__ __forceinline__ double cp_terms(const DevSheet &S, const double *__restrict__ x, const CpTerms &C, int a) {
    double e_loc = 0.0;
    if (a < S.n_cp) {
        const size_t ncp = S.n_cp;
        const int i = a % S.n_u, j = a / S.n_u;
        double accb[3] = {0.0, 0.0, 0.0};
#pragma unroll 4
        for (int s2 = 0; s2 < kSlots; ++s2) {
            const int di = slot_di(s2), dj = slot_dj(s2);
            const int ib = i + di, jb = j + dj;
            const bool okb = ib >= 0 && ib < S.n_u && jb < S.n_v;
            const double w = S.hbend[s2 * ncp + a];
            double d[3];
            displacement_t<CURVED>(S, x, okb ? ib : i, okb ? jb : j, d);
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) accb[cc] += okb ? w * d[cc] : 0.0;
            if (s2 == 0) continue;
            const int ic = i - di, jc = j - dj;
            const bool okc = ic >= 0 && ic < S.n_u && jc >= 0;
            const double w2 = S.hbend[s2 * ncp + (okc ? jc * S.n_u + ic : a)];
            displacement_t<CURVED>(S, x, okc ? ic : i, okc ? jc : j, d);
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) accb[cc] += okc ? w2 * d[cc] : 0.0;
        }
        // the bending energy: quadratic in d with the same stencil, 1/2 d^T K_b d, this CP's share
        double dself[3];
        displacement_t<CURVED>(S, x, i, j, dself);
        e_loc += 0.5 * (dself[0] * accb[0] + dself[1] * accb[1] + dself[2] * accb[2]);
        const double M = S.mass[a];
        const double grav[3] = {C.gx, C.gy, C.gz};
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            double gs = accb[cc];
            const double xc = x[cc * ncp + a];
            if (C.xhat) {
                const double dlt = xc - C.xhat[cc * ncp + a];
                gs += M * C.inv_dt2 * dlt;
                e_loc += 0.5 * M * C.inv_dt2 * dlt * dlt;
            }
            gs -= M * grav[cc];
            e_loc -= M * grav[cc] * xc;
            C.gpre[cc * ncp + a] = gs;
        }
    }
    return e_loc;
}

// Minimum waves per SIMD of the points pass: the FP32 instantiation (FP32 arithmetic and records)
// runs faster with its registers capped for three waves; the FP64 ones keep all their registers.
template <typename T, typename TP>
constexpr int kPointsWaves = (sizeof(T) == 4 && sizeof(TP) == 4) ? 3 : 1;

// The per-CP terms, the membrane points and the bending evaluations in one launch: blocks
// [0, ncb) take CPs (ncb = 0 without them), the next nbm membrane points, the rest bending
// evaluations; each block writes the sum of its energies to its own partial slot (CPs:
// pc[block], membrane: pm[block - ncb], bending: pb[block - ncb - nbm]), so the sums keep the
// order of separate launches. The parts are independent, and one grid lets the light bending
// and CP blocks fill the slots that the register-heavy membrane blocks leave free; the CP
// blocks, bound by the latency of their neighbour loads, come first so that it overlaps the rest.
template <typename T, bool HESS, bool CURVED, typename TA = T, typename TP = T, bool BEND = true>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kPointsWaves<T, TP>)))
k_points(DevSheet S, const double *__restrict__ x, TA *__restrict__ ptA,
                                                   TP *__restrict__ ptP, double *__restrict__ ptE,
                                                   double *__restrict__ pm, double *__restrict__ beD,
                                                   double *__restrict__ beE, double *__restrict__ pb, int ncb, int nbm,
                                                   CpTerms C, double *__restrict__ pc) {
    __shared__ double sh[kBlock / 64];
    const int b = int(blockIdx.x);
    const int role = b < ncb ? 2 : (b < ncb + nbm ? 0 : 1);
    const int blk = role == 2 ? b : (role == 0 ? b - ncb : b - ncb - nbm);
    const int q = blk * kBlock + threadIdx.x;
    double e_loc;
    if (role == 0) {
        e_loc = membrane_point<T, HESS, CURVED, TA, TP>(S, x, ptA, ptP, ptE, q);
    } else if (role == 1) {
        if constexpr (BEND) e_loc = bending_point<CURVED>(S, x, beD, beE, q);
        else e_loc = 0.0;
    } else {
        e_loc = cp_terms<CURVED>(S, x, C, q);
    }
    const double s = block_sum(e_loc, sh);
    if (threadIdx.x == 0) (role == 2 ? pc : (role == 0 ? pm : pb))[blk] = s;
}

// The energy of an assembly without |g|^2 (bsc_assemble), summed by the tile kernel's block 0
// from the points pass's partials (membrane, bending, CPs) in a fixed order; out null: none.
struct EnergySum {
    const double *p0, *p1, *p2;
    int n0, n1, n2;
    double *out;
};

// ---- stage 2, tiled: Hessian blocks from LDS, gradient ------------------------------------------
//
// One workgroup per tile of kAsmTileU x ty CPs. The membrane points of the elements that the
// tile's CPs touch (at most (kAsmTileU + 2) x (ty + 2) elements) are staged in LDS once: the
// weighted density Hessian A (21 entries) and the gradients of the 9 local basis functions
// (FP32) or the span coordinates (FP64, gradients recomputed). Work items (CP, slot): slots
// 0..12 are the upper-stencil Hessian blocks, slot 13 is the gradient with the per-CP energy
// terms (membrane stresses gathered from global memory, bending as K_b d from the constant
// bending stencil). Items are numbered slot-major
// with the slots by decreasing cost, and handed to waves in chunks of 64 from an LDS counter.
// Each item sums over elements and points in a fixed order, so the result does not depend on
// which wave takes it.
template <typename TA, typename TP, typename TG, bool CURVED>
__global__ void __launch_bounds__(kAsmThreads) k_assemble_tile(DevSheet S, int kind, const TA *__restrict__ ptA,
                                                               const TP *__restrict__ ptP, const double *__restrict__ gpre,
                                                               double inv_dt2, TA *__restrict__ hess, TG *__restrict__ gout,
                                                               double *__restrict__ gg_partials, EnergySum esum) {
    constexpr bool STAGE_DN = sizeof(TA) == 4;
    // kind of record (see AsmLds): FP32, mixed (float Hessian, double stress) or FP64
    constexpr int KIND = sizeof(TA) == 4 ? (sizeof(TP) == 4 ? kAsmF32 : kAsmMixed) : kAsmF64;
    constexpr int REC = KIND == kAsmF32 ? kAsmRecF
                      : (KIND == kAsmMixed ? kAsmRecM : kAsmRecD);
    // offsets (units of TA) of the stress P (FP64: P K^T) and, in mixed records, of the basis
    // gradients' rounding remainders; FP64 records hold the 1-D factors Nu, Du, Nv, Dv from OFF_N
    constexpr int OFF_P = KIND == kAsmF64 ? 33 : 44;
    constexpr int OFF_N = 21, OFF_LO = 56;
    extern __shared__ __align__(16) char lds[];
    __shared__ double sh[kAsmThreads / 64];
    const int ty = S.asm_ty[kind], maxp = S.asm_maxp[kind];
    const AsmLds L = asm_lds_layout(kAsmTileU, ty, maxp, KIND, CURVED);
    int *el_info = (int *)(lds + L.el_off);      // per tile-local element: count, first and further records
    int *counter = (int *)(lds + L.counter);
    TA *prec = (TA *)(lds + L.rec);

    // the tile: kAsmTileU CPs wide, h CP rows tall (ty inside, min(2, ty) near the edges)
    const int ntx = (S.n_u + kAsmTileU - 1) / kAsmTileU;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tx0 = (tile % ntx) * kAsmTileU;
    int ty0 = 0, h = 0;
    asm_tile_row(S.n_v, ty, tile / ntx, ty0, h);
    const int R = kAsmTileU * h;                 // CPs of the tile (some past the sheet's edge)
    const int k0 = max(0, tx0 - 2), k1 = min(S.Nu - 1, tx0 + kAsmTileU - 1);
    const int l0 = max(0, ty0 - 2), l1 = min(S.Nv - 1, ty0 + h - 1);
    const int nk = k1 - k0 + 1, nl = l1 - l0 + 1, ne = nk * nl;

    // The tile's table (built at create): its point count, the global point and tile-local
    // element of each record, and the per-element record indices, all read in one round of
    // independent loads (the record lists are padded to maxp).
    const int32_t *T = S.asm_tab[kind] + size_t(tile) * S.asm_stride[kind];
    const int32_t *tq = T + 1, *te = T + 1 + maxp;
    for (int t = threadIdx.x; t < ne; t += blockDim.x) el_info[t] = T[1 + 2 * maxp + t];
    if (threadIdx.x == 0) *counter = 0;
    {
        const int np = T[0];
        for (int t = threadIdx.x; t < np; t += blockDim.x) {
            const int q = tq[t], elr = te[t];
            const int r = elr / nk, kk = elr - r * nk;
            TA *rec = prec + size_t(t) * REC;
            if (hess) {
#pragma unroll
                for (int c = 0; c < 21; ++c) rec[c] = ptA[c * S.n_mp + q];
            }
            const double tu = S.mp_tu[q], tv = S.mp_tv[q];
            if constexpr (STAGE_DN) {
                if constexpr (KIND == kAsmMixed) {
                    // the gradients in FP64, stored as float plus float remainder
                    double dN[9][2];
                    local_grads<double>(S, mp_geo_t<CURVED>(S, q), k0 + kk, l0 + r, tu, tv, dN);
#pragma unroll
                    for (int m = 0; m < 9; ++m)
#pragma unroll
                        for (int g = 0; g < 2; ++g) {
                            const float hi = float(dN[m][g]);
                            rec[24 + 2 * m + g] = hi;
                            rec[OFF_LO + 2 * m + g] = float(dN[m][g] - double(hi));
                        }
                } else {
                    TA dN[9][2];
                    local_grads<TA>(S, mp_geo_t<CURVED>(S, q), k0 + kk, l0 + r, TA(tu), TA(tv), dN);
#pragma unroll
                    for (int m = 0; m < 9; ++m) {
                        rec[24 + 2 * m] = dN[m][0];
                        rec[24 + 2 * m + 1] = dN[m][1];
                    }
                }
            } else {
                // FP64: the gradient with respect to X of basis function (a, b) is K^T ghat with
                // ghat = (Du[a] Nv[b], Nu[a] Dv[b]) in the span's parameters, so the items' sums
                // of ga^T A^(gamma delta) gb equal those of ghat_a^T Ahat ghat_b with Ahat the
                // congruence (K x I3) A (K x I3)^T, and P dN = (P K^T) ghat: formed once per point
                double Nu[3], Du[3], Nv[3], Dv[3];
                pieces<double>(span_type(k0 + kk, S.Nu), tu, Nu, Du);
                pieces<double>(span_type(l0 + r, S.Nv), tv, Nv, Dv);
#pragma unroll
                for (int m = 0; m < 3; ++m) {
                    rec[OFF_N + m] = Nu[m];
                    rec[OFF_N + 3 + m] = Du[m];
                    rec[OFF_N + 6 + m] = Nv[m];
                    rec[OFF_N + 9 + m] = Dv[m];
                }
                const PtK K = mp_geo_t<CURVED>(S, q);
                const double Kg[2][2] = {{K.k00, K.k01}, {K.k10, K.k11}};
                if (hess) {
                    double A6[21];
#pragma unroll
                    for (int c = 0; c < 21; ++c) A6[c] = rec[c];
                    // Ahat[3g' + i][3d' + j] = sum_{g,d} K[g'][g] K[d'][d] A[3g + i][3d + j]
#pragma unroll
                    for (int R = 0; R < 6; ++R)
#pragma unroll
                        for (int C = R; C < 6; ++C) {
                            const int gp = R / 3, i = R % 3, dp = C / 3, jc = C % 3;
                            double v = 0.0;
#pragma unroll
                            for (int g = 0; g < 2; ++g)
#pragma unroll
                                for (int d = 0; d < 2; ++d) {
                                    const int r6 = 3 * g + i, c6 = 3 * d + jc;
                                    v += Kg[gp][g] * Kg[dp][d] * A6[u6(r6, c6)];
                                }
                            rec[u6(R, C)] = v;
                        }
                }
                TP *pp = (TP *)(rec + OFF_P);
                double P6[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) P6[c] = ptP[c * S.n_mp + q];
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int gp = 0; gp < 2; ++gp) pp[2 * i + gp] = Kg[gp][0] * P6[2 * i] + Kg[gp][1] * P6[2 * i + 1];
            }
            if constexpr (STAGE_DN) {
                TP *pp = (TP *)(rec + OFF_P);
#pragma unroll
                for (int c = 0; c < 6; ++c) pp[c] = ptP[c * S.n_mp + q];
            }
        }
    }
    __syncthreads();

    // slots by decreasing number of shared elements (13 = gradient), 4 bits each
    constexpr unsigned long long kO[14] = {0, 1, 5, 13, 4, 6, 2, 10, 3, 7, 9, 11, 8, 12};
    constexpr unsigned long long kPacked = kO[0] | kO[1] << 4 | kO[2] << 8 | kO[3] << 12 | kO[4] << 16 | kO[5] << 20 |
                                           kO[6] << 24 | kO[7] << 28 | kO[8] << 32 | kO[9] << 36 | kO[10] << 40 |
                                           kO[11] << 44 | kO[12] << 48 | kO[13] << 52;
    const int nitems = (hess ? kSlots + 1 : 1) * R;
    const int nchunks = (nitems + 63) / 64;
    const size_t ncp = S.n_cp;
    const int lane = threadIdx.x & 63;
    double gg_loc = 0.0;
    for (;;) {
        int ch = 0;
        if (lane == 0) ch = atomicAdd(counter, 1);
        ch = __shfl(ch, 0);
        if (ch >= nchunks) break;
        const int item = ch * 64 + lane;
        if (item >= nitems) continue;
        const int pos = item / R, c = item % R;
        const int s = hess ? int((kPacked >> (4 * pos)) & 15ull) : kSlots;
        const int i = tx0 + c % kAsmTileU, j = ty0 + c / kAsmTileU;
        if (i >= S.n_u || j >= S.n_v) continue;
        const int a = j * S.n_u + i;
        if (s < kSlots) {
            // Hessian block (a, b) of upper slot s
            const int ib = i + slot_di(s), jb = j + slot_dj(s);
            const int e0 = slot_entry(s);
            TA acc[3][3] = {{TA(0), TA(0), TA(0)}, {TA(0), TA(0), TA(0)}, {TA(0), TA(0), TA(0)}};
            const bool inside = ib >= 0 && ib < S.n_u && jb < S.n_v;
            const bool pinned = inside && (S.pinmask[a] != 0 || S.pinmask[jb * S.n_u + ib] != 0);
            if (inside && !pinned) {
                for (int l = max(0, max(j, jb) - 2); l <= min(min(j, jb), S.Nv - 1); ++l) {
                    for (int k = max(0, max(i, ib) - 2); k <= min(min(i, ib), S.Nu - 1); ++k) {
                        const int el = (l - l0) * nk + (k - k0);
                        const int la = i - k, lb = j - l, ma = ib - k, mb = jb - l;
                        const int oa = 24 + 2 * (3 * lb + la), ob = 24 + 2 * (3 * mb + ma);
                        const int info = el_info[el], cnt = asm_el_count(info);
                        const int r0 = asm_el_first(info), r1 = asm_el_rest(info) - 1;
                        for (int sq = 0; sq < cnt; ++sq) {
                            const TA *rec = prec + size_t(sq == 0 ? r0 : r1 + sq) * REC;
                            TA ga[2], gb[2];
                            if constexpr (STAGE_DN) {
                                TA Aq[21];
                                // 16-byte reads of the record: A in entries 0..20, gradients from 24
                                const float4 *r4 = (const float4 *)rec;
#pragma unroll
                                for (int v = 0; v < 5; ++v) {
                                    const float4 t4 = r4[v];
                                    Aq[4 * v] = t4.x; Aq[4 * v + 1] = t4.y; Aq[4 * v + 2] = t4.z; Aq[4 * v + 3] = t4.w;
                                }
                                Aq[20] = rec[20];
                                const float2 a2 = *(const float2 *)(rec + oa), b2 = *(const float2 *)(rec + ob);
                                ga[0] = a2.x; ga[1] = a2.y; gb[0] = b2.x; gb[1] = b2.y;
                                const TA c00 = ga[0] * gb[0], c01 = ga[0] * gb[1], c10 = ga[1] * gb[0], c11 = ga[1] * gb[1];
#pragma unroll
                                for (int r = 0; r < 3; ++r)
#pragma unroll
                                    for (int cc = 0; cc < 3; ++cc)
                                        acc[r][cc] += c00 * Aq[u6(r, cc)] + c01 * Aq[u6(r, 3 + cc)] +
                                                      c10 * Aq[u6(3 + r, cc)] + c11 * Aq[u6(3 + r, 3 + cc)];
                            } else {
                                // parametric gradients from the 1-D factors; rec holds Ahat
                                ga[0] = rec[OFF_N + 3 + la] * rec[OFF_N + 6 + lb];
                                ga[1] = rec[OFF_N + la] * rec[OFF_N + 9 + lb];
                                gb[0] = rec[OFF_N + 3 + ma] * rec[OFF_N + 6 + mb];
                                gb[1] = rec[OFF_N + ma] * rec[OFF_N + 9 + mb];
                                const TA c00 = ga[0] * gb[0], c01 = ga[0] * gb[1], c10 = ga[1] * gb[0], c11 = ga[1] * gb[1];
#pragma unroll
                                for (int r = 0; r < 3; ++r)
#pragma unroll
                                    for (int cc = 0; cc < 3; ++cc)
                                        acc[r][cc] += c00 * rec[u6(r, cc)] + c01 * rec[u6(r, 3 + cc)] +
                                                      c10 * rec[u6(3 + r, cc)] + c11 * rec[u6(3 + r, 3 + cc)];
                            }
                        }
                    }
                }
                const TA hb = TA(S.hbend[s * ncp + a]) + ((s == 0) ? TA(S.mass[a] * inv_dt2) : TA(0));
#pragma unroll
                for (int r = 0; r < 3; ++r) acc[r][r] += hb;
            } else if (pinned && s == 0) {
#pragma unroll
                for (int r = 0; r < 3; ++r) acc[r][r] = TA(1);
            }
            if (s == 0) {
                hess[(e0 + 0) * ncp + a] = acc[0][0];
                hess[(e0 + 1) * ncp + a] = acc[0][1];
                hess[(e0 + 2) * ncp + a] = acc[0][2];
                hess[(e0 + 3) * ncp + a] = acc[1][1];
                hess[(e0 + 4) * ncp + a] = acc[1][2];
                hess[(e0 + 5) * ncp + a] = acc[2][2];
            } else {
#pragma unroll
                for (int r = 0; r < 3; ++r)
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc) hess[(e0 + 3 * r + cc) * ncp + a] = acc[r][cc];
            }
        } else {
            // gradient: the membrane stresses of the CP's points (staged records) plus the per-CP
            // terms (bending, inertia, gravity) formed by the points pass
            double gp[3];
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) gp[cc] = gpre[cc * ncp + a];
            TG acc[3] = {TG(0), TG(0), TG(0)};
            // the stresses and basis gradients of the CP's points, all from the staged records
            for (int l = max(0, j - 2); l <= min(j, S.Nv - 1); ++l) {
                const int r = l - l0;
                for (int k = max(0, i - 2); k <= min(i, S.Nu - 1); ++k) {
                    const int el = r * nk + (k - k0), la = i - k, lb = j - l;
                    const int info = el_info[el], cnt = asm_el_count(info);
                    const int r0 = asm_el_first(info), r1 = asm_el_rest(info) - 1;
                    for (int sq = 0; sq < cnt; ++sq) {
                        const TA *rec = prec + size_t(sq == 0 ? r0 : r1 + sq) * REC;
                        TG dn[2];
                        if constexpr (KIND == kAsmF32) {
                            const float2 g2 = *(const float2 *)(rec + 24 + 2 * (3 * lb + la));
                            dn[0] = g2.x;
                            dn[1] = g2.y;
                        } else if constexpr (KIND == kAsmMixed) {
                            const int o = 2 * (3 * lb + la);
                            const float2 h2 = *(const float2 *)(rec + 24 + o), l2 = *(const float2 *)(rec + OFF_LO + o);
                            dn[0] = double(h2.x) + double(l2.x);
                            dn[1] = double(h2.y) + double(l2.y);
                        } else {
                            // parametric gradient; the staged stress is P K^T
                            dn[0] = rec[OFF_N + 3 + la] * rec[OFF_N + 6 + lb];
                            dn[1] = rec[OFF_N + la] * rec[OFF_N + 9 + lb];
                        }
                        const TP *pp = (const TP *)(rec + OFF_P);
#pragma unroll
                        for (int cc = 0; cc < 3; ++cc) acc[cc] += TG(pp[2 * cc]) * dn[0] + TG(pp[2 * cc + 1]) * dn[1];
                    }
                }
            }
            const bool pin = S.pinmask[a] != 0;
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                const double gs = double(acc[cc]) + gp[cc];
                const TG gv = pin ? TG(0) : TG(gs);
                gout[cc * ncp + a] = gv;
                gg_loc += double(gv) * double(gv);
            }
        }
    }
    if (gg_partials) {
        const double gg = block_sum(gg_loc, sh);
        if (threadIdx.x == 0) gg_partials[blockIdx.x] = gg;
    }
    // the energy from the points pass's partials, complete before this launch began
    if (esum.out && blockIdx.x == 0) {
        double v = 0.0;
        for (int t = threadIdx.x; t < esum.n0; t += blockDim.x) v += esum.p0[t];
        for (int t = threadIdx.x; t < esum.n1; t += blockDim.x) v += esum.p1[t];
        for (int t = threadIdx.x; t < esum.n2; t += blockDim.x) v += esum.p2[t];
        const double e = block_sum(v, sh);
        if (threadIdx.x == 0) esum.out[0] = e;
    }
}

// ---- per-element outputs -------------------------------------------------------------------

template <typename T>
__global__ void __launch_bounds__(kBlock) k_elem_hess(DevSheet S, const T *__restrict__ ptA, T *__restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int ent = blockIdx.y;                   // 0..377, upper triangle of 27x27, row-major
    if (e >= S.n_elem) return;
    int r = 0, rem = ent;
    while (rem >= 27 - r) { rem -= 27 - r; ++r; }
    const int c = r + rem;
    const int m = r / 3, ci = r % 3, n = c / 3, cj = c % 3;
    const int k = e % S.Nu, l = e / S.Nu;
    double acc = 0.0;
    for (int q = S.mp_off[e]; q < S.mp_off[e + 1]; ++q) {
        T ga[2], gb[2];
        const T tu = T(S.mp_tu[q]), tv = T(S.mp_tv[q]);
        const PtK K = mp_geo(S, q);
        one_grad<T>(S, K, k, l, m % 3, m / 3, tu, tv, ga);
        one_grad<T>(S, K, k, l, n % 3, n / 3, tu, tv, gb);
        T v = T(0);
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int d = 0; d < 2; ++d) v += ga[g] * gb[d] * ptA[u6(3 * g + ci, 3 * d + cj) * S.n_mp + q];
        acc += double(v);
    }
    if (ci == cj) {
        for (int q = S.be_off[e]; q < S.be_off[e + 1]; ++q) {
            double L[9];
            bend_L(S, be_geo(S, q), k, l, S.be_tu[q], S.be_tv[q], L);
            acc += S.be_w[q] * S.mu_bend * L[m] * L[n];
        }
    }
    out[size_t(ent) * S.n_elem + e] = T(acc);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_elem_grad(DevSheet S, const T *__restrict__ ptP, const double *__restrict__ beD,
                                                      const double *__restrict__ ptE, const double *__restrict__ beE,
                                                      T *__restrict__ eE, T *__restrict__ eg) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= S.n_elem) return;
    const int k = e % S.Nu, l = e / S.Nu;
    if (eg) {
        for (int m = 0; m < 9; ++m) {
            double acc[3] = {0.0, 0.0, 0.0};
            for (int q = S.mp_off[e]; q < S.mp_off[e + 1]; ++q) {
                T gm[2];
                one_grad<T>(S, mp_geo(S, q), k, l, m % 3, m / 3, T(S.mp_tu[q]), T(S.mp_tv[q]), gm);
                for (int c = 0; c < 3; ++c)
                    acc[c] += double(ptP[(2 * c) * S.n_mp + q] * gm[0] + ptP[(2 * c + 1) * S.n_mp + q] * gm[1]);
            }
            for (int q = S.be_off[e]; q < S.be_off[e + 1]; ++q) {
                double L[9];
                bend_L(S, be_geo(S, q), k, l, S.be_tu[q], S.be_tv[q], L);
                for (int c = 0; c < 3; ++c) acc[c] += beD[c * S.n_be + q] * L[m];
            }
            for (int c = 0; c < 3; ++c) eg[size_t(3 * m + c) * S.n_elem + e] = T(acc[c]);
        }
    }
    if (eE) {
        double s = 0.0;
        for (int q = S.mp_off[e]; q < S.mp_off[e + 1]; ++q) s += ptE[q];
        for (int q = S.be_off[e]; q < S.be_off[e + 1]; ++q) s += beE[q];
        eE[e] = T(s);
    }
}

// Sums three partial arrays in a fixed order into out[0] (the energy) and, if pg is given, the
// partials pg (|g|^2 of the assembly tiles) into out_g[0].
// With pub, the solver scalars (scal, which holds out and out_g) and flags are then read back to
// the host in the same launch.
__global__ void __launch_bounds__(kBlock) k_reduce(const double *__restrict__ p0, int n0, const double *__restrict__ p1,
                                                   int n1, const double *__restrict__ p2, int n2,
                                                   double *__restrict__ out, const double *__restrict__ pg, int ng,
                                                   double *__restrict__ out_g, const double *scal, int32_t *flags,
                                                   PubPtrs pub, int do_pub) {
    __shared__ double sh[kBlock / 64];
    double v = 0.0;
    for (int t = threadIdx.x; t < n0; t += blockDim.x) v += p0[t];
    for (int t = threadIdx.x; t < n1; t += blockDim.x) v += p1[t];
    for (int t = threadIdx.x; t < n2; t += blockDim.x) v += p2[t];
    const double s = block_sum(v, sh);
    if (threadIdx.x == 0) out[0] = s;
    if (pg) {
        double u = 0.0;
        for (int t = threadIdx.x; t < ng; t += blockDim.x) u += pg[t];
        const double sg = block_sum(u, sh);
        if (threadIdx.x == 0) out_g[0] = sg;
    }
    if (do_pub) {
        __syncthreads();
        publish_block(scal, flags, pub);
    }
}

inline int blocks(int n) { return (n + kBlock - 1) / kBlock; }

}  // namespace

int cp_blocks(const DevSheet &S) { return blocks(S.n_cp); }

hipError_t launch_points(const DevSheet &S, const DevBufs &B, int precision, bool hess, bool grad64,
                         const double *x, hipStream_t st, bool bending, const CpTerms *cpt) {
    // Partials layout: [0] membrane, [1] bending, [2] per-CP terms, [3] assembly tiles (|g|^2);
    // [4..7] are free for the kernels that follow (the warm start's dot products).
    double *pm = B.partials, *pb = B.partials + B.max_blocks, *pc = B.partials + 2 * B.max_blocks;
    // with the per-CP terms the bending energy comes from the stencil: no bending blocks
    const int ncb = cpt ? cp_blocks(S) : 0, nbm = blocks(S.n_mp), nb = ncb + nbm + (bending && !cpt ? blocks(S.n_be) : 0);
    const CpTerms Ct = cpt ? *cpt : CpTerms{nullptr, 0.0, 0.0, 0.0, 0.0, nullptr};
    auto go = [&](auto curved, auto bend) {
        constexpr bool C = decltype(curved)::value, BE = decltype(bend)::value;
        if (grad64 || precision == BSC_FP64) {
            double *P = grad64 ? B.ptP64 : (double *)B.ptP;
            if (hess && !grad64)
                k_points<double, true, C, double, double, BE><<<nb, kBlock, 0, st>>>(S, x, (double *)B.ptA, P, B.ptE, pm, B.beD,
                                                                                      B.beE, pb, ncb, nbm, Ct, pc);
            else
                k_points<double, false, C, double, double, BE><<<nb, kBlock, 0, st>>>(S, x, (double *)B.ptA, P, B.ptE, pm, B.beD,
                                                                                       B.beE, pb, ncb, nbm, Ct, pc);
        } else {
            if (hess)
                k_points<float, true, C, float, float, BE><<<nb, kBlock, 0, st>>>(S, x, (float *)B.ptA, (float *)B.ptP, B.ptE, pm,
                                                                                  B.beD, B.beE, pb, ncb, nbm, Ct, pc);
            else
                k_points<float, false, C, float, float, BE><<<nb, kBlock, 0, st>>>(S, x, (float *)B.ptA, (float *)B.ptP, B.ptE, pm,
                                                                                   B.beD, B.beE, pb, ncb, nbm, Ct, pc);
        }
    };
    auto go2 = [&](auto curved) {
        if (bending) go(curved, std::true_type{});
        else go(curved, std::false_type{});
    };
    if (S.curved) go2(std::true_type{});
    else go2(std::false_type{});
    return hipGetLastError();
}

// The Newton step's mixed-precision points in one pass: FP64 arithmetic, the stresses (for the
// FP64 gradient) stored in double and the projected density Hessian stored in float.
hipError_t launch_points_mixed(const DevSheet &S, const DevBufs &B, const double *x, hipStream_t st, const CpTerms *cpt) {
    double *pm = B.partials, *pb = B.partials + B.max_blocks, *pc = B.partials + 2 * B.max_blocks;
    const int ncb = cpt ? cp_blocks(S) : 0, nbm = blocks(S.n_mp), nb = ncb + nbm + (cpt ? 0 : blocks(S.n_be));
    const CpTerms Ct = cpt ? *cpt : CpTerms{nullptr, 0.0, 0.0, 0.0, 0.0, nullptr};
    auto go = [&](auto curved) {
        constexpr bool C = decltype(curved)::value;
        k_points<double, true, C, float, double><<<nb, kBlock, 0, st>>>(S, x, (float *)B.ptA, B.ptP64, B.ptE, pm, B.beD, B.beE,
                                                                         pb, ncb, nbm, Ct, pc);
    };
    if (S.curved) go(std::true_type{});
    else go(std::false_type{});
    return hipGetLastError();
}

int assemble_tiles(const DevSheet &S, int kind) {
    return ((S.n_u + kAsmTileU - 1) / kAsmTileU) * asm_tile_rows(S.n_v, S.asm_ty[kind]);
}

hipError_t launch_assemble(const DevSheet &S, const DevBufs &B, int kind, double inv_dt2, void *g, void *hess,
                           hipStream_t st, bool gnorm, double *out_e) {
    double *pg = gnorm ? B.partials + 3 * B.max_blocks : nullptr;
    const EnergySum esum{B.partials, B.partials + B.max_blocks, B.partials + 2 * B.max_blocks, blocks(S.n_mp), 0, cp_blocks(S),
                         out_e};
    const size_t lds = asm_lds_layout(kAsmTileU, S.asm_ty[kind], S.asm_maxp[kind], kind, S.curved != 0).total;
    const int nt = assemble_tiles(S, kind);
    auto go = [&](auto curved) {
        constexpr bool CV = decltype(curved)::value;
        if (kind == kAsmF32)
            k_assemble_tile<float, float, float, CV><<<nt, kAsmThreads, lds, st>>>(
                S, kind, (const float *)B.ptA, (const float *)B.ptP, B.gpre, inv_dt2, (float *)hess, (float *)g, pg, esum);
        else if (kind == kAsmF64)
            k_assemble_tile<double, double, double, CV><<<nt, kAsmThreads, lds, st>>>(
                S, kind, (const double *)B.ptA, (const double *)B.ptP, B.gpre, inv_dt2, (double *)hess, (double *)g, pg, esum);
        else
            k_assemble_tile<float, double, double, CV><<<nt, kAsmThreads, lds, st>>>(
                S, kind, (const float *)B.ptA, B.ptP64, B.gpre, inv_dt2, (float *)hess, (double *)g, pg, esum);
    };
    if (S.curved) go(std::true_type{});
    else go(std::false_type{});
    return hipGetLastError();
}

hipError_t launch_energy_reduce(const DevSheet &S, const DevBufs &B, int n_cp_partials, int n_gg_partials, double *out,
                                hipStream_t st, double *out_gg, const PubPtrs *pub) {
    static_assert(kBlock >= kScalars, "the read-back copies one scalar per thread");
    k_reduce<<<1, kBlock, 0, st>>>(B.partials, blocks(S.n_mp), B.partials + B.max_blocks, n_cp_partials ? 0 : blocks(S.n_be),
                                   B.partials + 2 * B.max_blocks, n_cp_partials, out,
                                   out_gg ? B.partials + 3 * B.max_blocks : nullptr, n_gg_partials, out_gg, B.scalars,
                                   B.iscalars, pub ? *pub : PubPtrs{nullptr, nullptr, nullptr}, pub ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_elem(const DevSheet &S, const DevBufs &B, int precision, void *eE, void *eg, void *eH, hipStream_t st) {
    if (precision == BSC_FP64) {
        if (eH) k_elem_hess<double><<<dim3(blocks(S.n_elem), 378), kBlock, 0, st>>>(S, (const double *)B.ptA, (double *)eH);
        if (eE || eg)
            k_elem_grad<double><<<blocks(S.n_elem), kBlock, 0, st>>>(S, (const double *)B.ptP, B.beD, B.ptE, B.beE, (double *)eE, (double *)eg);
    } else {
        if (eH) k_elem_hess<float><<<dim3(blocks(S.n_elem), 378), kBlock, 0, st>>>(S, (const float *)B.ptA, (float *)eH);
        if (eE || eg)
            k_elem_grad<float><<<blocks(S.n_elem), kBlock, 0, st>>>(S, (const float *)B.ptP, B.beD, B.ptE, B.beE, (float *)eE, (float *)eg);
    }
    return hipGetLastError();
}

}  // namespace bsc

using namespace bsc;

extern "C" {

bsc_status bsc_eval_egh(bsc_ctx *c, int32_t precision, const double *d_x, double *d_energy, void *d_elem_energy,
                        void *d_elem_grad, void *d_elem_hess) {
    if (!c) return BSC_E_INVAL;
    if (!c->ws) return fail(c, BSC_E_STATE, "no workspace bound");
    if (!d_x || !d_energy) return fail(c, BSC_E_INVAL, "null pointer");
    if (precision != BSC_FP64 && precision != BSC_FP32_MIXED) return fail(c, BSC_E_INVAL, "bad precision");
    const DevSheet &S = c->dev;
    bsc_status st = hip_check(c, launch_points(S, c->buf, precision, d_elem_hess != nullptr, false, d_x, c->stream, true), "eval points");
    if (st != BSC_OK) return st;
    st = hip_check(c, launch_energy_reduce(S, c->buf, 0, 0, d_energy, c->stream), "energy reduce");
    if (st != BSC_OK) return st;
    return hip_check(c, launch_elem(S, c->buf, precision, d_elem_energy, d_elem_grad, d_elem_hess, c->stream), "element gather");
}

bsc_status bsc_assemble(bsc_ctx *c, int32_t precision, const double *d_x, const double *d_xhat, double dt,
                        const double *gravity, double *d_energy, void *d_grad, void *d_hess) {
    if (!c) return BSC_E_INVAL;
    if (!c->ws) return fail(c, BSC_E_STATE, "no workspace bound");
    if (!d_x || !d_energy || !d_grad) return fail(c, BSC_E_INVAL, "null pointer");
    if (precision != BSC_FP64 && precision != BSC_FP32_MIXED) return fail(c, BSC_E_INVAL, "bad precision");
    double inv_dt2 = 0.0;
    if (d_xhat) {
        if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, BSC_E_INVAL, "dt must be positive");
        inv_dt2 = 1.0 / (dt * dt);
    }
    const DevSheet &S = c->dev;
    const CpTerms cpt{d_xhat, inv_dt2, gravity ? gravity[0] : 0.0, gravity ? gravity[1] : 0.0, gravity ? gravity[2] : 0.0,
                      c->buf.gpre};
    bsc_status st = hip_check(c, launch_points(S, c->buf, precision, d_hess != nullptr, false, d_x, c->stream, false, &cpt),
                              "eval points");
    if (st != BSC_OK) return st;
    const int kind = precision == BSC_FP64 ? kAsmF64 : kAsmF32;
    return hip_check(c, launch_assemble(S, c->buf, kind, inv_dt2, d_grad, d_hess, c->stream, false, d_energy), "assemble");
}

}  // extern "C"
