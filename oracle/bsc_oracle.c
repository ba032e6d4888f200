/*
 * bsc_oracle.c -- plain FP64 CPU reference ("oracle") for the hot path of the quadratic
 * B-spline cloth finite elements of arXiv 2506.18867: membrane and bending energy, gradient
 * and element Hessian at the separately reduced quadrature points, per-point PSD projection,
 * assembly onto the 5x5 control-point block pattern, lumped mass and the implicit-Euler
 * incremental potential.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the benchmark's CPU-baseline
 * leg may load this library. It is deliberately plain and slow: straight loops that follow the
 * paper's definitions in the paper's order, no blocking, no fusion, and no code shared with
 * the HIP library (neither includes or links the other).
 *
 * Conventions
 *   - Knot vectors are 0-based arrays of n+3 doubles (the paper indexes them from 1).
 *   - Control point (CP) (i,j), 0 <= i < n_u, 0 <= j < n_v, has index alpha = j*n_u + i.
 *   - World positions are AoS: x[3*alpha + c]. Rest positions: X[2*alpha + c].
 *   - The 3x2 deformation gradient F = [f1 f2]; vec(F) is column-major, r = 3*gamma + i.
 *   - An element is a knot span (k,l); its CPs are (k+a, l+b), a,b in {0,1,2}; local CP
 *     index 3*b + a, local DOF 3*(3*b+a) + c (27 DOFs).
 *   - Global Hessian ("stencil form"): H[(alpha*25 + s)*9 + 3*r + c] is the 3x3 block
 *     coupling CP alpha to CP alpha + (di, dj) with s = (dj+2)*5 + (di+2).
 *
 * Readings of the paper taken here (each is listed with its reason in the design notes):
 *   R-quad  quadrature weights = Gauss weights x area of the clipped dual cell / knot span.
 *   R-edge  edge half cells of the interior region carry two points on the knot line,
 *           corner quarter cells one point at the knot.
 *   R2      bending at a knot intersection = mean of the four one-sided evaluations, each
 *           made with the polynomial of one adjacent knot span.
 *   R-mass  lumped mass from 3x3 Gauss per knot span, rows of the consistent mass summed.
 *   R-stvk  StVK membrane with plane-stress Lame parameter E*nu/(1-nu^2), times thickness.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)

/* ------------------------------------------------------------------------------------------
 * 1. B-spline basis (Sec. 3.1.1, Eq. "B-spline basis"): the Cox-de Boor recursion, with any
 *    term whose denominator vanishes (repeated knots) set to zero.
 * ------------------------------------------------------------------------------------------ */

/* N_{i,p}(u) exactly as defined: the degree-0 functions are half-open indicators. */
double or_basis(const double *xi, int i, int p, double u)
{
    if (p == 0) return (xi[i] <= u && u < xi[i + 1]) ? 1.0 : 0.0;
    double left = 0.0, right = 0.0;
    double dl = xi[i + p] - xi[i];
    double dr = xi[i + p + 1] - xi[i + 1];
    if (dl != 0.0) left = (u - xi[i]) / dl * or_basis(xi, i, p - 1, u);
    if (dr != 0.0) right = (xi[i + p + 1] - u) / dr * or_basis(xi, i + 1, p - 1, u);
    return left + right;
}

/* The polynomial piece of N_{i,p} on knot interval [xi_s, xi_{s+1}), extended to every u:
 * the same recursion with the degree-0 indicator replaced by "interval index == s". Its
 * d-th derivative follows by differentiating the recursion (the standard derivative formula
 * N'_{i,p} = p/(xi_{i+p}-xi_i) N_{i,p-1} - p/(xi_{i+p+1}-xi_{i+1}) N_{i+1,p-1}). */
double or_basis_piece(const double *xi, int i, int p, int s, double u, int d)
{
    if (p == 0) return (d == 0 && i == s) ? 1.0 : 0.0;
    double dl = xi[i + p] - xi[i];
    double dr = xi[i + p + 1] - xi[i + 1];
    double left = 0.0, right = 0.0;
    if (d == 0) {
        if (dl != 0.0) left = (u - xi[i]) / dl * or_basis_piece(xi, i, p - 1, s, u, 0);
        if (dr != 0.0) right = (xi[i + p + 1] - u) / dr * or_basis_piece(xi, i + 1, p - 1, s, u, 0);
        return left + right;
    }
    if (dl != 0.0) left = p / dl * or_basis_piece(xi, i, p - 1, s, u, d - 1);
    if (dr != 0.0) right = p / dr * or_basis_piece(xi, i + 1, p - 1, s, u, d - 1);
    return left - right;
}

/* Index s of the k-th non-empty knot interval, or -1. */
static int knot_interval(const double *xi, int nk, int k)
{
    int count = 0;
    for (int s = 0; s + 1 < nk; ++s) {
        if (xi[s + 1] > xi[s]) {
            if (count == k) return s;
            ++count;
        }
    }
    return -1;
}

/* Checks that xi (n+3 entries) is an open, uniform quadratic knot vector starting at 0 with
 * integer knots (Sec. 3.1.2). Returns the number of spans N and the spacing h, or -1. */
int or_check_knots(const double *xi, int n, double *spacing)
{
    int nk = n + 3;
    if (n < 3) return -1;
    if (xi[0] != 0.0 || xi[1] != 0.0 || xi[2] != 0.0) return -1;
    if (xi[nk - 1] != xi[nk - 2] || xi[nk - 2] != xi[nk - 3]) return -1;
    double h = xi[3] - xi[2];
    if (!(h > 0.0) || h != floor(h)) return -1;
    for (int s = 2; s < nk - 3; ++s) {
        if (xi[s + 1] - xi[s] != h) return -1;
    }
    if (spacing) *spacing = h;
    return n - 2;
}

/* ------------------------------------------------------------------------------------------
 * 2. Reduced quadrature rules (Sec. 4.1 "Reduced Integration" and Sec. 4.2 "Reduced
 *    Integration"; Fig. "quadrature"). Coordinates are in span units (span k = [k, k+1]).
 *    Each output record is (u, v, wbar, k, l): wbar is the parametric weight, (k,l) the span
 *    whose polynomials evaluate the point.
 * ------------------------------------------------------------------------------------------ */

static const double G2 = 0.28867513459481288225;   /* 1/(2 sqrt 3): 2-point Gauss, +-offset */
static const double G3 = 0.38729833462074168852;   /* sqrt(3/5)/2: 3-point Gauss offset     */

static void gauss_1d(int npt, double *off, double *w)
{
    if (npt == 2) {
        off[0] = -G2; off[1] = G2; w[0] = w[1] = 0.5;
    } else {
        off[0] = -G3; off[1] = 0.0; off[2] = G3;
        w[0] = 5.0 / 18.0; w[1] = 8.0 / 18.0; w[2] = 5.0 / 18.0;
    }
}

static int push(double *out, int cap, int cnt, double u, double v, double w, int k, int l)
{
    if (cnt < cap && out) {
        out[5 * cnt + 0] = u; out[5 * cnt + 1] = v; out[5 * cnt + 2] = w;
        out[5 * cnt + 3] = k; out[5 * cnt + 4] = l;
    }
    return cnt + 1;
}

static int imin(int a, int b) { return a < b ? a : b; }

/* Quadrature variants. OR_QUAD_REDUCED is the paper's scheme (Sec. 4.1, 4.2). The others are
 * the comparison rules of its ablation study (Sec. 6.5): the standard 2x2 Gauss rule on every
 * interior knot span for membrane and bending (boundary spans unchanged), a single midpoint
 * per interior span for the membrane ("1x1", which admits hourglass modes), and 2x2 instead of
 * 3x3 Gauss on the four corner spans for the membrane. */
enum { OR_QUAD_REDUCED = 0, OR_QUAD_GAUSS2 = 1, OR_QUAD_INTERIOR1 = 2, OR_QUAD_CORNER2 = 3 };

/* Membrane rule. Boundary knot spans: 3x3 Gauss at the four corners, 3 (across) x 2 (along)
 * on the sides. Interior region [1,Nu-1]x[1,Nv-1]: cells of the dual grid (lines through the
 * control points, i.e. at half-integers) centred at knot (a,b), clipped to the region.
 * Full cells alternate 1x2 / 2x1 Gauss by the parity of a+b; edge half cells carry two
 * points on the knot line, corner quarter cells one point at the knot. Returns the count. */
int or_membrane_rule_q(int Nu, int Nv, int quad, double *out, int cap)
{
    int cnt = 0;
    double ou[3], wu[3], ov[3], wv[3];
    for (int l = 0; l < Nv; ++l) {
        for (int k = 0; k < Nu; ++k) {
            int bu = (k == 0 || k == Nu - 1), bv = (l == 0 || l == Nv - 1);
            int nu, nv;
            if (bu && bv) {
                nu = nv = (quad == OR_QUAD_CORNER2) ? 2 : 3;      /* corner spans */
            } else if (bu || bv) {
                nu = bu ? 3 : 2; nv = bv ? 3 : 2;                  /* side spans   */
            } else if (quad == OR_QUAD_GAUSS2) {
                nu = nv = 2;                                       /* interior, standard rule */
            } else if (quad == OR_QUAD_INTERIOR1) {
                cnt = push(out, cap, cnt, k + 0.5, l + 0.5, 1.0, k, l);   /* span midpoint */
                continue;
            } else {
                continue;                                          /* dual-grid cells below */
            }
            gauss_1d(nu, ou, wu);
            gauss_1d(nv, ov, wv);
            for (int b = 0; b < nv; ++b)
                for (int a = 0; a < nu; ++a)
                    cnt = push(out, cap, cnt, k + 0.5 + ou[a], l + 0.5 + ov[b], wu[a] * wv[b], k, l);
        }
    }
    if (quad == OR_QUAD_GAUSS2 || quad == OR_QUAD_INTERIOR1) return cnt;
    for (int b = 1; b <= Nv - 1; ++b) {
        for (int a = 1; a <= Nu - 1; ++a) {
            int edge_u = (a == 1 || a == Nu - 1), edge_v = (b == 1 || b == Nv - 1);
            double pts[2][2];
            int np;
            double w;
            if (edge_u && edge_v) {               /* corner quarter cell */
                np = 1; w = 0.25;
                pts[0][0] = a; pts[0][1] = b;
            } else if (edge_u) {                  /* half cell on a vertical edge */
                np = 2; w = 0.25;
                pts[0][0] = a; pts[0][1] = b - G2;
                pts[1][0] = a; pts[1][1] = b + G2;
            } else if (edge_v) {                  /* half cell on a horizontal edge */
                np = 2; w = 0.25;
                pts[0][0] = a - G2; pts[0][1] = b;
                pts[1][0] = a + G2; pts[1][1] = b;
            } else if ((a + b) % 2 == 0) {        /* full cell, 1 (u) x 2 (v) */
                np = 2; w = 0.5;
                pts[0][0] = a; pts[0][1] = b - G2;
                pts[1][0] = a; pts[1][1] = b + G2;
            } else {                              /* full cell, 2 (u) x 1 (v) */
                np = 2; w = 0.5;
                pts[0][0] = a - G2; pts[0][1] = b;
                pts[1][0] = a + G2; pts[1][1] = b;
            }
            for (int q = 0; q < np; ++q) {
                double u = pts[q][0], v = pts[q][1];
                int k = imin((int)floor(u), Nu - 1), l = imin((int)floor(v), Nv - 1);
                cnt = push(out, cap, cnt, u, v, w, k, l);
            }
        }
    }
    return cnt;
}

int or_membrane_rule(int Nu, int Nv, double *out, int cap)
{
    return or_membrane_rule_q(Nu, Nv, OR_QUAD_REDUCED, out, cap);
}

/* Bending rule: one point at the centre of every boundary knot span (weight 1) and one at
 * every interior knot (a,b), the centre of its dual cell, weighted by the clipped cell area.
 * Reading R2: the knot point is evaluated four times, once with the polynomials of each
 * adjacent span, each carrying a quarter of the weight. With OR_QUAD_GAUSS2 the interior spans
 * take 2x2 Gauss points instead of the knot points. Returns the number of evaluations. */
int or_bending_rule_q(int Nu, int Nv, int quad, double *out, int cap)
{
    int cnt = 0;
    for (int l = 0; l < Nv; ++l)
        for (int k = 0; k < Nu; ++k)
            if (k == 0 || k == Nu - 1 || l == 0 || l == Nv - 1)
                cnt = push(out, cap, cnt, k + 0.5, l + 0.5, 1.0, k, l);
    if (quad == OR_QUAD_GAUSS2) {              /* standard 2x2 Gauss on the interior spans */
        double o[3], w[3];
        gauss_1d(2, o, w);
        for (int l = 1; l < Nv - 1; ++l)
            for (int k = 1; k < Nu - 1; ++k)
                for (int b = 0; b < 2; ++b)
                    for (int a = 0; a < 2; ++a)
                        cnt = push(out, cap, cnt, k + 0.5 + o[a], l + 0.5 + o[b], w[a] * w[b], k, l);
        return cnt;
    }
    for (int b = 1; b <= Nv - 1; ++b) {
        for (int a = 1; a <= Nu - 1; ++a) {
            double lu = (a == 1 || a == Nu - 1) ? 0.5 : 1.0;
            double lv = (b == 1 || b == Nv - 1) ? 0.5 : 1.0;
            if (Nu == 2) lu = 0.0;
            if (Nv == 2) lv = 0.0;
            double w = lu * lv * 0.25;
            cnt = push(out, cap, cnt, a, b, w, a - 1, b - 1);
            cnt = push(out, cap, cnt, a, b, w, a, b - 1);
            cnt = push(out, cap, cnt, a, b, w, a - 1, b);
            cnt = push(out, cap, cnt, a, b, w, a, b);
        }
    }
    return cnt;
}

int or_bending_rule(int Nu, int Nv, double *out, int cap)
{
    return or_bending_rule_q(Nu, Nv, OR_QUAD_REDUCED, out, cap);
}

/* ------------------------------------------------------------------------------------------
 * 3. Sheet description and tensor-product basis at a point (Eq. "tensor product of B-spline
 *    basis", Eq. "general B-spline patch", Sec. 3.2).
 * ------------------------------------------------------------------------------------------ */

typedef struct {
    int n_u, n_v;               /* control points per direction */
    const double *knots_u;      /* n_u + 3 */
    const double *knots_v;      /* n_v + 3 */
    const double *rest;         /* 2*n_u*n_v, AoS (X1, X2) */
    int membrane;               /* 0 StVK, 1 FBW */
    double young, poisson, thickness;
    double mu_st1, mu_st2, mu_sh;
    double mu_bend;
    double rho_area;
    int quadrature;             /* OR_QUAD_*                                                  */
} or_sheet;

typedef struct {
    int cp[9];                  /* global CP index of local CP 3*b+a */
    double N[9], Nu[9], Nv[9], Nuu[9], Nvv[9], Nuv[9];
} tp_basis;

/* u, v in span units; the knot coordinate is knot_origin + spacing * u. */
static void eval_tp_basis(const or_sheet *S, int k, int l, double us, double vs, tp_basis *B)
{
    double hu, hv;
    or_check_knots(S->knots_u, S->n_u, &hu);
    or_check_knots(S->knots_v, S->n_v, &hv);
    int su = knot_interval(S->knots_u, S->n_u + 3, k);
    int sv = knot_interval(S->knots_v, S->n_v + 3, l);
    double u = us * hu, v = vs * hv;
    double Ru[3][3], Rv[3][3];      /* [local a][derivative order] */
    for (int a = 0; a < 3; ++a) {
        int i = su - 2 + a;
        for (int d = 0; d < 3; ++d) Ru[a][d] = or_basis_piece(S->knots_u, i, 2, su, u, d);
        int j = sv - 2 + a;
        for (int d = 0; d < 3; ++d) Rv[a][d] = or_basis_piece(S->knots_v, j, 2, sv, v, d);
    }
    for (int b = 0; b < 3; ++b) {
        for (int a = 0; a < 3; ++a) {
            int m = 3 * b + a;
            B->cp[m] = (sv - 2 + b) * S->n_u + (su - 2 + a);
            /* derivatives with respect to the span-unit coordinates */
            B->N[m] = Ru[a][0] * Rv[b][0];
            B->Nu[m] = Ru[a][1] * hu * Rv[b][0];
            B->Nv[m] = Ru[a][0] * Rv[b][1] * hv;
            B->Nuu[m] = Ru[a][2] * hu * hu * Rv[b][0];
            B->Nvv[m] = Ru[a][0] * Rv[b][2] * hv * hv;
            B->Nuv[m] = Ru[a][1] * hu * Rv[b][1] * hv;
        }
    }
}

/* Rest map derivatives at a point (Sec. 4.1, inverse function theorem; Sec. 4.2 for the
 * second derivatives). J[l][m] = dX_l/dxi_m, K = J^{-1} (K[m][b] = dxi_m/dX_b), detJ, and the
 * coefficients of the Laplacian in parametric space (Eq. "Laplacian in parametric space"):
 *   lap[0] = u1^2+u2^2, lap[1] = v1^2+v2^2, lap[2] = u11+u22, lap[3] = v11+v22,
 *   lap[4] = 2(u1 v1 + u2 v2).
 * The second derivatives come from d(K)/dxi_p = -K (dJ/dxi_p) K and the chain rule. */
static void rest_geometry(const or_sheet *S, const tp_basis *B, double K[2][2], double *detJ,
                          double lap[5])
{
    double J[2][2] = {{0, 0}, {0, 0}};
    double dJ[2][2][2] = {{{0}}};           /* dJ[p][l][m] = d J[l][m] / d xi_p */
    for (int m = 0; m < 9; ++m) {
        const double *X = S->rest + 2 * B->cp[m];
        for (int c = 0; c < 2; ++c) {
            J[c][0] += X[c] * B->Nu[m];
            J[c][1] += X[c] * B->Nv[m];
            dJ[0][c][0] += X[c] * B->Nuu[m];
            dJ[0][c][1] += X[c] * B->Nuv[m];
            dJ[1][c][0] += X[c] * B->Nuv[m];
            dJ[1][c][1] += X[c] * B->Nvv[m];
        }
    }
    double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    *detJ = det;
    K[0][0] = J[1][1] / det;  K[0][1] = -J[0][1] / det;
    K[1][0] = -J[1][0] / det; K[1][1] = J[0][0] / det;
    /* dK[p] = -K dJ[p] K */
    double dK[2][2][2];
    for (int p = 0; p < 2; ++p) {
        for (int r = 0; r < 2; ++r) {
            for (int c = 0; c < 2; ++c) {
                double s = 0.0;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) s += K[r][a] * dJ[p][a][b] * K[b][c];
                dK[p][r][c] = -s;
            }
        }
    }
    /* Laplacian of xi_m over X: sum_q d K[m][q] / d X_q = sum_q sum_p dK[p][m][q] K[p][q] */
    double lapxi[2];
    for (int m = 0; m < 2; ++m) {
        double s = 0.0;
        for (int q = 0; q < 2; ++q)
            for (int p = 0; p < 2; ++p) s += dK[p][m][q] * K[p][q];
        lapxi[m] = s;
    }
    lap[0] = K[0][0] * K[0][0] + K[0][1] * K[0][1];
    lap[1] = K[1][0] * K[1][0] + K[1][1] * K[1][1];
    lap[2] = lapxi[0];
    lap[3] = lapxi[1];
    lap[4] = 2.0 * (K[0][0] * K[1][0] + K[0][1] * K[1][1]);
}

/* ------------------------------------------------------------------------------------------
 * 4. Membrane energy densities (Sec. 4.1). F is 3x2, column-major vec (r = 3*gamma + i).
 * ------------------------------------------------------------------------------------------ */

/* StVK (reading R-stvk): E_G = (F^T F - I)/2, Psi = mu |E_G|^2 + lam/2 tr(E_G)^2 with
 * mu = E t / (2(1+nu)), lam = E t nu / (1 - nu^2). P = F S, S = 2 mu E_G + lam tr(E_G) I,
 * A[(g,i),(d,j)] = delta_ij S_gd + mu F_id F_jg + mu delta_gd (F F^T)_ij + lam F_ig F_jd. */
static void stvk_density(const double F[3][2], double mu, double lam, double *psi,
                         double P[3][2], double A[6][6])
{
    double C[2][2];
    for (int g = 0; g < 2; ++g)
        for (int d = 0; d < 2; ++d) {
            double s = 0.0;
            for (int i = 0; i < 3; ++i) s += F[i][g] * F[i][d];
            C[g][d] = s;
        }
    double E[2][2] = {{0.5 * (C[0][0] - 1.0), 0.5 * C[0][1]}, {0.5 * C[1][0], 0.5 * (C[1][1] - 1.0)}};
    double trE = E[0][0] + E[1][1];
    double EE = E[0][0] * E[0][0] + E[0][1] * E[0][1] + E[1][0] * E[1][0] + E[1][1] * E[1][1];
    *psi = mu * EE + 0.5 * lam * trE * trE;
    double Sm[2][2];
    for (int g = 0; g < 2; ++g)
        for (int d = 0; d < 2; ++d) Sm[g][d] = 2.0 * mu * E[g][d] + (g == d ? lam * trE : 0.0);
    for (int i = 0; i < 3; ++i)
        for (int g = 0; g < 2; ++g) P[i][g] = F[i][0] * Sm[0][g] + F[i][1] * Sm[1][g];
    double FFt[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) FFt[i][j] = F[i][0] * F[j][0] + F[i][1] * F[j][1];
    for (int g = 0; g < 2; ++g)
        for (int i = 0; i < 3; ++i)
            for (int d = 0; d < 2; ++d)
                for (int j = 0; j < 3; ++j) {
                    double a = (i == j ? Sm[g][d] : 0.0) + mu * F[i][d] * F[j][g]
                               + (g == d ? mu * FFt[i][j] : 0.0) + lam * F[i][g] * F[j][d];
                    A[3 * g + i][3 * d + j] = a;
                }
}

/* FBW (Eqs. "anisotropic invariants", "FBW stretching and shearing energy"):
 * I5(e1) = f1.f1, I5(e2) = f2.f2, I6 = f1.f2,
 * Psi = mu_sh I6^2 + mu_st1 (sqrt(I5(e1)) - 1)^2 + mu_st2 (sqrt(I5(e2)) - 1)^2. */
static void fbw_density(const double F[3][2], double mu1, double mu2, double msh, double *psi,
                        double P[3][2], double A[6][6])
{
    double f[2][3];
    for (int i = 0; i < 3; ++i) { f[0][i] = F[i][0]; f[1][i] = F[i][1]; }
    double I5[2], I6 = 0.0, len[2];
    for (int g = 0; g < 2; ++g) {
        I5[g] = f[g][0] * f[g][0] + f[g][1] * f[g][1] + f[g][2] * f[g][2];
        len[g] = sqrt(I5[g]);
    }
    for (int i = 0; i < 3; ++i) I6 += f[0][i] * f[1][i];
    double mu[2] = {mu1, mu2};
    *psi = msh * I6 * I6 + mu1 * (len[0] - 1.0) * (len[0] - 1.0) + mu2 * (len[1] - 1.0) * (len[1] - 1.0);
    for (int g = 0; g < 2; ++g)
        for (int i = 0; i < 3; ++i)
            P[i][g] = 2.0 * msh * I6 * f[1 - g][i] + 2.0 * mu[g] * (1.0 - 1.0 / len[g]) * f[g][i];
    for (int g = 0; g < 2; ++g) {
        for (int d = 0; d < 2; ++d) {
            for (int i = 0; i < 3; ++i) {
                for (int j = 0; j < 3; ++j) {
                    double a;
                    if (g == d) {
                        a = 2.0 * msh * f[1 - g][i] * f[1 - g][j]
                            + 2.0 * mu[g] * ((i == j ? 1.0 - 1.0 / len[g] : 0.0)
                                             + f[g][i] * f[g][j] / (len[g] * len[g] * len[g]));
                    } else {
                        /* d^2 Psi / d f_g,i d f_d,j = 2 mu_sh (f_d,i f_g,j + I6 delta_ij) */
                        a = 2.0 * msh * (f[d][i] * f[g][j] + (i == j ? I6 : 0.0));
                    }
                    A[3 * g + i][3 * d + j] = a;
                }
            }
        }
    }
}

void or_membrane_density(int model, const double *Fin /* 3x2 row-major */, double young,
                         double poisson, double thickness, double mu1, double mu2, double msh,
                         double *psi, double *Pout /* 3x2 row-major */, double *Aout /* 6x6 */)
{
    double F[3][2], P[3][2], A[6][6];
    for (int i = 0; i < 3; ++i) { F[i][0] = Fin[2 * i]; F[i][1] = Fin[2 * i + 1]; }
    if (model == 0) {
        double mu = young * thickness / (2.0 * (1.0 + poisson));
        double lam = young * thickness * poisson / (1.0 - poisson * poisson);
        stvk_density(F, mu, lam, psi, P, A);
    } else {
        fbw_density(F, mu1, mu2, msh, psi, P, A);
    }
    if (Pout) for (int i = 0; i < 3; ++i) { Pout[2 * i] = P[i][0]; Pout[2 * i + 1] = P[i][1]; }
    if (Aout) for (int r = 0; r < 6; ++r) for (int c = 0; c < 6; ++c) Aout[6 * r + c] = A[r][c];
}

/* ------------------------------------------------------------------------------------------
 * 5. PSD projection (Sec. 5.1, projected Newton): clamp the negative eigenvalues of the
 *    6x6 density Hessian to zero. Eigen-decomposition by the cyclic Jacobi method
 *    (Golub & Van Loan, symmetric Schur rotations), run to convergence.
 * ------------------------------------------------------------------------------------------ */

static void jacobi_eigen(int n, double A[6][6], double V[6][6])
{
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) V[r][c] = (r == c) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int r = 0; r < n; ++r)
            for (int c = 0; c < n; ++c) {
                tot += A[r][c] * A[r][c];
                if (r != c) off += A[r][c] * A[r][c];
            }
        if (off <= 1e-32 * tot || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                if (A[p][q] == 0.0) continue;
                double tau = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                for (int k = 0; k < n; ++k) {          /* A <- A J */
                    double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {          /* A <- J^T A */
                    double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {          /* V <- V J */
                    double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - s * vkq;
                    V[k][q] = s * vkp + c * vkq;
                }
            }
        }
    }
}

/* Projects the symmetric 6x6 matrix Ain (row-major) onto the PSD cone in place. */
void or_project_psd6(double *Ain)
{
    double A[6][6], V[6][6];
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) A[r][c] = 0.5 * (Ain[6 * r + c] + Ain[6 * c + r]);
    jacobi_eigen(6, A, V);
    double lam[6];
    for (int r = 0; r < 6; ++r) lam[r] = A[r][r] > 0.0 ? A[r][r] : 0.0;
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) {
            double s = 0.0;
            for (int m = 0; m < 6; ++m) s += V[r][m] * lam[m] * V[c][m];
            Ain[6 * r + c] = s;
        }
}

/* ------------------------------------------------------------------------------------------
 * 6. Element energy, gradient and 27x27 Hessian (Sec. 4.1, 4.2; the element is a knot span).
 * ------------------------------------------------------------------------------------------ */

static int rule_sizes(const or_sheet *S, int *Nu, int *Nv)
{
    *Nu = or_check_knots(S->knots_u, S->n_u, NULL);
    *Nv = or_check_knots(S->knots_v, S->n_v, NULL);
    return (*Nu > 0 && *Nv > 0) ? OR_OK : OR_EINVAL;
}

/* Parametric-to-physical weight. The rule weights are in span units (a span has unit size)
 * and J = dX/d(u,v) is taken with respect to the same span-unit coordinates, so
 * int f dX = sum wbar f |det J| (Sec. 3.2: integrals over the rest domain). */
static double phys_weight(const or_sheet *S, double wbar, double detJ)
{
    (void)S;
    return wbar * fabs(detJ);
}

/* One membrane quadrature point: adds w*Psi, w*dPsi/dC and w*d2Psi/dC2 (projected if asked)
 * to element arrays E (1), g (27), H (27x27). */
static void membrane_point(const or_sheet *S, const double *x, const double *rec, int project,
                           double *E, double *g, double *H)
{
    int k = (int)rec[3], l = (int)rec[4];
    tp_basis B;
    eval_tp_basis(S, k, l, rec[0], rec[1], &B);
    double K[2][2], detJ, lap[5];
    rest_geometry(S, &B, K, &detJ, lap);
    double w = phys_weight(S, rec[2], detJ);
    /* grad_X N_alpha (Eq. "deformation gradient"): dN/dX_b = N_u du/dX_b + N_v dv/dX_b */
    double dN[9][2];
    for (int m = 0; m < 9; ++m)
        for (int b = 0; b < 2; ++b) dN[m][b] = B.Nu[m] * K[0][b] + B.Nv[m] * K[1][b];
    double F[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    for (int m = 0; m < 9; ++m)
        for (int i = 0; i < 3; ++i)
            for (int b = 0; b < 2; ++b) F[i][b] += x[3 * B.cp[m] + i] * dN[m][b];
    double psi, P[3][2], A[6][6];
    if (S->membrane == 0) {
        double mu = S->young * S->thickness / (2.0 * (1.0 + S->poisson));
        double lam = S->young * S->thickness * S->poisson / (1.0 - S->poisson * S->poisson);
        stvk_density(F, mu, lam, &psi, P, A);
    } else {
        fbw_density(F, S->mu_st1, S->mu_st2, S->mu_sh, &psi, P, A);
    }
    if (project) or_project_psd6(&A[0][0]);
    *E += w * psi;
    for (int m = 0; m < 9; ++m)
        for (int i = 0; i < 3; ++i)
            g[3 * m + i] += w * (P[i][0] * dN[m][0] + P[i][1] * dN[m][1]);
    for (int m = 0; m < 9; ++m)
        for (int i = 0; i < 3; ++i)
            for (int n = 0; n < 9; ++n)
                for (int j = 0; j < 3; ++j) {
                    double s = 0.0;
                    for (int ga = 0; ga < 2; ++ga)
                        for (int de = 0; de < 2; ++de)
                            s += dN[m][ga] * A[3 * ga + i][3 * de + j] * dN[n][de];
                    H[(3 * m + i) * 27 + 3 * n + j] += w * s;
                }
}

/* One bending evaluation (Eqs. "general bending energy", "mean curvature", "Laplacian in
 * parametric space"): Psi_bd = mu_bd/2 |Laplacian(phi)|^2 with Laplacian(phi) = sum L_a C^a. */
static void bending_point(const or_sheet *S, const double *x, const double *rec, double *E,
                          double *g, double *H)
{
    int k = (int)rec[3], l = (int)rec[4];
    tp_basis B;
    eval_tp_basis(S, k, l, rec[0], rec[1], &B);
    double K[2][2], detJ, lap[5];
    rest_geometry(S, &B, K, &detJ, lap);
    double w = phys_weight(S, rec[2], detJ);
    double L[9];
    for (int m = 0; m < 9; ++m)
        L[m] = lap[0] * B.Nuu[m] + lap[1] * B.Nvv[m] + lap[2] * B.Nu[m] + lap[3] * B.Nv[m]
               + lap[4] * B.Nuv[m];
    double dphi[3] = {0, 0, 0};
    for (int m = 0; m < 9; ++m)
        for (int i = 0; i < 3; ++i) dphi[i] += L[m] * x[3 * B.cp[m] + i];
    double mu = S->mu_bend;
    *E += w * 0.5 * mu * (dphi[0] * dphi[0] + dphi[1] * dphi[1] + dphi[2] * dphi[2]);
    for (int m = 0; m < 9; ++m)
        for (int i = 0; i < 3; ++i) g[3 * m + i] += w * mu * L[m] * dphi[i];
    for (int m = 0; m < 9; ++m)
        for (int n = 0; n < 9; ++n)
            for (int i = 0; i < 3; ++i) H[(3 * m + i) * 27 + 3 * n + i] += w * mu * L[m] * L[n];
}

/* Per-element elastic (membrane + bending) energy, gradient and Hessian for every knot span.
 * E_e[N_u*N_v], g_e[27*N_u*N_v], H_e[729*N_u*N_v] (row-major 27x27), element e = l*N_u + k.
 * project != 0 applies the PSD projection to every membrane point's density Hessian. */
int or_element_egh(const or_sheet *S, const double *x, int project, double *E_e, double *g_e,
                   double *H_e)
{
    int Nu, Nv;
    if (rule_sizes(S, &Nu, &Nv) != OR_OK) return OR_EINVAL;
    int ne = Nu * Nv;
    memset(E_e, 0, sizeof(double) * ne);
    memset(g_e, 0, sizeof(double) * 27 * ne);
    if (H_e) memset(H_e, 0, sizeof(double) * 729 * ne);
    double *Hscratch = H_e ? NULL : (double *)calloc(729, sizeof(double));
    int nm = or_membrane_rule_q(Nu, Nv, S->quadrature, NULL, 0);
    double *rm = (double *)malloc(sizeof(double) * 5 * nm);
    or_membrane_rule_q(Nu, Nv, S->quadrature, rm, nm);
    for (int q = 0; q < nm; ++q) {
        const double *rec = rm + 5 * q;
        int e = (int)rec[4] * Nu + (int)rec[3];
        membrane_point(S, x, rec, project, E_e + e, g_e + 27 * e, H_e ? H_e + 729 * e : Hscratch);
    }
    free(rm);
    int nb = or_bending_rule_q(Nu, Nv, S->quadrature, NULL, 0);
    double *rb = (double *)malloc(sizeof(double) * 5 * nb);
    or_bending_rule_q(Nu, Nv, S->quadrature, rb, nb);
    for (int q = 0; q < nb; ++q) {
        const double *rec = rb + 5 * q;
        int e = (int)rec[4] * Nu + (int)rec[3];
        bending_point(S, x, rec, E_e + e, g_e + 27 * e, H_e ? H_e + 729 * e : Hscratch);
    }
    free(rb);
    free(Hscratch);
    return OR_OK;
}

/* ------------------------------------------------------------------------------------------
 * 7. Lumped mass (Sec. 5.1, Eq. "lumped mass matrix"): row sums of the consistent mass
 *    M_ab = int R0 N_a N_b dX (Sec. 3.2). By the partition of unity the row sum is
 *    int R0 N_a dX, integrated here with 3x3 Gauss on every knot span (reading R-mass).
 * ------------------------------------------------------------------------------------------ */
int or_lumped_mass(const or_sheet *S, double *M)
{
    int Nu, Nv;
    if (rule_sizes(S, &Nu, &Nv) != OR_OK) return OR_EINVAL;
    int ncp = S->n_u * S->n_v;
    memset(M, 0, sizeof(double) * ncp);
    double off[3], w[3];
    gauss_1d(3, off, w);
    for (int l = 0; l < Nv; ++l)
        for (int k = 0; k < Nu; ++k)
            for (int b = 0; b < 3; ++b)
                for (int a = 0; a < 3; ++a) {
                    tp_basis B;
                    eval_tp_basis(S, k, l, k + 0.5 + off[a], l + 0.5 + off[b], &B);
                    double K[2][2], detJ, lap[5];
                    rest_geometry(S, &B, K, &detJ, lap);
                    double wp = phys_weight(S, w[a] * w[b], detJ);
                    for (int m = 0; m < 9; ++m) {
                        /* consistent-mass row of CP m at this point: sum over n of N_m N_n
                         * (CPs outside the span have N_n = 0 here) */
                        double row = 0.0;
                        for (int n = 0; n < 9; ++n) row += S->rho_area * B.N[m] * B.N[n];
                        M[B.cp[m]] += wp * row;
                    }
                }
    return OR_OK;
}

/* ------------------------------------------------------------------------------------------
 * 8. Incremental potential and its derivatives (Sec. 3.2, Eq. "incremental_potential";
 *    Sec. 5.1 lumped mass, gravity, Dirichlet conditions by elimination):
 *      E(x) = sum_a M_a |x_a - xhat_a|^2 / (2 dt^2) - sum_a M_a grav . x_a + E_elastic(x).
 *    inv_dt2 = 1/dt^2 (0 disables inertia); xhat may be NULL when inv_dt2 == 0.
 *    pinned[ncp] (nullable): pinned CPs get g = 0 and identity rows/columns in H.
 *    H (nullable) is in stencil form, 25 blocks of 3x3 per CP.
 * ------------------------------------------------------------------------------------------ */
int or_assemble(const or_sheet *S, const double *x, const double *xhat, double inv_dt2,
                const double *grav, const int *pinned, int project, double *E_out, double *g,
                double *H)
{
    int Nu, Nv;
    if (rule_sizes(S, &Nu, &Nv) != OR_OK) return OR_EINVAL;
    int nu = S->n_u, ncp = S->n_u * S->n_v, ne = Nu * Nv;
    double *Ee = (double *)malloc(sizeof(double) * ne);
    double *ge = (double *)malloc(sizeof(double) * 27 * ne);
    double *He = H ? (double *)malloc(sizeof(double) * 729 * ne) : NULL;
    or_element_egh(S, x, project, Ee, ge, He);
    double E = 0.0;
    memset(g, 0, sizeof(double) * 3 * ncp);
    if (H) memset(H, 0, sizeof(double) * 225 * ncp);
    for (int l = 0; l < Nv; ++l) {
        for (int k = 0; k < Nu; ++k) {
            int e = l * Nu + k;
            E += Ee[e];
            for (int m = 0; m < 9; ++m) {
                int am = m % 3, bm = m / 3;
                int A = (l + bm) * nu + (k + am);
                for (int i = 0; i < 3; ++i) g[3 * A + i] += ge[27 * e + 3 * m + i];
                if (!H) continue;
                for (int n = 0; n < 9; ++n) {
                    int an = n % 3, bn = n / 3;
                    int s = (bn - bm + 2) * 5 + (an - am + 2);
                    for (int i = 0; i < 3; ++i)
                        for (int j = 0; j < 3; ++j)
                            H[(A * 25 + s) * 9 + 3 * i + j] += He[729 * e + (3 * m + i) * 27 + 3 * n + j];
                }
            }
        }
    }
    double *M = (double *)malloc(sizeof(double) * ncp);
    or_lumped_mass(S, M);
    for (int a = 0; a < ncp; ++a) {
        for (int i = 0; i < 3; ++i) {
            if (inv_dt2 != 0.0) {
                double d = x[3 * a + i] - xhat[3 * a + i];
                E += 0.5 * M[a] * inv_dt2 * d * d;
                g[3 * a + i] += M[a] * inv_dt2 * d;
                if (H) H[(a * 25 + 12) * 9 + 4 * i] += M[a] * inv_dt2;
            }
            if (grav) {
                E -= M[a] * grav[i] * x[3 * a + i];
                g[3 * a + i] -= M[a] * grav[i];
            }
        }
    }
    if (pinned) {
        for (int a = 0; a < ncp; ++a) {
            if (!pinned[a]) continue;
            for (int i = 0; i < 3; ++i) g[3 * a + i] = 0.0;
            if (!H) continue;
            int ia = a % nu, ja = a / nu;
            for (int s = 0; s < 25; ++s) {
                int di = s % 5 - 2, dj = s / 5 - 2;
                int ib = ia + di, jb = ja + dj;
                for (int t = 0; t < 9; ++t) H[(a * 25 + s) * 9 + t] = 0.0;
                if (ib < 0 || ib >= nu || jb < 0 || jb >= S->n_v) continue;
                int b = jb * nu + ib;
                int sb = (-dj + 2) * 5 + (-di + 2);
                for (int t = 0; t < 9; ++t) H[(b * 25 + sb) * 9 + t] = 0.0;
            }
            for (int i = 0; i < 3; ++i) H[(a * 25 + 12) * 9 + 4 * i] = 1.0;
        }
    }
    *E_out = E;
    free(M); free(Ee); free(ge); free(He);
    return OR_OK;
}

/* Energy only (used by the line search). */
int or_energy(const or_sheet *S, const double *x, const double *xhat, double inv_dt2,
              const double *grav, double *E_out)
{
    int ncp = S->n_u * S->n_v;
    double *g = (double *)malloc(sizeof(double) * 3 * ncp);
    int st = or_assemble(S, x, xhat, inv_dt2, grav, NULL, 0, E_out, g, NULL);
    free(g);
    return st;
}

/* Surface point S(u,v) = sum N_{i,j}(u,v) C^{i,j} (Eq. "general B-spline patch"), u, v in
 * knot coordinates, evaluated with the literal half-open basis (the last knot is mapped to
 * the last span by evaluating just inside it). */
void or_surface_point(const or_sheet *S, const double *x, double u, double v, double *out)
{
    double umax = S->knots_u[S->n_u + 2], vmax = S->knots_v[S->n_v + 2];
    if (u >= umax) u = umax * (1.0 - 1e-15);
    if (v >= vmax) v = vmax * (1.0 - 1e-15);
    out[0] = out[1] = out[2] = 0.0;
    for (int j = 0; j < S->n_v; ++j) {
        double Nj = or_basis(S->knots_v, j, 2, v);
        if (Nj == 0.0) continue;
        for (int i = 0; i < S->n_u; ++i) {
            double Ni = or_basis(S->knots_u, i, 2, u);
            for (int c = 0; c < 3; ++c) out[c] += Ni * Nj * x[3 * (j * S->n_u + i) + c];
        }
    }
}

/* Rest-map quantities at a point of span (k,l) (span units), for tests:
 * out = [K00, K01, K10, K11, detJ, lap0..lap4] (see rest_geometry). */
void or_point_geometry(const or_sheet *S, int k, int l, double u, double v, double *out)
{
    tp_basis B;
    eval_tp_basis(S, k, l, u, v, &B);
    double K[2][2], detJ, lap[5];
    rest_geometry(S, &B, K, &detJ, lap);
    out[0] = K[0][0]; out[1] = K[0][1]; out[2] = K[1][0]; out[3] = K[1][1];
    out[4] = detJ;
    for (int m = 0; m < 5; ++m) out[5 + m] = lap[m];
}
