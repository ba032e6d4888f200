// host.cpp -- context creation, validation and the one-time precompute of the device tables:
// reduced quadrature lists (Sec. 4.1 and 4.2), lumped mass (Sec. 5.1), constant bending
// Hessian stencil (the bending Hessian of a flat rest shape is constant, so it is precomputed;
// Sec. 6.5 step "bending Hessian precomputation"), workspace layout and the C ABI entry points
// that are not solver calls.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "bsc_internal.h"

namespace bsc {

bsc_status fail(bsc_ctx *ctx, bsc_status st, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return st;
}

bsc_status hip_check(bsc_ctx *ctx, hipError_t e, const char *what) {
    if (e == hipSuccess) return BSC_OK;
    return fail(ctx, BSC_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

namespace {

enum SpanType { kFirst = 0, kInner = 1, kLast = 2 };

int span_type(int k, int N) { return k == 0 ? kFirst : (k == N - 1 ? kLast : kInner); }

// Quadratic B-spline pieces on a span of an open uniform knot vector, local t in [0,1]:
// values, first and second derivatives of the three functions supported on the span.
void pieces(int type, double t, double N[3], double D[3], double D2[3]) {
    const double s = 1.0 - t;
    if (type == kInner) {
        N[0] = 0.5 * s * s; N[1] = 0.5 * (-2.0 * t * t + 2.0 * t + 1.0); N[2] = 0.5 * t * t;
        D[0] = -s; D[1] = 1.0 - 2.0 * t; D[2] = t;
        D2[0] = 1.0; D2[1] = -2.0; D2[2] = 1.0;
    } else if (type == kFirst) {
        N[0] = s * s; N[1] = 2.0 * t - 1.5 * t * t; N[2] = 0.5 * t * t;
        D[0] = -2.0 * s; D[1] = 2.0 - 3.0 * t; D[2] = t;
        D2[0] = 2.0; D2[1] = -3.0; D2[2] = 1.0;
    } else {
        N[0] = 0.5 * s * s; N[1] = 2.0 * s - 1.5 * s * s; N[2] = t * t;
        D[0] = -s; D[1] = 1.0 - 3.0 * t; D[2] = 2.0 * t;
        D2[0] = 1.0; D2[1] = -3.0; D2[2] = 2.0;
    }
}

// Greville abscissa of CP i in span units: 0, 1/2, 3/2, ..., N - 1/2, N.
double greville(int i, int n) {
    if (i == 0) return 0.0;
    if (i == n - 1) return double(n - 2);
    return i - 0.5;
}

// Rest-map geometry at span coordinates (tu, tv) of span (k, l), span units. J = dX/d(u,v)
// and the second derivatives of X come from the 9 rest CPs of the span; K = J^{-1} (Sec. 4.1,
// inverse function theorem). The Laplacian over X in parametric form (Sec. 4.2) is
//   Lap f = G_uu f_uu + G_vv f_vv + 2 G_uv f_uv + (Lap u) f_u + (Lap v) f_v,
// G_mn = grad xi_m . grad xi_n (rows of K). Lap xi follows from Lap X_c = 0 for the two
// coordinate functions: J Lap(xi) = -(G_uu X_uu + G_vv X_vv + 2 G_uv X_uv).
struct RestGeo { double K[2][2], det, cuu, cvv, cuv, lu, lv; };

RestGeo rest_geometry(const double *rest_xy, int n_u, int Nu, int Nv, int k, int l, double tu, double tv) {
    double Nu3[3], Du[3], D2u[3], Nv3[3], Dv[3], D2v[3];
    pieces(span_type(k, Nu), tu, Nu3, Du, D2u);
    pieces(span_type(l, Nv), tv, Nv3, Dv, D2v);
    double J[2][2] = {{0.0, 0.0}, {0.0, 0.0}}, Xuu[2] = {0.0, 0.0}, Xvv[2] = {0.0, 0.0}, Xuv[2] = {0.0, 0.0};
    for (int b = 0; b < 3; ++b)
        for (int a = 0; a < 3; ++a) {
            const double *X = rest_xy + 2 * (size_t(l + b) * n_u + (k + a));
            for (int c = 0; c < 2; ++c) {
                J[c][0] += X[c] * Du[a] * Nv3[b];
                J[c][1] += X[c] * Nu3[a] * Dv[b];
                Xuu[c] += X[c] * D2u[a] * Nv3[b];
                Xvv[c] += X[c] * Nu3[a] * D2v[b];
                Xuv[c] += X[c] * Du[a] * Dv[b];
            }
        }
    RestGeo g;
    g.det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    g.K[0][0] = J[1][1] / g.det; g.K[0][1] = -J[0][1] / g.det;
    g.K[1][0] = -J[1][0] / g.det; g.K[1][1] = J[0][0] / g.det;
    const double Guu = g.K[0][0] * g.K[0][0] + g.K[0][1] * g.K[0][1];
    const double Gvv = g.K[1][0] * g.K[1][0] + g.K[1][1] * g.K[1][1];
    const double Guv = g.K[0][0] * g.K[1][0] + g.K[0][1] * g.K[1][1];
    g.cuu = Guu; g.cvv = Gvv; g.cuv = 2.0 * Guv;
    double h[2];
    for (int c = 0; c < 2; ++c) h[c] = Guu * Xuu[c] + Gvv * Xvv[c] + 2.0 * Guv * Xuv[c];
    g.lu = -(g.K[0][0] * h[0] + g.K[0][1] * h[1]);
    g.lv = -(g.K[1][0] * h[0] + g.K[1][1] * h[1]);
    return g;
}

struct Pt { double u, v, w; int k, l; };

const double kG2 = 0.28867513459481288225;   // 1 / (2 sqrt 3)
const double kG3 = 0.38729833462074168852;   // sqrt(3/5) / 2

// Membrane rule (Sec. 4.1): 3x3 Gauss on corner spans, 3x2 / 2x3 on side spans, and in the
// interior region alternating 1x2 / 2x1 Gauss on dual-grid cells centred at the knots,
// clipped to the region (two points on the knot line for edge half cells, one at the knot
// for corner quarter cells). Weights: Gauss weights times the clipped cell area.
//
// Comparison rules (Sec. 6.5, selected by bsc_material.quadrature): BSC_QUAD_GAUSS2 puts 2x2
// Gauss on every interior span instead of the dual-grid cells, BSC_QUAD_INTERIOR1 one point at
// the centre of every interior span, BSC_QUAD_CORNER2 2x2 instead of 3x3 Gauss on the corner
// spans.
std::vector<Pt> membrane_points(int Nu, int Nv, int quad) {
    std::vector<Pt> out;
    const double o1[1] = {0.0}, w1[1] = {1.0};
    const double o2[2] = {-kG2, kG2}, w2[2] = {0.5, 0.5};
    const double o3[3] = {-kG3, 0.0, kG3}, w3[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
    auto order = [&](int npt, const double **o, const double **w) {
        *o = npt == 1 ? o1 : (npt == 2 ? o2 : o3);
        *w = npt == 1 ? w1 : (npt == 2 ? w2 : w3);
    };
    for (int l = 0; l < Nv; ++l) {
        for (int k = 0; k < Nu; ++k) {
            const bool eu = (k == 0 || k == Nu - 1), ev = (l == 0 || l == Nv - 1);
            int nu, nv;
            if (eu && ev) nu = nv = (quad == BSC_QUAD_CORNER2) ? 2 : 3;
            else if (eu || ev) { nu = eu ? 3 : 2; nv = ev ? 3 : 2; }
            else if (quad == BSC_QUAD_GAUSS2) nu = nv = 2;
            else if (quad == BSC_QUAD_INTERIOR1) nu = nv = 1;
            else continue;
            const double *ou, *wu, *ov, *wv;
            order(nu, &ou, &wu);
            order(nv, &ov, &wv);
            for (int b = 0; b < nv; ++b)
                for (int a = 0; a < nu; ++a) out.push_back({k + 0.5 + ou[a], l + 0.5 + ov[b], wu[a] * wv[b], k, l});
        }
    }
    if (quad == BSC_QUAD_GAUSS2 || quad == BSC_QUAD_INTERIOR1) return out;
    for (int b = 1; b < Nv; ++b) {
        for (int a = 1; a < Nu; ++a) {
            const bool hu = (a == 1 || a == Nu - 1), hv = (b == 1 || b == Nv - 1);
            double pu[2], pv[2], w;
            int np = 2;
            if (hu && hv) { np = 1; w = 0.25; pu[0] = a; pv[0] = b; }
            else if (hu) { w = 0.25; pu[0] = pu[1] = a; pv[0] = b - kG2; pv[1] = b + kG2; }
            else if (hv) { w = 0.25; pv[0] = pv[1] = b; pu[0] = a - kG2; pu[1] = a + kG2; }
            else if (((a + b) & 1) == 0) { w = 0.5; pu[0] = pu[1] = a; pv[0] = b - kG2; pv[1] = b + kG2; }
            else { w = 0.5; pv[0] = pv[1] = b; pu[0] = a - kG2; pu[1] = a + kG2; }
            for (int q = 0; q < np; ++q) {
                int k = std::min(int(std::floor(pu[q])), Nu - 1);
                int l = std::min(int(std::floor(pv[q])), Nv - 1);
                out.push_back({pu[q], pv[q], w, k, l});
            }
        }
    }
    return out;
}

// Bending rule (Sec. 4.2): one point per boundary span centre, one per interior knot weighted
// by its clipped dual cell; each knot point is evaluated in its four adjacent spans with a
// quarter of the weight (mean of the one-sided values).
// With BSC_QUAD_GAUSS2 the interior spans take 2x2 Gauss points instead of the knot points.
std::vector<Pt> bending_points(int Nu, int Nv, int quad) {
    std::vector<Pt> out;
    for (int l = 0; l < Nv; ++l)
        for (int k = 0; k < Nu; ++k)
            if (k == 0 || k == Nu - 1 || l == 0 || l == Nv - 1) out.push_back({k + 0.5, l + 0.5, 1.0, k, l});
    if (quad == BSC_QUAD_GAUSS2) {
        for (int l = 1; l < Nv - 1; ++l)
            for (int k = 1; k < Nu - 1; ++k)
                for (int b = 0; b < 2; ++b)
                    for (int a = 0; a < 2; ++a)
                        out.push_back({k + 0.5 + (a ? kG2 : -kG2), l + 0.5 + (b ? kG2 : -kG2), 0.25, k, l});
        return out;
    }
    for (int b = 1; b < Nv; ++b) {
        for (int a = 1; a < Nu; ++a) {
            const double cu = (a == 1 || a == Nu - 1) ? 0.5 : 1.0;
            const double cv = (b == 1 || b == Nv - 1) ? 0.5 : 1.0;
            const double w = 0.25 * cu * cv;
            for (int dl = -1; dl <= 0; ++dl)
                for (int dk = -1; dk <= 0; ++dk) out.push_back({double(a), double(b), w, a + dk, b + dl});
        }
    }
    return out;
}

// Sorts points by element and fills the SoA tables plus per-element offsets.
void fill_tables(const std::vector<Pt> &pts, int Nu, int n_elem, double wscale, std::vector<int32_t> &elem,
                 std::vector<int32_t> &off, std::vector<double> &tu, std::vector<double> &tv,
                 std::vector<double> &w) {
    off.assign(n_elem + 1, 0);
    for (const Pt &p : pts) off[p.l * Nu + p.k + 1]++;
    for (int e = 0; e < n_elem; ++e) off[e + 1] += off[e];
    std::vector<int32_t> cur(off.begin(), off.end() - 1);
    const size_t n = pts.size();
    elem.assign(n, 0); tu.assign(n, 0.0); tv.assign(n, 0.0); w.assign(n, 0.0);
    for (const Pt &p : pts) {
        const int e = p.l * Nu + p.k;
        const int d = cur[e]++;
        elem[d] = e; tu[d] = p.u - p.k; tv[d] = p.v - p.l; w[d] = p.w * wscale;
    }
}

bool knots_ok(const double *kn, int n, double *spacing) {
    const int nk = n + 3;
    if (n < 5) return false;
    if (kn[0] != 0.0 || kn[1] != 0.0 || kn[2] != 0.0) return false;
    if (kn[nk - 1] != kn[nk - 2] || kn[nk - 2] != kn[nk - 3]) return false;
    const double h = kn[3] - kn[2];
    if (!(h > 0.0) || h != std::floor(h)) return false;
    for (int s = 2; s < nk - 3; ++s)
        if (kn[s + 1] - kn[s] != h) return false;
    *spacing = h;
    return true;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

DevSheet dev_sheet(const bsc_ctx *ctx) { return ctx->dev; }

void host_pieces(int type, double t, double N[3], double D[3], double D2[3]) { pieces(type, t, N, D, D2); }

size_t layout_workspace(const bsc_ctx *c, DevBufs *b, char *base) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    const size_t ncp = c->n_cp, nmp = c->n_mp, nbe = c->n_be, ne = c->n_elem;
    const int max_items = int(std::max(std::max(nmp, nbe), std::max(ncp, ne)));
    // at least 256: the fixed-grid reductions (dot products, max-norm) launch 256 blocks
    // also >= the SpMV grid (64 rows per block) and the CG grid (kCgTileU x kCgTileV tiles)
    const int cg_tiles = ((c->n_u + kCgTileU - 1) / kCgTileU) * ((c->n_v + kCgTileV - 1) / kCgTileV);
    int asm_tiles = 0;                 // the assembly grid (energy partials), smallest tile height
    for (int kind = 0; kind < 3; ++kind)
        asm_tiles = std::max(asm_tiles, ((c->n_u + kAsmTileU - 1) / kAsmTileU) *
                                            asm_tile_rows(c->n_v, std::max(1, c->dev.asm_ty[kind])));
    const int max_blocks = std::max(std::max(256, std::max(cg_tiles, asm_tiles) + 1),
                                    std::max((max_items + kBlock - 1) / kBlock + 1, int(ncp / 64) + 2));
    DevBufs t{};
    t.max_blocks = max_blocks;
    t.mp_elem = (int32_t *)take(4 * nmp);
    t.mp_off = (int32_t *)take(4 * (ne + 1));
    t.mp_tu = (double *)take(8 * nmp);
    t.mp_tv = (double *)take(8 * nmp);
    t.mp_w = (double *)take(8 * nmp);
    t.be_elem = (int32_t *)take(4 * nbe);
    t.be_off = (int32_t *)take(4 * (ne + 1));
    t.be_tu = (double *)take(8 * nbe);
    t.be_tv = (double *)take(8 * nbe);
    t.be_w = (double *)take(8 * nbe);
    t.mass = (double *)take(8 * ncp);
    t.hbend = (double *)take(8 * kSlots * ncp);
    t.mp_K = (double *)take(8 * c->mp_K.size());
    t.be_L = (double *)take(8 * c->be_L.size());
    t.rest = (double *)take(8 * c->rest.size());
    t.pinmask = (int32_t *)take(4 * ncp);
    t.asm_tab = (int32_t *)take(4 * c->asm_tab.size());
    t.pin_idx = (int32_t *)take(4 * ncp);
    t.ptA = take(8 * 21 * nmp);
    t.ptP = take(8 * 6 * nmp);
    t.ptE = (double *)take(8 * nmp);
    t.ptP64 = (double *)take(8 * 6 * nmp);
    t.beD = (double *)take(8 * 3 * nbe);
    t.beE = (double *)take(8 * nbe);
    t.partials = (double *)take(8 * 8 * size_t(max_blocks));
    t.bsr_rowptr = (int32_t *)take(4 * (ncp + 1));
    t.scalars = (double *)take(8 * kScalars);
    t.iscalars = (int32_t *)take(4 * 64);          // directly after the scalars (kScalars * 8 is a multiple of 256)
    double **vecs[] = {&t.g, &t.xn, &t.xhat, &t.dir, &t.r, &t.p0, &t.p1, &t.q, &t.tmp, &t.phat, &t.r2, &t.q2, &t.p2, &t.gpre};
    for (double **v : vecs) *v = (double *)take(8 * 3 * ncp);
    t.pinv = (double *)take(8 * 6 * ncp);
    t.mg_x0 = t.r2;                                // unused by the multigrid solver otherwise
    t.mg_t0 = t.q2;
    t.mg_levels = mg_level_count(c->n_u, c->n_v);
    {
        int nuf = c->n_u, nvf = c->n_v;
        for (int l = 0; l < t.mg_levels; ++l) {
            MgLevel &L = t.mg[l];
            L.n_u = (nuf - 2) / 2 + 2;
            L.n_v = (nvf - 2) / 2 + 2;
            const size_t nl = size_t(L.n_u) * L.n_v;
            L.H = take(8 * size_t(kHessEntries) * nl);
            L.pinv = take(8 * 6 * nl);
            L.Hmid = take(8 * size_t(kHessEntries) * size_t(L.n_u) * nvf);
            L.r = (double *)take(24 * nl);
            L.xa = (double *)take(24 * nl);
            L.xb = (double *)take(24 * nl);
            L.t = (double *)take(24 * nl);
            nuf = L.n_u;
            nvf = L.n_v;
        }
    }
    t.hess = take(8 * size_t(kHessEntries) * ncp);
    t.net_w = (float *)take(4 * BSC_NET_PARAMS);
    t.net_w_fwd = (float *)take(4 * BSC_NET_PARAMS);
    t.net_wr = (float *)take(4 * BSC_NET_PARAMS);
    t.net_in = (float *)take(4 * 3 * ncp);
    t.net_out = (float *)take(4 * 3 * ncp);
    t.net_act0 = (float *)take(4 * 32 * ncp);
    t.net_act1 = (float *)take(4 * 32 * ncp);
    t.net_scale = (float *)take(4 * 1024);
    t.net_lpart = (double *)take(8 * 1024 * 64 * 3);
    if (b) *b = t;
    return off;
}

}  // namespace bsc

using namespace bsc;

extern "C" {

const char *bsc_status_string(bsc_status s) {
    switch (s) {
        case BSC_OK: return "ok";
        case BSC_E_INVAL: return "invalid argument";
        case BSC_E_KNOTS: return "invalid knot vector";
        case BSC_E_NOMEM: return "out of memory";
        case BSC_E_HIP: return "HIP runtime error";
        case BSC_E_NOT_CONVERGED: return "Newton did not converge";
        case BSC_E_LINESEARCH: return "line search failed";
        case BSC_E_NONFINITE: return "non-finite value";
        case BSC_E_PCG_BREAKDOWN: return "PCG breakdown";
        case BSC_E_STATE: return "invalid call order";
    }
    return "unknown status";
}

const char *bsc_last_error(const bsc_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

void bsc_destroy(bsc_ctx *ctx) { delete ctx; }

bsc_status bsc_create(bsc_ctx **out, int32_t n_u, int32_t n_v, const double *knots_u, const double *knots_v,
                      const double *rest_xy, const bsc_material *mat, void *hip_stream) {
    if (!out) return BSC_E_INVAL;
    *out = nullptr;
    if (!knots_u || !knots_v || !rest_xy || !mat) return BSC_E_INVAL;
    if (n_u < 5 || n_v < 5 || n_u > 32768 || n_v > 32768 || int64_t(n_u) * n_v > (int64_t(1) << 24))
        return BSC_E_INVAL;
    double hu = 0, hv = 0;
    if (!knots_ok(knots_u, n_u, &hu) || !knots_ok(knots_v, n_v, &hv)) return BSC_E_KNOTS;
    if (mat->membrane == BSC_MEMBRANE_STVK) {
        if (!(mat->young >= 0.0) || !(mat->thickness > 0.0) || !(mat->poisson > -1.0 && mat->poisson <= 0.5))
            return BSC_E_INVAL;
    } else if (mat->membrane == BSC_MEMBRANE_FBW) {
        if (!(mat->mu_st1 >= 0.0 && mat->mu_st2 >= 0.0 && mat->mu_sh >= 0.0)) return BSC_E_INVAL;
    } else {
        return BSC_E_INVAL;
    }
    if (!(mat->mu_bend >= 0.0) || !(mat->rho_area > 0.0)) return BSC_E_INVAL;
    if (mat->quadrature < BSC_QUAD_REDUCED || mat->quadrature > BSC_QUAD_CORNER2) return BSC_E_INVAL;
    for (int64_t a = 0; a < 2 * int64_t(n_u) * n_v; ++a)
        if (!std::isfinite(rest_xy[a])) return BSC_E_INVAL;

    bsc_ctx *c = new (std::nothrow) bsc_ctx;
    if (!c) return BSC_E_NOMEM;
    c->n_u = n_u; c->n_v = n_v; c->Nu = n_u - 2; c->Nv = n_v - 2;
    c->n_cp = n_u * n_v; c->n_elem = c->Nu * c->Nv;
    c->mat = *mat;
    c->stream = (hipStream_t)hip_stream;
    if (const char *gr = std::getenv("BSC_GRAPHS")) c->use_graphs = gr[0] == '1';
    if (hipGetDevice(&c->device) != hipSuccess) c->device = 0;

    // The rest map X(u,v) = sum N_a X^a is affine iff the CPs are an affine image of the
    // Greville abscissae (linear precision); read A and b off three corners and test. An affine
    // rest keeps K and the Laplacian coefficients as sheet constants; any other rest map gets
    // per-point tables (the general path).
    auto R = [&](int i, int j, int comp) { return rest_xy[2 * (int64_t(j) * n_u + i) + comp]; };
    const int Nu = c->Nu, Nv = c->Nv;
    double A[2][2], b[2];
    for (int comp = 0; comp < 2; ++comp) {
        b[comp] = R(0, 0, comp);
        A[comp][0] = (R(n_u - 1, 0, comp) - b[comp]) / Nu;
        A[comp][1] = (R(0, n_v - 1, comp) - b[comp]) / Nv;
    }
    double ext = std::fabs(A[0][0]) * Nu + std::fabs(A[0][1]) * Nv + std::fabs(A[1][0]) * Nu + std::fabs(A[1][1]) * Nv;
    bool affine = ext > 0.0;
    for (int j = 0; j < n_v && affine; ++j)
        for (int i = 0; i < n_u && affine; ++i)
            for (int comp = 0; comp < 2; ++comp) {
                double want = A[comp][0] * greville(i, n_u) + A[comp][1] * greville(j, n_v) + b[comp];
                if (std::fabs(R(i, j, comp) - want) > 1e-12 * ext) affine = false;
            }
    const bool curved = !affine;
    auto reject = [&](const char *why) {   // the context is not returned, so no error text
        (void)why;
        delete c;
        return BSC_E_INVAL;
    };
    double det = 1.0, K[2][2] = {{1.0, 0.0}, {0.0, 1.0}};
    if (affine) {
        det = A[0][0] * A[1][1] - A[0][1] * A[1][0];
        if (!(det > 0.0)) return reject("rest map is not orientation preserving");
        K[0][0] = A[1][1] / det; K[0][1] = -A[0][1] / det;
        K[1][0] = -A[1][0] / det; K[1][1] = A[0][0] / det;
    }

    // quadrature tables (weights times |det J|: the constant here, per point below)
    fill_tables(membrane_points(Nu, Nv, mat->quadrature), Nu, c->n_elem, det, c->mp_elem, c->mp_off, c->mp_tu, c->mp_tv, c->mp_w);
    fill_tables(bending_points(Nu, Nv, mat->quadrature), Nu, c->n_elem, det, c->be_elem, c->be_off, c->be_tu, c->be_tv, c->be_w);
    c->n_mp = int(c->mp_elem.size());
    c->n_be = int(c->be_elem.size());

    // Laplacian in parametric space for an affine rest: only the second-derivative terms remain.
    const double c_uu = K[0][0] * K[0][0] + K[0][1] * K[0][1];
    const double c_vv = K[1][0] * K[1][0] + K[1][1] * K[1][1];
    const double c_uv = 2.0 * (K[0][0] * K[1][0] + K[0][1] * K[1][1]);

    if (curved) {
        // per-point geometry; det J > 0 is required at every point (an orientation-preserving,
        // locally invertible rest map)
        const size_t nmp = c->n_mp, nbe = c->n_be, ncp = c->n_cp;
        c->mp_K.assign(4 * nmp, 0.0);
        c->be_L.assign(5 * nbe, 0.0);
        c->rest.assign(2 * ncp, 0.0);
        for (size_t a = 0; a < ncp; ++a) { c->rest[a] = rest_xy[2 * a]; c->rest[ncp + a] = rest_xy[2 * a + 1]; }
        for (size_t q = 0; q < nmp; ++q) {
            const int e = c->mp_elem[q];
            const RestGeo g = rest_geometry(rest_xy, n_u, Nu, Nv, e % Nu, e / Nu, c->mp_tu[q], c->mp_tv[q]);
            if (!(g.det > 0.0)) return reject("det J <= 0 at a membrane quadrature point");
            c->mp_w[q] *= g.det;
            c->mp_K[q] = g.K[0][0]; c->mp_K[nmp + q] = g.K[0][1];
            c->mp_K[2 * nmp + q] = g.K[1][0]; c->mp_K[3 * nmp + q] = g.K[1][1];
        }
        for (size_t q = 0; q < nbe; ++q) {
            const int e = c->be_elem[q];
            const RestGeo g = rest_geometry(rest_xy, n_u, Nu, Nv, e % Nu, e / Nu, c->be_tu[q], c->be_tv[q]);
            if (!(g.det > 0.0)) return reject("det J <= 0 at a bending evaluation point");
            c->be_w[q] *= g.det;
            c->be_L[q] = g.cuu; c->be_L[nbe + q] = g.cvv; c->be_L[2 * nbe + q] = g.cuv;
            c->be_L[3 * nbe + q] = g.lu; c->be_L[4 * nbe + q] = g.lv;
        }
    }

    // Lumped mass: row sums of the consistent mass = int rho N_a dX (partition of unity), 3x3
    // Gauss per span. For an affine rest it factorises as rho |det A| (int N_i du)(int N_j dv).
    const double o3[3] = {-kG3, 0.0, kG3}, w3[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
    c->mass.assign(c->n_cp, 0.0);
    if (affine) {
        auto integrals = [&](int n, int N) {
            std::vector<double> m(n, 0.0);
            for (int k = 0; k < N; ++k) {
                double Nv3[3], D[3], D2[3];
                for (int g = 0; g < 3; ++g) {
                    pieces(span_type(k, N), 0.5 + o3[g], Nv3, D, D2);
                    for (int a = 0; a < 3; ++a) m[k + a] += w3[g] * Nv3[a];
                }
            }
            return m;
        };
        std::vector<double> mu1 = integrals(n_u, Nu), mv1 = integrals(n_v, Nv);
        for (int j = 0; j < n_v; ++j)
            for (int i = 0; i < n_u; ++i) c->mass[j * n_u + i] = mat->rho_area * det * mu1[i] * mv1[j];
    } else {
        for (int l = 0; l < Nv; ++l)
            for (int k = 0; k < Nu; ++k)
                for (int gb = 0; gb < 3; ++gb)
                    for (int ga = 0; ga < 3; ++ga) {
                        const double tu = 0.5 + o3[ga], tv = 0.5 + o3[gb];
                        const RestGeo g = rest_geometry(rest_xy, n_u, Nu, Nv, k, l, tu, tv);
                        if (!(g.det > 0.0)) return reject("det J <= 0 at a mass quadrature point");
                        double Nu3[3], Nv3[3], D[3], D2[3];
                        pieces(span_type(k, Nu), tu, Nu3, D, D2);
                        pieces(span_type(l, Nv), tv, Nv3, D, D2);
                        const double wq = mat->rho_area * w3[ga] * w3[gb] * g.det;
                        for (int bb = 0; bb < 3; ++bb)
                            for (int aa = 0; aa < 3; ++aa) c->mass[(l + bb) * n_u + (k + aa)] += wq * Nu3[aa] * Nv3[bb];
                    }
    }

    // Constant bending Hessian: scalar stencil h[s][a] = sum over evaluations of
    // w mu L_a L_b for the upper-stencil slot s linking CP a to CP b (the 3x3 block is h I).
    c->hbend.assign(size_t(kSlots) * c->n_cp, 0.0);
    for (int q = 0; q < c->n_be; ++q) {
        const int e = c->be_elem[q], k = e % Nu, l = e / Nu;
        double Nu3[3], Du[3], D2u[3], Nv3[3], Dv[3], D2v[3];
        pieces(span_type(k, Nu), c->be_tu[q], Nu3, Du, D2u);
        pieces(span_type(l, Nv), c->be_tv[q], Nv3, Dv, D2v);
        double cu = c_uu, cv = c_vv, cuv = c_uv, lu = 0.0, lv = 0.0;
        if (curved) {
            const size_t nbe = c->n_be;
            cu = c->be_L[q]; cv = c->be_L[nbe + q]; cuv = c->be_L[2 * nbe + q];
            lu = c->be_L[3 * nbe + q]; lv = c->be_L[4 * nbe + q];
        }
        double L[9];
        for (int bb = 0; bb < 3; ++bb)
            for (int aa = 0; aa < 3; ++aa)
                L[3 * bb + aa] = cu * D2u[aa] * Nv3[bb] + cv * Nu3[aa] * D2v[bb] + cuv * Du[aa] * Dv[bb] +
                                 lu * Du[aa] * Nv3[bb] + lv * Nu3[aa] * Dv[bb];
        const double wm = c->be_w[q] * mat->mu_bend;
        for (int m = 0; m < 9; ++m)
            for (int n = 0; n < 9; ++n) {
                const int di = n % 3 - m % 3, dj = n / 3 - m / 3;
                const int s = upper_slot(di, dj);
                if (s < 0) continue;
                const int a = (l + m / 3) * n_u + (k + m % 3);
                c->hbend[size_t(s) * c->n_cp + a] += wm * L[m] * L[n];
            }
    }

    DevSheet &S = c->dev;
    S.n_u = n_u; S.n_v = n_v; S.Nu = Nu; S.Nv = Nv; S.n_cp = c->n_cp; S.n_elem = c->n_elem;
    S.n_mp = c->n_mp; S.n_be = c->n_be;
    S.A00 = A[0][0]; S.A01 = A[0][1]; S.A10 = A[1][0]; S.A11 = A[1][1]; S.b0 = b[0]; S.b1 = b[1];
    S.K00 = K[0][0]; S.K01 = K[0][1]; S.K10 = K[1][0]; S.K11 = K[1][1];
    S.c_uu = c_uu; S.c_vv = c_vv; S.c_uv = c_uv;
    S.curved = curved ? 1 : 0;
    S.membrane = mat->membrane;
    S.mu = mat->young * mat->thickness / (2.0 * (1.0 + mat->poisson));
    S.lam = mat->young * mat->thickness * mat->poisson / (1.0 - mat->poisson * mat->poisson);
    S.mu1 = mat->mu_st1; S.mu2 = mat->mu_st2; S.msh = mat->mu_sh;
    S.mu_bend = mat->mu_bend;

    // Tiled assembly: for each precision combination the tallest interior tile height (16 x ty
    // CPs, ty in 8, 4, 2, 1; edge rows min(2, ty)) whose staged points fit kAsmLdsMax bytes of
    // LDS in every tile.
    for (int kind = 0; kind < 3; ++kind) {
        S.asm_ty[kind] = 0;
        for (int ty = 8; ty >= 1 && S.asm_ty[kind] == 0; ty /= 2) {
            int maxp = 0;
            for (int tr = 0; tr < asm_tile_rows(n_v, ty); ++tr)
                for (int tx0 = 0; tx0 < n_u; tx0 += kAsmTileU) {
                    int ty0 = 0, h = 0;
                    asm_tile_row(n_v, ty, tr, ty0, h);
                    const int k0 = std::max(0, tx0 - 2), k1 = std::min(Nu - 1, tx0 + kAsmTileU - 1);
                    const int l0 = std::max(0, ty0 - 2), l1 = std::min(Nv - 1, ty0 + h - 1);
                    int np = 0;
                    for (int l = l0; l <= l1; ++l) np += c->mp_off[l * Nu + k1 + 1] - c->mp_off[l * Nu + k0];
                    maxp = std::max(maxp, np);
                }
            if (asm_lds_layout(kAsmTileU, ty, maxp, kind, curved).total <= kAsmLdsMax) {
                S.asm_ty[kind] = ty;
                S.asm_maxp[kind] = maxp;
            }
        }
        if (S.asm_ty[kind] == 0) { delete c; return BSC_E_INVAL; }
    }
    // the tile tables, one per distinct (tile height, point bound)
    c->asm_tab.clear();
    for (int kind = 0; kind < 3; ++kind) {
        const int ty = S.asm_ty[kind], maxp = S.asm_maxp[kind];
        S.asm_stride[kind] = asm_tab_stride(ty, maxp);
        int same = -1;
        for (int k2 = 0; k2 < kind; ++k2)
            if (S.asm_ty[k2] == ty && S.asm_maxp[k2] == maxp) same = k2;
        if (same >= 0) { c->asm_tab_off[kind] = c->asm_tab_off[same]; continue; }
        if (maxp >= (1 << 14)) { delete c; return BSC_E_INVAL; }
        const int ntx = (n_u + kAsmTileU - 1) / kAsmTileU, nt = ntx * asm_tile_rows(n_v, ty), stride = S.asm_stride[kind];
        c->asm_tab_off[kind] = c->asm_tab.size();
        c->asm_tab.resize(c->asm_tab.size() + size_t(nt) * stride, 0);
        int32_t *base = c->asm_tab.data() + c->asm_tab_off[kind];
        for (int tile = 0; tile < nt; ++tile) {
            const int tx0 = (tile % ntx) * kAsmTileU;
            int ty0 = 0, h = 0;
            asm_tile_row(n_v, ty, tile / ntx, ty0, h);
            const int k0 = std::max(0, tx0 - 2), k1 = std::min(Nu - 1, tx0 + kAsmTileU - 1);
            const int l0 = std::max(0, ty0 - 2), l1 = std::min(Nv - 1, ty0 + h - 1);
            const int nk = k1 - k0 + 1, ne = nk * (l1 - l0 + 1);
            int32_t *T = base + size_t(tile) * stride;
            int n0 = 0, np = 0;
            for (int el = 0; el < ne; ++el) {
                const int e = (l0 + el / nk) * Nu + k0 + el % nk, cnt = c->mp_off[e + 1] - c->mp_off[e];
                if (cnt > 15) { delete c; return BSC_E_INVAL; }
                n0 += cnt > 0;
                np += cnt;
            }
            int32_t *rq = T + 1, *re = T + 1 + maxp, *info = T + 1 + 2 * maxp;
            T[0] = np;
            int i0 = 0, i1 = n0;
            for (int el = 0; el < ne; ++el) {
                const int e = (l0 + el / nk) * Nu + k0 + el % nk, q0 = c->mp_off[e], cnt = c->mp_off[e + 1] - q0;
                info[el] = cnt | (i0 << 4) | (i1 << 18);
                for (int s = 0; s < cnt; ++s) {
                    const int r = s == 0 ? i0 : i1 + s - 1;
                    rq[r] = q0 + s;
                    re[r] = el;
                }
                if (cnt > 0) { ++i0; i1 += cnt - 1; }
            }
        }
    }
    c->hu = hu;
    c->hv = hv;
    *out = c;
    return BSC_OK;
}

bsc_status bsc_sizes(const bsc_ctx *c, int32_t *n_cp, int32_t *n_elem, int32_t *n_mp, int32_t *n_be) {
    if (!c) return BSC_E_INVAL;
    if (n_cp) *n_cp = c->n_cp;
    if (n_elem) *n_elem = c->n_elem;
    if (n_mp) *n_mp = c->n_mp;
    if (n_be) *n_be = c->n_be;
    return BSC_OK;
}

bsc_status bsc_workspace_size(const bsc_ctx *c, size_t *bytes) {
    if (!c || !bytes) return BSC_E_INVAL;
    *bytes = layout_workspace(c, nullptr, nullptr);
    return BSC_OK;
}

bsc_status bsc_bind_workspace(bsc_ctx *c, void *d_ws, size_t bytes) {
    if (!c || !d_ws) return BSC_E_INVAL;
    if ((reinterpret_cast<uintptr_t>(d_ws) & 255) != 0) return fail(c, BSC_E_INVAL, "workspace must be 256-byte aligned");
    const size_t need = layout_workspace(c, nullptr, nullptr);
    if (bytes < need) return fail(c, BSC_E_NOMEM, "workspace too small");
    c->ws = (char *)d_ws;
    c->ws_bytes = bytes;
    layout_workspace(c, &c->buf, c->ws);
    DevBufs &B = c->buf;
    struct Up { void *dst; const void *src; size_t n; } ups[] = {
        {B.mp_elem, c->mp_elem.data(), 4 * c->mp_elem.size()}, {B.mp_off, c->mp_off.data(), 4 * c->mp_off.size()},
        {B.mp_tu, c->mp_tu.data(), 8 * c->mp_tu.size()}, {B.mp_tv, c->mp_tv.data(), 8 * c->mp_tv.size()},
        {B.mp_w, c->mp_w.data(), 8 * c->mp_w.size()},
        {B.be_elem, c->be_elem.data(), 4 * c->be_elem.size()}, {B.be_off, c->be_off.data(), 4 * c->be_off.size()},
        {B.be_tu, c->be_tu.data(), 8 * c->be_tu.size()}, {B.be_tv, c->be_tv.data(), 8 * c->be_tv.size()},
        {B.be_w, c->be_w.data(), 8 * c->be_w.size()},
        {B.mass, c->mass.data(), 8 * c->mass.size()}, {B.hbend, c->hbend.data(), 8 * c->hbend.size()},
        {B.mp_K, c->mp_K.data(), 8 * c->mp_K.size()}, {B.be_L, c->be_L.data(), 8 * c->be_L.size()},
        {B.rest, c->rest.data(), 8 * c->rest.size()},
        {B.asm_tab, c->asm_tab.data(), 4 * c->asm_tab.size()},
    };
    for (const Up &u : ups) {
        if (u.n == 0) continue;
        bsc_status st = hip_check(c, hipMemcpyAsync(u.dst, u.src, u.n, hipMemcpyHostToDevice, c->stream), "upload tables");
        if (st != BSC_OK) return st;
    }
    bsc_status st = hip_check(c, hipMemsetAsync(B.pinmask, 0, 4 * size_t(c->n_cp), c->stream), "clear pins");
    if (st != BSC_OK) return st;
    std::vector<int32_t> rowptr(c->n_cp + 1);
    int32_t nnzb = 0;
    bsc_bsr_pattern(c, rowptr.data(), nullptr, &nnzb);
    st = hip_check(c, hipMemcpyAsync(B.bsr_rowptr, rowptr.data(), 4 * rowptr.size(), hipMemcpyHostToDevice, c->stream), "upload pattern");
    if (st != BSC_OK) return st;
    st = hip_check(c, hipMemsetAsync(B.iscalars, 0, 4 * 64, c->stream), "clear scalars");
    if (st != BSC_OK) return st;
    // the Newton direction starts at zero: the first recycled warm start of a context sees p = 0
    // and falls back to the zero start
    st = hip_check(c, hipMemsetAsync(B.dir, 0, 24 * size_t(c->n_cp), c->stream), "clear direction");
    if (st != BSC_OK) return st;
    st = hip_check(c, hipStreamSynchronize(c->stream), "bind workspace");
    if (st != BSC_OK) return st;
    c->pins.clear();
    c->net_loaded = false;
    c->log_g = c->log_p = nullptr;
    c->log_cap = c->log_count = 0;
    for (auto &row : c->cg_graph)
        for (auto &g : row)
            if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
    for (auto &row : c->mg_graph)
        for (auto &g : row)
            if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
    DevSheet &S = c->dev;
    S.mp_elem = B.mp_elem; S.mp_off = B.mp_off; S.mp_tu = B.mp_tu; S.mp_tv = B.mp_tv; S.mp_w = B.mp_w;
    S.be_elem = B.be_elem; S.be_off = B.be_off; S.be_tu = B.be_tu; S.be_tv = B.be_tv; S.be_w = B.be_w;
    S.mass = B.mass; S.hbend = B.hbend; S.pinmask = B.pinmask;
    S.mp_K = S.curved ? B.mp_K : nullptr;
    S.be_L = S.curved ? B.be_L : nullptr;
    S.rest = S.curved ? B.rest : nullptr;
    for (int kind = 0; kind < 3; ++kind) S.asm_tab[kind] = B.asm_tab + c->asm_tab_off[kind];
    return BSC_OK;
}

bsc_status bsc_set_pins(bsc_ctx *c, const int32_t *idx, int32_t n) {
    if (!c) return BSC_E_INVAL;
    if (!c->ws) return fail(c, BSC_E_STATE, "bind a workspace before setting pins");
    if (n < 0 || n > c->n_cp || (n > 0 && !idx)) return fail(c, BSC_E_INVAL, "bad pin list");
    std::vector<int32_t> mask(c->n_cp, 0);
    for (int a = 0; a < n; ++a) {
        if (idx[a] < 0 || idx[a] >= c->n_cp) return fail(c, BSC_E_INVAL, "pin index out of range");
        if (mask[idx[a]]) return fail(c, BSC_E_INVAL, "duplicate pin index");
        mask[idx[a]] = 1;
    }
    bsc_status st = hip_check(c, hipMemcpyAsync(c->buf.pinmask, mask.data(), 4 * size_t(c->n_cp), hipMemcpyHostToDevice, c->stream), "upload pins");
    if (st != BSC_OK) return st;
    if (n > 0) {
        st = hip_check(c, hipMemcpyAsync(c->buf.pin_idx, idx, 4 * size_t(n), hipMemcpyHostToDevice, c->stream), "upload pins");
        if (st != BSC_OK) return st;
    }
    st = hip_check(c, hipStreamSynchronize(c->stream), "set pins");
    if (st != BSC_OK) return st;
    c->pins.assign(idx, idx + n);
    return BSC_OK;
}

bsc_status bsc_set_sample_log(bsc_ctx *c, float *d_g, float *d_p, int32_t capacity) {
    if (!c) return BSC_E_INVAL;
    if (capacity < 0 || (capacity > 0 && (!d_g || !d_p))) return fail(c, BSC_E_INVAL, "bad sample log");
    c->log_g = d_g;
    c->log_p = d_p;
    c->log_cap = capacity;
    c->log_count = 0;
    return BSC_OK;
}

bsc_status bsc_sample_log_count(const bsc_ctx *c, int32_t *count) {
    if (!c || !count) return BSC_E_INVAL;
    *count = c->log_count;
    return BSC_OK;
}

bsc_status bsc_bsr_pattern(const bsc_ctx *c, int32_t *row_ptr, int32_t *col_idx, int32_t *nnzb) {
    if (!c || !nnzb) return BSC_E_INVAL;
    int32_t cnt = 0;
    for (int j = 0; j < c->n_v; ++j)
        for (int i = 0; i < c->n_u; ++i) {
            if (row_ptr) row_ptr[j * c->n_u + i] = cnt;
            for (int jb = std::max(0, j - 2); jb <= std::min(c->n_v - 1, j + 2); ++jb)
                for (int ib = std::max(0, i - 2); ib <= std::min(c->n_u - 1, i + 2); ++ib) {
                    if (col_idx) col_idx[cnt] = jb * c->n_u + ib;
                    ++cnt;
                }
        }
    if (row_ptr) row_ptr[c->n_cp] = cnt;
    *nnzb = cnt;
    return BSC_OK;
}

}  // extern "C"
