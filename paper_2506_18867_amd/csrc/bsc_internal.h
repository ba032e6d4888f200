// bsc_internal.h -- shared declarations of the HIP library behind include/bsc.h.
//
// Device data layout (all in the caller-owned workspace):
//   membrane points  mp_*  sorted by element, SoA: element index, local span coordinates
//                          (t_u, t_v) in [0,1], physical weight w = wbar |det dX/d(u,v)|
//   bending evals    be_*  same layout; weight w (the bending stiffness is applied in-kernel)
//   per CP           mass (lumped), hbend[13][n_cp] (constant bending Hessian, scalar per
//                          upper-stencil slot), pinmask
//   per point        ptA[21][n_mp] w * projected density Hessian (upper triangle of 6x6),
//                    ptP[6][n_mp] w * first Piola stress, ptE[n_mp] w * Psi
//   per bending eval beD[3][n_be] w * mu_bend * Laplacian(phi), beE[n_be]
//   Hessian          hess[114][n_cp] upper-stencil form (see bsc_assemble)
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <type_traits>
#include <string>
#include <vector>

#include "../../include/bsc.h"

namespace bsc {

constexpr int kBlock = 256;
constexpr int kScalars = 64;           // solver scalars (doubles); the int flags follow them
constexpr int kSlots = 13;            // diagonal + 12 upper offsets
constexpr int kHessEntries = BSC_HESS_ENTRIES;
// CG iteration tile: kCgTileU x kCgTileV control points per workgroup (one wave of rows)
constexpr int kCgTileU = 64, kCgTileV = 2;
// Hessian blocks per wave that the FP32 CG kernel loads before its prologue reduction (3 or more
// need more than the 128 VGPRs that keep two workgroups on a CU)
// CG grids of more workgroups than this have the previous launch's partials summed once, by a
// one-block kernel between the launches, instead of by every workgroup (quadratic in the grid)
constexpr int kCgPrefetch = 2;
constexpr int kCgPreSumBlocks = 2048;

// Upper-stencil slot offsets (di, dj); slot 0 is the diagonal.
constexpr int kSlotDi[kSlots] = {0, 1, 2, -2, -1, 0, 1, 2, -2, -1, 0, 1, 2};
constexpr int kSlotDj[kSlots] = {0, 0, 0, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2};

// The same offsets computed arithmetically: a runtime index into the tables above becomes a
// memory load on the device, which stalls the loads whose addresses depend on it.
__host__ __device__ constexpr int slot_di(int s) { return s <= 2 ? s : (s <= 7 ? s - 5 : s - 10); }
__host__ __device__ constexpr int slot_dj(int s) { return s == 0 ? 0 : (s <= 2 ? 0 : (s <= 7 ? 1 : 2)); }

// First Hessian entry of a slot: 0 for the diagonal (6 entries), 6 + 9 (s - 1) otherwise.
__host__ __device__ constexpr int slot_entry(int s) { return s == 0 ? 0 : 6 + 9 * (s - 1); }

constexpr bool slot_offsets_agree() {
    for (int s = 0; s < kSlots; ++s)
        if (slot_di(s) != kSlotDi[s] || slot_dj(s) != kSlotDj[s]) return false;
    return true;
}
static_assert(slot_offsets_agree(), "slot offsets");

// Slot of an offset, or -1 for a lower offset / outside the 5x5 neighbourhood.
__host__ __device__ inline int upper_slot(int di, int dj) {
    if (di < -2 || di > 2 || dj < 0 || dj > 2) return -1;
    if (dj == 0) return di < 0 ? -1 : di;      // 0, 1, 2
    return 3 + (dj - 1) * 5 + (di + 2);
}

// Solver scalars (doubles) and flags (int32) in the workspace, shared by the solvers and read
// back by the host in one copy.
enum { S_TOL2 = 0, S_ALPHA0, S_ALPHA1, S_GAMMA0, S_GAMMA1, S_E, S_GG, S_C1, S_C2, S_DEM, S_PMAX, S_RTOL, S_ETA, S_GPREV,
       S_WS0, S_WS1, S_WS2, S_WS3, S_RHO, S_WSA, S_WSB, S_G0, S_MGRHO0 = 40, S_MGRHO1 = 41, S_CGSUM = 44 /* 3 slots */,
       S_XMAX = 47 };
enum { I_DONE = 0, I_ITA, I_ITB, I_BREAK, I_MAXIT, I_ITERS, I_WS, I_LSACC };
// I_WS: the warm start was kept; I_LSACC: the device's line-search trial at alpha = 1 (0 rejected,
// 1 accepted and applied, 2 the direction is below the stagnation scale, x untouched)
constexpr int I_PUBSEQ = 60;                 // sequence number of the last published read-back
// Largest PCG relative tolerance of the Eisenstat-Walker forcing term (and its first value):
// loose under the step-length stopping rule, tighter under the gradient rule, which has to reach
// the region of fast local convergence.
constexpr double kEtaMaxStep = 0.5, kEtaMaxGrad = 0.1;
// Relative size (to |x0|_inf) below which a Newton direction only moves x by rounding.
constexpr double kStagnation = 16.0 * 2.220446049250313e-16;

// Multigrid levels below the fine grid (knot halvings), at most kMgMaxLevels.
constexpr int kMgMaxLevels = 6;
struct MgLevel {
    int n_u, n_v;
    void *H, *pinv, *Hmid;                   // Galerkin operator, its block-Jacobi inverse, the u-pass result
    double *r, *xa, *xb, *t;                 // restricted residual, smoothed iterate, level output, residual
};

// Everything a kernel needs to know about the sheet (passed by value).
struct DevSheet {
    int n_u, n_v, Nu, Nv, n_cp, n_elem, n_mp, n_be;
    double A00, A01, A10, A11, b0, b1;      // rest map X = A (u, v) + b, span units
    double K00, K01, K10, K11;              // K = A^{-1}: K[m][b] = d u_m / d X_b
    double c_uu, c_vv, c_uv;                // Laplacian coefficients (affine rest)
    // General rest map (curved != 0): per-point tables replace the constants above. mp_K
    // [4][n_mp] holds K = J^{-1} (k00, k01, k10, k11) at each membrane point, be_L [5][n_be]
    // the Laplacian coefficients (c_uu, c_vv, c_uv, l_u, l_v) at each bending evaluation,
    // rest [2][n_cp] the rest CPs. The weights mp_w, be_w include |det J| per point.
    int curved;
    const double *mp_K, *be_L, *rest;
    int membrane;                           // BSC_MEMBRANE_*
    double mu, lam;                         // StVK per-area Lame parameters
    double mu1, mu2, msh;                   // FBW stiffnesses
    double mu_bend;
    const int32_t *mp_elem, *mp_off;
    const double *mp_tu, *mp_tv, *mp_w;
    const int32_t *be_elem, *be_off;
    const double *be_tu, *be_tv, *be_w;
    const double *mass, *hbend;
    const int32_t *pinmask;
    // tiled assembly (k_assemble_tile): tile height and the per-tile maximum of the membrane
    // points of the elements a tile touches, per precision combination (AsmKind), and each
    // kind's tile table (asm_tile_table; asm_stride ints per tile)
    int asm_ty[3], asm_maxp[3], asm_stride[3];
    const int32_t *asm_tab[3];
};

// Tiled assembly: tiles of kAsmTileU x ty CPs; the precision combinations of the per-point
// Hessian (A), stress (P) and outputs.
#ifndef BSC_ASM_TILE_U
#define BSC_ASM_TILE_U 16
#endif
#ifndef BSC_ASM_THREADS
#define BSC_ASM_THREADS 512
#endif
// Dynamic LDS per assembly workgroup: two workgroups (plus their small static arrays, under
// 256 bytes) share a CU's 160 KB.
#ifndef BSC_ASM_LDS_BYTES
#define BSC_ASM_LDS_BYTES (80 * 1024 - 256)
#endif
constexpr int kAsmTileU = BSC_ASM_TILE_U;
constexpr int kAsmThreads = BSC_ASM_THREADS;
enum AsmKind { kAsmF32 = 0, kAsmF64 = 1, kAsmMixed = 2 };   // (A, P, g) = (f, f, f), (d, d, d), (f, d, d)
constexpr size_t kAsmLdsMax = BSC_ASM_LDS_BYTES;

// LDS layout of one assembly tile (offsets in bytes): local membrane point offsets of the
// (tx + 2) x (ty + 2) elements, the first global point of each element row, the work counter,
// then one record per membrane point holding what the tile's items read of that point:
//   FP32 (kAsmF32, floats, 16-byte aligned): the weighted density Hessian A (21 entries, padded
//     to 24), the gradients of the 9 local basis functions (18, from 24), the weighted first
//     Piola stress P (6, from 44): kAsmRecF floats.
//   mixed (kAsmMixed, floats, 16-byte aligned): A and the basis gradients as in FP32 (float, for
//     the FP32 Hessian; the gradients rounded from FP64), then for the FP64 gradient P in double
//     (from float 44) and the rounding remainders of the 18 basis gradients (from 56; the float
//     pair holds each FP64 gradient to about 48 bits): kAsmRecM floats, for any rest map.
//   FP64 (kAsmF64, doubles): everything in the span's parametric coordinates (u, v), where the
//     gradient of basis function (a, b) is (Du[a] Nv[b], Nu[a] Dv[b]): the density Hessian
//     congruent to A under the inverse Jacobian K (21), the 1-D factors Nu, Du, Nv, Dv (21..32)
//     and the stress P K^T (6, from 33): kAsmRecD doubles, for any rest map.
// The float record lengths in 16-byte units are odd or twice odd, so the neighbouring records
// that the lanes of a wave read fall on different LDS banks.
constexpr int kAsmRecF = 52, kAsmRecM = 76, kAsmRecD = 39;
struct AsmLds {
    size_t el_off, rows, counter, rec, rec_bytes, total;
};
__host__ __device__ inline size_t align16(size_t v) { return (v + 15) & ~size_t(15); }
__host__ __device__ inline size_t asm_rec_bytes(int kind, bool curved) {
    return kind == kAsmF32 ? 4 * kAsmRecF
                           : (kind == kAsmMixed ? 4 * kAsmRecM : 8 * kAsmRecD);
}
__host__ __device__ inline AsmLds asm_lds_layout(int tx, int ty, int maxp, int kind, bool curved) {
    AsmLds L;
    const size_t ne = size_t(tx + 2) * (ty + 2);
    L.el_off = 0;                                   // local membrane point offsets (ne + 1)
    L.rows = align16(L.el_off + 4 * (ne + 1));      // global first point of each element row (ty + 2)
    L.counter = align16(L.rows + 4 * size_t(ty + 2));
    L.rec = align16(L.counter + 4);
    L.rec_bytes = asm_rec_bytes(kind, curved);
    L.total = align16(L.rec + L.rec_bytes * size_t(maxp));
    return L;
}
// Tile rows of the assembly: the four CP rows at each edge of the sheet get tile rows of height
// e = min(2, ty) (their elements, next to the boundary, carry the boundary spans' extra
// quadrature points, which would otherwise set the LDS size of every tile), the interior rows
// tile rows of height ty; sheets with fewer than 9 CP rows use height e throughout.
__host__ __device__ inline int asm_tile_rows(int n_v, int ty) {
    const int e = ty < 2 ? 1 : 2;
    return n_v >= 9 ? 8 / e + (n_v - 8 + ty - 1) / ty : (n_v + e - 1) / e;
}
__host__ __device__ inline void asm_tile_row(int n_v, int ty, int tr, int &y0, int &h) {
    const int e = ty < 2 ? 1 : 2;
    if (n_v < 9) {
        y0 = e * tr;
        h = n_v - y0 < e ? n_v - y0 : e;
        return;
    }
    const int ne = 4 / e, nint = (n_v - 8 + ty - 1) / ty;
    if (tr < ne) {
        y0 = e * tr;
        h = e;
    } else if (tr < ne + nint) {
        y0 = 4 + (tr - ne) * ty;
        h = n_v - 4 - y0 < ty ? n_v - 4 - y0 : ty;
    } else {
        y0 = n_v - 4 + e * (tr - ne - nint);
        h = e;
    }
}

// Tile table of the tiled assembly, built at create: tile t (t = tile row * tiles per row +
// tile column) owns asm_stride ints from t * asm_stride: the number np of staged points, then
// for each record r < np the global membrane point (np ints) and the tile-local element
// (l - l0) nk + (k - k0) it belongs to (np ints; both padded to the kind's maxp), then one int
// per tile-local element: point count | first record << 4 | further records << 18. A span's
// first point goes to region 0 (the first points of the tile's spans in element order), its
// further points, in order, to region 1 (contiguous per span, after region 0): every interior
// span carries exactly two points under the paper's rule, so the lanes of a wave that read the
// s-th point of neighbouring spans read neighbouring records.
__host__ __device__ inline int asm_tab_stride(int ty, int maxp) {
    return 1 + 2 * maxp + (BSC_ASM_TILE_U + 2) * (ty + 2);
}
__host__ __device__ inline int asm_el_count(int info) { return info & 15; }
__host__ __device__ inline int asm_el_first(int info) { return (info >> 4) & 0x3fff; }
__host__ __device__ inline int asm_el_rest(int info) { return (info >> 18) & 0x3fff; }

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2). Give every
// XCD a contiguous range of tiles so that neighbouring tiles, which read each other's halo
// (stencil neighbours, shared elements), are usually in the same L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int x = b & 7, k = b >> 3, q = nb >> 3, r = nb & 7;
    return x * q + (x < r ? x : r) + k;
}

// Device buffers carved out of the workspace.
struct DevBufs {
    // tables
    int32_t *mp_elem, *mp_off, *be_elem, *be_off, *pinmask, *pin_idx;
    double *mp_tu, *mp_tv, *mp_w, *be_tu, *be_tv, *be_w, *mass, *hbend;
    double *mp_K, *be_L, *rest;              // general rest map only (zero bytes when affine)
    int32_t *asm_tab;                        // assembly tile tables (asm_tile_table)
    // per-point intermediates (sized for double; float uses the front half)
    void *ptA, *ptP;
    double *ptE, *ptP64, *beD, *beE;
    // reductions
    double *partials;                        // 8 arrays of max_blocks
    int32_t *bsr_rowptr;                     // n_cp + 1 (standard BSR export)
    double *scalars;                         // solver scalars (see solve.hip)
    int32_t *iscalars;
    // solver vectors (3 n_cp doubles each) and the block-Jacobi inverse (6 n_cp)
    double *g, *xn, *xhat, *dir, *r, *p0, *p1, *q, *pinv, *tmp, *phat;
    double *gpre;                                // per-CP gradient terms of the assembly (bending, inertia, gravity)
    double *r2, *q2, *p2;                    // second halves of the CG double buffers
    void *hess;                              // kHessEntries n_cp doubles
    // warm-start network
    float *net_w, *net_w_fwd, *net_wr, *net_in, *net_out, *net_act0, *net_act1, *net_scale;
    double *net_lpart;                        // loss partials: 1024 samples x 64 blocks x 3
    int max_blocks;
    // multigrid hierarchy (mg_levels = 0: not available for this grid)
    int mg_levels;
    MgLevel mg[kMgMaxLevels];
    double *mg_x0, *mg_t0;                   // fine-level smoother vectors
};

// Contact-mesh conversion buffers (one caller-owned workspace, see contact.hip).
struct ContactBufs {
    int32_t *vspan, *voff, *vlist;           // span of each vertex; vertices grouped by span
    double *vw;                              // 9 interpolation weights per vertex
    unsigned long long *key1a, *key1b, *ukey1, *key2a, *key2b, *ukey2;
    unsigned int *val1a, *val1b, *cnt1, *off1, *val2a, *val2b, *cnt2, *off2, *small;
    double *hlin, *glin;                     // vertex-pair blocks, vertex gradients
    int32_t *pa, *pb;                        // vertices of each distinct vertex pair
    double *hsp;                             // vertex-pair blocks in span-pair order
    int32_t *pas, *pbs;                      // their vertices, same order
    unsigned long long *spk, *spk_s, *uksp;  // span-pair keys of the vertex pairs (sorted, distinct)
    unsigned int *spv, *spv_s, *cntsp, *offsp;
    void *tmp;                               // sort / run-length / scan temporary storage
    size_t tmp_bytes;
};

}  // namespace bsc

struct bsc_ctx {
    int n_u = 0, n_v = 0, Nu = 0, Nv = 0, n_cp = 0, n_elem = 0, n_mp = 0, n_be = 0;
    double hu = 1.0, hv = 1.0;               // knot spacings (parameter units per span)
    bsc_material mat{};
    bsc::DevSheet dev{};
    hipStream_t stream = nullptr;
    int device = 0;
    // host tables
    std::vector<int32_t> mp_elem, mp_off, be_elem, be_off;
    std::vector<double> mp_tu, mp_tv, mp_w, be_tu, be_tv, be_w, mass, hbend;
    std::vector<double> mp_K, be_L, rest;    // general rest map: SoA per-point geometry, rest CPs
    std::vector<int32_t> pins;
    // assembly tile tables (AsmKind kinds with the same tile height share one): offset of each
    // kind's table in asm_tab and the ints per tile; layout in asm_tile_table
    std::vector<int32_t> asm_tab;
    size_t asm_tab_off[3] = {0, 0, 0};
    // workspace
    char *ws = nullptr;
    size_t ws_bytes = 0;
    bsc::DevBufs buf{};
    bool net_loaded = false;
    std::string err;
    // replayable bursts of CG iterations (kernel arguments depend only on the workspace): graphs
    // of 1..8 chunks of launches per precision (index [precision][chunks])
    hipGraphExec_t cg_graph[2][9] = {};
    hipGraphExec_t mg_graph[2][9] = {};      // the same for multigrid-preconditioned CG iterations
    bool use_graphs = false;         // BSC_GRAPHS=1 in the environment at create: bursts replayed from graphs
    // PCG iterations of the previous step's solves, by Newton iteration (sizes first bursts)
    int pcg_hist[64] = {};
    // (g, p) sample log of the Newton iterations (device float buffers owned by the caller)
    float *log_g = nullptr, *log_p = nullptr;
    int log_cap = 0, log_count = 0;
    // timing events of a step (a pool that grows to the largest step; read at the step's end)
    std::vector<hipEvent_t> ev_pool;
    bool ev_failed = false;
    // pinned host buffer for the step's small read-backs (solver scalars followed by the flags)
    char *pinned = nullptr;
    char *pinned_dev = nullptr;              // its device address (host-mapped, coherent), or null
    // contact mesh embedded in the surface (bsc_contact_setup): per-vertex span and weights
    int ct_nvert = 0, ct_max_pairs = 0, ct_max_vpairs = 0;
    std::vector<int32_t> ct_span, ct_voff, ct_vlist;
    std::vector<double> ct_w;
    size_t ct_tmp_bytes = 0;
    char *ct_ws = nullptr;
    size_t ct_ws_bytes = 0;
    bsc::ContactBufs ct{};
    ~bsc_ctx() {
        for (auto &row : cg_graph)
            for (auto &g : row)
                if (g) (void)hipGraphExecDestroy(g);
        for (auto &row : mg_graph)
            for (auto &g : row)
                if (g) (void)hipGraphExecDestroy(g);
        for (auto &e : ev_pool) (void)hipEventDestroy(e);
        if (pinned) (void)hipHostFree(pinned);
    }
};

namespace bsc {

bsc_status fail(bsc_ctx *ctx, bsc_status st, const std::string &msg);
bsc_status hip_check(bsc_ctx *ctx, hipError_t e, const char *what);
size_t layout_workspace(const bsc_ctx *ctx, DevBufs *b, char *base);
size_t contact_layout(const bsc_ctx *ctx, ContactBufs *b, char *base);
int mg_level_count(int n_u, int n_v);
hipError_t mg_setup(const DevSheet &S, const DevBufs &B, int prec, hipStream_t st);
hipError_t mg_cg_iteration(const DevSheet &S, const DevBufs &B, int prec, double *r, double *z, double *p, double *q,
                           double *rz_part, double *pq_part, double *rr_part, hipStream_t st);
size_t contact_tmp_bytes(int max_pairs, int max_vpairs);
// Quadratic B-spline pieces on a span (type 0 first, 1 inner, 2 last), local t in [0, 1].
void host_pieces(int type, double t, double N[3], double D[3], double D2[3]);
DevSheet dev_sheet(const bsc_ctx *ctx);

// Read-back into host-mapped pinned memory: the scalars and the first 8 flags, then the next
// sequence number (kept in the device flags) stored with system-scope release, on which the host
// spins. Run by one block (at least kScalars threads) once the values it copies are final in the
// block's view; every thread of the block calls it.
struct PubPtrs {
    double *hs;          // host copy of the scalars
    int32_t *hf;         // host copy of the flags
    int32_t *hseq;       // host sequence number
};
__device__ __forceinline__ void publish_block(const double *scal, int32_t *flags, const PubPtrs &P) {
    const int t = threadIdx.x;
    if (t < kScalars) P.hs[t] = scal[t];
    if (t < 8) P.hf[t] = flags[t];
    const int32_t seq = flags[I_PUBSEQ] + 1;
    __threadfence_system();
    __syncthreads();
    if (t == 0) {
        flags[I_PUBSEQ] = seq;
        __hip_atomic_store(P.hseq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// The per-CP terms of an assembly that need no quadrature point: the bending gradient K_b d, the
// inertia M (x - xhat) / dt^2 (when xhat is given) and the gravity load -M g, summed into gpre
// ([3][n_cp], double), with their energies (the bending energy as d^T K_b d / 2).
struct CpTerms {
    const double *xhat;
    double inv_dt2, gx, gy, gz;
    double *gpre;
};

// ---- launchers (eval.hip) ----
// Membrane points (w Psi, w P and, with hess, w A+) and either the bending evaluations or, with
// cpt, the per-CP terms (bending energy included; their energy partials in partial array 2,
// cp_blocks of them); element gather;
// tiled assembly, after a points pass with cpt, of the per-CP gradient (membrane stresses plus
// B.gpre) and (hess != NULL) the upper-stencil Hessian blocks (kind: AsmKind; gnorm: also
// per-tile partials of |g|^2; out_e: the energy of the points pass, summed by the tile kernel's
// block 0, where no |g|^2 is needed); energy reduction (n_cp_partials: cp_blocks after a points pass
// with cpt, else 0; n_gg_partials: the tile count of an assembly run with gnorm, summed into
// out_gg; with pub the solver scalars and flags are then published to the host in the same
// launch). The mixed-precision Newton points: FP64 arithmetic, FP32 Hessian and FP64 stresses
// in one pass.
hipError_t launch_points(const DevSheet &S, const DevBufs &B, int precision, bool hess, bool grad64,
                         const double *x, hipStream_t st, bool bending, const CpTerms *cpt = nullptr);
hipError_t launch_points_mixed(const DevSheet &S, const DevBufs &B, const double *x, hipStream_t st, const CpTerms *cpt);
int assemble_tiles(const DevSheet &S, int kind);
int cp_blocks(const DevSheet &S);
hipError_t launch_assemble(const DevSheet &S, const DevBufs &B, int kind, double inv_dt2, void *g, void *hess,
                           hipStream_t st, bool gnorm = false, double *out_e = nullptr);
hipError_t launch_energy_reduce(const DevSheet &S, const DevBufs &B, int n_cp_partials, int n_gg_partials, double *out,
                                hipStream_t st, double *out_gg = nullptr, const PubPtrs *pub = nullptr);
hipError_t launch_elem(const DevSheet &S, const DevBufs &B, int precision, void *eE, void *eg, void *eH,
                       hipStream_t st);

// ---- launchers (solve.hip) ----
hipError_t launch_spmv(const DevSheet &S, int precision, const void *hess, const double *in, double *out,
                       hipStream_t st);
hipError_t launch_export_bsr(const DevSheet &S, int precision, const void *hess, const int32_t *row_ptr,
                             const int32_t *col_idx, void *vals, hipStream_t st);
bsc_status newton_step(bsc_ctx *ctx, const bsc_step_opts *o, double *x, double *v, const double *pin_tgt,
                       bsc_step_stats *stats);
// H x = b for the upper-stencil matrix held in the workspace (B.hess) by the fused block-Jacobi PCG
// from x0 = 0 to |r| <= rtol |b|; overwrites the workspace's CG vectors, B.g, B.tmp and B.dir.
bsc_status stencil_pcg(bsc_ctx *ctx, int prec, const double *b, double *x, double rtol, int max_iter, int *iters);

// ---- launchers (net.hip) ----
hipError_t net_forward_impl(int n_u, int n_v, int batch, const float *w, const float *in, float *out, float *acts,
                            float *tmp0, float *tmp1, float *scale, float *wr, bool reordered, hipStream_t st);
hipError_t net_backward(int n_u, int n_v, int batch, const float *w, const float *in, const float *acts,
                        const float *dout, float *dw, float *din, void *scratch, hipStream_t st);
size_t net_scratch_bytes(int n_u, int n_v, int batch);
hipError_t net_adam(int n, float *p, const float *g, float *m, float *v, float lr, float b1, float b2,
                    float eps, int t, hipStream_t st);
hipError_t net_loss(int n_cp, int batch, const float *in, const float *pred, const float *tgt, float *loss,
                    float *dpred, double *part, hipStream_t st);

}  // namespace bsc
