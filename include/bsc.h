/*
 * bsc.h -- C ABI of the MI355X (gfx950) hot path of quadratic B-spline cloth finite elements
 * (arXiv 2506.18867, "Efficient B-Spline Finite Elements for Cloth Simulation").
 *
 * The library evaluates the membrane and bending energy, gradient and Hessian of a quadratic
 * B-spline sheet at the paper's separately reduced quadrature points (Sec. 4.1 and 4.2), projects
 * every membrane point's density Hessian onto the PSD cone (Sec. 5.1), assembles the global
 * 3x3-block Hessian on its fixed control-point pattern by a per-block gather (Sec. 5.2), and runs
 * the projected-Newton minimisation of the implicit-Euler incremental potential (Sec. 3.2,
 * Eq. "incremental_potential"; Sec. 5.1) with a hand-written block-Jacobi PCG.
 *
 * General rules
 *   - Every call returns a bsc_status (0 = OK, < 0 = error) and never throws or aborts.
 *     bsc_last_error() gives a message for the last failing call on a context.
 *   - Pointers named d_* are device pointers (HIP global memory of the context's device);
 *     everything else is host memory. The caller owns every buffer it passes, including the
 *     workspace; the context owns only host-side tables. Nothing is freed across the boundary.
 *   - Calls are asynchronous on the context's HIP stream unless stated otherwise; the caller
 *     synchronises before reading results on the host.
 *   - One context per host thread. Calls that overlap on one context race.
 *   - Layouts. Control point (CP) (i,j), 0 <= i < n_u, 0 <= j < n_v, has index a = j*n_u + i.
 *     Vectors over CPs are structure-of-arrays: v[c*n_cp + a] for component c in {0,1,2}
 *     (a (3, n_v, n_u) contiguous tensor). An element is a knot span (k,l), index
 *     e = l*(n_u-2) + k; its CPs are (k+a', l+b'), a',b' in {0,1,2}, local CP 3*b'+a',
 *     local DOF r = 3*(3*b'+a') + c.
 *   - Precision: BSC_FP64 computes everything in double. BSC_FP32_MIXED computes element
 *     quantities, assembly and SpMV in float (float outputs), keeps the PSD eigen-problems in
 *     double, and the Newton step keeps the gradient, energy differences, PCG residual and
 *     dot products in double.
 */
#ifndef BSC_H
#define BSC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bsc_ctx bsc_ctx;

typedef enum {
    BSC_OK = 0,
    BSC_E_INVAL = -1,           /* bad argument, size or unsupported input                       */
    BSC_E_KNOTS = -2,           /* knot vector is not open, uniform, integer, starting at 0        */
    BSC_E_NOMEM = -3,           /* host allocation failed or workspace too small                   */
    BSC_E_HIP = -4,             /* a HIP runtime call failed                                       */
    BSC_E_NOT_CONVERGED = -5,   /* Newton hit max_newton before the stopping test                  */
    BSC_E_LINESEARCH = -6,      /* no energy decrease after 20 step halvings                       */
    BSC_E_NONFINITE = -7,       /* NaN or Inf in the state, gradient or energy                     */
    BSC_E_PCG_BREAKDOWN = -8,   /* p^T H p <= 0 inside PCG                                         */
    BSC_E_STATE = -9            /* call order violated (e.g. no workspace bound)                   */
} bsc_status;

enum { BSC_MEMBRANE_STVK = 0, BSC_MEMBRANE_FBW = 1 };
enum { BSC_FP64 = 0, BSC_FP32_MIXED = 1 };
enum { BSC_STOP_GRAD = 0, BSC_STOP_STEP = 1 };

/* Quadrature rule of the membrane and bending energies. BSC_QUAD_REDUCED is the paper's
 * reduced integration (Sec. 4.1 and 4.2, Fig. "quadrature"): 3x3 Gauss on corner spans, 3x2 on
 * side spans, alternating 1x2 / 2x1 Gauss on the dual-grid cells of the interior for the
 * membrane; span centres on the boundary and the interior knots for bending. The others are the
 * comparison rules of the ablation (Sec. 6.5), all with the same boundary placement except as
 * stated: BSC_QUAD_GAUSS2 the standard 2x2 Gauss rule on every interior span for membrane and
 * bending; BSC_QUAD_INTERIOR1 one midpoint per interior span for the membrane (admits hourglass
 * modes); BSC_QUAD_CORNER2 2x2 instead of 3x3 Gauss on the four corner spans for the membrane. */
enum { BSC_QUAD_REDUCED = 0, BSC_QUAD_GAUSS2 = 1, BSC_QUAD_INTERIOR1 = 2, BSC_QUAD_CORNER2 = 3 };

/* Material and discretisation (Sec. 4). StVK: membrane energy per rest area
 * t [mu |E_G|^2 + lam/2 tr(E_G)^2], E_G = (F^T F - I)/2, mu = E/(2(1+nu)), lam = E nu/(1-nu^2).
 * FBW (Eq. "FBW stretching and shearing energy"): mu_st1, mu_st2, mu_sh per rest area. Bending
 * (Eq. "general bending energy"): mu_bend/2 |Laplacian(phi)|^2 per rest area. rho_area: rest
 * mass per area R^0. quadrature: BSC_QUAD_* (0 is the paper's rule); others return
 * BSC_E_INVAL from bsc_create. */
typedef struct {
    int32_t membrane;
    double young, poisson, thickness;
    double mu_st1, mu_st2, mu_sh;
    double mu_bend;
    double rho_area;
    int32_t quadrature;
} bsc_material;

/* Options of one implicit-Euler step (Sec. 3.2, Sec. 5.1).
 *   stop_mode BSC_STOP_GRAD: stop when |g_free|_2 <= rtol |g0_free|_2 (g0 at the first iterate);
 *   stop_mode BSC_STOP_STEP: stop when |p|_inf / dt <= atol (the paper's rule).
 *   fixed_newton_iters > 0 runs exactly that many iterations instead (for comparisons).
 *   pcg_rtol: PCG stops when |r|_2 <= pcg_rtol |g|_2. warm_start: the PCG initial guess, one of
 *   BSC_WARM_* below; a predicted start is scaled by its energy-optimal multiple and kept only
 *   when it lowers the initial residual below |g|_2, else the solve starts from zero.
 *   pcg_adaptive: 1 chooses the PCG tolerance per Newton iteration by the Eisenstat-Walker rule
 *   eta_k = 0.9 (|g_k| / |g_{k-1}|)^2 (not below 0.9 eta_{k-1}^2 when that exceeds 0.1),
 *   clamped to [pcg_rtol, eta_max] (eta_0 = eta_max), eta_max = pcg_eta_max if set, else 0.5
 *   under BSC_STOP_STEP and 0.1 under BSC_STOP_GRAD; with
 *   BSC_STOP_STEP a stop is only accepted on a direction solved to pcg_rtol. */
/* PCG warm starts. NONE: x0 = 0. NET: the loaded network's prediction from the gradient (the
 * learned warm start; needs bsc_warmstart_load). PREVIOUS: the previous Newton direction of the
 * same step (recycled: in the linearly converging phase of projected Newton successive
 * directions are close; the first Newton iteration of a step starts from zero; not in the
 * paper). Both decide on the device, with no host round trip. */
enum { BSC_WARM_NONE = 0, BSC_WARM_NET = 1, BSC_WARM_PREVIOUS = 2 };
/* PCG preconditioners. JACOBI: 3x3 block Jacobi, one fused kernel per iteration. MULTIGRID: one
 * symmetric V(1,1) cycle on the hierarchy of the patch's knot halvings (exact B-spline
 * prolongation, Galerkin coarse operators, damped block-Jacobi smoothing); used when both span
 * counts are even (otherwise, and with the warm start, the step falls back to JACOBI). */
enum { BSC_PRECOND_JACOBI = 0, BSC_PRECOND_MULTIGRID = 1 };
/* First Newton iterate x0 (pinned CPs at their targets in both). PREVIOUS: x^n. PREDICTOR: the
 * inertial prediction xhat = x^n + dt v^n, the minimiser of the inertia term alone; the paper
 * leaves the start open (Sec. 5.1 follows IPC, whose x^n start keeps a contact barrier finite;
 * without contact any start is admissible). */
enum { BSC_START_PREVIOUS = 0, BSC_START_PREDICTOR = 1 };

typedef struct {
    double dt;
    double gravity[3];
    int32_t precision;
    int32_t stop_mode;
    double rtol, atol;
    int32_t max_newton, max_pcg;
    double pcg_rtol;
    int32_t warm_start;
    int32_t fixed_newton_iters;
    int32_t pcg_adaptive;
    int32_t preconditioner;     /* BSC_PRECOND_JACOBI (default) or BSC_PRECOND_MULTIGRID */
    int32_t start;              /* BSC_START_PREVIOUS (default) or BSC_START_PREDICTOR */
    double pcg_eta_max;         /* cap of the adaptive PCG tolerance; 0 = 0.5 under BSC_STOP_STEP,
                                   0.1 under BSC_STOP_GRAD; else in [pcg_rtol, 0.9] */
    int32_t timing;             /* BSC_TIMING_CG (default), BSC_TIMING_PHASES or BSC_TIMING_OFF */
} bsc_step_opts;
/* GPU timing of a step (bsc_step_stats). Every timing event is a marker between two kernels on the
 * context's stream and delays the second by a few microseconds, so the default records only what
 * ms_cg_kernels needs. CG: one event at the start of each burst of PCG launches and one after its
 * last CG launch. PHASES: also ms_assemble, ms_pcg, ms_linesearch and ms_warmstart (about 14
 * events per Newton iteration; diagnostics). OFF: none (the GPU fields of the stats stay 0). */
enum { BSC_TIMING_CG = 0, BSC_TIMING_PHASES = 1, BSC_TIMING_OFF = 2 };

/* Statistics of one step. ms_assemble, ms_pcg, ms_linesearch and ms_warmstart are GPU phase
 * times from HIP events on the context's stream, recorded under BSC_TIMING_PHASES only (else 0;
 * read once at the end of the step; ms_warmstart
 * is the network's forward pass, the warm start's product, dots and decision count in ms_pcg;
 * warm_start_used / warm_start_fallbacks count the Newton iterations whose prediction was kept /
 * dropped); ms_total is
 * the host wall-clock time of the call. The PCG iterations run as launches of one fused kernel (one per
 * iteration, enqueued in fixed-size chunks; launches after convergence exit at once):
 * cg_launches counts them, cg_active_launches those that performed an iteration, and
 * ms_cg_kernels is their GPU time from HIP events recorded on the context's stream around
 * the CG launches of each burst of chunks (not under BSC_TIMING_OFF; with BSC_GRAPHS=1 in the
 * environment at bsc_create a burst is one graph launch, which ends with the kernel that
 * publishes the solver state to the host). */
typedef struct {
    int32_t newton_iters, pcg_iters_total, ls_halvings, warm_start_used, warm_start_fallbacks;
    double g0_norm, g_norm, energy;
    double ms_assemble, ms_pcg, ms_linesearch, ms_warmstart, ms_total;
    int32_t cg_launches, cg_active_launches;
    double ms_cg_kernels;
} bsc_step_stats;

/* Sizes of a context: CPs, elements, membrane quadrature points, bending evaluations (four per
 * interior knot, one per boundary span), stored Hessian entries per CP (BSC_HESS_ENTRIES). */
#define BSC_HESS_ENTRIES 114

/* Creates a context for an n_u x n_v control grid (Sec. 3.1.2, Eq. "general B-spline patch").
 *   knots_u / knots_v: host, n_u+3 / n_v+3 doubles; must be open uniform quadratic knot vectors
 *     starting at 0 with integer knots (Sec. 3.1.2); n_u, n_v >= 5 (at least 3 spans), each at
 *     most 32768, and n_u*n_v <= 2^24 (16.7 M CPs: every offset into the device tables, such as
 *     entry * n_cp for the 114 Hessian entries, stays below 2^31); otherwise BSC_E_INVAL.
 *   rest_xy: host, 2*n_u*n_v doubles, AoS (X1, X2) per CP (Sec. 3.2). Any rest map whose
 *     Jacobian determinant is positive at every quadrature point (membrane, bending and the
 *     3x3 Gauss mass points) is accepted; otherwise BSC_E_INVAL. An affine rest (control points
 *     at the Greville abscissae of an affine image of the parameter rectangle) keeps the
 *     inverse Jacobian and the Laplacian coefficients as sheet constants; any other rest map
 *     gets them per quadrature point (Sec. 4.1 inverse function theorem; Sec. 4.2 Laplacian in
 *     parametric space, with its first-derivative terms): 32 more workspace bytes per membrane
 *     point, 40 per bending evaluation and 16 per CP.
 *   mat: host; E, thickness, rho_area > 0, nu in (-1, 0.5] for StVK (plane stress stays finite at
 *   0.5); mu_* >= 0 for FBW.
 *   hip_stream: hipStream_t on which all work is enqueued (NULL = default stream).
 * On success *out owns the host tables; free it with bsc_destroy. Host-only, synchronous. */
bsc_status bsc_create(bsc_ctx **out, int32_t n_u, int32_t n_v, const double *knots_u,
                      const double *knots_v, const double *rest_xy, const bsc_material *mat,
                      void *hip_stream);

bsc_status bsc_sizes(const bsc_ctx *ctx, int32_t *n_cp, int32_t *n_elem, int32_t *n_membrane_pts,
                     int32_t *n_bending_evals);

/* Bytes of device workspace the context needs (tables, per-point buffers, solver vectors,
 * the Hessian and the warm-start network). */
bsc_status bsc_workspace_size(const bsc_ctx *ctx, size_t *bytes);

/* Binds caller-owned device memory (>= bsc_workspace_size bytes, 256-byte aligned) and uploads
 * the precomputed tables into it. Synchronises the context's stream before returning. */
bsc_status bsc_bind_workspace(bsc_ctx *ctx, void *d_ws, size_t bytes);

/* Sets the pinned CPs (Dirichlet conditions, Sec. 5.1: eliminated DOFs). cp_idx: host list of
 * n distinct CP indices (n = 0 clears). Needs a bound workspace. Synchronous. */
bsc_status bsc_set_pins(bsc_ctx *ctx, const int32_t *cp_idx, int32_t n);

/* Per-element elastic (membrane + bending) energy, gradient and 27x27 Hessian (Sec. 4.1, 4.2,
 * Sec. 5.2 step 1) with every membrane point's density Hessian projected to PSD.
 *   d_x: 3*n_cp doubles (SoA), world CP positions.
 *   d_energy: 1 double, total elastic energy (required).
 *   d_elem_energy: n_elem values or NULL; d_elem_grad: 27*n_elem values or NULL, layout
 *     [r][e]; d_elem_hess: 378*n_elem values or NULL, upper triangle (r <= c) of the
 *     symmetric 27x27 matrix in row-major order, layout [entry][e].
 *   Output values are double for BSC_FP64 and float for BSC_FP32_MIXED (d_energy is always
 *   double). No pins, inertia or gravity are applied. */
bsc_status bsc_eval_egh(bsc_ctx *ctx, int32_t precision, const double *d_x, double *d_energy,
                        void *d_elem_energy, void *d_elem_grad, void *d_elem_hess);

/* Incremental potential of Eq. "incremental_potential" with lumped mass (Eq. "lumped mass
 * matrix"), gravity and eliminated pinned DOFs, assembled by per-block gather (Sec. 5.2):
 *   E = sum_a M_a |x_a - xhat_a|^2 / (2 dt^2) - sum_a M_a grav.x_a + E_elastic(x).
 *   d_xhat: 3*n_cp doubles, or NULL to drop the inertia term (dt is then ignored).
 *   gravity: host, 3 doubles, or NULL for none.
 *   d_energy: 1 double. d_grad: 3*n_cp values (SoA), zero on pinned CPs.
 *   d_hess: BSC_HESS_ENTRIES*n_cp values, or NULL: the symmetric Hessian in upper-stencil
 *     form, layout [entry][a]. Entries 0..5 are the diagonal block (xx,xy,xz,yy,yz,zz);
 *     entry 6 + 9*(s-1) + 3*r + c is row r, column c of the block coupling CP a to CP a+d_s
 *     for the upper offsets d_1..d_12 = (1,0),(2,0),(-2,1),(-1,1),(0,1),(1,1),(2,1),
 *     (-2,2),(-1,2),(0,2),(1,2),(2,2) in (di,dj). Blocks reaching outside the grid are 0;
 *     pinned CPs have an identity diagonal block and zero coupling blocks.
 *   Values are double for BSC_FP64 and float for BSC_FP32_MIXED. */
bsc_status bsc_assemble(bsc_ctx *ctx, int32_t precision, const double *d_x, const double *d_xhat,
                        double dt, const double *gravity, double *d_energy, void *d_grad,
                        void *d_hess);

/* y = H x for a Hessian in upper-stencil form (as written by bsc_assemble with the same
 * precision). d_in, d_out: 3*n_cp doubles, SoA; must not alias. */
bsc_status bsc_spmv(bsc_ctx *ctx, int32_t precision, const void *d_hess, const double *d_in,
                    double *d_out);

/* Standard 3x3-block CSR (BSR) pattern of the Hessian: every CP pair with |di| <= 2 and
 * |dj| <= 2 (the 5x5 control-point neighbourhood). row_ptr: host, n_cp+1 ints; col_idx: host,
 * nnzb ints (pass NULL to query *nnzb). Columns ascending within a row. Host-only. */
bsc_status bsc_bsr_pattern(const bsc_ctx *ctx, int32_t *row_ptr, int32_t *col_idx, int32_t *nnzb);

/* Expands an upper-stencil Hessian into BSR values on the device: d_bsr_vals holds 9*nnzb
 * values (row-major 3x3 blocks in the order of bsc_bsr_pattern), same precision as d_hess. */
bsc_status bsc_export_bsr(bsc_ctx *ctx, int32_t precision, const void *d_hess, void *d_bsr_vals);

/* One implicit-Euler step by projected Newton (Sec. 5.1): x0 = x^n (or xhat, opts.start) with
 * pinned CPs at their targets, xhat = x^n + dt v^n; per iteration assemble, stop test, block-Jacobi PCG for the
 * direction on the free DOFs, backtracking from alpha = 1 halving until the energy difference
 * (computed in double) is <= 0, update; finally v = (x - x^n)/dt.
 *   d_x: in x^n, out x^{n+1} (3*n_cp doubles); d_v: in v^n, out v^{n+1}.
 *   d_pin_targets: 3*n_pins doubles, SoA [c][pin] in the order given to bsc_set_pins (may be
 *     NULL when there are no pins). stats: host, may be NULL. Synchronous.
 * Returns BSC_E_NOT_CONVERGED, BSC_E_LINESEARCH, BSC_E_NONFINITE or BSC_E_PCG_BREAKDOWN on
 * failure; x and v then hold the last iterate. */
bsc_status bsc_newton_step(bsc_ctx *ctx, const bsc_step_opts *opts, double *d_x, double *d_v,
                           const double *d_pin_targets, bsc_step_stats *stats);

/* Energy difference of the incremental potential along a direction, as the line search of
 * bsc_newton_step evaluates it (Sec. 5.1, backtracking on a monotone decrease of the potential
 * of Sec. 3.2, Eq. "incremental_potential"): d_de[k] = E(x + alphas[k] p) - E(x) with E as in
 * bsc_assemble without pins (inertia with d_xhat and dt, gravity, membrane and bending). The
 * inertia, gravity and bending terms are quadratics in alpha whose coefficients are summed over
 * CPs and bending evaluations; the membrane term is summed point by point as
 * w (Psi(F + alpha dF) - Psi(F)) from the strain increment, so the difference carries no
 * cancellation against E itself. All arithmetic is double.
 *   d_x, d_p: 3*n_cp doubles (SoA); d_xhat: 3*n_cp doubles or NULL (no inertia term; dt is then
 *     ignored); gravity: host, 3 doubles or NULL.
 *   alphas: host, n_alpha step lengths (1 <= n_alpha <= 64, finite); d_de: n_alpha doubles.
 *   Uses the workspace's per-point buffers (overwrites what bsc_eval_egh / bsc_assemble left
 *   there). Asynchronous. */
bsc_status bsc_energy_difference(bsc_ctx *ctx, const double *d_x, const double *d_xhat, double dt,
                                 const double *gravity, const double *d_p, int32_t n_alpha,
                                 const double *alphas, double *d_de);

/* Sample log for training the warm start: while capacity > 0, every Newton iteration of
 * bsc_newton_step appends its free-DOF gradient g and its PCG direction p (the solve of
 * H p = -g at the step's pcg_rtol) as floats, SoA [c][a], at d_g + 3*n_cp*k and d_p + 3*n_cp*k
 * for k = 0, 1, ... up to capacity samples. The caller owns both device buffers. capacity = 0
 * disables logging. bsc_sample_log_count returns how many samples have been written. */
bsc_status bsc_set_sample_log(bsc_ctx *ctx, float *d_g, float *d_p, int32_t capacity);
bsc_status bsc_sample_log_count(const bsc_ctx *ctx, int32_t *count);

/* Learned PCG warm start (a method extension; not in the paper). A bias-free 6-layer 3x3
 * convolutional net over the CP grid (3 -> 32 -> 32 -> 32 -> 32 -> 32 -> 3 channels, zero
 * padding, LeakyReLU(0.1) between layers) maps the normalised gradient g/rms(g) to a
 * direction p_hat; the step uses alpha* p_hat with alpha* = -g.p_hat / p_hat.H p_hat (the
 * energy-optimal multiple, of either sign) as the PCG initial guess when it lowers the 2-norm of
 * the residual, else zero.
 * Weights: BSC_NET_PARAMS floats, layer by layer, each [c_out][c_in][3][3]. */
#define BSC_NET_PARAMS 38592
bsc_status bsc_warmstart_load(bsc_ctx *ctx, const float *d_weights, int32_t n_params);

/* Network forward for a batch of B grids of the context's size (training and inference).
 *   d_in: B*3*n_cp floats [b][c][a]; d_out: B*3*n_cp floats; d_acts: B*5*32*n_cp floats,
 *   the outputs of layers 1..5 after LeakyReLU, layout [layer][b][channel][a], kept for the
 *   backward pass (NULL for inference only). d_weights: BSC_NET_PARAMS floats. */
bsc_status bsc_net_forward(bsc_ctx *ctx, int32_t batch, const float *d_weights, const float *d_in,
                           float *d_out, float *d_acts);

/* Network backward: given d_dout (dLoss/dOut, B*3*n_cp floats) and the d_acts saved by the
 * forward, writes dLoss/dWeights (BSC_NET_PARAMS floats, overwritten, deterministic) and, if
 * d_din is not NULL, dLoss/dIn. d_scratch: bsc_net_scratch_size() bytes. */
bsc_status bsc_net_backward(bsc_ctx *ctx, int32_t batch, const float *d_weights, const float *d_in,
                            const float *d_acts, const float *d_dout, float *d_dweights, float *d_din,
                            void *d_scratch);
bsc_status bsc_net_scratch_size(const bsc_ctx *ctx, int32_t batch, size_t *bytes);

/* bsc_net_backward without the d_scratch argument, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight training or serving loops, harnesses that forbid
 * hipMalloc). Same arguments, kernels and results as bsc_net_backward; the scratch is a static
 * device array of BSC_NET_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends. Calls no
 * hipMalloc, hipFree or allocating library routine.
 *   Limit: bsc_net_scratch_size(ctx, batch) must not exceed BSC_NET_NOALLOC_SCRATCH_BYTES
 *   (32 MiB: a 226 x 226 grid at batch 1, a 128 x 128 grid up to batch 5); larger requests return
 *   BSC_E_INVAL before anything is enqueued.
 *   Every call on one GPU shares that GPU's array and leaves its contents behind (the kernels
 *   overwrite every byte they read, so nothing needs clearing): calls that overlap on one GPU,
 *   from any context or stream, race. Asynchronous on the context's stream. */
#define BSC_NET_NOALLOC_SCRATCH_BYTES (32u << 20)
bsc_status bsc_net_backward_noalloc(bsc_ctx *ctx, int32_t batch, const float *d_weights, const float *d_in,
                                    const float *d_acts, const float *d_dout, float *d_dweights, float *d_din);

/* Adam update of n parameters in place (step counter t >= 1). */
bsc_status bsc_adam_step(bsc_ctx *ctx, int32_t n, float *d_param, const float *d_grad, float *d_m,
                         float *d_v, float lr, float beta1, float beta2, float eps, int32_t t);

/* Training loss of the warm-start net for a batch: for each sample b, over the CPs where the
 * network input d_in is not zero in all three components (pinned CPs have a zero gradient),
 * L_b = 1 - (p_hat.p)^2 / (|p_hat|^2 |p|^2), the squared relative error of the best scalar
 * multiple of p_hat against the solved step p. Writes the mean loss (1 float, device) and
 * dL/dp_hat (B*3*n_cp floats, zero on masked CPs). */
bsc_status bsc_net_loss(bsc_ctx *ctx, int32_t batch, const float *d_in, const float *d_pred,
                        const float *d_target, float *d_loss, float *d_dpred);

/* ---- Contact Hessian conversion (Sec. 4.3 contact barrier; Sec. 5.2 Alg. "Contact Hessian
 * conversion and assembly") ---------------------------------------------------------------
 * A triangle contact mesh is embedded in the surface: vertex a has fixed parametric coordinates,
 * so its position is sum_ij N_ij(u_a, v_a) C^{ij} over the 9 CPs of its span (Eq. "trig mesh node
 * from control points"). A contact model (not part of this library) gives, per contact pair of
 * 2 to 4 mesh vertices, the Hessian and gradient of its energy with respect to those vertices.
 * The conversion applies the chain rule (Eq. "gradient and hessian of contact barrier"; the
 * second-derivative term vanishes because vertices are linear in the CPs):
 *   H_CP(i, j) = sum over vertex pairs (a, b) of w_a(i) w_b(j) H(a, b),  g_CP(i) = sum_a w_a(i) g_a.
 *
 * bsc_contact_setup: host, synchronous. n_vert vertices at uv (host, 2*n_vert doubles, (u, v) per
 *   vertex in the units of the knot vectors given to bsc_create, inside the parameter
 *   rectangle). max_pairs (1..2^20) bounds n_pairs per call; max_vpairs bounds the distinct
 *   vertex pairs per call (0: 16*max_pairs, the worst case). Sizes the contact workspace, which
 *   grows by about 40 bytes x 81 per vertex pair of capacity. Replaces any earlier setup.
 * bsc_contact_workspace_size / bsc_contact_bind_workspace: caller-owned device memory (256-byte
 *   aligned) for the vertex tables and the sort buffers; binding uploads the tables and
 *   synchronises the context's stream.
 * bsc_contact_hessian: converts n_pairs contact pairs (0..max_pairs).
 *   d_pair_verts: device, 4*n_pairs int32 vertex indices per pair; -1 marks an unused slot.
 *   d_pair_hess: device, 144*n_pairs doubles: the 12x12 Hessian of each pair over (slot, xyz),
 *     row-major, row 3*s + k; rows and columns of unused slots are ignored.
 *   d_pair_grad: device, 12*n_pairs doubles (slot, xyz), or NULL.
 *   Outputs (device, caller-owned): d_row_ptr (n_cp+1), d_col_idx (cap_blocks) and d_vals
 *   (9*cap_blocks, row-major 3x3 per block): the CP Hessian as block CSR with both triangles,
 *   columns ascending in each row, one block per CP pair reached by a nonzero weight product;
 *   *nnzb (host) the block count; d_grad (3*n_cp, SoA like the state, or NULL) the CP gradient.
 *   Enqueued on the context's stream; synchronises it twice (the sizes of the two sorts). The
 *   result is bitwise reproducible. BSC_E_INVAL for a vertex index outside [-1, n_vert);
 *   BSC_E_NOMEM if the distinct vertex pairs exceed max_vpairs or the blocks exceed cap_blocks
 *   (then *nnzb holds the count needed). */
bsc_status bsc_contact_setup(bsc_ctx *ctx, int32_t n_vert, const double *uv, int32_t max_pairs, int32_t max_vpairs);
bsc_status bsc_contact_workspace_size(const bsc_ctx *ctx, size_t *bytes);
bsc_status bsc_contact_bind_workspace(bsc_ctx *ctx, void *d_ws, size_t bytes);
bsc_status bsc_contact_hessian(bsc_ctx *ctx, int32_t n_pairs, const int32_t *d_pair_verts, const double *d_pair_hess,
                               const double *d_pair_grad, int32_t cap_blocks, int32_t *d_row_ptr, int32_t *d_col_idx,
                               double *d_vals, int32_t *nnzb, double *d_grad);

/* ---- Partial factorization (Sec. 5.3, Eq. "per iteration solve", Eq. "Woodbury", Eq. "Neumann
 * expansion", the Gershgorin bound) ------------------------------------------------------------
 * Solves the Newton system with a contact Hessian, (H + H_c) x = b.
 *   H: d_hess, the inertia-plus-elasticity Hessian in upper-stencil form and the given precision,
 *     as bsc_assemble writes it (pinned CPs with identity diagonal blocks); H_c: the contact
 *     (barrier) Hessian in block CSR with both triangles, as bsc_contact_hessian writes it
 *     (d_row_ptr: n_cp + 1 ints with d_row_ptr[n_cp] == nnzb, d_col_idx: nnzb ints in
 *     [0, n_cp), d_vals: 9 nnzb doubles, row-major 3x3 per block); H_c must be positive
 *     semi-definite (as a projected barrier Hessian is). dt: the step, for the lumped inertia
 *     M_a / dt^2 in the bound. d_b, d_x: 3 n_cp doubles (SoA), distinct.
 * Split: H_c = (its 3x3 CP self-blocks) + B; D = H + self-blocks keeps the stencil pattern.
 * Rows and columns of H_c at pinned CPs are dropped. Trigger: rho = max_i sum_j |B_ij| /
 * min over free CPs of (M_a / dt^2 + max(0, Gershgorin lower bound of H_c[a, a])) bounds
 * |D^-1 B|_op (H's elastic part and H_c are PSD). If rho <= rho_max (and < 1), the Neumann series
 * x = sum_{k<=K} (-D^-1 B)^k D^-1 b with K the smallest integer such that rho^(K+1)/(1-rho) <=
 * series_tol (at most max_terms terms), each D^-1 by the fused block-Jacobi stencil PCG to
 * pcg_rtol; else PCG on D + B (block Jacobi on D's diagonal blocks) to pcg_rtol. force: 0 lets
 * the bound decide, 1 takes the series (max_terms terms if rho >= 1), 2 the merged solve.
 * Uses the workspace's Hessian buffer and solver vectors (overwrites what bsc_assemble or
 * bsc_newton_step left there); d_hess must be a caller buffer. Synchronous. BSC_E_INVAL for a
 * column index outside [0, n_cp) or d_row_ptr[n_cp] != nnzb; BSC_E_PCG_BREAKDOWN if an inner
 * solve meets p^T A p <= 0. */
typedef struct {
    double rho_max;        /* trigger threshold of the bound (e.g. 0.5) */
    double series_tol;     /* truncation target of the series (e.g. 1e-12) */
    int32_t max_terms;     /* 1..1000 */
    double pcg_rtol;       /* relative residual of every inner and merged PCG solve */
    int32_t max_pcg;       /* iterations per PCG solve */
    int32_t force;         /* 0 bound decides, 1 series, 2 merged */
} bsc_pf_opts;
typedef struct {
    int32_t triggered, terms, pcg_iters;     /* series taken; terms summed; PCG iterations in all */
    double rho_bound, b_bound, d_bound;      /* the bound, its numerator and denominator */
    double ms_total;                         /* host wall-clock time of the call */
} bsc_pf_stats;
bsc_status bsc_contact_solve(bsc_ctx *ctx, int32_t precision, const void *d_hess, double dt, const int32_t *d_row_ptr,
                             const int32_t *d_col_idx, const double *d_vals, int32_t nnzb, const double *d_b,
                             double *d_x, const bsc_pf_opts *opts, bsc_pf_stats *stats);

const char *bsc_status_string(bsc_status s);
const char *bsc_last_error(const bsc_ctx *ctx);
void bsc_destroy(bsc_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* BSC_H */
