/*
 * librgp: reversed-gradient-polarity (RGP) susceptibility-distortion correction on one MI355X.
 *
 * C ABI of the hot path of PyHySCO (Julian and Ruthotto): column-wise 1D optimal-transport
 * initialisation, objective and gradient of the discretised problem, Gauss-Newton
 * Hessian-vector products, Jacobi-preconditioned CG, and the coarse-to-fine Gauss-Newton solve
 * that ends in the Jacobian-modulation correction.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Volumes are C-contiguous [m0][m1][m2] arrays in DEVICE memory owned by the caller.  Images
 *    are cell-centred (m0*m1*m2 values).  The field map b and every vector of the Gauss-Newton
 *    solve live on the staggered grid of Sec. 2.1: cell centres across the phase-encoding (PE)
 *    axis and nodes along it, i.e. shape [m0][m1][m2] with m[pe] replaced by m[pe] + 1.
 *  - "field" arrays (b, gradients, Hessian data, PCG vectors) have the arithmetic type
 *    (RGP_F64 or RGP_F32); images may also be RGP_BF16 (storage only; arithmetic stays in the
 *    field type).  Inner products and reductions are always accumulated in FP64.
 *  - Scalars produced on the device (J, iteration counts, ...) are written to caller-owned
 *    DEVICE memory; no call synchronises the host.  Every call is enqueued on `stream` (a
 *    hipStream_t; NULL is the default stream) and returns as soon as the work is enqueued.
 *  - `ws`/`ws_bytes` is a caller-owned device workspace of at least rgp_workspace_size() bytes,
 *    256-byte aligned and ZERO-FILLED before its first use; the library keeps the parts it relies
 *    on at zero between calls, so a workspace can be reused by any entry point afterwards.  The
 *    library never allocates device memory.  Calls that share a workspace must not overlap.
 *  - Argument errors are reported synchronously through the return value; nothing is enqueued
 *    then.  A violated barrier (|d b / d v| >= 1 somewhere) is a value, J = +inf, not an error.
 */
#ifndef RGP_H
#define RGP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RGP_OK = 0,
  RGP_EINVAL = -1,      /* null pointer, bad option value or enum */
  RGP_ESHAPE = -2,      /* grid extents out of range */
  RGP_EDTYPE = -3,      /* unsupported dtype combination */
  /* The next three are found on the device while a correction runs, so they are never returned
   * by a call: the solve reports the first of them in its stats header (RGP_STAT_HEADER). */
  RGP_ENONFINITE = -4,  /* an input image holds a NaN or an infinity: no Gauss-Newton step is
                           taken on any level, and the initial field is zero (OT) or b_init */
  RGP_EBARRIER = -5,    /* a level started from a field with |d b / d v| >= 1 somewhere, where the
                           barrier of Eq. (3) is infinite (a caller's b_init, or an OT field with
                           the guard off): that level stops with b unchanged */
  RGP_ELINESEARCH = -6, /* no Armijo trial was accepted in some Gauss-Newton step (Sec. 2.3.1):
                           that level stops with b unchanged; later levels still run */
  RGP_EHIP = -7,        /* a HIP runtime call failed (see rgp_last_hip_error) */
  RGP_EWORKSPACE = -8   /* workspace missing or smaller than rgp_workspace_size() */
} rgp_status;

typedef enum { RGP_F64 = 0, RGP_F32 = 1, RGP_BF16 = 2 } rgp_dtype;

/* Grid of one volume.  m: cells per axis (caller order, each >= 1, m[pe] >= 2, at most 2^28
 * field nodes, and at most 512 field nodes along the contiguous axis m[2], i.e. m[2] <= 512, or
 * m[2] <= 511 when pe == 2; other grids give RGP_ESHAPE); pe: phase-encoding axis 0..2; h: voxel
 * sizes (> 0).  b is measured in the units of h. */
typedef struct {
  int64_t m[3];
  int32_t pe;
  int32_t reserved;
  double h[3];
} rgp_grid;

/* Per-level optimiser of the full solve. */
typedef enum {
  RGP_SOLVER_GN = 0,    /* Gauss-Newton with Jacobi-preconditioned CG (Sec. 2.3.1), the default */
  RGP_SOLVER_LBFGS = 1, /* L-BFGS on the explicit gradient (Sec. 2.3.3) */
  RGP_SOLVER_ADMM = 2   /* ADMM with column-parallel PCG and a transform z-update (Sec. 2.3.2) */
} rgp_solver;

/* Options of the full solve (rgp_correct).  rgp_default_opts() fills the paper's defaults. */
typedef struct {
  double alpha;          /* smoothness weight (300 in Sec. 2.1) */
  double beta;           /* barrier weight (1e-4 in Sec. 2.1) */
  int32_t levels;        /* pyramid levels, >= 1; coarse-to-fine */
  int32_t gn_iters;      /* Gauss-Newton iterations per level, >= 0 */
  int32_t pcg_iters;     /* PCG iterations per GN step, 1..1000 (10 in Sec. 2.3.1) */
  int32_t ls_max_trials; /* Armijo trials gamma = 1, 1/2, ..., at most 10 */
  double pcg_rtol;       /* PCG stops when |r|/|grad J| < pcg_rtol (0.1 in Sec. 2.3.1; 0 = never) */
  double armijo_c;       /* sufficient-decrease constant (1e-4) */
  double ot_eps;         /* positivity shift of the OT init: eps * max|I| (1e-3) */
  int32_t ot_guard;      /* clip OT slopes to +-0.99 and re-integrate (1) */
  int32_t use_b_init;    /* 1: start from b_init on the coarsest level instead of OT */
  int32_t ot_blur;       /* 1: blur the OT field (rgp_blur_field) before the first GN step (0) */
  int32_t solver;        /* rgp_solver (RGP_SOLVER_GN) */
  int32_t lbfgs_memory;  /* RGP_SOLVER_LBFGS: curvature pairs kept, 1..32 (10).  With L-BFGS,
                            gn_iters counts L-BFGS steps per level; pcg_iters and pcg_rtol are
                            not used.  A step's direction is -H g by the two-loop recursion with
                            H0 = (s^T y / y^T y) I of the newest pair, a pair is kept only when
                            s^T y > 1e-10 |s| |y|, and a step without pairs (the first of every
                            level) takes d = -g / max|g|; the step size is the Armijo search of
                            the Gauss-Newton solve.  In a stats record the PCG iteration field
                            holds the pairs used and the PCG residual field holds H0's scale
                            (1 / max|g| without pairs). */
  int32_t batch_march;   /* batched corrections (rgp_correct_batch_plan, rgp_correct_batch), 0..64:
                            0 (the default) gives every pair's PCG launches the plane march of
                            its own rgp_correct, so a pair's field is bitwise its solo result;
                            N > 0 makes each batched PCG step march at least min(N, planes)
                            planes per work unit (fewer, longer units: a batch has units to
                            spare on coarse levels, where a solo plan keeps them short to fill
                            the chip), which reorders the FP64 block sums of the PCG scalars, so
                            a pair's field then agrees with its solo one to rounding only.
                            Ignored by the single-pair calls.  Else RGP_EINVAL. */
  double admm_rho0;      /* RGP_SOLVER_ADMM: initial augmentation parameter rho on every level
                            (<= 0: alpha).  With ADMM, gn_iters counts ADMM iterations per level,
                            each one Gauss-Newton step on F(b) + (rho vol / 2)|b - z + u|^2 with
                            F = D + alpha S_PE + beta P (the search direction by Jacobi PCG on
                            every PE column independently: pcg_iters iterations at most, a
                            column stopping at relative residual pcg_rtol), then
                            z = argmin alpha (S_A + S_B)(z) + (rho vol / 2)|b - z + u|^2 with
                            periodic differences across the PE axis, u += b - z, and rho doubled
                            (u halved) when |b - z| > 10 rho |z - z_old|, halved (u doubled) when
                            rho |z - z_old| > 10 |b - z|.  z = b, u = 0 at the start of every
                            level; b is the result.  In a stats record S holds
                            S_PE + (rho / alpha)(vol / 2)|b - z + u|^2 (J = D + alpha S + beta P is
                            the b-update's objective), the PCG fields the largest column
                            iteration count and relative residual, and field 11 the rho used.
                            Supports at most 512 field nodes along PE and 1024 along the other
                            axes (else RGP_ESHAPE). */
} rgp_solver_opts;

/* Number of doubles per Gauss-Newton record in the stats buffer of rgp_correct. */
#define RGP_STAT_FIELDS 12
/* Stats buffer layout: [0] OT guarded cells, [1] OT shift, [2] status of the solve (0, or the
 * first of RGP_ENONFINITE, RGP_EBARRIER, RGP_ELINESEARCH that happened), [3] reserved, then one
 * record of RGP_STAT_FIELDS doubles per GN step, coarsest level first:
 * J, D, S, P, |grad J|, grad.q, PCG iterations, PCG relative residual, gamma, Armijo trials,
 * accepted (0/1), reserved.  Records of steps that did not run (the solve stopped) are NaN. */
#define RGP_STAT_HEADER 4

typedef enum {
  RGP_OP_OT_INIT = 0,
  RGP_OP_LOSS_GRAD = 1,
  RGP_OP_GN_HVP = 2,
  RGP_OP_PCG_SOLVE = 3,
  RGP_OP_CORRECT = 4,
  RGP_OP_APPLY_CORRECTION = 5
} rgp_op;

const char* rgp_status_string(rgp_status s);
/* Last HIP error code seen by the library on this thread (0 if none). */
int rgp_last_hip_error(void);
void rgp_default_opts(rgp_solver_opts* o);

/* Workspace bytes needed by `op` on `grid` (opts is read for RGP_OP_CORRECT and
 * RGP_OP_PCG_SOLVE only; real_t is the field type).  Writes *bytes. */
rgp_status rgp_workspace_size(rgp_op op, const rgp_grid* grid, rgp_dtype real_t,
                              const rgp_solver_opts* opts, size_t* bytes);

/* Column-wise 1D optimal-transport initialisation (Sec. 2.2, and Fig. 2).
 * Per PE column: images shifted positive by s = max(0, -min I) + ot_eps * max|I| (one global
 * scalar over both images), nodal CDFs C+ and C- (FP64 scans), linear-spline pseudo-inverses,
 * and b0_k = h_pe/4 [C+^{-1}(C-_k) - C-^{-1}(C+_k)] - the average of the displacement of the
 * halfway map T- and the negated displacement of T+.  Columns with no mass get b0 = 0, and so
 * does every column when an image holds a NaN or an infinity.  If
 * `guard` is set, a column whose slope |D b0| exceeds 0.99 somewhere gets its slopes clipped to
 * +-0.99 and is re-integrated from b0_0 = 0; the number of clipped cells is written to
 * *n_guarded_dev (nullable, uint64 on the device).  b0: field array (real_t) written in full.
 * Columns of more than 8192 cells along the PE axis give RGP_ESHAPE (the correction entry points:
 * on the coarsest level, unless the correction starts from a given field). */
rgp_status rgp_ot_init(const rgp_grid* grid, rgp_dtype img_t, const void* I_plus,
                       const void* I_minus, rgp_dtype real_t, void* b0, double ot_eps,
                       int32_t guard, uint64_t* n_guarded_dev, void* ws, size_t ws_bytes,
                       void* stream);

/* Optional smoothing of an OT initial field (Sec. 2.2, last step; Sec. 2.4, the OT
 * initialisation's blurring operator): b_out = G * b_in with the 3x3x3 Gaussian of standard
 * deviation 1 voxel, weights exp(-|d|^2/2) over the offsets d in {-1,0,1}^3 normalised to sum 1,
 * periodic over the node grid of `grid` (the paper applies it as an FFT convolution, which
 * wraps around).  b_in, b_out: distinct device field arrays of real_t (RGP_F32 or RGP_F64; b_in ==
 * b_out gives RGP_EINVAL).  Enqueued on `stream`; needs no workspace. */
rgp_status rgp_blur_field(const rgp_grid* grid, rgp_dtype real_t, const void* b_in, void* b_out,
                          void* stream);

/* Restriction of one image to the next coarser level of the multilevel pyramid that the
 * coarse-to-fine scheme solves on (Sec. 3.4; the same transfer rgp_correct applies between its
 * levels): coarse cell c is the mean of the existing fine cells of its 2x2x2 block, ceil(m/2)
 * cells per axis.  `grid` describes the FINE image; only its m is read (pe and h are ignored).
 * src: device cell array of img_t in the fine shape; dst: device cell array of real_t in the
 * coarse shape, written in full; distinct buffers.  Summed in FP64 and rounded once to real_t.
 * Types as for rgp_loss_grad (img_t == real_t, or RGP_BF16 images with an RGP_F32 or RGP_F64
 * result, or RGP_F32 images with an RGP_F64 result).  Enqueued on `stream`; no workspace. */
rgp_status rgp_restrict_image(const rgp_grid* grid, rgp_dtype img_t, const void* src,
                              rgp_dtype real_t, void* dst, void* stream);

/* Adjoint of rgp_restrict_image, for gradients taken through the pyramid (differentiation
 * extension): fine cell f receives g_coarse at its coarse cell divided by the number of existing
 * fine cells of that cell's block (1, 2, 4 or 8).  `grid` describes the FINE image (only m is
 * read).  g_coarse: device cell array of real_t (RGP_F32 or RGP_F64) in the coarse shape;
 * g_fine: device cell array of real_t in the fine shape, overwritten, or added to when
 * accumulate != 0; distinct buffers.  Enqueued on `stream`; no workspace. */
rgp_status rgp_restrict_image_adjoint(const rgp_grid* grid, rgp_dtype real_t,
                                      const void* g_coarse, void* g_fine, int32_t accumulate,
                                      void* stream);

/* Objective J = D + alpha S + beta P of Eq. (6) at b, with D the SSD of the mass-preserving
 * transforms of Eq. (1)-(2), S the smoothness term of Eq. (5) (seven-point negative Laplacian on
 * the staggered field, Neumann boundaries) and P the barrier of Eq. (3); all with weight vol/2.
 * jdsp_dev (device, 4 doubles, nullable): J, D, S, P (J = P = +inf when the barrier is violated).
 * Optional outputs (field arrays, nullable): grad = grad J; hdiag/hoff = the Gauss-Newton
 * Hessian of Sec. 2.3.1 in banded form - hdiag its diagonal (the Jacobi preconditioner) and
 * hoff[k] the coupling of PE nodes k and k+1 (0 at the last node); the cross-axis couplings are
 * -alpha vol / h_d^2.  hdiag and hoff are both given or both NULL.  Their contents are
 * unspecified when J = +inf. */
rgp_status rgp_loss_grad(const rgp_grid* grid, rgp_dtype img_t, const void* I_plus,
                         const void* I_minus, rgp_dtype real_t, const void* b, double alpha,
                         double beta, double* jdsp_dev, void* grad, void* hdiag, void* hoff,
                         void* ws, size_t ws_bytes, void* stream);

/* rgp_loss_grad without a workspace, for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments,
 * outputs and arithmetic as rgp_loss_grad (bitwise the same results), minus ws/ws_bytes: the
 * state block and the per-block FP64 sums live in a fixed library-owned device array of
 * 512.25 KiB per GPU (one copy on each device the library runs on, held until the process
 * ends), looked up on the first call on each device.  The call allocates nothing and needs the
 * stream's device to be the current device.  Every call on a GPU uses that GPU's one array, so
 * calls that overlap on one GPU (two streams, two threads, or a concurrent capture replay) race
 * and must be serialised by the caller; each call writes all of the array it reads, so nothing
 * needs clearing between calls.  Errors as rgp_loss_grad; RGP_EWORKSPACE if a launch would need
 * more block sums than the array holds (not reachable with the current launch plans), RGP_EHIP
 * if the array's device address cannot be obtained. */
rgp_status rgp_loss_grad_noalloc(const rgp_grid* grid, rgp_dtype img_t, const void* I_plus,
                                 const void* I_minus, rgp_dtype real_t, const void* b,
                                 double alpha, double beta, double* jdsp_dev, void* grad,
                                 void* hdiag, void* hoff, void* stream);

/* Gauss-Newton Hessian-vector product Hv = H_J v (Sec. 2.3.1, Eq. 7) with H_J given by the
 * hdiag/hoff produced by rgp_loss_grad at the same grid and alpha.  vHv_dev (nullable, device
 * double) receives v^T H v. */
rgp_status rgp_gn_hvp(const rgp_grid* grid, rgp_dtype real_t, const void* hdiag,
                      const void* hoff, double alpha, const void* v, void* Hv, double* vHv_dev,
                      void* ws, size_t ws_bytes, void* stream);

/* Jacobi-preconditioned CG for H_J x = rhs from x0 = 0 (Sec. 2.3.1): at most maxit iterations,
 * stopping early when |r| / |rhs| < rtol or when p^T H p <= 0.  x: field array written in full.
 * iters_dev (int32) and relres_dev (double): device outputs, nullable. */
rgp_status rgp_pcg_solve(const rgp_grid* grid, rgp_dtype real_t, const void* hdiag,
                         const void* hoff, double alpha, const void* rhs, void* x, int32_t maxit,
                         double rtol, int32_t* iters_dev, double* relres_dev, void* ws,
                         size_t ws_bytes, void* stream);

/* Gradient of the objective with respect to the two images (only the distance term of Eq. 2
 * depends on them): dJ/dI+ = vol A+^T (r (1 + d_v b)) and dJ/dI- = -vol A-^T (r (1 - d_v b)),
 * where A+- is the 1D linear interpolation at x +- b v (zero outside the column) and
 * r = T+ - T- the residual of Eq. 1.  The backward of the objective with respect to I+-
 * (differentiation extension).  gI_plus/gI_minus: cell arrays of real_t (both required), written
 * in full.  Needs |d_v b| < 1 everywhere (then the sample positions are monotone along every
 * column and each output value is accumulated by one thread without atomics); otherwise the
 * output is unspecified (finite writes only, in bounds). */
rgp_status rgp_loss_grad_images(const rgp_grid* grid, rgp_dtype img_t, const void* I_plus,
                                const void* I_minus, rgp_dtype real_t, const void* b,
                                void* gI_plus, void* gI_minus, void* stream);

/* Jacobian-modulation correction (Sec. 2.4.7): T+ = I+(x + b v)(1 + d_v b) and
 * T- = I-(x - b v)(1 - d_v b) at the cell centres, with the 1D linear image model (zero outside
 * the column).  T_plus/T_minus: arrays of img_t (nullable). */
rgp_status rgp_apply_correction(const rgp_grid* grid, rgp_dtype img_t, const void* I_plus,
                                const void* I_minus, rgp_dtype real_t, const void* b,
                                void* T_plus, void* T_minus, void* stream);

/* Least-squares correction (Sec. 2.4.7): one corrected image from both inputs and the field.
 * Per PE column the field defines the push-forward matrices M+ and M- that carry a true image to
 * the two distorted ones - the mass-conserving remap of the distortion model: true cell j (between
 * the nodes x_j and x_{j+1}) moves to [x_j +- b_j, x_{j+1} +- b_{j+1}], its mass spread evenly
 * there and integrated over the output cells, mass leaving the column lost - and I_out minimises
 * |M+ I - I+|^2 + |M- I - I-|^2, found by CGLS from I = 0: at most maxit (1..100000)
 * iterations, a column stopping when |M^T r| < rtol |M^T [I+; I-]| or when its search direction
 * vanishes.  I_out: cell array of img_t (written in full); iters_dev: nullable device int32 array
 * of one count per column, columns numbered by their two cross-axis indices in the arrays' order
 * (slower axis first).  Needs |d_v b| < 1 (else the output is unspecified, finite writes only).
 * Columns of more than 2340 cells (FP32 field) or 1170 cells (FP64) give RGP_ESHAPE.  Enqueued on
 * `stream`; needs no workspace. */
rgp_status rgp_correct_lsq(const rgp_grid* grid, rgp_dtype img_t, const void* I_plus,
                           const void* I_minus, rgp_dtype real_t, const void* b, int32_t maxit,
                           double rtol, void* I_out, int32_t* iters_dev, void* stream);

/* The whole hot path: image pyramid (2x2x2 means, `levels` levels), OT initialisation on the
 * coarsest level (or b_init there when opts->use_b_init; b_init has the coarsest level's
 * staggered shape), then on every level from coarse to fine `gn_iters` Gauss-Newton steps
 * b <- b + gamma q with H_J q = -grad J solved by `pcg_iters` PCG iterations and gamma chosen by
 * Armijo backtracking (Sec. 2.3.1), linear prolongation of b between levels, and finally the
 * Jacobian-modulation correction of the finest images.  A step that no trial accepts stops the
 * level with b unchanged.  b_out: finest field (real_t); T_plus/T_minus (nullable, img_t);
 * stats_dev: nullable device buffer of RGP_STAT_HEADER + levels*gn_iters*RGP_STAT_FIELDS
 * doubles.  Failures found on the device (a non-finite input, a level starting outside the
 * barrier, a failed line search: RGP_ENONFINITE, RGP_EBARRIER, RGP_ELINESEARCH) do not abort:
 * the first one is written to stats_dev[2], and b_out is still written. */
rgp_status rgp_correct(const rgp_grid* grid, rgp_dtype img_t, const void* I_plus,
                       const void* I_minus, rgp_dtype real_t, const rgp_solver_opts* opts,
                       const void* b_init, void* b_out, void* T_plus, void* T_minus,
                       double* stats_dev, void* ws, size_t ws_bytes, void* stream);

/* Captured solve: the whole sequence of rgp_correct (same arguments, same buffers) recorded once
 * into a HIP graph on `stream` (a non-default hipStream_t), so that rgp_plan_launch replays the
 * entire correction with one launch.  Every replay recomputes from the current contents of the
 * input buffers and overwrites the outputs; the buffers and the workspace must stay alive and
 * unchanged in size until rgp_plan_destroy.  For callers that repeat one correction shape (a
 * serving loop, a benchmark). */
typedef struct rgp_plan_s* rgp_plan;
rgp_status rgp_correct_plan(const rgp_grid* grid, rgp_dtype img_t, const void* I_plus,
                            const void* I_minus, rgp_dtype real_t, const rgp_solver_opts* opts,
                            const void* b_init, void* b_out, void* T_plus, void* T_minus,
                            double* stats_dev, void* ws, size_t ws_bytes, void* stream,
                            rgp_plan* plan);
rgp_status rgp_plan_launch(rgp_plan plan, void* stream);
rgp_status rgp_plan_destroy(rgp_plan plan);

/* Batched correction (batching extension): n volume pairs of their own shapes, PE axes and
 * buffers corrected by one captured HIP graph (replayed with rgp_plan_launch) in which every
 * Gauss-Newton kernel - loss_grad, the PCG scalar phase and steps, the Armijo passes and
 * decisions, the step update - is ONE launch covering all pairs, each pair's workgroups reading
 * their arguments from a table in the workspace; the pyramid, OT, prolongation and correction
 * kernels run pair by pair inside the same graph.  Per pair the arithmetic is that of
 * rgp_correct (same options for all pairs; use_b_init must be 0; at most 1024 pairs; the
 * contiguous field axis of every pair at most 256 nodes, else RGP_ESHAPE).  I_plus, I_minus,
 * b_out: host arrays of n device pointers; T_plus, T_minus, stats_dev: NULL or host arrays of n
 * device pointers (all entries non-NULL).  ws: one zero-filled workspace of at least
 * rgp_batch_workspace_size bytes holding every pair's workspace and the launch tables, which
 * this call writes (it synchronises `stream` once, to upload them, then captures on it).
 * Buffers and workspace must outlive the plan. */
rgp_status rgp_batch_workspace_size(int32_t n, const rgp_grid* grids, rgp_dtype real_t,
                                    const rgp_solver_opts* opts, size_t* bytes);
rgp_status rgp_correct_batch_plan(int32_t n, const rgp_grid* grids, rgp_dtype img_t,
                                  const void* const* I_plus, const void* const* I_minus,
                                  rgp_dtype real_t, const rgp_solver_opts* opts,
                                  void* const* b_out, void* const* T_plus, void* const* T_minus,
                                  double* const* stats_dev, void* ws, size_t ws_bytes,
                                  void* stream, rgp_plan* plan);

/* The batched correction without a graph: the same arguments, launches and results as
 * rgp_correct_batch_plan followed by one rgp_plan_launch, enqueued directly on `stream` (each
 * Gauss-Newton kernel one launch over all pairs).  It synchronises `stream` once, to upload the
 * launch tables into ws, before it enqueues the correction (RGP_EINVAL while the stream is being
 * captured).  Launches are seen by a kernel-timing session (rgp_timing_start), each record
 * carrying the cells and nodes summed over the pairs. */
rgp_status rgp_correct_batch(int32_t n, const rgp_grid* grids, rgp_dtype img_t,
                             const void* const* I_plus, const void* const* I_minus,
                             rgp_dtype real_t, const rgp_solver_opts* opts, void* const* b_out,
                             void* const* T_plus, void* const* T_minus, double* const* stats_dev,
                             void* ws, size_t ws_bytes, void* stream);

/* Autotuner of the PCG tile shape (batching extension): for every pyramid level of `grid` under
 * `opts` (one level when opts is NULL) it times the candidate march lengths of the PCG step - a
 * work unit is 256 consecutive positions of the contiguous node plane times XL planes - on the
 * workspace's own vectors (a correction workspace; their contents are overwritten, the parts the
 * library relies on are left as rgp_correct needs them) and records the fastest in a
 * process-wide table that every later plain or batched launch on that geometry and field type
 * uses.  A candidate's figure is the median kernel duration of 9 timed launches (events taken at
 * each kernel's start and end; a timing session of rgp_timing_start does not see these launches).
 * Synchronises `stream`; RGP_EINVAL while the stream is being captured.  xl_out: host
 * array of opts->levels int32 (nullable) receiving the chosen XL per level, finest first. */
rgp_status rgp_autotune(const rgp_grid* grid, rgp_dtype real_t, const rgp_solver_opts* opts,
                        void* ws, size_t ws_bytes, void* stream, int32_t* xl_out);

/* Kernel timing (instrumentation; not part of the method).  rgp_timing_start(capacity) creates
 * `capacity` pairs of HIP events (host API objects, no device memory) and from then on every
 * launch of a hot kernel that is not being captured into a graph records one pair at the start
 * and the end of the kernel itself (hipExtLaunchKernelGGL), until the pairs run out.
 * rgp_timing_stop() ends the recording, waits for the recorded events, writes up to `max`
 * records (in launch order) to the HOST array `out`, stores their number in *n and releases the
 * events.  `kernel` is an rgp_kernel_kind; `cells`/`nodes` give the volume the launch covered
 * (cells of the images, nodes of the field; 0 when not applicable).  Not thread-safe against
 * concurrent launches from other threads' timing sessions: one session per process at a time.
 * Errors: RGP_EINVAL (capacity < 1 or > 1<<20; out or n null), RGP_EHIP (event calls). */
typedef enum {
  RGP_KERNEL_PCG_STEP = 0,   /* one Jacobi-PCG iteration (Sec. 2.3.1) incl. w = H p */
  RGP_KERNEL_LOSS_GRAD = 1,  /* objective, gradient and GN Hessian diagonals (Sec. 2.3) */
  RGP_KERNEL_TRIAL = 2,      /* Armijo trial objectives */
  RGP_KERNEL_HVP = 3,        /* stand-alone GN Hessian-vector product */
  RGP_KERNEL_OT = 4,         /* column-wise optimal-transport initialisation (Sec. 2.2) */
  RGP_KERNEL_SHIFT = 5,      /* positivity shift of the OT initialisation */
  RGP_KERNEL_BLUR = 6,       /* optional Gaussian blur of the OT field */
  RGP_KERNEL_DHT = 7,        /* ADMM z-update: one Hartley pass along a cross axis (Sec. 2.3.2) */
  RGP_KERNEL_BLOCK_PCG = 8,  /* ADMM b-update: per-column Jacobi PCG (Sec. 2.3.2) */
  RGP_KERNEL_LBFGS = 9,      /* L-BFGS direction, one of its three phases (Sec. 2.3.3) */
  RGP_KERNEL_LSQ = 10        /* least-squares correction, CGLS per column (Sec. 2.4.7) */
} rgp_kernel_kind;
typedef struct {
  int32_t kernel;
  int32_t tag;       /* PCG step: the PCG iteration (0 = first); trial: candidates; loss_grad:
                        1 when it also applies the previous step; Hartley pass: the pass mode
                        (0 first, 1 scaling, 2 plain, 3 last) + 4 x the transform length; block
                        PCG: the iteration limit; L-BFGS: the phase (0 pair and inner products,
                        1 scalar recursion, 2 combination); else 0 */
  uint32_t grid;     /* workgroups */
  uint32_t pad;
  int64_t cells;
  int64_t nodes;
  double ms;         /* kernel duration */
} rgp_timing_record;
rgp_status rgp_timing_start(int32_t capacity);
rgp_status rgp_timing_stop(rgp_timing_record* out, int32_t max, int32_t* n);

#ifdef __cplusplus
}
#endif

#endif /* RGP_H */
