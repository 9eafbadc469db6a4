/*
 * vps.h -- C ABI of the MI355X vertex-patch multigrid library (libvps.so).
 *
 * Method: Wichrowski, Munch, Kronbichler, Kanschat, "Smoothers with localized
 * residual computations for geometric multigrid methods" (arXiv 2407.02100).
 * The library solves A u = b (Section 2, eq:matrix) for the Q_k Laplacian
 * -div(rho grad u) = f on [0,1]^d, d in {2,3}, homogeneous Dirichlet data
 * (Appendix A.2), uniform Cartesian meshes with N cells per direction, by CG
 * preconditioned with a geometric-multigrid V-cycle whose smoother is the
 * multiplicative vertex-patch smoother (Section 2.1, eq:s-ell) in its
 * combined, colorized form (Section 3.2, Algorithm 4): per color, every patch
 * gathers its closure, computes its local residual (eq:main:4), applies the
 * fast-diagonalization inverse (Appendix A.3, eq:fdm:inverse) and scatters the
 * update of its interior (eq:scatter).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Vectors.  A level with N_l cells per direction stores the full nodal grid of
 *   n_l = (k*N_l + 1)^d values, x fastest (index = ix + n1*iy + n1^2*iz).
 *   Node positions inside a cell are the Gauss-Lobatto points of degree k.
 *   Dirichlet entries (any ix, iy, iz equal to 0 or n1-1) of inputs must be
 *   0; the library writes 0 to Dirichlet entries of every vector it outputs.
 * Memory.  Every vector pointer is a DEVICE pointer owned by the caller; the
 *   library never frees it.  Work vectors, level constants and the coarse
 *   solver belong to the context and are freed by vps_destroy.
 * Levels.  Level 0 is the coarsest (N_0 = N / 2^(n_levels-1) cells), level
 *   n_levels-1 the finest (N cells).
 * Patches.  One patch per interior vertex v in [1, N_l-1]^d, numbered
 *   lexicographically (x fastest).  Color of a patch: sum_e (v_e mod 2) 2^e.
 *   A patch has (2k+1)^d closure nodes and q^d = (2k-1)^d interior nodes.
 * Streams.  Every call enqueues its work on the context's HIP stream (given at
 *   creation, 0 = the null stream) and returns without synchronising, except
 *   vps_solve, vps_vcycle_iterate, vps_mlp_infer_patches and vps_sync, which
 *   synchronise.  Errors of asynchronous work surface at the next
 *   synchronising call.
 * Errors.  Argument errors are detected on the host before any work is
 *   enqueued; they return a negative vps_status and set the context's
 *   message (vps_last_error).  A context is not thread-safe.
 */
#ifndef VPS_H
#define VPS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vps_context vps_context;

typedef enum {
  VPS_OK = 0,
  VPS_E_ARG = -1,           /* invalid argument (null pointer, bad level, ...) */
  VPS_E_UNSUPPORTED = -2,   /* valid but unsupported configuration */
  VPS_E_HIP = -3,           /* a HIP runtime call failed */
  VPS_E_NOMEM = -4,         /* device allocation failed */
  VPS_E_NOT_CONVERGED = -5, /* solver hit maxit before the tolerance */
  VPS_E_NONFINITE = -6,     /* NaN or Inf met in a solver scalar */
  VPS_E_STATE = -7          /* call not valid in the context's current state */
} vps_status;

typedef enum { VPS_F64 = 0, VPS_F32 = 1 } vps_dtype;

typedef enum {
  VPS_COEF_CONST = 0,          /* rho = 1: exact FDM local solver */
  VPS_COEF_CELL_MEAN_FDM = 1,  /* rho per cell: residual with rho, FDM with patch mean of rho */
  VPS_COEF_CELL_LEARNED = 2,   /* as 1, each FDM eigenmode scaled by a per-patch factor */
  VPS_COEF_CELL_EXACT = 3      /* rho per cell, exact dense local solvers A_j(rho)^{-1} (eq:main:2),
                                  formed by vps_set_coefficient: the ceiling for any per-patch
                                  correction of the FDM inverse; Q2, 3D, FP64 V-cycle, whole
                                  colors (per color: the global residual, then the dense patch
                                  solves), 5.8 KB of device memory per patch */
} vps_coef;

/* Smoother algorithm: the two colorized forms of Section 3.2. */
typedef enum {
  VPS_ALG_COMBINED = 0,  /* Algorithm 4: per color, each patch forms its local residual from its closure */
  VPS_ALG_SEPARATED = 1  /* Algorithm 3: per color, the global residual b - A u, then the local solves;
                            3D, rho = 1, degree 2..4 */
} vps_algorithm;

typedef struct {
  int dim;               /* 2 or 3 */
  int degree;            /* k, 1..5 (5: 3D smoother on the generic kernel, 3D operator and
                            transfers always on the streaming kernels) */
  int n_cells;           /* N on the finest level; divisible by 2^(n_levels-1) */
  int n_levels;          /* 1..16; coarsest level must have >= 2 cells per direction */
  int pre_sweeps;        /* forward sweeps before the coarse correction, >= 0 */
  int post_sweeps;       /* reverse sweeps after it, >= 0 */
  int vcycle_dtype;      /* vps_dtype of everything inside the V-cycle */
  int coef;              /* vps_coef */
  int patches_per_block; /* 0 = automatic (3D rho = 1: one patch per wavefront);
                            1, 2, 4 = batches of that many patches along x per
                            256-thread workgroup of the LDS-staged kernel
                            (VPS_E_UNSUPPORTED where the batch exceeds the LDS
                            in the V-cycle dtype) */
  int stream_min_cells;  /* the operator and the residual (rho = 1) and the grid
                            transfers use the plane- (3D) or row-streaming (2D)
                            kernels on levels with at least this many cells per
                            direction (for a transfer: on its coarse level),
                            single-pass tile kernels below; 0 = default (32; 2D
                            transfers 256, and the 2D restriction keeps the tiles
                            at degree 5), 1 = always; must be >= 0 */
  int algorithm;         /* vps_algorithm of every smoothing step (vps_smooth_color,
                            vps_smooth, the V-cycle) */
  int patch_order;       /* 3D, rho = 1, one patch per wavefront: order in which the
                            workgroups of a color visit its patches (dispatch-order
                            study): 0 = lexicographic, one contiguous slab per XCD
                            (default); 1 = lexicographic, dealt round-robin over
                            the XCDs; 2 = Morton curve, one slab per XCD; 3 = tiles
                            of 4x4x4 patches, one slab per XCD */
  int batch_layers;      /* batch processing (Algorithm 5, Section 4.1) in vps_smooth and
                            the V-cycle: 0 = whole colors (Algorithm 4); B > 0 = on levels
                            with more than 2B vertex layers per direction, for each slab
                            of B vertex layers along the slowest direction, all colors of
                            its patches in turn (reverse sweeps: the whole sequence
                            backwards); smaller levels sweep whole colors.  Even B visits
                            every pair of interacting patches in the colorized order, i.e.
                            gives Algorithm 4's iterate.  Combined algorithm only; >= 0 */
  int patches_per_wave;  /* 3D, rho = 1, combined algorithm, patch_order 0: patches of a
                            color per wavefront in the smoother: 1 = one patch; 2 = two
                            x-adjacent patches that share a closure face (their boundary
                            columns are loaded together; degree 2..4); 3 = a row of
                            floor(63 / 2k) x-adjacent patches (lanes on node columns,
                            closure rows loaded as contiguous runs; degree 2..4), at
                            degree 5 a row of 5 patches per workgroup of two wavefronts
                            (one on the closure columns, one on the patch rows);
                            0 = automatic (3 at degree 2 from 32 cells per direction,
                            at degrees 3 to 5 from 64; else 2 from 32 cells except
                            FP32 at degree 4 and at degree 5; 1 otherwise).
                            VPS_E_UNSUPPORTED for 2 or 3 outside these cases.  Same
                            update either way, different rounding order */
  int vcycle_graph;      /* 1: the finest-level V-cycle of vps_vcycle and vps_solve is
                            captured once per (input, output) buffer pair into a HIP
                            graph on a stream of the library's own and replayed on the
                            context stream (kernel by kernel while the phase timer
                            runs); 0 (default): launched kernel by kernel.  Same
                            kernels, same results */
  int wave_rows_2d;      /* 2D, rho = 1, degree 2..5, automatic patches_per_block: the
                            smoother kernel.  0 = automatic: a row of x-adjacent
                            patches of a color per wavefront (their shared closure
                            columns loaded once, as rows of up to 61 values) on levels
                            of at least 64 cells per direction, the LDS-staged kernel
                            below; 1 = always the row kernel; 2 = never.  Same
                            update, different rounding order */
} vps_config;

typedef struct {
  int iterations;           /* CG iterations done */
  double rel_residual_true; /* ||b - A u||_2 / ||b||_2 over all nodes, FP64 */
  double seconds;           /* wall time of the solve measured with HIP events */
  long long fallback_patches; /* patches whose learned scaling fell back to 1 */
} vps_solve_info;

/* ---- set-up (paper: the mesh hierarchy and the level spaces, Section 2) ---- */

/* Create a context: validates cfg, builds the level constants (1D Q_k mass and
 * stiffness matrices, the FDM factors of the patch interior, the transfer
 * matrices, the coarse solver) on the host in FP64 and uploads them, and
 * allocates the V-cycle work vectors of every level in cfg->vcycle_dtype.
 * hip_stream: a hipStream_t (may be NULL for the null stream).
 * Returns VPS_E_UNSUPPORTED for degree outside 1..5, dim outside {2,3},
 * N not divisible by 2^(n_levels-1), a coarsest level below 2 cells, more
 * than 2e9 nodes, or (3D, rho = 1, degree 2..4) a finest level whose vector in
 * the V-cycle dtype reaches 4 GiB (the patch kernels use 32-bit byte offsets).
 * A context whose coarsest grid is too large for the coarse solver (rho = 1:
 * more than 15 free nodes per direction in 3D, 63 in 2D; cell coefficient:
 * more than 4096 free nodes) is still created: its smoother, operator and
 * transfers work, and the calls that need the coarse solver return
 * VPS_E_UNSUPPORTED. */
vps_status vps_create(const vps_config* cfg, void* hip_stream, vps_context** out);

/* Free the context and everything it owns.  NULL is accepted. */
vps_status vps_destroy(vps_context* ctx);

/* Replace the stream all later calls enqueue on. */
vps_status vps_set_stream(vps_context* ctx, void* hip_stream);

/* Nodes (k N_l + 1)^d of a level, or 0 for an invalid level. */
size_t vps_level_nodes(const vps_context* ctx, int level);

/* Cells per direction N_l of a level, or 0 for an invalid level. */
int vps_level_cells(const vps_context* ctx, int level);

/* Number of patches (N_l - 1)^d of a level, or 0 for an invalid level. */
long long vps_level_patches(const vps_context* ctx, int level);

/* Per-cell coefficient rho on the finest level: N^d FP64 values on the
 * device, cells lexicographic (x fastest), all > 0.  Coarser levels get the
 * mean of the 2^d children.  Only for coef != VPS_COEF_CONST.  With
 * VPS_COEF_CELL_EXACT it also forms every level's dense local inverses.  Rebuilds the
 * dense coarse solver (host FP64 Cholesky inverse of the coarsest operator,
 * at most 4096 free nodes).  Synchronises. */
vps_status vps_set_coefficient(vps_context* ctx, const double* rho_cells_dev);

/* Learned per-patch, per-eigenmode scaling of one level: n_patches(level) x q^d
 * FP32 values on the device (patch-major; mode index lexicographic over the
 * 1D eigenvector indices, x fastest) copied into the context; NULL resets to 1.
 * Only for coef == VPS_COEF_CELL_LEARNED. */
vps_status vps_set_patch_scaling(vps_context* ctx, int level, const float* c_dev);

/* ---- level operators ---- */

/* Au = A_l u (Section 2, eq:matrix: A_l is the bilinear form applied to the
 * basis functions of V_l), matrix-free: the cell operator of Appendix A.1 as
 * the Kronecker sum of 1D mass and stiffness matrices, by sum factorisation.
 * u, Au: level vectors of dtype t (distinct buffers); Dirichlet rows of Au are 0. */
vps_status vps_apply(vps_context* ctx, int level, const void* u, void* Au, vps_dtype t);

/* r = b - A_l u: the residual that the local solvers act on (Section 2.1, the
 * remark after eq:main:2 that A v amounts to b - A u).  b, u, r: level vectors
 * of dtype t; r may not alias u. */
vps_status vps_residual(vps_context* ctx, int level, const void* b, const void* u, void* r,
                        vps_dtype t);

/* Restriction (Section 2: the adjoint of the embedding with respect to the
 * Euclidean products, i.e. the transpose of the prolongation matrix):
 * r_coarse = P^T r_fine from level fine_level (>= 1) to fine_level-1.
 * Vectors of dtype t on their levels; r_coarse is overwritten. */
vps_status vps_restrict(vps_context* ctx, int fine_level, const void* r_fine, void* r_coarse,
                        vps_dtype t);

/* Prolongation (Section 2: the embedding V_{l-1} -> V_l of the nested spaces;
 * P[f][c] is the coarse basis function c at fine node f):
 * u_fine += P e_coarse from level fine_level-1 to fine_level (fine_level >= 1). */
vps_status vps_prolongate_add(vps_context* ctx, int fine_level, const void* e_coarse,
                              void* u_fine, vps_dtype t);

/* x = A_0^{-1} b on the coarsest level, the exact coarse solve of the V-cycle
 * (Section 2; its cost is negligible in the time split of Section 4.1):
 * fast diagonalization (Appendix A.3 applied to the whole coarse grid) for
 * rho = 1, a dense explicit inverse (host FP64 Cholesky) otherwise.  b, x:
 * level-0 vectors of dtype t.  VPS_E_UNSUPPORTED if the coarse grid exceeds
 * the limits given at vps_create. */
vps_status vps_coarse_solve(vps_context* ctx, const void* b, void* x, vps_dtype t);

/* ---- the smoother (Algorithm 4, combined and colorized) ---- */

/* One color of the smoother on a level, in place on u: every patch of the
 * color computes r_j = b_j - Abar_j ubar_j and u_j += B_j r_j.  color in
 * [0, 2^d).  u and b: level vectors of dtype t. */
vps_status vps_smooth_color(vps_context* ctx, int level, void* u, const void* b, vps_dtype t,
                            int color);

/* `sweeps` sweeps of the smoother on a level, in place on u.  A sweep runs the
 * colors 0..2^d-1 (reverse = 0) or 2^d-1..0 (reverse != 0), one launch each. */
vps_status vps_smooth(vps_context* ctx, int level, void* u, const void* b, vps_dtype t,
                      int sweeps, int reverse);

/* ---- multigrid and the outer solver ---- */

/* z = V r: one V-cycle (Section 2: smoother S_l on every level, restriction,
 * coarse-level recursion, prolongation) on the finest level from a zero
 * initial guess: pre_sweeps forward sweeps of eq:colorized, residual,
 * restriction, recursion, prolongate-add, post_sweeps reverse sweeps (which
 * makes the V-cycle symmetric), the exact coarse solve on level 0; computed in
 * cfg->vcycle_dtype (FP64 r and z are converted at the ends).  r, z: finest
 * FP64 vectors (distinct). */
vps_status vps_vcycle(vps_context* ctx, const double* r, double* z);

/* Solve eq:matrix, A u = b on the finest level, from u = 0 by CG
 * preconditioned with the V-cycle (the multigrid solver of Section 4.1's
 * timings; the paper does not name its Krylov method: flexible CG when the
 * V-cycle runs in FP32), all Krylov vectors,
 * dot products and updates in FP64, until ||b - A u|| <= rtol ||b|| with the
 * true residual recomputed at the end.  Synchronises.  info may be NULL.
 * Returns VPS_E_NOT_CONVERGED after maxit iterations (u holds the iterate),
 * VPS_E_NONFINITE if a CG scalar is NaN/Inf. */
vps_status vps_solve(vps_context* ctx, const double* b, double* u, double rtol, int maxit,
                     vps_solve_info* info);

/* Stationary iteration u <- u + V(b - A u), `iters` times, starting from the
 * given u (FP64, device): the multigrid method of Section 2 used as a solver,
 * whose residual ratio per iteration is the convergence factor that judges a
 * local solver (not in the paper).  res_hist (host, iters+1 doubles, may be NULL)
 * receives ||b - A u||_2 before the first and after every iteration.
 * Synchronises. */
vps_status vps_vcycle_iterate(vps_context* ctx, const double* b, double* u, int iters,
                              double* res_hist);

/* ---- learned eigenmode scaling (variable coefficient, d = 3) ----
 * Not in the paper.  The paper allows approximate local solvers (the remark
 * after eq:main:2); these calls build one: the fast-diagonalization inverse
 * of Appendix A.3 (eq:fdm:inverse) formed for the patch mean of rho, with
 * every eigenmode scaled by a factor that a small MLP predicts from the
 * patch's cell coefficients.  Every pointer below is a device pointer owned
 * by the caller, FP32 unless stated. */

/* Features of every patch of a level (MLP input; not in the paper):
 * x[j][c] = log(rho_c / rhobar_j) over the patch's 2^d cells (lexicographic,
 * x fastest), rhobar_j their arithmetic mean, FP32, n_patches x 2^d. */
vps_status vps_patch_features(vps_context* ctx, int level, float* x_dev);

/* Cell coefficients of every patch of a level (the cells of the vertex patch
 * Omega_j, Section 2.1 item 1): rho8[j][c] for the patch's 2^d cells
 * (lexicographic, x fastest), FP64, n_patches x 2^d (device). */
vps_status vps_patch_rho8(vps_context* ctx, int level, double* rho8_dev);

/* Features of n arbitrary patches from their cell coefficients (not in the
 * paper):
 * x[j][c] = log(rho8[j][c] / mean_c rho8[j][c]), FP32, n x 2^d (device). */
vps_status vps_rho8_features(vps_context* ctx, const double* rho8_dev, long long n, float* x_dev);

/* Training targets from exact dense patch operators (Q2, d = 3).  rho8: n x 8
 * FP64 per-cell coefficients of n patches (device).  Per patch: assemble
 * A_j(rho), Y = S^T A_j S, solve (Y o Y) d = diag(Y) by Cholesky,
 * c*_m = rhobar Lambda_m d_m: the per-mode scaling of the FDM inverse that
 * minimises ||I - A_j^{1/2} B_j A_j^{1/2}||_F (a reading of the remark that
 * approximate local solvers are allowed, after eq:main:2).  cstar: n x 27
 * FP64 (device).  log_target (device, may be NULL): n x 27 FP32 values
 * log(clamp(c*, 1/4, 4)), the regression target of the MLP. */
vps_status vps_patch_targets(vps_context* ctx, const double* rho8_dev, long long n,
                             double* cstar_dev, float* log_target_dev);

/* Not in the paper.
 * MLP n_in -> n_h (tanh) -> n_h (tanh) -> n_out with n_in = 2^d, n_h = 64,
 * n_out = q^d, FP32.  params: flat W1 (n_h x n_in, row-major), b1, W2, b2, W3
 * (n_out x n_h), b3.  x: n x n_in.  y: n x n_out.  act_cache (may be NULL):
 * n x 2 n_h, the two hidden activations, needed by vps_mlp_backward. */
vps_status vps_mlp_forward(vps_context* ctx, const float* params, const float* x, long long n,
                           float* y, float* act_cache);

/* Not in the paper.
 * dy = d(loss)/dy for loss = mean over n x n_out of (y - t)^2; loss_out
 * (device, 1 float, may be NULL) receives the loss. */
vps_status vps_mlp_loss_grad(vps_context* ctx, const float* y, const float* t, long long n,
                             float* dy, float* loss_out);

/* Not in the paper.
 * dparams = gradient of sum(dy * y) w.r.t. params (overwritten); x is the
 * forward input (the first layer's weight gradient needs it), act_cache the
 * forward's hidden activations, dy n x n_out.  dparams must not alias params. */
vps_status vps_mlp_backward(vps_context* ctx, const float* params, const float* x,
                            const float* act_cache, const float* dy, long long n,
                            float* dparams);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same gradient
 * as vps_mlp_backward, same kernels and same result, but its work memory (the
 * per-sample deltas and the partial gradients of up to 64 sample splits) is a
 * static device array of 4 MiB (1 Mi floats) that the library holds on every
 * GPU it runs on until the process ends, so the call allocates nothing.
 * n must not exceed (2^20 - 64 P) / 128 samples, P the MLP parameter count
 * (4946 for 8 -> 64 -> 64 -> 27); larger n returns VPS_E_ARG before any work.
 * Every call on one GPU uses that GPU's one array: calls that overlap in time
 * on one GPU (several streams or threads) race and give wrong results; calls
 * in order on one stream are safe.  Nothing in the array needs clearing (each
 * call overwrites what it reads). */
vps_status vps_mlp_backward_noalloc(vps_context* ctx, const float* params, const float* x,
                                    const float* act_cache, const float* dy, long long n,
                                    float* dparams);

/* Not in the paper.
 * One Adam step (step counts from 1) on params with moments m, v, in place;
 * params, dparams, m, v: mlp parameter count each. */
vps_status vps_mlp_adam(vps_context* ctx, float* params, const float* dparams, float* m,
                        float* v, int step, float lr, float b1, float b2, float eps);

/* Not in the paper (the approximate local solver of the remark after
 * eq:main:2, with eq:fdm:inverse's 1/Lambda_m scaled per mode).
 * Run the MLP on every patch of a level and store c = clamp(exp(y), 1/4, 4) as
 * the level's scaling; patches with non-finite outputs fall back to c = 1.
 * fallback (host, may be NULL) receives their number.  Synchronises. */
vps_status vps_mlp_infer_patches(vps_context* ctx, int level, const float* params,
                                 long long* fallback);

/* ---- phase timing (the time split of the multigrid solve, the analogue of
 * the split Section 4.1 reports for its solver) ---- */

#define VPS_MAX_LEVELS 16

typedef struct {
  int n_levels;
  double smooth_s[VPS_MAX_LEVELS];          /* smoother sweeps, per level */
  long long smooth_sweeps[VPS_MAX_LEVELS];  /* sweeps done, per level (2^d color launches each) */
  double residual_s[VPS_MAX_LEVELS];        /* r = b - A u inside the V-cycle, per level */
  double restrict_s[VPS_MAX_LEVELS];        /* restriction from this level to the next coarser */
  double prolong_s[VPS_MAX_LEVELS];         /* prolongation from the next coarser to this level */
  double coarse_s;                          /* coarse solves */
  double cg_operator_s;                     /* CG matrix-vector products (finest level, FP64) */
  double cg_vector_s;                       /* CG dots, updates, precision conversions */
  long long vcycles;
} vps_timing;

/* enable != 0: from now on record HIP events on the context's stream around
 * every phase (small overhead) and reset the totals; 0: stop recording. */
vps_status vps_timing_enable(vps_context* ctx, int enable);

/* Totals of the recorded phases since the last vps_timing_enable(ctx, 1).
 * Synchronises. */
vps_status vps_timing_get(vps_context* ctx, vps_timing* out);

/* ---- misc ---- */

/* Wait for the context's stream; reports asynchronous HIP errors. */
vps_status vps_sync(vps_context* ctx);

/* Static description of a status code. */
const char* vps_status_string(vps_status s);

/* Message of the last error on this context ("" if none); valid until the next
 * call.  ctx = NULL: message of the calling thread's last failed vps_create. */
const char* vps_last_error(const vps_context* ctx);

#ifdef __cplusplus
}
#endif

#endif /* VPS_H */
