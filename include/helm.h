/*
 * helm.h -- C ABI of the MI355X FD-Helmholtz ORAS-FGMRES solver.
 *
 * Solves A x = b, the 27-point mixed-grid finite-difference discretisation of
 * the frequency-domain Helmholtz equation (Delta + k^2(x)) u = b, k = omega/c,
 * c complex in viscous media (Dolean et al., EAGE 2021, arXiv 2103.14921:
 * eq. eqh and eq. eq1 of the FD-vs-FE section), with absorbing layers (PML) on
 * the vertical and bottom faces and a homogeneous Dirichlet top.  The solver
 * is right-preconditioned flexible GMRES with the one- or two-level Optimized
 * Restricted Additive Schwarz preconditioner (eq. oras and eq. 2lvl of the
 * domain-decomposition section): absorbing (Robin) conditions on the subdomain
 * interfaces, local problems solved by a direct method, and a coarse problem
 * solved by 10 GMRES iterations preconditioned by one-level ORAS.
 *
 * Conventions used by every entry point:
 *   - Grid node (ix, iy, iz) sits at (ix h, iy h, iz h), z is depth (down).
 *     Fields are complex128 (interleaved re, im doubles), C order
 *     [nz][ny][nx] (x fastest); a batch of nrhs fields is [nrhs][nz][ny][nx]
 *     (each right-hand side one contiguous field).
 *   - Time dependence e^{-i omega t}; the Dirichlet top is the ghost plane
 *     iz = -1; every neighbour outside the grid is a zero ghost.
 *   - Pointers may be host or device memory (detected per call); the caller
 *     owns every buffer it passes in.  The handle owns all device memory it
 *     allocates; only helm_destroy releases it.
 *   - Return codes: HELM_OK = 0; positive = warning with outputs valid;
 *     negative = error with outputs untouched.  helm_last_error(h) gives the
 *     message of the last failure of a call on handle h, helm_last_error(NULL)
 *     that of the last failure on the calling thread.
 *   - One solve in flight per handle; handles are independent.
 */
#ifndef HELM_H_
#define HELM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HELM_OK = 0,
  HELM_NOT_CONVERGED = 1, /* some right-hand side reached maxit; residuals are reported */
  HELM_PENDING = 2,       /* an asynchronous solve is still running (helm_request_query) */
  HELM_EINVAL = -1,       /* bad sizes or values (non-finite, Re c <= 0, boxes too small) */
  HELM_ENOMEM = -2,       /* device footprint exceeds the memory budget */
  HELM_EDEVICE = -3,      /* HIP runtime error or no device */
  HELM_EBREAKDOWN = -4    /* a numerically singular pivot in a local factorisation */
} helm_status;

typedef struct helm_handle helm_handle_t;

typedef struct {
  int32_t nx, ny, nz; /* nodes per axis, each >= 3 */
  double h;           /* grid spacing in metres, > 0 */
} helm_grid_t;

/* PML thickness in nodes per side (0 = none).  npml_ztop = 0 gives the
 * homogeneous Dirichlet top of the paper.  Damping gamma(d) = gamma_max (d/L)^2,
 * gamma_max = 3 vmax/(2L) ln(1/R), L = npml h; R <= 0 selects R = 1e-3. */
typedef struct {
  int32_t npml_x, npml_y, npml_zbot, npml_ztop;
  double R;
} helm_pml_t;

/* Mixed-grid stencil weights (FD-vs-FE section: stiffness and consistent mass
 * on rotated systems, weights fitted by least squares on the dispersion).
 * Stiffness: w1 Cartesian 7-point, w2 mean of the three 45-degree rotated
 * systems, w3 the body-diagonal system, w1+w2+w3 = 1.  Mass: wm1 centre,
 * wm2 face, wm3 edge, wm4 corner neighbours, wm1+6wm2+12wm3+8wm4 = 1. */
typedef struct {
  double w1, w2, w3, wm1, wm2, wm3, wm4;
} helm_weights_t;

enum { HELM_FP64 = 0, HELM_MIXED = 1, HELM_SINGLE_LOCAL = 2, HELM_APPROX_LOCAL = 3 };

/* Decomposition and solver options (domain-decomposition section).  Boxes
 * split each axis into p ranges (floor(n/p), the first n mod p one longer),
 * extended by `overlap` layers on every interior side; Boolean partition of
 * unity.  levels = 2 adds the coarse grid at 2h with E = Z^T A Z solved by
 * coarse_iters GMRES iterations.  precision = HELM_MIXED factors and applies
 * the fine level's local solves in complex FP32 and keeps FGMRES,
 * orthogonalisation, Givens, residuals and the coarse level in FP64.
 * HELM_SINGLE_LOCAL also factors and applies the coarse level's local solves
 * (the one-level preconditioner of the coarse GMRES) in complex FP32; the
 * coarse GMRES itself, E and the transfers stay FP64 (the numerical-results
 * section runs every part in single precision with unchanged iteration
 * counts, Table 2).  HELM_APPROX_LOCAL makes the fine level's local solves
 * approximate, as the paper's incomplete Cholesky factors do (numerical-results
 * section, Table 2: cheaper and smaller local solves, FGMRES unchanged): the
 * plane inverses, factored in complex FP32, are kept as complex FP16 with a
 * power-of-two scale per plane (half the memory), and the sweeps multiply them
 * on FP16 matrix cores (FP32 accumulation) by the operand rounded to FP16 with
 * a power-of-two scale per column; everything else is as in HELM_MIXED.  Its
 * fine planes are limited to 960 nodes. */
typedef struct {
  int32_t px, py, pz;     /* subdomains per axis, >= 1 */
  int32_t overlap;        /* added layers per interior side, >= 1 */
  int32_t levels;         /* 1 or 2 */
  int32_t coarse_iters;   /* GMRES iterations of the coarse solve (paper: 10) */
  int32_t precision;      /* HELM_FP64, HELM_MIXED, HELM_SINGLE_LOCAL or HELM_APPROX_LOCAL */
  int32_t restart;        /* FGMRES restart length m, >= 1 */
  int32_t robin;          /* 1: absorbing interfaces (ORAS); 0: Dirichlet (RAS) */
  int32_t nrhs_chunk;     /* right-hand sides per batch; 0 = planner's choice */
  int32_t adaptive;       /* 1: adaptive stencil coefficients (helm_fit_weight_table); 0: one weight set */
} helm_decomp_t;

/* Least-squares fit of the mixed-grid weights on the dispersion relation
 * (FD-vs-FE section): minimises sum (stiffness/(kappa h)^2 - mass)^2 over
 * G = gmin..gmax points per wavelength (ng values) and nang x nang directions in
 * the first octant, subject to the two sum constraints.  Host only; needs no GPU. */
helm_status helm_fit_weights(double gmin, double gmax, int32_t ng, int32_t nang, helm_weights_t* out);

/* Adaptive stencil coefficients (FD-vs-FE section: coefficients matched to the
 * local wavespeed).  out[j], j < n, is the weight set fitted as in
 * helm_fit_weights on the band of three G values from G_j / 1.05 to
 * G_j * 1.05, G_j = g0 + j dg, with nang x nang directions.  With
 * dec->adaptive = 1, helm_setup fits the table g0 = 3, dg = 0.25, n = 29,
 * nang = 15 (G from 3 to 10: above, every consistent stencil is accurate and
 * the fit loses its conditioning) and gives each node the weights interpolated
 * linearly in its G = Re(c)/(f h) (clamped at the table's ends); every edge
 * takes the mean of its two end nodes' stiffness weights and the mean of
 * wm sigma at its ends as its mass coupling, so the operator stays complex
 * symmetric; helm_setup's weights argument is then ignored.  Host only. */
helm_status helm_fit_weight_table(double g0, double dg, int32_t n, int32_t nang, helm_weights_t* out);

/* Kinds of velocity array accepted by helm_setup. */
enum {
  HELM_VEL_COMPLEX128 = 0, /* complex c (interleaved re, im doubles): attenuation c (1 - i/(2Q)) */
  HELM_VEL_REAL64 = 1      /* real c (doubles): a medium without attenuation */
};

/* Set up the operator, the decomposition and the factorisations on the current
 * HIP device: the Helmholtz operator of eq. eqh discretised by the 27-point
 * mixed-grid stencil of eq. eq1 (FD-vs-FE section) with k = 2 pi freq_hz / c,
 * the overlapping subdomains with absorbing interfaces and their direct local
 * factorisations of eq. oras, and for dec->levels = 2 the coarse operator
 * E = Z^T A Z with its own local factorisations (eq. 2lvl; domain-decomposition
 * section).
 *   grid:      node counts (each >= 3) and spacing h > 0 (metres).
 *   velocity:  [nz][ny][nx] (x fastest), host or device memory, of the kind
 *              vel_kind names; every value finite with Re c > 0.  Copied: the
 *              caller may free it on return.  A real array sets up exactly the
 *              operator of the complex array with zero imaginary parts.
 *   freq_hz:   frequency > 0.
 *   pml, dec:  see the structs above; weights == NULL uses
 *              helm_fit_weights(4, 10, 7, 15).
 * On success *out receives a handle that owns every device allocation of the
 * problem (released by helm_destroy).  Errors: HELM_EINVAL (sizes, values,
 * vel_kind, boxes narrower than 2 overlap + 1), HELM_ENOMEM (the footprint does
 * not fit the device), HELM_EDEVICE, HELM_EBREAKDOWN (a numerically singular
 * local factor); *out is then NULL and helm_last_error(NULL) holds the reason. */
helm_status helm_setup(const helm_grid_t* grid, const void* velocity, int32_t vel_kind, double freq_hz,
                       const helm_pml_t* pml, const helm_weights_t* weights,
                       const helm_decomp_t* dec, helm_handle_t** out);

enum {
  HELM_X0 = 1u,   /* X holds the initial guess on entry */
  HELM_BLOCK = 2u /* block FGMRES: one Krylov space shared by the right-hand sides of each batch */
};

/* Solve A X[r] = B[r], r < nrhs, by right-preconditioned flexible GMRES (the
 * Krylov solver of the domain-decomposition section) with the handle's one- or
 * two-level ORAS preconditioner (eq. oras / eq. 2lvl), one Krylov space per
 * right-hand side.  Stop when |g_{j+1}|/||b|| <= tol (FGMRES estimate), then
 * confirm with the FP64 true residual ||b - A x||/||b|| and restart from x
 * while it is above tol.  maxit bounds the outer iterations of each
 * right-hand side; x0 = 0 unless flags has HELM_X0 (X holds the guess).
 *   B, X: complex128 [nrhs][nz][ny][nx], host or device memory, owned by the
 *         caller; X is written only on HELM_OK / HELM_NOT_CONVERGED.
 *   iters[nrhs], relres_est[nrhs], relres_true[nrhs]: host arrays (may be NULL).
 * With HELM_BLOCK in flags the right-hand sides of each batch (at most 32;
 * nrhs_chunk or the planner's choice) share one Krylov space (block FGMRES,
 * the paper's many sources per frequency taken together): block j applies the
 * preconditioner to the s basis vectors, orthogonalises A Z_j against the
 * basis by two block classical Gram-Schmidt passes and factors it by two
 * Cholesky-QR passes; the block least-squares problem is solved on the host
 * and every right-hand side stops when all of its batch are at tol (iters
 * counts block iterations).  Zero right-hand sides get X = 0 and no iteration;
 * a numerically rank-deficient block at a (re)start makes the batch continue
 * with one Krylov space per right-hand side.  Results depend on the batch.
 * Returns HELM_NOT_CONVERGED when some right-hand side reached maxit (its
 * residuals are reported), HELM_EINVAL for bad arguments or a handle with a
 * request in flight, HELM_ENOMEM when not even one right-hand side's Krylov
 * workspace fits, HELM_EDEVICE on a runtime error. */
helm_status helm_solve(helm_handle_t* h, int32_t nrhs, const void* B, void* X, double tol,
                       int32_t maxit, uint32_t flags, int32_t* iters, double* relres_est,
                       double* relres_true);

/* Asynchronous form of helm_solve for callers that overlap solves of several
 * handles (continuous batching of a serving loop): the arguments are checked
 * at once, then the solve runs on a library thread with the handle's device
 * current, in the same order of device work as helm_solve, so its results are
 * bitwise those of helm_solve.  stream (a hipStream_t of the handle's device;
 * NULL = the handle's own stream) receives every device operation of the
 * solve, so work the caller enqueued on it before this call (producing B, say)
 * is ordered before the solve; the caller enqueues nothing more on that stream
 * until helm_request_wait returns.  The FGMRES loop is driven from the host
 * (each outer iteration reads the convergence counters), hence the library
 * thread.  B, X and the result arrays belong to the caller and must stay
 * valid until helm_request_wait returns.  One solve at a time per handle: helm_solve, helm_solve_async and
 * helm_release_workspace on a handle with a request in flight return
 * HELM_EINVAL; helm_destroy waits for it (the request stays valid for
 * helm_request_wait, which must not run concurrently with helm_destroy of the
 * same handle).  On success *req receives a request that the caller must pass
 * to helm_request_wait exactly once. */
typedef struct helm_request helm_request_t;
helm_status helm_solve_async(helm_handle_t* h, int32_t nrhs, const void* B, void* X, double tol,
                             int32_t maxit, uint32_t flags, int32_t* iters, double* relres_est,
                             double* relres_true, void* stream, helm_request_t** req);
/* HELM_PENDING while the solve runs, then its helm_solve status (the request
 * stays valid). */
helm_status helm_request_query(const helm_request_t* req);
/* Block until the solve has finished, free the request and return its
 * helm_solve status; on failure helm_last_error (in the calling thread) holds
 * the solve's message. */
helm_status helm_request_wait(helm_request_t* req);

/* Device bytes the handle needs for this grid and decomposition plus the
 * Krylov workspace of nrhs_chunk right-hand sides (admission control). */
size_t helm_footprint(const helm_grid_t* grid, const helm_decomp_t* dec, int32_t nrhs_chunk);

/* Device bytes of the Krylov workspace alone for nrhs_chunk right-hand sides
 * (the part of helm_footprint that a solve on an already set-up handle
 * allocates; released by helm_release_workspace).  0 on invalid arguments,
 * with the reason in helm_last_error. */
size_t helm_workspace_bytes(const helm_grid_t* grid, const helm_decomp_t* dec, int32_t nrhs_chunk);

/* Device bytes the handle holds now (factors, operators, cached workspace):
 * the sizes of the blocks it was given, which the library's device cache may
 * round up by as much as an eighth of a request. */
size_t helm_resident_bytes(const helm_handle_t* h);

/* Timings of the last setup / solve in seconds, measured with HIP events on the
 * handle's stream: out[0] setup, out[1] solve, out[2] fine factorisation,
 * out[3] coarse set-up, out[4] number of outer iterations summed over RHS. */
helm_status helm_last_timings(const helm_handle_t* h, double out[5]);

/* Lower bound of the last solve on this handle: every kernel launch of the
 * solve (the local-solve sweeps of eq. oras, the 27-point products of eq. eq1,
 * the coarse correction of eq. 2lvl, the Krylov passes, staging) contributes
 * max(algorithmic bytes / 8 TB/s, algorithmic flops / peak), with the FP64
 * (78.6 TFLOP/s) or FP32 (157.3 TFLOP/s) peak of its arithmetic.  out[0] the
 * bound in seconds, out[1] algorithmic bytes, out[2] algorithmic flops.  The
 * solve's roofline fraction is out[0] over the measured solve time. */
helm_status helm_solve_bound(const helm_handle_t* h, double out[3]);

/* Live timing of the batched local solves (the one-level ORAS sweep of eq.
 * oras, one kernel launch per application): when enabled, HIP events on the
 * handle's stream bracket every sweep launch; helm_sweep_stats returns, for
 * level 0 (fine) or 1 (coarse), out[0] launches, out[1] total milliseconds,
 * out[2] algorithmic real flops (8 b^2 per plane product and right-hand side,
 * b the unpadded plane size, 2 ez - 1 plane products per box) and out[3]
 * algorithmic bytes (every factor once per application plus the plane
 * vectors), summed over the launches since enabling.  Enabling resets them. */
helm_status helm_set_sweep_timing(helm_handle_t* h, int32_t enable);
helm_status helm_sweep_stats(const helm_handle_t* h, int32_t level, double out[4]);

/* The autotuned launch of the batched local solves (eq. oras) of level 0 (fine)
 * or 1 (coarse) on batches of nrhs right-hand sides under the current sweep
 * policy: out[0] right-hand-side group, out[1] waves per item (0 for the
 * pipelined sweep), out[2] the variant, numbered as the sweep policy that
 * forces it (1 one item per workgroup, 2 pipelined, 3 low-register build,
 * 4 pipelined with 16 waves, 5 paired, 6 plane solutions in LDS, paired or
 * one group), out[3] waves per workgroup; all zero
 * if that batch width has not been tuned yet.  HELM_EINVAL for a bad level
 * or nrhs <= 0. */
helm_status helm_sweep_config(const helm_handle_t* h, int32_t level, int32_t nrhs, int32_t out[4]);
/* Environment: HELM_TUNE_FILE=path persists the sweep tuner's decisions --
 * decisions recorded in the file are used as tuned, new ones are appended --
 * so that separate processes launch the same sweeps (an entry naming a launch
 * that cannot run on the problem is ignored and tuned again); HELM_TUNE_VERBOSE=1
 * prints every candidate the tuners time; HELM_NO_TUNE=1 skips tuning. */

/* With the same timing on, the fine-grid 27-point products of eq. eq1 inside
 * solves are bracketed too: helm_stencil_stats gives, for kind 0 (y = A x,
 * the Arnoldi product) or 1 (y = b - A x: the (I - A Q) term of eq. 2lvl and
 * the true residuals), out[0] launches, out[1] total milliseconds, out[2]
 * algorithmic real flops (27 complex multiply-adds per node and right-hand
 * side) and out[3] algorithmic bytes (16 B per node and right-hand side for
 * x read and y written, and for b in a residual, plus 16 B per node for
 * s k^2 and 16 B per node for the stored row diagonal), summed since timing
 * was enabled. */
helm_status helm_stencil_stats(const helm_handle_t* h, int32_t kind, double out[4]);

/* Captured iterations (batching form).  With graphs enabled (the default),
 * each outer FGMRES iteration -- the two-level preconditioner of eq. 2lvl with
 * its ten inner coarse GMRES iterations, the operator product and the Arnoldi
 * step -- is captured once as a HIP graph per iteration index, batch width,
 * tolerance and iteration limit, after the first direct run has tuned the
 * sweeps, and replayed from then on; results are bitwise those of direct
 * launches.  Sweep timing stays live inside graphs (external event nodes).
 * helm_set_graphs(h, 0) launches directly and drops the captured graphs;
 * helm_graph_stats gives out[0] captures and out[1] replays since set-up.
 * Graphs are dropped whenever the workspace is reallocated or released. */
helm_status helm_set_graphs(helm_handle_t* h, int32_t enable);
helm_status helm_graph_stats(const helm_handle_t* h, double out[2]);

/* Process-wide choice among the implementations of the batched local solves
 * (the one-level ORAS sweep of eq. oras): 0 (default) times the admissible
 * variants once per problem shape and keeps the fastest; 1 restricts to the
 * one-workgroup-per-box sweep; 2 uses the pipelined persistent sweep (two
 * boxes per compute unit, operand build overlapped with the matrix-core
 * product) wherever its two operand slots fit in LDS; 3 uses the
 * one-workgroup-per-box sweep built for two workgroups per compute unit
 * (complex FP64, groups of 32 right-hand sides, planes of up to 144 nodes)
 * wherever it exists, else as 1; 4 uses the pipelined sweep with eight
 * producer waves beside the eight consumers (16 waves) wherever the pipelined
 * sweep fits, else as 1; 5 uses the paired sweep (two right-hand-side groups of
 * one box per workgroup, each on half of its waves, so that both stream the
 * box's factors in step and the second read hits L2) wherever the batch
 * splits into an even number of groups whose two operands fit in LDS, else
 * as 0; 6 uses the sweep that also keeps each item's last plane solution in
 * LDS (groups of 16 whose operands and solutions fit), so that a plane step
 * needs only a workgroup barrier: paired where the complex FP64 groups pair,
 * else one group per workgroup (the approximate form's FP16 sweep too), else
 * as 0.
 * Planes whose operand does not fit in LDS
 * (complex FP64 above 600 nodes, complex FP32 above 1200) keep it in global
 * memory under every policy.  Results agree to rounding.  Graphs captured
 * under one policy are not replayed under another. */
helm_status helm_set_sweep_policy(int32_t policy);

/* Process-wide schedule of the 27-point products (the fine operator of eq. eq1
 * and the coarse operator E of eq. 2lvl) for batches of 4 or more right-hand
 * sides.  2, 4 or 8: row tiles, each thread computing that many consecutive
 * nodes of a grid row; HELM_TILE_MARCH | n (n = 2 or 3): plane-marching, each
 * thread keeping n nodes of a row and marching through a chunk of planes, for
 * batches of 16 k right-hand sides (other batches then take row tiles of 4);
 * 0 (default) times every admissible schedule once per grid and batch size and
 * keeps the fastest.  Every schedule sums the 27 terms of an output in the
 * same order from the same coefficients, so results are bitwise identical.
 * Returns HELM_EINVAL for any other value. */
enum { HELM_TILE_MARCH = 0x100 };
helm_status helm_set_row_tiling(int32_t nodes_per_thread);

/* Process-wide panel width of the blocked Gauss-Jordan inversion of the plane
 * Schur complements (the local factorisation of eq. oras, done by set-up):
 * 0 (default) times the admissible widths on the first plane of each new
 * (precision, plane size, box count) and keeps the fastest; 4, 8 or 16 forces
 * that width wherever it is admissible (16 or 8 for planes of up to 512 rows,
 * 8 or 4 above).  Widths change only the rounding of the inverses.  Returns
 * HELM_EINVAL for any other value. */
helm_status helm_set_lu_panel(int32_t columns);

/* Return the handle's cached Krylov workspace (sized for its last batch) to
 * the library's device cache, keeping operators and factors resident: lets a
 * server hold many set-up problems and pay workspace only while solving. */
helm_status helm_release_workspace(helm_handle_t* h);

/* Device blocks freed by handles are kept in a process-wide cache and reused
 * for requests of the same size class; this returns them all to the HIP
 * runtime (for other allocators in the process) and reports the bytes freed. */
size_t helm_trim_cache(void);

/* Device bytes the library never allocates into on the current device: 1 % of
 * its memory, at least 1 GiB (the runtime allocates for itself at dispatch --
 * kernel arguments, signals, graph instantiation -- and a failure there aborts
 * the queue instead of returning an error).  Callers that allocate device
 * memory beside the library, such as staging buffers, keep the same margin. */
size_t helm_device_headroom(void);

void helm_destroy(helm_handle_t* h);

/* Message of the last failed call on handle h (the solve's own failure for an
 * asynchronous request), or with h == NULL of the last failure on the calling
 * thread (e.g. a helm_setup that returned no handle).  The string stays valid
 * in the calling thread until its next helm_last_error call; "" if none. */
const char* helm_last_error(const helm_handle_t* h);

/* Bind later kernels of this handle to a HIP stream (hipStream_t; NULL = the
 * handle's own stream). */
helm_status helm_set_stream(helm_handle_t* h, void* stream);

/* ---- operator-level entry points (parity tests, tools) ----------------- */

/* Y = A X for nrhs fields (eq. eq1). */
helm_status helm_apply_A(helm_handle_t* h, int32_t nrhs, const void* X, void* Y);

/* Z = M^{-1} R: the preconditioner the handle was set up with (eq. oras for
 * levels = 1, eq. 2lvl for levels = 2). */
helm_status helm_apply_M(helm_handle_t* h, int32_t nrhs, const void* R, void* Z);

/* Z = M1^{-1} R, the one-level ORAS sum_i R_i^T D_i A_i^{-1} R_i (eq. oras)
 * on level 0 (fine grid) or level 1 (coarse grid, fields of the coarse shape
 * ceil(n/2) per axis). */
helm_status helm_apply_oras(helm_handle_t* h, int32_t level, int32_t nrhs, const void* R, void* Z);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): Z = M1^{-1} R
 * as helm_apply_oras computes it, with no allocation of any kind.  R and Z are
 * device arrays owned by the caller, complex128 [nrhs][n of the level] (x
 * fastest); R is not modified.  The node-major staging of R and Z and the
 * sweep's plane vectors live in a fixed scratch array of 64 MiB per GPU, which
 * the library holds from its first use on that GPU until the process ends; a
 * level and batch needing more return HELM_EINVAL (helm_apply_oras has no such
 * limit).  A shape the sweep autotuner has not timed yet takes its default
 * launch shape.  The work is enqueued on the handle's stream and the call
 * returns without waiting for it.  Every call on one GPU shares that GPU's
 * scratch, which keeps the last call's contents: calls that overlap on one
 * GPU (other handles, streams or threads) race, so callers order them. */
helm_status helm_apply_oras_noalloc(helm_handle_t* h, int32_t level, int32_t nrhs, const void* R, void* Z);

/* X = A_i^{-1} R for one subdomain s of a level (the local problem of eq.
 * oras, with its absorbing interface fold), through the same factors and
 * sweep kernels as the preconditioner.  R, X: complex128 [nrhs][ez][ey][ex]
 * in the extended box's natural order (x fastest; see helm_subdomain_box). */
helm_status helm_local_solve(helm_handle_t* h, int32_t level, int32_t s, int32_t nrhs, const void* R, void* X);

/* Coarse transfers (eq. 2lvl): C = Z^T R (restriction, fine -> coarse) and
 * R = Z C (trilinear prolongation, coarse -> fine). */
helm_status helm_restrict(helm_handle_t* h, int32_t nrhs, const void* R, void* C);
helm_status helm_prolong(helm_handle_t* h, int32_t nrhs, const void* C, void* R);

/* Y = E X on the coarse grid, E = Z^T A Z (eq. 2lvl). */
helm_status helm_apply_E(helm_handle_t* h, int32_t nrhs, const void* X, void* Y);

/* Q = Z GMRES_coarse(E, Z^T R): the coarse correction Q R of eq. 2lvl. */
helm_status helm_apply_Q(helm_handle_t* h, int32_t nrhs, const void* R, void* Q);

/* Geometry of the decomposition: number of subdomains of a level, and for
 * subdomain s its extended box elo[3], ehi[3] and core lo[3], hi[3] (x, y, z). */
int32_t helm_num_subdomains(const helm_handle_t* h, int32_t level);
helm_status helm_subdomain_box(const helm_handle_t* h, int32_t level, int32_t s, int32_t box[12]);

#ifdef __cplusplus
}
#endif
#endif /* HELM_H_ */
