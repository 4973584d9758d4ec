/*
 * nosdd.h -- C ABI of libnosdd: two-level Schwarz flexible-GMRES solver for
 * 2D E_z FDFD (Helmholtz) problems with UPML, on one AMD Instinct MI355X.
 *
 * The problem statement follows the paper's two-level Schwarz algorithm
 * (Algorithm 3 inputs: permittivity map, source, PML, subdomain partition,
 * coarse-space size, subdomain solver, subdomain and global thresholds):
 *
 *   curl curl E - k0^2 eps E = -i omega J            (Eq. 1, E_z form)
 *   d_n E + i k E = g  on subdomain interfaces       (Eq. 2, Robin data,
 *                                                    exp(+i omega t) convention)
 *
 * Units are normalised (c = eps0 = mu0 = 1), so omega = k0 = 2 pi / wavelength,
 * and the grid spacing h is in the same length unit as the wavelengths.
 *
 * Layout conventions used by every call:
 *   - a scalar field on the grid is [ny][nx], row-major, x fastest;
 *   - complex values are interleaved (re, im) single precision (nosdd_c32);
 *   - a batch of right-hand sides is [n_wl][n_src][ny][nx]: RHS index
 *     r = wl * n_src + src.
 *
 * Ownership: the caller owns every buffer it passes.  The library copies eps
 * at problem_create and never keeps a caller pointer after a call returns.
 * Library objects are released only by their *_destroy call.
 *
 * Errors: a negative status is a failure; output buffers are then
 * unspecified and nosdd_last_error() describes the failure.  A positive
 * status (NOSDD_NOT_CONVERGED) is a warning: outputs are valid.
 *
 * Threading: one host thread at a time per context.  All GPU work of a
 * context is issued on one HIP stream (the caller's, or the library's own).
 */
#ifndef NOSDD_H
#define NOSDD_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { float re, im; } nosdd_c32;
typedef struct { double re, im; } nosdd_c64;

typedef enum {
    NOSDD_OK = 0,
    NOSDD_NOT_CONVERGED = 1,    /* tolerance not reached within max_iters; outputs valid */
    NOSDD_EINVAL = -1,          /* invalid argument (null pointer, size, option)         */
    NOSDD_ENOMEM = -2,          /* device or host allocation failed                      */
    NOSDD_EHIP = -3,            /* HIP runtime error                                     */
    NOSDD_EPARTITION = -4,      /* partition does not fit the grid / PML                 */
    NOSDD_EBREAKDOWN = -5,      /* Krylov breakdown before any progress                  */
    NOSDD_ENONFINITE = -6,      /* NaN or Inf met in a residual                          */
    NOSDD_ENOWEIGHTS = -7,      /* neural subdomain solver requested without weights     */
    NOSDD_ESTATE = -8           /* call out of order (e.g. solve before setup)           */
} nosdd_status;

typedef struct nosdd_ctx nosdd_ctx;
typedef struct nosdd_problem nosdd_problem;

/* Grid: nx * ny cells of size h; a PML of npml cells on every side with
 * conductivity profile sigma(d) = sigma_max d^pml_m and ideal reflection
 * exp(pml_lnR) (Methods, UPML equations).  Defaults used by the benchmarks:
 * h = 0.05, npml = 12, pml_m = 2, pml_lnR = -30.  nx, ny >= 4 and
 * nx * ny < 2^29 (NOSDD_EINVAL otherwise). */
typedef struct {
    int nx, ny;
    double h;
    int npml;
    int pml_m;
    double pml_lnR;
} nosdd_grid;

/* Rectangular partition (Methods, "partitioner"): core widths core_x[ncx]
 * (sum = nx) and heights core_y[ncy] (sum = ny) tile the grid; every core is
 * extended by overlap/2 cells across each side that is not on the global
 * boundary.  overlap must be even and >= 2, overlap/2 + 1 <= every core, and
 * no interface may lie inside the PML of its normal direction
 * (NOSDD_EPARTITION otherwise). */
typedef struct {
    const int *core_x;
    int ncx;
    const int *core_y;
    int ncy;
    int overlap;
} nosdd_partition;

/* Subdomain solver and coarse space (Algorithm 3 set-up block).
 * sub_solver: 0 = exact subdomain LU (block-tridiagonal factorisation),
 *             1 = per-subdomain flexible GMRES preconditioned by the Fourier
 *                 neural operator read from nn_weights (Algorithm 1 inference).
 * k_coarse:   coarse basis functions per subdomain (0 = one-level).
 * k_trial:    pseudo-plane-wave probes per subdomain (>= k_coarse; 8 if 0).
 * inner_max, inner_tol: inner FGMRES step limit and relative threshold
 *             (NN solver only). */
typedef struct {
    int sub_solver;
    int k_coarse;
    int k_trial;
    const char *nn_weights;
    int inner_max;
    float inner_tol;
} nosdd_setup_opts;

/* Outer flexible GMRES(restart) on A x = b, right-preconditioned by the
 * two-level Schwarz sweep.  Stops when ||b - A x|| / ||b|| <= tol (checked on
 * an explicit residual) or after max_iters preconditioner applications; a
 * right-hand side whose explicit residual did not decrease over a whole
 * restart cycle is stopped early (stagnation: the solve then returns
 * NOSDD_NOT_CONVERGED and nosdd_last_error says so).
 * x0 (nullable) is an initial guess laid out like E_out. */
typedef struct {
    double tol;
    int restart;
    int max_iters;
    const nosdd_c32 *x0;
} nosdd_solve_opts;

/* Create a context on HIP device hip_device.  hip_stream is a hipStream_t
 * (nullable: the library creates its own default-priority stream). */
nosdd_status nosdd_ctx_create(int hip_device, void *hip_stream, nosdd_ctx **out);
void nosdd_ctx_destroy(nosdd_ctx *ctx);                /* NULL is accepted */
/* Message of the last failure on this context; owned by the context and
 * valid until the next call on it.  Never NULL. */
const char *nosdd_last_error(const nosdd_ctx *ctx);

/* Create a problem (destroy it before its context): eps is a host [ny][nx] real permittivity map (copied);
 * every entry must be finite and positive, since the Robin condition's local wavenumber k0 sqrt(eps) is
 * taken real (NOSDD_EINVAL otherwise); wavelengths[n_wl] are solved together, one operator per
 * wavelength. */
nosdd_status nosdd_problem_create(nosdd_ctx *ctx, const nosdd_grid *grid, const float *eps,
                                  const nosdd_partition *part, const double *wavelengths,
                                  int n_wl, nosdd_problem **out);
/* Create a problem over an explicit list of subdomain cores (Methods,
 * "partitioner": any arrangement of subdomains that covers the domain, for
 * instance a quad-tree whose quadrants are split while larger than about five
 * wavelengths).  cores is a host array [n_cores][4] of half-open rectangles
 * (cx0, cx1, cy0, cy1) in cells (copied); they must cover every cell exactly
 * once.  Subdomain i is core i extended by overlap/2 cells across every side
 * that is not on the global boundary, so a side may border several
 * neighbours (T-junctions).  Same rules as nosdd_problem_create otherwise:
 * overlap even and >= 2, overlap/2 + 1 <= every core side (with more than one
 * core), no interface inside the PML of its normal direction, extended
 * subdomains with an even short side <= 128 cells and a long side <= 256
 * (NOSDD_EPARTITION otherwise; NOSDD_EINVAL for null pointers, n_cores <= 0
 * or n_wl <= 0).  Every solve, sweep and set-up call works on it unchanged. */
nosdd_status nosdd_problem_create_cores(nosdd_ctx *ctx, const nosdd_grid *grid, const float *eps,
                                        const int *cores, int n_cores, int overlap,
                                        const double *wavelengths, int n_wl, nosdd_problem **out);
/* Build every per-wavelength subdomain factorisation, the coarse space and,
 * for sub_solver = 1, load the network.  Must precede any solve. */
nosdd_status nosdd_problem_setup(nosdd_problem *p, const nosdd_setup_opts *opts);
void nosdd_problem_destroy(nosdd_problem *p);          /* NULL is accepted */

/* Solve for n_src current densities J[n_src][ny][nx] (host) at every
 * wavelength: E = A^-1 (-i omega J) with A the Eq. 1 operator, by flexible
 * GMRES(restart) preconditioned by one two-level Schwarz sweep per iteration
 * (the Algorithm 3 loop body: subdomain Robin solves of Eq. 2 with exact LU
 * or the Algorithm 1 network-preconditioned inner solver, then the coarse
 * correction of the Methods two-level subsection).  Outputs (host): E_out[n_wl][n_src][ny][nx];
 * resid_hist[n_wl][n_src][max_iters] relative residual estimate after each
 * preconditioner application, -1 padded (nullable); iters[n_wl][n_src]
 * preconditioner applications (nullable); final_resid[n_wl][n_src] explicit
 * relative residual (nullable). */
nosdd_status nosdd_solve(nosdd_problem *p, const nosdd_c32 *J, int n_src,
                         const nosdd_solve_opts *opts, nosdd_c32 *E_out, float *resid_hist,
                         int *iters, float *final_resid);
/* Same as nosdd_solve (Eq. 1 solved by the Algorithm 3 sweep inside
 * flexible GMRES), but J, x0 and E_out are device pointers, ordered on the
 * context stream; resid_hist, iters and final_resid stay host pointers.
 * This is the call whose time the benchmark reports (inputs resident in HBM). */
nosdd_status nosdd_solve_device(nosdd_problem *p, const nosdd_c32 *J_dev, int n_src,
                                const nosdd_solve_opts *opts, nosdd_c32 *E_dev, float *resid_hist,
                                int *iters, float *final_resid);

/* Same as nosdd_solve_device, with the field returned as the outer FGMRES's
 * FP64 iterate (E64_dev, device, [n_wl][n_src][ny][nx] complex128) instead
 * of its complex64 rounding: the iterate and every restart residual are FP64
 * (refinement around FP32 Krylov cycles), so tolerances below single
 * precision are reached and kept in the returned field. */
nosdd_status nosdd_solve_device_c64(nosdd_problem *p, const nosdd_c32 *J_dev, int n_src,
                                    const nosdd_solve_opts *opts, nosdd_c64 *E64_dev, float *resid_hist,
                                    int *iters, float *final_resid);

/* The paper's own outer loop (Algorithm 3): stationary sweeps over the Robin
 * data g of every subdomain's interface entries, starting from g = 0,
 *   u_i = B_i^-1 (R_i b + inj(g_i)),  x = sum_i Rt_i^T u_i (core-only assembly),
 *   g_new = Robin traces of x (Eq. 2 data),  e = g_new - g,
 *   g <- m g + (1 - m) g_new [+ (m Q + (1 - m) T Q) z],
 * with momentum m in [0, 1) and, when coarse is set (requires k_coarse > 0 at
 * set-up), the Robin-space coarse correction of the Methods two-level
 * subsection: z solves the normal equations of (I - T) Q z = e (T the
 * Robin-to-Robin map, Q the rotated probe data of each subdomain's coarse
 * columns), in FP64.  Stops when ||b - A x|| / ||b|| <= tol after a sweep or
 * after max_iters sweeps.  Exact subdomain solves only (sub_solver 0). */
typedef struct {
    double momentum;
    int coarse;
    double tol;
    int max_iters;
} nosdd_paper_opts;
/* J_dev and E_dev are device pointers on the context stream, laid out as in
 * nosdd_solve_device; resid_hist[n_wl][n_src][max_iters] (-1 padded), iters
 * (sweeps) and final_resid (relative residual after the last sweep) are host
 * pointers (nullable).  Returns NOSDD_NOT_CONVERGED when some right-hand side
 * did not reach tol; E_dev then holds its last sweep. */
nosdd_status nosdd_solve_paper_device(nosdd_problem *p, const nosdd_c32 *J_dev, int n_src,
                                      const nosdd_paper_opts *opts, nosdd_c32 *E_dev, float *resid_hist,
                                      int *iters, float *final_resid);

/* ---- Steps of one Schwarz sweep, exposed for testing and composition. ----
 * All vectors are device pointers on the context stream, laid out
 * [n_wl][n_src][ny][nx]; n_src is the number of vectors per wavelength. */

/* y = A x, or y = b - A x when b is not NULL (Eq. 1 operator with UPML). */
nosdd_status nosdd_apply_operator(nosdd_problem *p, const nosdd_c32 *x, const nosdd_c32 *b,
                                  nosdd_c32 *y, int n_src);
/* One-level restricted additive Schwarz sweep with Robin transmission:
 * z = sum_i Rt_i^T B_i^-1 R_i v  (gather across overlaps, exact subdomain
 * solve, core-only scatter).  Equivalent to one boundary-update step of the
 * paper's domain-decomposition loop applied to the residual v. */
nosdd_status nosdd_schwarz_sweep(nosdd_problem *p, const nosdd_c32 *v, nosdd_c32 *z, int n_src);
/* Full two-level preconditioner: z = z1 + Phi c, Az = A z1 + W c with
 * c = G^-1 W^H (v - A z1) (coarse correction, FP64 solve). Az nullable. */
nosdd_status nosdd_precond_apply(nosdd_problem *p, const nosdd_c32 *v, nosdd_c32 *z, nosdd_c32 *Az,
                                 int n_src);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * two-level preconditioner as nosdd_precond_apply for a problem set up with
 * exact subdomain solves (sub_solver 0), z = z1 + Phi c and Az = A z
 * (Az required), computed without any allocation.  The job queue of the
 * subdomain solves and the coarse coefficients (FP64 W^H t and c) live in a
 * fixed per-device scratch array of NOSDD_NOALLOC_SCRATCH_BYTES inside the
 * library, whose device address is looked up when a context is created on
 * that device; a batch needs 8 n_tiles n_rhs + 24 n_rhs n_coarse bytes (each
 * part rounded up to 256), n_rhs = n_wl * n_src, and larger batches are
 * rejected with NOSDD_EINVAL before any work is issued.  The subdomain solves
 * always use the one-source kernel.  Nothing is synchronised: the work is
 * ordered on the context stream.  Every call on one GPU shares that GPU's
 * scratch (which keeps the last call's contents; every entry is written
 * before it is read), so calls that overlap on one device race.
 * NOSDD_ESTATE before set-up or with sub_solver 1. */
#define NOSDD_NOALLOC_SCRATCH_BYTES (16u << 20)
nosdd_status nosdd_precond_apply_noalloc(nosdd_problem *p, const nosdd_c32 *v, nosdd_c32 *z, nosdd_c32 *Az,
                                         int n_src);
/* Subdomain solves on subdomain-local vectors with the configured sub-solver:
 * for tile t (index ty*ncx+tx) and wavelength wl, u = B_{t,wl}^-1 rhs.
 * sub_solver 0: exact block-Thomas LU.  sub_solver 1: the inner NN-FGMRES of
 * Algorithm 1 (inference branch; x0 = 0, no restart, at most inner_max steps,
 * stop once |gamma_{k+1}| / ||rhs|| <= inner_tol), u over the whole tile.
 * rhs and u are [n_wl][n_tiles][ly_t][lx_t] packed in tile order (tile sizes
 * differ; use nosdd_tile_info for offsets), one vector per (wl, tile). */
nosdd_status nosdd_local_solve(nosdd_problem *p, const nosdd_c32 *rhs, nosdd_c32 *u);
/* Apply the subdomain neural operator once to every subdomain-local vector
 * (Fig. 2 network as loaded at setup, BF16 MFMA channel mixes, truncated DFTs
 * on BF16 MFMA with operands split into high and low parts, near FP32):
 * e = NN(v) for v, e laid out [n_wl][n_tiles][ly_t][lx_t] like
 * nosdd_local_solve.  Needs a problem set up with sub_solver = 1. */
nosdd_status nosdd_nn_apply(nosdd_problem *p, const nosdd_c32 *v, nosdd_c32 *e);
/* Robin traces g_p(x) = (x_q - x_p)/h + i kappa_p (x_q + x_p)/2 on every
 * interface-ring entry of every tile, for one global field per wavelength.
 * g is [n_wl][n_entries]; entry order per tile: counter-clockwise ring walk
 * from the lower-left node, bottom/right/top/left at corners. */
nosdd_status nosdd_robin_trace(nosdd_problem *p, const nosdd_c32 *x, nosdd_c32 *g);

/* Geometry queries (host). info[10] = {x0, x1, y0, y1, cx0, cx1, cy0, cy1,
 * local_offset (cells, within one wavelength's packed local vector),
 * trace_offset (entries)}.  Totals: n_tiles, local cells per wavelength,
 * trace entries per wavelength. */
nosdd_status nosdd_tile_info(const nosdd_problem *p, int tile, long long info[10]);
nosdd_status nosdd_sizes(const nosdd_problem *p, int *n_tiles, long long *local_cells,
                         long long *trace_entries, int *n_coarse);

/* Coarse basis fields of wavelength wl (host copy), for inspection and tests:
 * phi[n_coarse] boxes concatenated in tile order, column l of tile t being
 * [bh][bw] cells of the tile's core grown by one cell (clipped to the grid);
 * box[4 * n_tiles] = {bx0, by0, bw, bh} per tile.  Either pointer may be NULL. */
nosdd_status nosdd_coarse_basis(const nosdd_problem *p, int wl, nosdd_c32 *phi, long long *box);

/* Kernel timing of the solve path (HIP events recorded on the context stream
 * around every launch group while enabled).  Classes: 0 = subdomain solves
 * (gather, block-Thomas, core scatter), 1 = operator and residuals,
 * 2 = Arnoldi (Gram-Schmidt passes, reductions, Givens, scaling),
 * 3 = coarse correction.  nosdd_profile(p, 1) enables and resets the
 * counters, nosdd_profile(p, 0) disables.  units[0] counts (subdomain, RHS)
 * solves. */
nosdd_status nosdd_profile(nosdd_problem *p, int enable);
nosdd_status nosdd_kernel_times(const nosdd_problem *p, double ms[4], long long launches[4], long long units[4]);

/* Gradient of the inverse-design figure of merit (adjoint-variables method of
 * the paper's inverse-design section, with implicit differentiation of the
 * converged fields):
 *   FoM = sum over wavelengths, sources and focal cells f of |E(r_f)|^2,
 *   grad[iy][ix] = dFoM/d eps(ix, iy) = sum 2 k0^2 Re(E lam),  A^T lam = P conj(E).
 * The adjoint field is obtained from the same two-level Schwarz-FGMRES: with
 * S = diag(s_x s_y) (centre PML stretches) S A is complex symmetric, so
 * lam = S mu with A mu = S^-1 P conj(E).  Two solves per call (forward, then
 * adjoint) with the options o (x0 ignored).  J: device [n_src][ny][nx];
 * focal: host int [n_focal][2] = (ix, iy), repeats allowed; grad: device
 * float [ny][nx] (every cell; mask the design region yourself); fom: host
 * double, nullable; iters: host int [2][n_wl * n_src] (forward, adjoint
 * outer iterations), nullable.  Returns NOSDD_NOT_CONVERGED (outputs valid)
 * if either solve stopped at max_iters. */
nosdd_status nosdd_fom_gradient_device(nosdd_problem *p, const nosdd_c32 *J, int n_src, const int *focal,
                                       int n_focal, const nosdd_solve_opts *o, double *fom, float *grad,
                                       int *iters);

/* Launch-parameter autotuning (enabled by default).  At the first solve of a
 * given batch shape, before any graph capture, the library times candidate
 * launch parameters on the problem's own buffers and keeps the fastest: the
 * number of workgroups per right-hand side of the Gram-Schmidt passes (per
 * basis-size bucket j + 1 <= 8, 16, 24, 32) and the prefetch depth of the
 * batched subdomain solve (the depths the subdomain block size allows).  The
 * arithmetic is the same for every candidate.  Disabling restores the
 * defaults.  nosdd_tuning reports out[6] = {solve prefetch depth (0 =
 * default), workgroups per RHS for the four buckets, flags: 1 Gram-Schmidt
 * tuned, 2 subdomain solve tuned}. */
nosdd_status nosdd_autotune(nosdd_problem *p, int enable);
nosdd_status nosdd_tuning(const nosdd_problem *p, int out[6]);

/* Launch mode of the solve loop.  Enabled (the default): every Arnoldi step
 * of a restart cycle (subdomain solves, operator, coarse correction,
 * Gram-Schmidt passes, Givens) is captured once into a HIP graph on a private
 * stream and replayed on the context stream; convergence is read from pinned
 * host memory two steps behind, so the host never blocks the device inside a
 * cycle.  Graphs are rebuilt when buffers, sizes or solve options change.
 * Disabled, or while nosdd_profile is on: the same kernels are launched one
 * by one.  Results are bit-identical in both modes. */
nosdd_status nosdd_graphs(nosdd_problem *p, int enable);
/* Subdomain solves of the FGMRES preconditioner when a wavelength has at
 * least 4 sources (blocks at most 112 cells wide, grid and packed subdomain
 * vectors at most 2^23 cells, so that one group's vectors stay below 2^31
 * bytes): enabled (default),
 * one workgroup per subdomain, wavelength and group of 32 (16 above 80-cell
 * blocks) sources reads each factor block once and forms the block's products
 * for the whole group as FP32 MFMA contractions; disabled, one workgroup per
 * subdomain and source (the right-hand sides share the factor stream only
 * through the caches).  Same arithmetic per product up to summation order. */
nosdd_status nosdd_multi_source(nosdd_problem *p, int enable);
/* Second Gram-Schmidt pass of the outer FGMRES (both forms orthogonalise
 * twice against the basis; flexible GMRES, Algorithm 1 recurrence): enabled
 * (default), the second pass's correction and the normalisation of each new
 * basis vector are kept in a small triangular FP64 map from the stored
 * vectors to the orthonormal basis, so a step makes two passes over the
 * vectors (dots; update fused with the second dots) and the preconditioner
 * is applied to the stored vector; disabled, the second pass runs where the
 * Daniel-Gragg-Kaufman-Stewart test asks for it and a third pass writes the
 * normalised vector.  Same Krylov space in exact arithmetic. */
nosdd_status nosdd_stored_basis(nosdd_problem *p, int enable);

/* Exact-LU fallback of the neural subdomain solver.  Every subdomain is
 * factorised at set-up whatever the subdomain solver, so in each sweep of a
 * problem set up with sub_solver = 1 an inner NN-FGMRES solve (one subdomain,
 * one right-hand side) whose recurrence meets a NaN or Inf, or whose final
 * residual estimate is not below 0.99 of its right-hand side's norm (the
 * network did not reduce the subdomain residual), is replaced by the exact
 * block-Thomas solve of that subdomain in the same sweep (Algorithm 1 leaves
 * the inner solve's quality to the network; exact subdomain LU is the solver
 * the network approximates).  *count receives the number of such
 * replacements since the current or last solve began (sweeps and local
 * solves outside a solve add to it); 0 for sub_solver = 0. */
nosdd_status nosdd_fallback_count(const nosdd_problem *p, long long *count);

/* Timing of the last solve (ms, GPU events): setup, total solve, iterations. */
nosdd_status nosdd_last_timing(const nosdd_problem *p, double *setup_ms, double *solve_ms,
                               int *outer_iters);

#ifdef __cplusplus
}
#endif
#endif /* NOSDD_H */
