/*
 * specmg: multiscale spectral multigrid preconditioned CG for the TPFA
 * pressure system of Darcy flow on a 3D Cartesian grid (arXiv 2403.19342),
 * implemented with hand-written HIP kernels for gfx950 (MI355X).
 *
 * Problem (Section 2): -div(K grad p) = f in the unit box with no-flow
 * boundaries, K = kappa I or diag(kappa_x, kappa_y, kappa_z), discretised by lowest-order Raviart-Thomas
 * elements with trapezoidal quadrature; eliminating the velocity gives the
 * symmetric positive semidefinite system A p = f (eq. p), a 7-point stencil
 * whose face coefficients are harmonic means of kappa/h^2 (eq. discrete
 * varia and fig. kappa edge).  The source must have zero sum and the
 * returned pressure has zero mean (Section 2.1, space W).
 *
 * Conventions shared by every entry point:
 *  - Cell vectors are float64 arrays of nx*ny*nz values, index
 *    i + nx*(j + ny*k) (x fastest), resident in device memory and owned by
 *    the caller; the library never frees or retains them past the call.
 *  - `stream` is a hipStream_t (may be NULL for the null stream).  Work is
 *    enqueued on it; calls return after the work they enqueued is complete
 *    unless stated otherwise.
 *  - Every int-returning call returns SPECMG_OK (0) or a negative error
 *    code; specmg_last_error() then holds a message for the calling thread.
 *    A context stays usable after SPECMG_ENOCONV and SPECMG_EBREAKDOWN.
 *  - A context is not thread-safe: calls on one context must not overlap.
 */
#ifndef SPECMG_H
#define SPECMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPECMG_OK 0
#define SPECMG_EINVAL (-1)       /* bad sizes, options or pointers          */
#define SPECMG_EINVAL_PERM (-2)  /* permeability not positive and finite    */
#define SPECMG_ERHS (-3)         /* |sum f| > 1e-12 sum |f| (no compatible source) */
#define SPECMG_ENOCONV (-4)      /* max_iter reached; x holds the last iterate */
#define SPECMG_EBREAKDOWN (-5)   /* p^T A p <= 0 or not finite in CG, or a
                                    singular Hessenberg column in GMRES     */
#define SPECMG_EEIG (-6)         /* a local eigensolve did not converge     */
#define SPECMG_EFACT (-7)        /* a smoother pivot or the coarsest factor is not SPD */
#define SPECMG_EDEVICE (-8)      /* HIP runtime error                       */

#define SPECMG_FP64 0            /* every level in float64                  */
#define SPECMG_FP32_VCYCLE 1     /* V-cycle in float32, CG and coarsest in float64 */
#define SPECMG_FP32_BASIS 2      /* float64 throughout, the level-2 basis stored
                                    in float32 (restriction and prolongation
                                    read it and sum in float64)               */
#define SPECMG_FP32_STORE 3      /* the fine level of the V-cycle stores kappa~,
                                    the IC(0) pivots, the level-2 basis and its
                                    vectors u and t in float32 and computes in
                                    float64 (every residual formed in float64
                                    from the stored values); coarse levels,
                                    the coarsest solve and CG in float64;
                                    flexible CG with residual replacement     */

#define SPECMG_WS_NONE 0         /* cold-started local eigensolves          */
#define SPECMG_WS_CNN 1          /* warm starts predicted by the 3D CNN     */

typedef struct specmg_ctx specmg_ctx;

/* Grid: nx, ny, nz cells with spacings hx, hy, hz, any positive values
 * (Section 5 uses the unit cube, h = 1/N; Section 6 a grid whose three
 * spacings differ).  The normalised permeability of eq. (velocity) is
 * kappa / h_d^2 on the faces of axis d and the weight of eq. (spepb) is its
 * trace.  The learned warm start needs equal spacings.  `sub` is the edge
 * of the level-2 elements in cells (the coarse grid T_c; only 8 is
 * supported), `agg` the number of level-l elements per axis in one
 * level-(l+1) element (2 or 4).  Each of nx, ny, nz
 * must be divisible by sub * agg^(levels-2). */
typedef struct {
    int32_t nx, ny, nz;
    double hx, hy, hz;
    int32_t sub;
    int32_t agg;
} specmg_grid;

/* Options.  levels >= 2 is the number of grids (Algorithm 1 has three);
 * eigs_per_subdomain (1..8) is the target count of eigenvectors kept per
 * level-2 element (L_c, strategy 1 of Section 5; with eig_threshold > 0 the
 * number of candidates of strategy 2), grown or shrunk by at most
 * 3 so that no cluster of equal eigenvalues is split (relative gap
 * cluster_rtol).  Levels >= 3 use eigs_coarse (L_cc) the same way, or, when
 * eig_threshold_coarse > 0, keep the eigenvectors whose eigenvalues lie below
 * that threshold (B_cc, strategy 2 of Section 5; at least one, at most
 * eigs_coarse, then the cluster rule).  Each level's arrays are padded to its
 * own width, target + 3.  nu (fine level) and nu_c (coarse levels) are the
 * numbers of block-Jacobi sweeps before and after the coarse correction
 * (Section 5: nu, nu_c in {1, 2}; the repeated sweep is
 * u += M^-1 (f - A u)).  eig_tol is the residual tolerance of the
 * local eigensolves relative to the spectral radius of the local pencil. */
typedef struct {
    int32_t levels;
    int32_t eigs_per_subdomain;
    int32_t nu;
    int32_t precision;       /* SPECMG_FP64, _FP32_VCYCLE, _FP32_BASIS or _FP32_STORE */
    int32_t warm_start;      /* SPECMG_WS_NONE or SPECMG_WS_CNN   */
    const void* cnn_weights; /* WS_CNN only (eigs_per_subdomain even): device
                                pointer to the network's bf16 parameter vector
                                for k = eigs_per_subdomain (layout below,
                                specmg_cnn_param_count(k) values); read during
                                specmg_setup only */
    double eig_tol;          /* default 1e-12 when <= 0 */
    double cluster_rtol;     /* default 1e-6 when <= 0  */
    double ws_resid_tol;     /* WS_CNN: default 1e-3 when <= 0.  Each level-2
                                element's eigensolve starts from the predicted
                                block and stops at this residual (relative to
                                the spectral bound of the local pencil, as
                                eig_tol); an element that does not reach it
                                within 4 Chebyshev cycles falls back to the
                                exact solve (eig_tol) from the cold start */
    int32_t eigs_coarse;     /* L_cc, 0..20; 0 = eigs_per_subdomain.  With
                                agg 4 and four or more levels at most 9.
                                Above 10 the coarse-coarse eigensolves use a
                                block of 20 or 26 vectors, and a level of
                                width L_cc + 3 > 13 runs the wide (spilling)
                                form of the coarse smoother */
    double eig_threshold_coarse; /* B_cc >= 0; 0 = fixed count eigs_coarse.
                                Eigenvalues are those of eq. spectral cc with
                                S-normalised bases (dimensionless) */
    int32_t nu_c;            /* coarse-level sweeps nu_c (1 or 2); 0 = nu */
    double eig_threshold;    /* B_c >= 0; 0 = fixed count eigs_per_subdomain.
                                Strategy 2 of Section 5 at the level-2
                                elements: keep the eigenvalues of eq. spepb
                                below B_c (S-normalised, dimensionless), at
                                least one and at most eigs_per_subdomain
                                candidates, then the cluster rule */
} specmg_opts;

/* Device allocator for a context's memory (specmg_setup_alloc): alloc
 * returns `bytes` bytes of device memory usable on `stream` (the stream
 * given to set-up), or NULL; free releases a pointer alloc returned.  `user`
 * is passed back unchanged.  The callbacks are called from the calling
 * thread during specmg_setup_alloc, during the first specmg_gmres_solve
 * calls (its workspace) and during specmg_destroy, so they and `user` must
 * stay valid until the context is destroyed.  A PyTorch binding passes its
 * caching allocator here, so that PyTorch owns every device byte. */
typedef struct {
    void* (*alloc)(size_t bytes, void* stream, void* user);
    void (*free)(void* ptr, void* user);
    void* user;
} specmg_allocator;

/* Outcome of a solve.  iters counts products A p (one per CG iteration). */
typedef struct {
    int32_t iters;
    int32_t converged;
    double rel_resid;        /* recursive ||r|| / ||b|| at exit        */
    double rel_resid_true;   /* ||b - A x|| / ||b|| of the returned x  */
    double setup_ms;         /* wall time of specmg_setup               */
    double solve_ms;         /* wall time of this solve                 */
    int32_t n_levels;
    int32_t dims[8];         /* dims[0] = n, dims[l-1] = dim W_l        */
    int32_t eig_unconverged; /* local eigensolves that hit the cycle cap */
    int32_t ws_fallbacks;    /* WS_CNN: elements that fell back to the exact solve */
    int32_t replacements;    /* true-residual replacements in CG        */
} specmg_solve_info;

/* Set-up phase (Section 3 and Section 5): harmonic-mean transmissibilities,
 * local spectral problems on every element of every coarse level (eq. spepb,
 * eq. spectral cc), Galerkin coarse operators A_{l+1} = R A_l R^T, IC(0)
 * and block-IC(0) smoother factors, and the factored coarsest operator.
 * perm_dev: device float64 permeability, read during the call only:
 * perm_components = 1: kappa, nx*ny*nz values (isotropic K = kappa I);
 * perm_components = 3: kappa_x, kappa_y, kappa_z one after the other, 3 nx*ny*nz
 * values (orthotropic K = diag(kappa_x, kappa_y, kappa_z), Section 2.1; the
 * faces of axis d take the harmonic mean of kappa_d / h_d^2, the weight of
 * eq. spepb is the sum of the three; needs precision SPECMG_FP64 or
 * SPECMG_FP32_BASIS and no learned warm start).
 * On success *out receives a new context, released with specmg_destroy.
 * Errors: SPECMG_EINVAL, SPECMG_EINVAL_PERM, SPECMG_EEIG (context still
 * returned; info reports the count), SPECMG_EFACT, SPECMG_EDEVICE. */
int specmg_setup(const double* perm_dev, int32_t perm_components, const specmg_grid* grid,
                 const specmg_opts* opts, void* stream, specmg_ctx** out);

/* specmg_setup with every device allocation of the context (its arrays, the
 * set-up's transient workspaces, the GMRES workspace) taken from `allocator`
 * (NULL: hipMalloc and hipFree, as specmg_setup).  Errors as specmg_setup,
 * plus SPECMG_EINVAL for an allocator without both callbacks and
 * SPECMG_EDEVICE when alloc returns NULL. */
int specmg_setup_alloc(const double* perm_dev, int32_t perm_components, const specmg_grid* grid,
                       const specmg_opts* opts, const specmg_allocator* allocator, void* stream,
                       specmg_ctx** out);

/* One application of the preconditioner, z = P^{-1} r: Algorithm 1 applied
 * recursively (pre-smooth, restrict, coarse map, prolong, post-smooth) with
 * the pseudo-inverse at the coarsest level.  r_dev, z_dev: device float64
 * cell vectors (must not alias).  Asynchronous: returns once enqueued. */
int specmg_apply_precond(specmg_ctx* ctx, const double* r_dev, double* z_dev, void* stream);

/* Preconditioned CG on A x = rhs to ||b - A x|| <= tol ||b||.  rhs_dev must
 * sum to zero (SPECMG_ERHS otherwise).  x_dev: in: initial guess when
 * use_x0 != 0, out: solution shifted to zero mean.  info may be NULL.
 * Errors: SPECMG_ERHS, SPECMG_EINVAL (tol <= 0, max_iter < 1),
 * SPECMG_ENOCONV, SPECMG_EBREAKDOWN, SPECMG_EDEVICE. */
int specmg_pcg_solve(specmg_ctx* ctx, const double* rhs_dev, double* x_dev, int32_t use_x0,
                     double tol, int32_t max_iter, specmg_solve_info* info, void* stream);

/* Restarted flexible GMRES with the preconditioner applied on the right,
 * the outer Krylov solver of the paper's experiments (Section 5: GMRES,
 * relative tolerance 1e-6; restart length 30 is that library's default).
 * Solves A x = rhs to ||b - A x|| <= tol ||b||: a cycle of at most
 * `restart` Arnoldi steps (classical Gram-Schmidt applied twice) ends when
 * the Arnoldi residual reaches tol ||b||, then the true residual decides;
 * if it is still above, GMRES restarts from it.  The stored directions
 * z_j = P^{-1} v_j make the FP32 V-cycle (a preconditioner that is not a
 * fixed linear map) admissible.  rhs_dev must sum to zero; x_dev as for
 * specmg_pcg_solve (out: zero mean).  info->iters counts Arnoldi steps,
 * info->replacements the restarts.  Workspace: (2 restart + 2) float64 cell
 * vectors, allocated on the first call that needs them and kept by the
 * context.  Errors: SPECMG_ERHS, SPECMG_EINVAL (tol <= 0, max_iter < 1,
 * restart outside [1, 64], rhs_dev == x_dev), SPECMG_ENOCONV,
 * SPECMG_EBREAKDOWN (a singular Hessenberg column), SPECMG_EDEVICE. */
int specmg_gmres_solve(specmg_ctx* ctx, const double* rhs_dev, double* x_dev, int32_t use_x0,
                       int32_t restart, double tol, int32_t max_iter, specmg_solve_info* info,
                       void* stream);

/* Velocity recovery v = M_t^{-1} B^T p (Section 2.2; the two-point flux of
 * eq. (velocity)): vx_dev[i] (vy, vz) receives the flux through the +x (+y,
 * +z) face of cell i, -kappa_f (p_j - p_i) / h with the harmonic mean
 * kappa_f of the two cells' permeabilities, and 0 on the no-flow boundary.
 * p_dev: float64 cell vector (a pressure from specmg_pcg_solve or
 * specmg_gmres_solve); all arrays n float64 values, x fastest, caller-owned,
 * none may alias another.  Asynchronous.  Errors: SPECMG_EINVAL,
 * SPECMG_EDEVICE. */
int specmg_recover_flux(specmg_ctx* ctx, const double* p_dev, double* vx_dev, double* vy_dev,
                        double* vz_dev, void* stream);

/* Cell mass balance of a face flux (Section 2.2, conservation on a fine
 * element): res_dev[i] = (1/h) sum_axes (v_{+} - v_{-}) - f_dev[i], the
 * discrete divergence of v minus the source, with v_{-} the + face of the
 * lower neighbour (0 at the boundary).  For the flux recovered from p it
 * equals (A p - f)_i up to rounding.  Layout and ownership as for
 * specmg_recover_flux.  Asynchronous.  Errors: SPECMG_EINVAL,
 * SPECMG_EDEVICE. */
int specmg_mass_balance(specmg_ctx* ctx, const double* vx_dev, const double* vy_dev,
                        const double* vz_dev, const double* f_dev, double* res_dev, void* stream);

/* y = A x with the fine TPFA operator (eq. p).  Asynchronous. */
int specmg_apply_operator(specmg_ctx* ctx, const double* x_dev, double* y_dev, void* stream);

/* ------------------------------------------------------------------------
 * Two-phase flow (Section 6, eqs. v, div_v, trans_S and the improved IMPES
 * scheme, eqs. IMP and ES).  Water saturation S, fluid law of Section 6:
 * S* = clamp((S - 0.2)/0.6, 0, 1), k_w = S*^2, k_o = (1 - S*)^2,
 * mu_w = 0.3, mu_o = 3.0, lambda = k_w/mu_w + k_o/mu_o,
 * f_w = (k_w/mu_w)/lambda.  Rate-controlled wells: q > 0 injects water,
 * q < 0 produces the cell's mixture (q_w = f_w(S) q).  Pressure steps use
 * specmg_setup on the permeability lambda(S) kappa and a solve warm-started
 * from the previous pressure; these calls need no context.
 * ---------------------------------------------------------------------- */

/* perm_eff_dev[i] = perm_dev[i] * lambda(s_dev[i]) for i < n (eq. v: the
 * pressure system of a step has the permeability lambda(S) K).  Device
 * arrays of n doubles, owned by the caller; perm_eff_dev may alias
 * perm_dev.  Asynchronous.  Errors: SPECMG_EINVAL (null pointer, n < 0),
 * SPECMG_EDEVICE. */
int specmg_total_mobility(const double* perm_dev, const double* s_dev, double* perm_eff_dev, int64_t n,
                          void* stream);

/* `substeps` explicit Euler steps of the saturation equation (eq. ES) with
 * the face velocity held fixed:
 *   phi_i (S_i' - S_i)/dt + sum_d (F_+ - F_-)/h_d = q_w,i,
 * F = f_w(S_upstream) v on the faces of axis d,
 * the upstream cell being the one the face velocity leaves, and
 * dt = ds_max / max_i |dS_i/dt| (0 when every rate is zero), so that no cell
 * changes by more than ds_max per sub-step.
 * grid: nx, ny, nz >= 1 (any sizes), hx, hy, hz > 0; sub and agg unused.
 * phi_dev, q_dev: porosity (> 0) and total source density per cell;
 * vx/vy/vz_dev: the velocity through the +x/+y/+z face of every cell (the
 * layout of specmg_recover_flux; values on boundary faces are not read);
 * s_dev: in: S at the start, out: S after the sub-steps.  All (nz, ny, nx),
 * x fastest, doubles.  work_dev: caller-owned scratch of at least
 * 2 n + 2048 doubles.  t_dev: out, one double, the summed sub-step lengths.
 * ds_max in (0, 1], substeps >= 0.  Asynchronous; no host synchronisation
 * between sub-steps.  Errors: SPECMG_EINVAL, SPECMG_EDEVICE. */
int specmg_transport(const specmg_grid* grid, const double* phi_dev, const double* q_dev, const double* vx_dev,
                     const double* vy_dev, const double* vz_dev, double* s_dev, int32_t substeps, double ds_max,
                     double* work_dev, double* t_dev, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, hosts that forbid hipMalloc): specmg_transport
 * without the work argument.  The workspace is a device array built into the
 * library, one per GPU, for grids of at most SPECMG_TRANSPORT_NOALLOC_MAX_CELLS
 * cells (32 MiB + 16 KiB, held from the library's load until the process
 * ends); its address is looked up once per device on the first call there.
 * The call allocates nothing.  All calls on one GPU share that workspace:
 * calls that overlap on one GPU (other threads or streams) race, so callers
 * serialise them.  Arguments, layout, results and asynchrony as for
 * specmg_transport.  Errors: SPECMG_EINVAL (as specmg_transport, or more
 * than SPECMG_TRANSPORT_NOALLOC_MAX_CELLS cells), SPECMG_EDEVICE. */
#define SPECMG_TRANSPORT_NOALLOC_MAX_CELLS 2097152
int specmg_transport_noalloc(const specmg_grid* grid, const double* phi_dev, const double* q_dev,
                             const double* vx_dev, const double* vy_dev, const double* vz_dev, double* s_dev,
                             int32_t substeps, double ds_max, double* t_dev, void* stream);

/* Set-up information: dims[l-1] = dim W_l for l = 1..levels, the element
 * counts per level, and widths[l-1] = the padded per-element width of level
 * l (its target count plus 3; widths[0] = 1).  Arrays must hold 8 entries;
 * any pointer may be NULL. */
int specmg_get_info(specmg_ctx* ctx, int32_t* levels, int32_t* dims, int32_t* elems,
                    int32_t* widths, specmg_solve_info* setup_info);

/* Copy one set-up array of coarse level `level` (2..levels) to host memory,
 * for inspection and tests.  `which`:
 * With W = widths[level-1] and Wlo = widths[level-2] from specmg_get_info:
 *   0 nkeep   int32  [m]
 *   1 lambda  float64 [m][W]          ascending local eigenvalues (padded with 0)
 *   2 basis   float64 level 2: [m][W][512] columns of R_c^T per element,
 *             S-normalised; level >= 3: [m][W][agg^3*Wlo] columns of R^T
 *   3 Adiag   float64 [m][W][W] diagonal blocks of A_l
 *   4 Aoff    float64 [m][3][W][W] blocks A_l(e, e + x|y|z)
 *   5 status  int32  [m]  Chebyshev cycles used by the local eigensolve, -1 if
 *             it stopped at the cycle cap
 * `bytes` must equal the array size; returns SPECMG_EINVAL otherwise. */
int specmg_copy_level(specmg_ctx* ctx, int32_t level, int32_t which, void* host_dst, size_t bytes);

/* Per-kernel timing of later specmg_pcg_solve calls (on != 0) or off.
 * Each fine-level kernel of the CG iteration and the coarsest product are
 * timed by HIP events the dispatch itself stamps on the solve's stream; the
 * coarse part of the V-cycle as a whole is bracketed by events recorded
 * around it.  Turning it on resets the accumulated totals. */
int specmg_set_profiling(specmg_ctx* ctx, int32_t on);

/* Accumulated event times (ms) and launch counts per kernel class since
 * profiling was turned on, and the algorithmic bytes one launch of the class
 * moves (compulsory HBM traffic of its inputs and outputs).  Classes:
 * 0 CG operator (A p, p.Ap)            1 pre-smoothing (r update, IC(0))
 * 2 residual + restriction             3 prolongation
 * 4 post-smoothing (its residual, IC(0), r.z)
 * 5 coarse part of the V-cycle (every kernel of levels 2..L, the coarsest
 *   product included)                  6 coarsest product alone
 * 7 CG direction update (p = z + beta p, the deferred x update).
 * Bytes of classes 5 and 6 count kept widths (not the padded storage).
 * Arrays hold 8 entries. */
int specmg_get_profile(specmg_ctx* ctx, double* ms, int32_t* launches, double* bytes);

/* Releases every device and host resource of the context (NULL is a no-op). */
void specmg_destroy(specmg_ctx* ctx);

/* Message of the last error on the calling thread ("" if none). */
const char* specmg_last_error(void);

/* ------------------------------------------------------------------------
 * Learned warm start (an extension of the method; not in the paper).  A
 * 3-layer 3D CNN maps each level-2 element's log-permeability patch to k
 * cell vectors that start the element's eigensolve (Section 3, eq. spepb).
 *
 *   patch: log kappa on the 8^3 cells and a one-cell halo (10^3 values, x
 *          fastest; outside the domain the nearest boundary cell repeats),
 *          standardised by its own mean and standard deviation (population,
 *          1e-6 added under the root).
 *   c_j:  the k lowest cosine modes of the homogeneous element (the cold
 *         start block), cos(pi p (x+1/2)/8) cos(pi q (y+1/2)/8)
 *         cos(pi r (z+1/2)/8) with (p,q,r) = (000), (100), (010), (001),
 *         (110), (101), (011), (111) in this order
 *   a1 = relu(conv([patch, c_0..c_{k-1}], W1) + b1)  1+k -> 32 channels, no
 *        padding (-> 8^3); the mode channels are evaluated on the patch grid
 *   a2 = relu(conv(a1, W2) + b2)      32 -> 32 channels, zero padding 1
 *   X  = c + conv(a2, W3) + b3        32 -> k channels, zero padding 1
 * conv(x, W)[o][p] = sum_c sum_{t in {0,1,2}^3} W[o][c][t] x[c][p + t - pad].
 * k is 2, 4, 6 or 8.  Parameter vector, in this order: W1[32][1+k][27],
 * b1[32], W2[32][32][27], b2[32], W3[k][32][27], b3[k]; taps
 * t = 9 dz + 3 dy + dx.  Weights are used as bfloat16 values and every
 * product is accumulated in float32.
 *
 * Network outputs are float32 [count][k][512], cell order x fastest.
 *
 * Training loss of one element: with S its weight diagonal (tr K~, any
 * positive scale; normalised to mean 1 inside) and Phi its first k
 * eigenvectors (Phi^T S Phi = I up to the same scale), the S-distance of
 * Phi from span(X): || Phi - X^T C* ||_S^2, C* = (X S X^T)^-1 X S Phi.  The
 * batch loss is the mean over elements.
 * ---------------------------------------------------------------------- */

typedef struct specmg_cnn specmg_cnn;   /* network workspace, owned by the library */

/* Length of the parameter vector for k outputs (k = 2, 4, 6, 8), -1 otherwise. */
int64_t specmg_cnn_param_count(int32_t k);

/* Workspace for batches of at most max_batch elements (activations and
 * gradients: about 256 KiB per element).  EINVAL for k not in {2, 4, 6, 8}. */
int specmg_cnn_create(int32_t k, int32_t max_batch, specmg_cnn** out);
void specmg_cnn_destroy(specmg_cnn* net);

/* Load parameters: exactly one of theta32 (float32 master values, rounded
 * to bf16 here) and theta16 (bf16 values) is non-NULL; device pointers of
 * specmg_cnn_param_count(k) values, read before the call returns on the
 * stream's timeline. */
int specmg_cnn_load(specmg_cnn* net, const float* theta32, const uint16_t* theta16, void* stream);

/* Patches of level-2 elements e0 .. e0+count-1 (x-fastest element order of
 * the 8^3 tiling of `grid`, whose nx, ny, nz must be multiples of 8, hx > 0):
 * patches_dev receives count*1000 floats; s_dev (optional) receives the
 * elements' weight diagonals tr K~ = 3 kappa / hx^2, count*512 doubles (the
 * normalisation of the set-up's level-2 basis, Section 3).  EINVAL for a
 * bad grid or range. */
int specmg_cnn_patches(const double* perm_dev, const specmg_grid* grid, int32_t e0, int32_t count,
                       float* patches_dev, double* s_dev, void* stream);

/* X_dev = network(patches_dev), 1 <= count <= max_batch.  Keeps the hidden
 * activations for a following specmg_cnn_loss_backward on the same batch. */
int specmg_cnn_forward(specmg_cnn* net, const float* patches_dev, int32_t count, float* X_dev, void* stream);

/* Loss of the batch (mean over elements) and its gradient w.r.t. the
 * parameter vector (grad_dev: specmg_cnn_param_count(k) floats,
 * overwritten).  X_dev is the output of the preceding forward call with the
 * same patches_dev and count (EINVAL otherwise); phi_dev holds the target
 * vectors [count][ldphi][512] (the first k rows are used); s_dev the
 * weights [count][512].  loss (host, optional) is written after the call
 * synchronises the stream. */
int specmg_cnn_loss_backward(specmg_cnn* net, const float* patches_dev, const float* X_dev, const double* phi_dev,
                             int32_t ldphi, const double* s_dev, int32_t count, double* loss, float* grad_dev,
                             void* stream);

/* One Adam step (bias-corrected, step >= 1) on n float32 parameters with
 * moment buffers m1, m2 (zero before step 1); theta16_dev (optional)
 * receives the updated values rounded to bf16. */
int specmg_cnn_adam(float* theta_dev, const float* grad_dev, float* m1_dev, float* m2_dev, int64_t n, double lr,
                    double beta1, double beta2, double eps, int32_t step, uint16_t* theta16_dev, void* stream);

#ifdef __cplusplus
}
#endif
#endif
