/*
 * slrf.h -- C ABI of the shifted-Laplace rational filter (SLRF) eigensolver for
 * gfx950 (AMD Instinct MI355X).
 *
 * Problem (Wang, Meerbergen, Vandebril, An, Mo, arXiv:2503.21618, Section 1):
 * every eigenpair (lambda, x) of A x = lambda B x with lambda in (0, gamma], for
 * sparse symmetric positive definite A (stiffness) and B (mass).
 *
 * Method (Algorithm 1, Section 3): rational-filter subspace iteration.  Each
 * outer iteration applies the filter Phi(A, B) = sum_j 2 Re(w_j (A - sigma_j B)^{-1} B)
 * to an n x L block (N complex shifted solves per column, conjugate poles folded
 * into the real part, Section 3), then Rayleigh-Ritz, then relative residuals
 * rho_i = ||A x_i - theta_i B x_i||_2 / (|theta_i| ||B x_i||_2).  Poles lie on the
 * shifted-Laplace line sigma_j = x_j (1 + alpha i) (Section 3.1, equation of
 * the lines L+-).
 *
 * Conventions for every call:
 *  - Dense blocks are row-major (n, L) float64 on the DEVICE: element (i, l) at
 *    ptr[i * L + l] (a contiguous torch tensor of shape (n, L)).
 *  - CSR arrays passed to slrf_create are HOST pointers, int32 row pointers and
 *    column indices, float64 values, columns sorted within each row.
 *  - The caller owns every buffer.  The library never allocates device memory:
 *    all device scratch lives in the caller's workspace (size from
 *    slrf_workspace_bytes), which must outlive the context.
 *  - Work is enqueued on the HIP stream given at create; calls that return host
 *    data synchronise that stream before returning.
 *  - A context is not thread-safe; use one context per stream.
 *  - Errors: the return value is the status; slrf_last_error(ctx) gives detail.
 *    No C++ exception crosses the ABI.
 */
#ifndef SLRF_H
#define SLRF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct slrf_ctx_s* slrf_ctx;

typedef enum {
  SLRF_OK = 0,
  SLRF_E_INVALID_ARG = 1,        /* bad size, NULL pointer, unsorted/out-of-range CSR, NaN, A or B not symmetric */
  SLRF_E_NOT_SPD = 2,            /* a diagonal entry of A or B is <= 0 or missing */
  SLRF_E_WORKSPACE = 3,          /* workspace too small or misaligned (256 B) */
  SLRF_E_DEVICE = 4,             /* a HIP runtime call failed */
  SLRF_E_NOT_CONVERGED = 5,      /* outer iteration limit reached; partial result written */
  SLRF_E_SUBSPACE_TOO_SMALL = 6, /* every one of the L Ritz values lies in (0, gamma] */
  SLRF_E_BREAKDOWN = 7           /* projected problem not solvable (non-finite Gram) */
} slrf_status;

typedef enum { SLRF_FP64 = 0, SLRF_MIXED = 1 } slrf_precision;

/* Pole set in the upper half plane (Section 3: the N conjugate partners are
 * implied).  sigma and weight point to 2N HOST doubles, (re, im) interleaved;
 * Im(sigma_j) > 0 is required. */
typedef struct {
  int32_t n_poles;
  const double* sigma;
  const double* weight;
} slrf_poles;

typedef struct {
  int32_t precision;   /* slrf_precision.  FP64: complex FP64 inner solves.  MIXED:
                          complex FP32 inner solves with FP64 defect correction */
  double inner_tol;    /* relative residual ||f - S y|| / ||f|| of each shifted solve
                          (paper Section 4.2: 1e-13) */
  int32_t inner_maxit; /* inner-solver iteration limit per solve (paper: 1000) */
  double outer_tol;    /* tau of the residual test (paper Section 4.2: 1e-8) */
  int32_t outer_maxit; /* outer (subspace) iteration limit */
  int32_t check_every; /* inner iterations between host polls of the convergence count */
  uint64_t seed;       /* SplitMix64 seed of the Gaussian start block when V0 is NULL */
  int32_t precond;     /* preconditioner M_j of the shifted operator A - sigma_j B:
                          0 auto: ILU(0) if the merged pattern has nnz <= 5 n, else Jacobi
                          1 point Jacobi, M_j = diag(A) - sigma_j diag(B)
                          2 ILU(0) on the merged pattern (requires nnz <= 5 n)
                          3 node block Jacobi for three unknowns per node (unknowns
                            3k, 3k+1, 3k+2 form node k; requires n divisible by 3):
                            M_j = blockdiag of the 3x3 node blocks of A - sigma_j B
                          4 multicolour symmetric Gauss-Seidel (COCG only):
                            M_j = (D + L) D^{-1} (D + U) with D the diagonal of
                            A - sigma_j B and L / U its couplings to unknowns of lower /
                            higher colour in a greedy colouring of the pattern's
                            graph (natural order; the parity classes on structured
                            grids); applied in the split form with one backward and one
                            forward colour sweep per iteration
                          5 the same with the 3x3 node blocks as D for a pencil made of
                            nodes (n divisible by 3 and at least half of its rows in
                            triples 3k..3k+2 with one column pattern), the point form
                            of 4 for any other pencil; a batch may hold both kinds
                          The shifted operator preconditioner of Section 4.2 is an ILU
                          (drop tolerance 1e-4) with RCM ordering; 4 and 5 are
                          symmetric stand-ins whose sweeps run in parallel. */
  int32_t profile;     /* 1: time the sparse-product and vector-update kernels with HIP
                          events and count the column tiles each launch processes
                          (stats fields spmm_* and update_*); 0: off */
  int32_t graph;       /* 1: capture check_every inner iterations (and the poll of the
                          active count) once per Krylov run as a hipGraph and replay it;
                          needs a non-NULL stream and profile = 0, else ignored.  0: off */
  /* Work decomposition of the Krylov kernels (0 = default).  They change the
   * order of floating-point sums, not the method. */
  int32_t tile_rows;   /* rows per row block (default 16, or 24 for a batch of
                          node-triple pencils only; 1..64) */
  int32_t tile_wgs;    /* workgroups per XCD (default 128, 1..256; grid = 8 * this) */
  int32_t band_rows;   /* rows per sub-band of the sparse-product row order (default
                          1024; -1 = natural row order); applied when a pencil is built */
  int32_t tune;        /* 1: autotune (tile_rows, tile_wgs) per batch shape: the first
                          filter application of a shape not seen before in the process
                          times two inner iterations per candidate and keeps the
                          fastest (cached per process); overrides tile_rows/tile_wgs */
  int32_t solver;      /* inner solver of the shifted systems: 0 BiCGStab (Section 2,
                          the paper's choice), 1 COCG, conjugate gradients with the
                          bilinear form u^T v for the complex-symmetric A - sigma_j B
                          (one sparse product per iteration; symmetric
                          preconditioners only: 1 point Jacobi (also what
                          precond 0 selects), 3 node block Jacobi, 4 and 5 the
                          multicolour SGS; 2 (ILU(0)) is rejected with
                          SLRF_E_INVALID_ARG) */
  int32_t recycle;     /* 1 (mixed precision): each outer iteration after a pencil's
                          first starts its shifted solves from the previous one's
                          solutions carried to the new block, Y0 = Y_prev (X_prev^T B
                          X_new) (exact when X_new lies in span(X_prev)).  Each pencil
                          keeps Y_prev and B X_prev (n x N L complex and n x L real
                          FP64) with its own buffers, which the workspace sizes
                          include.  Default 0 (cold starts, x_0 = 0) */
  double sgs_omega;    /* relaxation factor of the multicolour SGS (precond 4 and 5):
                          symmetric SOR, D replaced by D / omega in
                          M = (D + L) D^{-1} (D + U); a value in (0, 2) applies to
                          every pencil (1: plain SGS).  0 (default): by block size,
                          0.7 for 3x3 node blocks (fewer iterations than 1 on the
                          elasticity pencils measured) and 1 for point blocks */
} slrf_options;

typedef struct {
  int32_t max_iterations;   /* largest inner-solver iteration count over the columns */
  double mean_iterations;   /* mean inner-solver iterations per (pole, column) */
  int64_t spmv;             /* single-vector products with A - sigma_j B (BiCGStab: 2 per
                               full iteration, 1 when a solve stops at the half step;
                               COCG: 1 per iteration; MIXED adds the FP64 defect's
                               product per column and correction round) */
  int32_t n_breakdown;      /* columns stopped by a zero denominator */
  int32_t n_maxit;          /* columns that hit inner_maxit */
  int32_t refinements;      /* MIXED: defect-correction rounds in which this pencil had an
                               open column */
  double max_relres;        /* largest final relative residual over the columns */
  double seconds;           /* wall time of the call */
  /* profile = 1 only (else 0): kernel time from HIP events, launches, and the
   * algorithmic HBM bytes of those launches (each processed column tile reads
   * its input block and writes its output block once; the merged CSR is read
   * once per launch) */
  double spmm_seconds;
  int64_t spmm_launches;
  double spmm_bytes;
  double spmm_columns;      /* columns those launches multiplied (each over all n rows) */
  double update_seconds;
  int64_t update_launches;
  double update_bytes;
} slrf_filter_stats;

typedef struct {
  int32_t outer_iterations;
  int64_t spmv_total;       /* paper Table 4 "spMV" */
  int32_t n_found;          /* converged Ritz pairs in (0, gamma] */
  double max_resid;         /* largest rho_i over those pairs */
  double seconds;           /* wall time of the call */
  double filter_seconds;    /* of which in filter application */
  double inner_iterations;  /* mean inner-solver iterations per (pole, column), all outer its */
  slrf_filter_stats kernels;/* profile = 1: spmm_* / update_* summed over the call */
} slrf_solve_stats;

/* Defaults: FP64, inner_tol 1e-13, inner_maxit 1000, outer_tol 1e-8,
 * outer_maxit 40, check_every 10, seed 1, precond 0 (auto), profile 0, graph 0,
 * tile_rows / tile_wgs / band_rows 0 (defaults), tune 0, solver 0 (BiCGStab), recycle 0,
 * sgs_omega 0 (by block size). */
void slrf_default_options(slrf_options* opt);

/* SLRF pole/weight design, Section 3.1: minimise the delta-weighted L2 distance
 * between Phi(x) = sum_j 2 Re(w_j/(x - sigma_j)) and the step h (1 on [0, gamma],
 * 0 on (gamma, 10 gamma]), delta = beta on [0, gamma], 1 on (gamma, 10 gamma],
 * over sigma_j = x_j (1 + alpha i), x_j in (0, gamma], and complex w_j, plus a
 * ridge term 1e-6 gamma^-2 sum |w_j|^2 that keeps the poles distinct (without it
 * the infimum is a merged pole with unbounded weights).  Host-only.
 * Outputs: sigma_out, weight_out: 2N doubles each, sorted by Re(sigma);
 * sep_factor_out (may be NULL): |Phi'(gamma)| (Definition 3.1).
 * Errors: INVALID_ARG for N < 1 or N > 16, alpha <= 0, beta <= 0, gamma <= 0. */
slrf_status slrf_design_poles(int32_t N, double alpha, double beta, double gamma,
                              double* sigma_out, double* weight_out, double* sep_factor_out);

/* Quadrature-rule filters of Section 3.2 (the filters the SLRF is compared
 * with): N nodes in the upper half-plane on the circle with centre gamma/2 and
 * radius gamma/2, from the midpoint (rule 0), Gauss-Legendre (rule 1) or
 * Gauss-Chebyshev (rule 2) rule in the angle; weights of the contour integral
 * of the spectral projector, so that Phi(x) = sum_j 2 Re(w_j/(x - sigma_j)) is
 * close to 1 inside [0, gamma] and to 0 outside.  Host-only.  Outputs as for
 * slrf_design_poles (2N doubles each, sorted by Re(sigma)); usable as the
 * slrf_poles of slrf_filter_apply and slrf_solve_interval.
 * Errors: INVALID_ARG for an unknown rule, N < 1 or N > 64, gamma <= 0. */
slrf_status slrf_quadrature_poles(int32_t rule, int32_t N, double gamma, double* sigma_out, double* weight_out);

/* Bytes of device workspace slrf_create needs for a pencil with n rows and
 * nnz_union entries in the union of the patterns of A and B, subspace size up
 * to L and up to N poles, at the given precision, with the automatic
 * preconditioner choice (precond = 0). */
slrf_status slrf_workspace_bytes(int64_t n, int64_t nnz_union, int64_t L, int32_t N,
                                 int32_t precision, size_t* bytes);

/* The same for the precision, preconditioner and warm starts (recycle) of opt
 * (NULL: defaults). */
slrf_status slrf_workspace_bytes_for(int64_t n, int64_t nnz_union, int64_t L, int32_t N,
                                     const slrf_options* opt, size_t* bytes);

/* Validates A and B (square, sorted in-range columns, finite values, positive
 * diagonals, symmetric: |m_ij - m_ji| <= 1e-10 sqrt(m_ii m_jj) for M = A and
 * M = B, an entry stored on one side only counting as zero; SLRF_E_INVALID_ARG
 * otherwise), merges them into one CSR over the union
 * pattern with (a_ij, b_ij) value pairs, and uploads it into the workspace.
 * d_workspace: device, 256-byte aligned, ws_bytes from slrf_workspace_bytes_for
 * with the largest L and N that later calls use and the same options.  hip_stream: a hipStream_t
 * (NULL = default stream).  opt may be NULL (defaults).  On failure *out may
 * still hold a context: read slrf_last_error(*out), then slrf_destroy(*out). */
slrf_status slrf_create(slrf_ctx* out, int64_t n,
                        const int32_t* a_rowptr, const int32_t* a_col, const double* a_val,
                        const int32_t* b_rowptr, const int32_t* b_col, const double* b_val,
                        void* d_workspace, size_t ws_bytes, int64_t max_L, int32_t max_poles,
                        const slrf_options* opt, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that forbid hipMalloc, harnesses without an
 * allocator): slrf_create without a workspace argument.  The context lives in a
 * file-scope device array of SLRF_STATIC_SCRATCH_BYTES (64 MiB) that the
 * library holds on every device it runs on until the process ends; the device
 * is the current one at this call.  The call and every later call on the
 * context allocate no device memory.  Arguments, validation and the returned
 * context are those of slrf_create; the caller still passes the dense blocks.
 * Limits and errors:
 *  - SLRF_E_WORKSPACE if the pencil needs more than SLRF_STATIC_SCRATCH_BYTES
 *    (slrf_workspace_bytes_for gives the need), or if another context made by
 *    this call still holds the device's array: one such context per device at
 *    a time; slrf_destroy releases it (after waiting for its stream).
 *  - SLRF_E_DEVICE if the array's device address cannot be obtained.
 * The array keeps the last call's contents; the library clears what it needs
 * cleared on each call.  Work on the context is queued on its stream, as for
 * any context: overlapping calls on it from several threads race. */
#define SLRF_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
slrf_status slrf_create_static(slrf_ctx* out, int64_t n,
                               const int32_t* a_rowptr, const int32_t* a_col, const double* a_val,
                               const int32_t* b_rowptr, const int32_t* b_col, const double* b_val,
                               int64_t max_L, int32_t max_poles, const slrf_options* opt,
                               void* hip_stream);

/* One filter application (Algorithm 1, the "Solve" loop and "Compute U"):
 *   U = sum_j 2 Re(w_j Y_j),  (A - sigma_j B) Y_j = B X  for j = 1..N,
 * every (pole, column) system solved by right-preconditioned BiCGStab (the
 * preconditioner of slrf_options.precond), x_0 = 0 and shadow residual B X, or by
 * COCG with point or node block Jacobi or the multicolour SGS (slrf_options.solver = 1).
 * d_X, d_U: device (n, L) row-major float64
 * (may not alias).  stats may be NULL.  Returns SLRF_OK even if some columns hit
 * inner_maxit or broke down; stats reports them. */
slrf_status slrf_filter_apply(slrf_ctx ctx, const slrf_poles* poles, int64_t L,
                              const double* d_X, double* d_U, slrf_filter_stats* stats);

/* All eigenpairs in (0, gamma] by Algorithm 1.  poles: NULL designs N = 4,
 * alpha = 1, beta = 0.01 (Section 4.2).  d_V0: device (n, L) start block, or
 * NULL for a seeded Gaussian block.  Outputs: n_found (host), h_evals (host, L
 * doubles: all Ritz values ascending, the first n_found are the eigenvalues in
 * (0, gamma]), d_evecs (device (n, L), B-orthonormal Ritz vectors in the same
 * order), h_resid (host, L doubles: rho_i).  stats may be NULL.
 * Stopping: every Ritz value in (0, gamma] has rho_i <= outer_tol and their
 * number is unchanged from the previous outer iteration. */
slrf_status slrf_solve_interval(slrf_ctx ctx, double gamma, int64_t L, const slrf_poles* poles,
                                const double* d_V0, int64_t* n_found, double* h_evals,
                                double* d_evecs, double* h_resid, slrf_solve_stats* stats);

void slrf_destroy(slrf_ctx ctx);
const char* slrf_status_string(slrf_status s);
const char* slrf_last_error(slrf_ctx ctx);

/* ---- Batches: many pencils, one launch per Krylov step ---------------------
 *
 * A batch runs Algorithm 1 on a changing set of pencils at once.  Each outer
 * step applies the filter to every unfinished pencil in ONE batched Krylov solve
 * (each kernel launch covers every pole x column of every pencil; the per-
 * pencil sizes, offsets and CSR pointers sit in a device table), then does
 * Rayleigh-Ritz, residuals and the stopping test per pencil.  The arithmetic of
 * each pencil is that of slrf_solve_interval with the same options, poles and
 * start block (the per-column reductions are summed in a fixed order that does
 * not depend on the other pencils or the grid size, so a pencil's result is
 * bitwise the same alone or in a batch).  With recycle = 1 every pencil
 * warm-starts from its own previous step, as it would alone, whichever pencils
 * join or leave the batch; a pencil whose first step shares a filter
 * application with warm-started pencils starts from Y = 0 through the warm
 * path, which computes what its cold start computes, so its result too is
 * bitwise the solve alone.
 *
 * Workspace (device, 256-byte aligned, caller-owned): a filter arena of
 * arena_bytes shared by the pencils of one step, and a pool for each pencil's
 * persistent data (merged CSR, subspace blocks).  slrf_batch_footprint gives
 * both parts for one pencil; the arena needed by a set of pencils is at most
 * the sum of their transient parts.  Pencils can be added between steps
 * (continuous batching) and removed once finished, which frees their pool
 * space.  Not thread-safe; one batch per stream. */
typedef struct slrf_batch_s* slrf_batch;

/* Bytes one pencil needs: persistent_bytes in the pool (kept from add to
 * remove; in mixed precision with room for the warm-start blocks of
 * options.recycle) and transient_bytes of filter arena while it is
 * unfinished. */
slrf_status slrf_batch_footprint(int64_t n, int64_t nnz_union, int64_t L, int32_t N,
                                 int32_t precision, size_t* persistent_bytes,
                                 size_t* transient_bytes);

/* The same for the precision and preconditioner of opt (NULL: defaults); a
 * batch whose options select the multicolour SGS preconditioner (precond 4 or
 * 5) sizes its pencils with this one. */
slrf_status slrf_batch_footprint_for(int64_t n, int64_t nnz_union, int64_t L, int32_t N,
                                     const slrf_options* opt, size_t* persistent_bytes,
                                     size_t* transient_bytes);

/* d_workspace: device, 256-byte aligned, ws_bytes >= arena_bytes + 2 KiB; the
 * rest after the arena becomes the pool.  max_poles: largest N of any pencil
 * (1..16).  opt may be NULL.  On failure *out may hold a batch: read
 * slrf_batch_last_error(*out), then slrf_batch_destroy(*out). */
slrf_status slrf_batch_create(slrf_batch* out, void* d_workspace, size_t ws_bytes,
                              size_t arena_bytes, int32_t max_poles,
                              const slrf_options* opt, void* hip_stream);

/* Adds a pencil (CSR arrays as for slrf_create, host) to find every eigenpair in
 * (0, gamma] with an L-column subspace; poles NULL designs N = 4 as in
 * slrf_solve_interval; d_V0 device (n, L) start block or NULL (seeded
 * Gaussian), copied before return.  *id receives its handle.  SLRF_E_WORKSPACE
 * if the pool or the arena (with the unfinished pencils) cannot take it: the
 * caller may retry after a step finishes or removes pencils. */
slrf_status slrf_batch_add(slrf_batch b, int64_t n,
                           const int32_t* a_rowptr, const int32_t* a_col, const double* a_val,
                           const int32_t* b_rowptr, const int32_t* b_col, const double* b_val,
                           double gamma, int64_t L, const slrf_poles* poles,
                           const double* d_V0, int32_t* id);

/* One outer iteration for every unfinished pencil.  *n_active (may be NULL)
 * gets the number still unfinished.  A device or breakdown error ends every
 * pencil of the step with that status. */
slrf_status slrf_batch_step(slrf_batch b, int32_t* n_active);

/* done = 1 once the pencil has stopped (converged, too small, limit, error). */
slrf_status slrf_batch_query(slrf_batch b, int32_t id, int32_t* done, int32_t* outer_iterations);

/* Results of a finished pencil, as slrf_solve_interval returns them; the
 * return value is that pencil's final status. */
slrf_status slrf_batch_result(slrf_batch b, int32_t id, int64_t* n_found, double* h_evals,
                              double* d_evecs, double* h_resid, slrf_solve_stats* stats);

/* Starts the pencil's solve again from the start block d_V0 (device (n, L), or
 * NULL for the seeded Gaussian block), with its gamma, L and poles, keeping the
 * pencil's device data: the next slrf_batch_step runs its first outer
 * iteration.  Its previous result is discarded (warm starts begin afresh).  A
 * stream of solves of one pencil then needs no new slrf_batch_add. */
slrf_status slrf_batch_restart(slrf_batch b, int32_t id, const double* d_V0);

/* Frees the pencil's pool space; the id becomes invalid. */
slrf_status slrf_batch_remove(slrf_batch b, int32_t id);
void slrf_batch_destroy(slrf_batch b);
const char* slrf_batch_last_error(slrf_batch b);

#ifdef __cplusplus
}
#endif
#endif /* SLRF_H */
