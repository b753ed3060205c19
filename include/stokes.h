/*
 * stokes.h -- C ABI of the MI355X (gfx950) generalized Stokes solver.
 *
 * Problem (Creff & Guermond, arXiv 2407.01783, Sec. 2.2, the saddle-point
 * system A U - B^T P = F, B U = 0, with A = (1/dt) M_V + mu (viscous term)):
 * on the unit square (dim 2) or unit cube (dim 3) split into n^dim cells, each
 * cut into dim! Kuhn simplices, with Taylor-Hood P2 velocity / P1 pressure,
 * find (u, p) with
 *
 *     (alpha M_V + mu L_V + gamma mu B^T M_Q^{-1} B) U - B^T P = F~,   B U = g,
 *
 * alpha = 1/dt, L_V the vector Laplacian (the paper's A~_{lambda,3} block of
 * Sec. 3.2), gamma the augmented-Lagrangian weight (Sec. 2.3, Eq.
 * "def_of_Alambda", written lambda there), Dirichlet velocity on the whole
 * boundary (Sec. 3.1), F~ = (M_V f)_I - A_{I,Gamma} G the lifted load of a
 * nodal forcing f, g = -B_Gamma G made mean-free, and the pressure returned
 * with zero integral.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All solver arrays are DEVICE pointers to float64, owned by the caller; the
 *   library reads and writes them on the context's HIP stream and never keeps
 *   them past the call.  Host pointers are marked _host.
 * - Velocity-shaped arrays (f, ubc, u, x0_u, lam_u, dJdu, dJdf) are laid out
 *   [nrhs][dim][n_p2]: component-major over ALL P2 nodes in the natural
 *   numbering (P2 node (I,J[,K]) of the refined (2n+1)^dim grid has id
 *   I + (2n+1) J [+ (2n+1)^2 K]).  Pressure-shaped arrays (p, x0_p, lam_p,
 *   dJdp) are [nrhs][n_p1] over the vertices (i,j[,k]), id i + (n+1) j [+ ...].
 * - Return value: STOKES_OK (0), STOKES_NOT_CONVERGED (1, outputs hold the
 *   best iterate), or a negative error code; stokes_last_error() then gives a
 *   message (thread-local).  Arguments are validated before any HIP call.
 *   After an error the output arrays are unspecified.
 * - The solve entry points return STOKES_ERR_NONFINITE (-4) when the
 *   right-hand side they form from f and ubc (or the adjoint's dJdu, dJdp)
 *   is not finite, when the first residual of a given initial guess is not
 *   finite, or when an iterate or a residual of the solve becomes non-finite;
 *   a NaN or Inf is never reported as convergence.
 * - One context per host thread at a time; calls on one context serialise on
 *   its stream.
 */
#ifndef STOKES_H
#define STOKES_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stokes_ctx stokes_ctx; /* opaque; owned by the library */
typedef int32_t stokes_status;

enum {
  STOKES_OK = 0,
  STOKES_NOT_CONVERGED = 1,
  STOKES_ERR_ARG = -1,
  STOKES_ERR_ALLOC = -2,
  STOKES_ERR_HIP = -3,
  STOKES_ERR_NONFINITE = -4,
  STOKES_ERR_BREAKDOWN = -5,
  STOKES_ERR_STATE = -6,
  STOKES_ERR_UNSUPPORTED = -7
};

/* stokes_solve_opts.precision */
enum { STOKES_FP64 = 0, STOKES_MIXED = 1 };
/* stokes_solve_opts.inner_mode: inner solves to a tolerance ("th" in the
 * paper, Sec. 3.3) or a fixed polynomial ("2Vc" counterpart). */
enum { STOKES_INNER_TOL = 0, STOKES_INNER_FIXED = 1 };
/* stokes_solve_opts.schur_pc: the Cahouet-Chabard family of Sec. 4.1,
 * alpha X^{-1} + mu (1 + gamma) M_Q^{-1} with X = L_Q (C^Delta),
 * B Lambda_V^{-1} B^T (C^Lambda) or B M_V^{-1} B^T (C). */
enum { STOKES_CC_LAPLACE = 0, STOKES_CC_LUMPED = 1, STOKES_CC_MASS = 2 };
/* stokes_solve_opts.coupled_pc: block preconditioners of Sec. 2.4:
 * FULL = the three-factor inexact factorisation (Eq.
 * "inexact_factorization_of_Alambda", two A~^{-1} per step), LOWER = the
 * "incomplete Full" of Sec. 6.2 (left factor dropped), UPPER = block upper
 * triangular [[A~, -B^T], [0, S~]]. */
enum { STOKES_PC_FULL = 0, STOKES_PC_UPPER = 1, STOKES_PC_LOWER = 2 };
/* stokes_problem.flags: STOKES_FLAG_STRAIN selects the paper's own velocity
 * matrix A = alpha M_V + mu (L_V + D) of Sec. 3.2 (D the grad-div matrix;
 * equal to the strain-rate form 2 mu eps(u):eps(v) on H^1_0) instead of the
 * vector-Laplacian block alpha M_V + mu L_V.  The inner velocity
 * preconditioner stays A~_{lambda,3} = alpha M_V + mu L_V (Sec. 3.2); the
 * Dirichlet lifting and dJ/dmu use the same A. */
enum { STOKES_FLAG_STRAIN = 1 };
/* stokes_problem.flags: STOKES_FLAG_P3 selects the Taylor-Hood P3/P2 pair,
 * the paper's second element pair (Sec. 1; Sec. 3.3, Table 4, P3 rows):
 * velocity in the continuous P3 space, pressure in the continuous P2 space.
 * The velocity nodes are then the points of the (3n+1)^dim lattice, id
 * I + (3n+1) J [+ (3n+1)^2 K]; the pressure nodes are the (2n+1)^dim P2
 * points.  Every "n_p2" / velocity-shaped array below counts P3 nodes and
 * every "n_p1" / pressure-shaped array P2 nodes.  Local P3 order: vertices,
 * then per local edge (a, b) the node next to a and the node next to b, then
 * the faces (0,1,2), (0,1,3), (0,2,3), (1,2,3) (2D: the interior node).  The
 * P2 pressure nodes of the mesh with n cells are the vertices of the mesh
 * with 2n cells, so both pressure multigrids (ops 6 and 8) run on P3/P2 with
 * the P1 space of the mesh as their first coarse level; the velocity
 * multigrid (vel_pc = STOKES_VEL_MG, op 9) needs the P2/P1 pair and returns
 * STOKES_ERR_UNSUPPORTED.  Combines with STOKES_FLAG_STRAIN. */
enum { STOKES_FLAG_P3 = 2 };
/* stokes_solve_opts.vel_pc: the preconditioner of A~_{lambda,3} = alpha M_V
 * + mu L_V inside the velocity solves -- a Chebyshev-Jacobi polynomial of
 * degree cheb_degree, or one geometric-multigrid V-cycle on the nested Kuhn
 * meshes (the counterpart of the paper's AMG V-cycles, Sec. 3.3), whose cost
 * and iteration counts do not grow with 1/h when mu dt / h^2 is large. */
enum { STOKES_VEL_CHEB = 0, STOKES_VEL_MG = 1 };
/* stokes_solve_opts.arnoldi_fp64: precision of the mixed FGMRES cycle. */
enum { STOKES_ARNOLDI_FP32 = 0, STOKES_ARNOLDI_FP64 = 1, STOKES_ARNOLDI_FP64_K = 2 };

typedef struct {
  int32_t dim;        /* 2 or 3 */
  int32_t n;          /* cells per side, >= 1 (>= 2 for a unique pressure) */
  uint64_t mesh_seed; /* seed of the interior-vertex jitter */
  double jitter;      /* jitter amplitude as a fraction of h, in [0, 0.2] */
  double mu;          /* viscosity, > 0 */
  double alpha;       /* 1/dt, > 0 */
  double gamma;       /* augmented-Lagrangian weight, >= 0 */
  int32_t flags;      /* 0, STOKES_FLAG_STRAIN, STOKES_FLAG_P3, or both */
} stokes_problem;

typedef struct {
  int32_t precision;      /* STOKES_FP64 or STOKES_MIXED (FP32 inner solves) */
  double rtol;            /* target true relative residual of the coupled FP64
                             system ||b - K x||_2 / ||b||_2 (per right-hand side) */
  int32_t max_outer;      /* cap on outer Krylov iterations, summed over sweeps */
  int32_t restart;        /* FGMRES restart length m (1..64) */
  int32_t max_inner;      /* cap on each inner CG */
  int32_t inner_mode;     /* STOKES_INNER_TOL or STOKES_INNER_FIXED */
  int32_t cheb_degree;    /* Chebyshev-Jacobi degree of the velocity block (1..16) */
  double inner_rtol_u;    /* relative tolerance of inner velocity CG */
  double inner_rtol_p;    /* relative tolerance of inner pressure CG */
  int32_t schur_pc;       /* STOKES_CC_* */
  int32_t coupled_pc;     /* STOKES_PC_* */
  int32_t max_refine;     /* cap on iterative-refinement sweeps */
  int32_t profile;        /* 1: time the dominant SpMV with HIP events (one
                             launch in seven, on the solver's stream); 2: also
                             the phase times of stokes_solve_info */
  int32_t inner_its_u;    /* > 0: every inner velocity CG runs exactly this many
                             iterations (no convergence checks); 0: use inner_rtol_u */
  int32_t inner_its_p;    /* the same for the inner pressure CG (0: inner_rtol_p) */
  int32_t vel_pc;         /* velocity-block preconditioner: STOKES_VEL_CHEB or STOKES_VEL_MG */
  int32_t arnoldi_fp64;   /* STOKES_MIXED coupled solves (each refinement sweep
                             asks a 1e-5 reduction of its own FP64 residual):
                             STOKES_ARNOLDI_FP32 = FGMRES basis, Gram-Schmidt
                             updates and K_gamma products in FP32 (sums in FP64);
                             STOKES_ARNOLDI_FP64 (default) = basis and
                             orthogonalization in FP64, K_gamma products with
                             the FP32 matrices; STOKES_ARNOLDI_FP64_K = also
                             K_gamma in FP64.  Ignored for STOKES_FP64 and the
                             Schur method. */
} stokes_solve_opts;

typedef struct {
  int32_t converged;      /* 1 if every right-hand side met rtol */
  int32_t outer_iters;    /* outer Krylov iterations (all sweeps) */
  int32_t inner_iters_u;  /* inner velocity CG iterations (all solves) */
  int32_t inner_iters_p;  /* inner pressure CG iterations */
  int32_t refinements;    /* sweeps of the refinement loop */
  int32_t spmv_launches;  /* timed launches of the dominant SpMV (profile = 1) */
  double rel_res;         /* max over right-hand sides of the final true residual */
  double seconds_total;   /* wall time of the call */
  double spmv_seconds;    /* summed duration of the timed SpMV launches */
  double spmv_bytes;      /* algorithmic bytes of one timed SpMV launch */
  /* Phase times (opts->profile = 2; 0 otherwise): GPU time summed over every
   * application of the phase, measured by HIP events on the solver's stream
   * (so work queued ahead of the host is attributed correctly). */
  double seconds_inner_u; /* velocity-block solves A~^{-1} (Sec. 3) */
  double seconds_inner_p; /* pressure-block applications: the Cahouet-Chabard
                             operator (Sec. 4.1), including its X^{-1} solves */
  double seconds_orth;    /* Gram-Schmidt passes of the FGMRES cycles (CGS2) */
  /* Residual history, CALLER-OWNED host buffer (may be NULL): entry k is the
   * relative residual after outer iteration k as the outer method estimates
   * it (FGMRES: its least-squares residual, Schur CG: the Schur residual),
   * divided by ||b||, the largest over the right-hand sides of a batch;
   * batches of more than 8 right-hand sides append in order.  Set res_hist
   * and res_hist_cap before the call (they are kept); the call writes at most
   * res_hist_cap entries and sets res_hist_len to the number written. */
  double* res_hist;
  int32_t res_hist_cap;
  int32_t res_hist_len;
  /* Algorithmic HBM bytes of the kernels the call launched, counted by the
   * library from its layouts (always, at no device cost): each stored
   * operator once per product (every padded entry's values and the column
   * index structure it reads), each streamed vector once per pass, each
   * gathered vector once.  bytes_alg / seconds_total over the device's HBM
   * bandwidth is the solve-level roofline fraction. */
  double bytes_alg;
} stokes_solve_info;

/* Fill *opts with defaults: FP64, rtol 1e-8, FGMRES(30), Chebyshev degree 4,
 * inner tolerances 1e-6 / 1e-4, C^Lambda, FULL, 8 refinement sweeps. */
void stokes_default_opts(stokes_solve_opts* opts);

/* Sizes of the problem without building anything (host only, no GPU):
 * sizes[0..9] = n_p2, n_p1, n_free_nodes, nnz(A_II), nnz(B_I one plane),
 * nnz(M_Q), n_elem, dim, nnz(full P2 scalar pattern), nnz(B full one plane). */
stokes_status stokes_problem_sizes(const stokes_problem* prob, int64_t sizes[10]);

/* Host-only mesh construction (no GPU): vertex coordinates [n_p1][dim],
 * simplex vertex ids [n_elem][dim+1], P2 node coordinates [n_p2][dim], and the
 * P2 node ids of every simplex [n_elem][n_loc] (local order: vertices, then
 * edges (0,1),(0,2),(0,3),(1,2),(1,3),(2,3) / (0,1),(0,2),(1,2)).  Any pointer
 * may be NULL to skip that output. */
stokes_status stokes_build_mesh_host(const stokes_problem* prob, double* vcoords_host,
                                     int32_t* elems_host, double* p2coords_host,
                                     int32_t* p2_host);

/* Host-only sparsity pattern (no GPU), CSR with sorted columns.
 * which: 0 = P2 x P2 over all nodes, 1 = interior P2 x interior P2 (natural
 * ids of interior nodes renumbered 0.. in increasing order), 2 = P1 x all P2
 * (B), 3 = P1 x interior P2 (B_I), 4 = P1 x P1.  Call with rowptr_host and
 * cols_host NULL to get *nrows / *nnz, then again with arrays of that size. */
stokes_status stokes_host_pattern(const stokes_problem* prob, int32_t which, int64_t* nrows,
                                  int64_t* nnz, int32_t* rowptr_host, int32_t* cols_host);

/* Build the mesh, assemble every operator on the GPU (Sec. 2.2, 3.2, 4.1:
 * M_V, L_V, B, M_Q, L_Q, Lambda_V), estimate the Chebyshev bounds and return a
 * context bound to hip_stream (NULL = default stream) and the current device. */
stokes_status stokes_assemble(const stokes_problem* prob, void* hip_stream, stokes_ctx** out);

/* Method 1 (Sec. 2.3): flexible CG on the pressure Schur complement
 * S = B A^{-1} B^T preconditioned by the Cahouet-Chabard operator
 * (Sec. 4.1), inside an FP64 iterative-refinement loop on the coupled
 * residual.  f: nodal forcing; ubc: Dirichlet data (boundary entries read;
 * NULL = 0); x0_u, x0_p: initial guess (NULL = 0); u, p: outputs (boundary
 * entries of u equal ubc; p has zero integral).  info may be NULL. */
stokes_status stokes_solve_schur(stokes_ctx* ctx, int32_t nrhs, const double* f,
                                 const double* ubc, const double* x0_u, const double* x0_p,
                                 double* u, double* p, const stokes_solve_opts* opts,
                                 stokes_solve_info* info);

/* Method 2 (Sec. 2.4): right-preconditioned flexible GMRES(m) on the coupled
 * matrix [[A_gamma, -B^T], [B, 0]] with a block preconditioner
 * (opts->coupled_pc), restarts checked against the true FP64 residual.
 * Same arguments as stokes_solve_schur. */
stokes_status stokes_solve_coupled(stokes_ctx* ctx, int32_t nrhs, const double* f,
                                   const double* ubc, const double* x0_u, const double* x0_p,
                                   double* u, double* p, const stokes_solve_opts* opts,
                                   stokes_solve_info* info);

/* One rotational incremental pressure-correction step, the comparator of
 * Sec. 7.5 and Table 8 (a momentum solve, then a pressure Poisson solve and a
 * pressure-mass solve), from p_old ([nrhs][n_p1], NULL = 0):
 *     A u = F~ + B^T p_old,  d = B u - g,  L_Q phi = -alpha d,  M_Q psi = d,
 *     p = p_old + phi - mu psi  (zero integral),
 * with (F~, g) the lifted right-hand side of stokes_solve_schur (A without
 * the augmented-Lagrangian term).  Each linear solve reaches a true FP64
 * relative residual <= opts->rtol (inner CG in the opts precision with FP64
 * refinement; velocity preconditioner opts->vel_pc, pressure Laplacian CG
 * preconditioned by a multigrid V-cycle of M_Q + L_Q, mass CG by
 * Chebyshev-Jacobi).  info->rel_res is the largest of the three final
 * residuals.  Layouts as in stokes_solve_schur. */
stokes_status stokes_projection_step(stokes_ctx* ctx, int32_t nrhs, const double* f, const double* ubc,
                                     const double* p_old, double* u, double* p, const stokes_solve_opts* opts,
                                     stokes_solve_info* info);

/* Adjoint of the solve: given the forward velocity u ([nrhs][dim][n_p2]) and
 * the loss gradients dJdu ([nrhs][dim][n_p2], boundary entries ignored) and
 * dJdp ([nrhs][n_p1], NULL = 0), solve the transposed coupled system
 * [[A, B^T], [-B, 0]] (lam_u, lam_p) = (dJ/dU_I, dJ/dP) and return
 * lam_u ([nrhs][dim][n_p2], zero on the boundary), lam_p ([nrhs][n_p1]),
 * dJdf = M_V[I,:]^T lam_u ([nrhs][dim][n_p2]) and
 * dJdmu[r] = -lam_u^T L_V[I,:] u ([nrhs], device).  Uses the coupled solver
 * with opts (solved as the forward system after lam_p -> -lam_p). */
stokes_status stokes_solve_adjoint(stokes_ctx* ctx, int32_t nrhs, const double* u,
                                   const double* dJdu, const double* dJdp, double* lam_u,
                                   double* lam_p, double* dJdf, double* dJdmu,
                                   const stokes_solve_opts* opts, stokes_solve_info* info);

/* Apply one assembled operator in FP64 (precision 0) or FP32 (1) to device
 * arrays in the caller layout.  op: 0 = y = A_gamma=0 x on interior nodes
 * (x, y velocity-shaped, boundary entries of x ignored, of y set to 0; A is
 * the context's velocity matrix, alpha M + mu (L + D) with
 * STOKES_FLAG_STRAIN);
 * 1 = y = B x (x velocity-shaped, y pressure-shaped); 2 = y = B^T x (x
 * pressure, y velocity, boundary 0); 3 = M_Q x; 4 = L_Q x; 5 = the coupled
 * operator: (y_u, y_p) = (A u - B^T p, B u) with x = (x_u, x_p) packed as
 * [nrhs][dim][n_p2] followed by [nrhs][n_p1]; 6 = one geometric multigrid
 * V-cycle for eps M_Q + L_Q (eps = 1), the pressure preconditioner of
 * Sec. 4.2 (x, y pressure-shaped); 7 = y = B_I Lambda_V^-1 B_I^T x, the
 * lumped-mass pressure operator of Sec. 4.3, assembled explicitly (x, y
 * pressure-shaped); 8 = one V-cycle of the Galerkin multigrid hierarchy of
 * B_I Lambda_V^-1 B_I^T + M_Q, the preconditioner of that operator (x, y
 * pressure-shaped); 9 = one velocity-multigrid V-cycle for alpha M_V + mu L_V
 * (x, y velocity-shaped, boundary entries ignored / set to 0); 10 = the
 * FIXED-mode velocity preconditioner: the degree-6 Chebyshev-Jacobi
 * polynomial of A~_{lambda,3} = alpha M_V + mu L_V on the interval of
 * stokes_bounds[0..1] (x, y velocity-shaped; precision 1 reads a
 * half-precision copy of A D^-1 and keeps the Chebyshev direction in
 * bfloat16, so it agrees with precision 0 to about 1e-3). */
stokes_status stokes_apply(stokes_ctx* ctx, int32_t op, int32_t precision, int32_t nrhs,
                           const double* x, double* y);

/* True relative residual ||b - K x|| / ||b|| of the plain coupled system for
 * the given forcing, boundary data and solution (all device, caller layout);
 * rel_res_host[nrhs] receives one value per right-hand side. */
stokes_status stokes_residual(stokes_ctx* ctx, int32_t nrhs, const double* f, const double* ubc,
                              const double* u, const double* p, double* rel_res_host);

/* Allocation-free variant of stokes_residual, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): same arguments, same result, but it calls
 * no hipMalloc/hipFree and no allocating library routine.  Its temporaries
 * live in a fixed device array of 128 MiB that the library holds on every GPU
 * it has run on until the process ends (its address is looked up when a
 * context is assembled).  Right-hand sides are processed one at a time, each
 * needing 16 (n_int dim + n_p1) bytes (n_int = stokes_query sizes[2]); a mesh
 * beyond 128 MiB returns STOKES_ERR_UNSUPPORTED (the 64^3 cube needs 103 MB).
 * Every call on one GPU shares that array: calls that overlap on one GPU
 * (from several host threads or contexts) race and must be serialised by the
 * caller. */
stokes_status stokes_residual_noalloc(stokes_ctx* ctx, int32_t nrhs, const double* f, const double* ubc,
                                      const double* u, const double* p, double* rel_res_host);

/* sizes[0..9] as in stokes_problem_sizes, for an assembled context;
 * sizes[10] = entries of B_I Lambda_V^-1 B_I^T (export_csr which 9),
 * sizes[11] = slices of 64 A_II rows whose columns the velocity kernels
 * compute (one base per slot and at most one jump across the slice) instead
 * of loading (0 with STOKES_VEL_AF=0 in the environment at assembly). */
stokes_status stokes_query(const stokes_ctx* ctx, int64_t sizes[12]);

/* Change mu and re-form A = alpha M + mu L on the device. */
stokes_status stokes_set_mu(stokes_ctx* ctx, double mu);

/* Rebind the context to another HIP stream of the same device. */
stokes_status stokes_set_stream(stokes_ctx* ctx, void* hip_stream);

/* Copy the P2 node coordinates [n_p2][dim] and simplex P2 ids
 * [n_elem][n_loc] to host arrays (either may be NULL). */
stokes_status stokes_export_mesh(const stokes_ctx* ctx, double* p2coords_host, int32_t* p2_host);

/* Copy an assembled FP64 matrix to host CSR arrays in the natural numbering
 * of stokes_host_pattern.  which: 0 = M_s (all P2), 1 = L_s (all P2),
 * 2..4 = B plane x, y, z (P1 x all P2), 5 = M_Q, 6 = L_Q, 7 = A_II (interior,
 * pattern 1), 8 = Lambda_V (diagonal: rowptr/cols ignored, vals [n_p2]),
 * 9 = B_I Lambda_V^-1 B_I^T (P1 x P1, stokes_query sizes[10] entries),
 * 10 + dim a + b = grad-div block D[a][b] (all P2, int d_a phi_i d_b phi_j;
 * STOKES_FLAG_STRAIN contexts only). */
stokes_status stokes_export_csr(const stokes_ctx* ctx, int32_t which, int32_t* rowptr_host,
                                int32_t* cols_host, double* vals_host);

/* Chebyshev interval estimates [lo, hi] of the Jacobi-scaled operators:
 * bounds_host[0..7] = A_II, M_V, M_Q, M_Q + L_Q. */
stokes_status stokes_bounds(const stokes_ctx* ctx, double bounds_host[8]);

/* Measurement helper (not part of the solve): achievable HBM bandwidth of a
 * device-to-device copy and of a read-only stream of `bytes` bytes on the
 * current device, each the mean over `reps` launches after one warm-up,
 * timed with HIP events on hip_stream (NULL = default stream).
 * gbs_host[0] = copy GB/s (read + write bytes), gbs_host[1] = read GB/s.
 * Allocates and frees two buffers of `bytes`. */
stokes_status stokes_bandwidth_probe(void* hip_stream, int64_t bytes, int32_t reps, double* gbs_host);

/* Free the context and every device buffer it owns.  NULL is a no-op. */
void stokes_destroy(stokes_ctx* ctx);

/* Message of the last error on this thread ("" if none). */
const char* stokes_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* STOKES_H */
