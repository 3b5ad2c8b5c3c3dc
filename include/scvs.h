/*
 * scvs.h -- C ABI of the MI355X (gfx950) spectral complex-valued Stokes library.
 *
 * The method (Meng, Bhattacharjee & Esmaily, arXiv 2009.06725) turns a
 * time-periodic creeping flow into independent Fourier modes (section 2.1,
 * Eqs. vaptransform and stokes_complex). For every mode w_k it solves the
 * complex Taylor-Hood (quadratic velocity, linear pressure) saddle-point
 * system of section 2.3 (Eqs. linear_sys_def and LS_construction)
 *     [ I_d (x) (mu Ks + j w rho M)   G ] [u]   [f_u]
 *     [ G^T                           0 ] [p] = [f_p]
 * and reconstructs the fields in time (section 2.4, Eq. sol_reconstruct).
 *
 * Conventions used by every entry point:
 *  - Status codes: 0 = success, negative = error (see SCVS_E_*). On error
 *    scvs_last_error() returns a thread-local message. No entry point throws
 *    or aborts across the ABI. Validation errors write no output.
 *  - Pointers documented "host" are read or written synchronously. Pointers
 *    documented "device" must be device memory of the context's device; the
 *    caller owns them (the library never frees them). Work on device buffers
 *    is ordered on the context's stream; entry points that return host data
 *    synchronize that stream.
 *  - Complex numbers are (re, im) pairs of double ("c128").
 *  - Numbering (section 2.3, Eq. shape_fun, with this library's reading):
 *    quadratic node A < nv is vertex A; node nv + e is the midside node of
 *    edge e, where edges are the unique vertex pairs {a<b} of all cells
 *    sorted lexicographically. Cell-local node order: the d+1 vertices, then
 *    edges (0,1),(1,2),(0,2) and in 3D (0,3),(1,3),(2,3).
 *  - Unknown layout of one system ("DOF vector", length ndof = d*n2 + nv):
 *    velocity of node A, component c at index d*A + c, then pressure of
 *    vertex v at index d*n2 + v.
 *  - Dirichlet (wall and prescribed-inflow) unknowns stay in the numbering;
 *    their rows and columns of the system are identity and their value is
 *    the prescribed one.
 */
#ifndef SCVS_H
#define SCVS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SCVS_OK 0
#define SCVS_E_INVALID (-1)   /* bad argument (null, negative size, out-of-range index) */
#define SCVS_E_MESH (-2)      /* malformed mesh (degenerate cell, node index range) */
#define SCVS_E_NOMEM (-3)     /* device or host allocation failed */
#define SCVS_E_HIP (-4)       /* a HIP runtime call failed */
#define SCVS_E_STATE (-5)     /* call out of order (e.g. solve before assemble) */
#define SCVS_E_CAPACITY (-6)  /* a fixed internal capacity was exceeded */

/* Boundary-condition kinds per boundary tag (section 2.1, Eq. steady_stokes). */
#define SCVS_BC_FREE 0      /* zero traction */
#define SCVS_BC_WALL 1      /* u = 0 (no slip) */
#define SCVS_BC_DIRICHLET 2 /* u = g, g supplied per system at the Dirichlet nodes */
#define SCVS_BC_TRACTION 3  /* normal-pressure traction h = -P n, P supplied per system */

/* Precedence where tags meet: WALL over DIRICHLET over traction/free. */

typedef struct scvs_ctx_s* scvs_ctx;
typedef struct scvs_mesh_s* scvs_mesh;

/* Thread-local message of the last failed call on this thread ("" if none). */
const char* scvs_last_error(void);

/* Library version string (static storage). */
const char* scvs_version(void);

/* Create a context on HIP device `device`. `stream` is a hipStream_t (may be
 * NULL for the null stream); the library launches all work on it and does not
 * take ownership. */
int scvs_ctx_create(int device, void* stream, scvs_ctx* out);
int scvs_ctx_destroy(scvs_ctx ctx);

/* Memory cap of a context: the device bytes that one scvs_solve (or one group of
 * scvs_solve_groups) may take for its pool of Krylov slots, on top of its inputs,
 * outputs and the mesh's own matrices and hierarchies. The modes are independent
 * (section 2.4, step 3), so the cap only decides how many are solved at once: the
 * pool holds min(nsys, max_batch, what fits) slots and refills them from the
 * remaining systems. 0 (the default) = 90% of the free device memory at the call;
 * a nonzero cap is used when it is smaller than that. A cap below one system's
 * workspace makes the solve fail with SCVS_E_NOMEM. */
int scvs_ctx_set_mem_cap(scvs_ctx ctx, uint64_t bytes);

/* ---- a1: mesh ingest, numbering, sparsity (section 2.3, Eq. shape_fun) ----
 * dim 2 (triangles) or 3 (tets). Host inputs, copied:
 *   xyz    double[nv][dim]    vertex coordinates
 *   cells  int32[nc][dim+1]   vertex indices (any orientation)
 *   bfaces int32[nf][dim]     boundary facets, ordered so their normal points
 *                             out of the domain (2D: domain on the left of
 *                             a->b; 3D: (b-a)x(c-a) outward)
 *   btags  int32[nf]          tag per facet (any non-negative integers)
 * Builds on the device: vertex->cell adjacency, the canonical edge list, the
 * cell->node map and the sorted CSR pattern S2 of quadratic node pairs that
 * share a cell. The vertex-vertex pattern C21 is the vertex-column prefix of
 * each S2 row, and the transpose pattern C12 equals the S2 rows of vertices.
 * Errors: SCVS_E_INVALID (null/negative), SCVS_E_MESH (index out of range),
 * SCVS_E_CAPACITY (a row needs more than 4096 candidate entries). */
int scvs_mesh_create(scvs_ctx ctx, int dim, int64_t nv, const double* xyz, int64_t nc,
                     const int32_t* cells, int64_t nf, const int32_t* bfaces,
                     const int32_t* btags, scvs_mesh* out);
int scvs_mesh_destroy(scvs_mesh mesh);

typedef struct {
  int32_t dim;
  int64_t nv, nc, nf, ne, n2; /* vertices, cells, facets, edges, quadratic nodes */
  int64_t ndof;               /* dim*n2 + nv complex unknowns per system */
  int64_t nnz_s2, nnz_c21;    /* pattern sizes */
  int64_t ndir;               /* number of DIRICHLET (non-wall) nodes, after set_bc */
  int32_t ntraction;          /* number of TRACTION tags, after set_bc */
  int32_t assembled;          /* 1 after scvs_assemble */
} scvs_mesh_info_t;
int scvs_mesh_info(scvs_mesh mesh, scvs_mesh_info_t* info);

/* Curved boundary (section 3.1: inserted boundary nodes are projected onto the
 * curved surface). `n` edges given by their two vertex indices (any order)
 * and the position of their midside node (host, double[n][dim]). Call order:
 * scvs_mesh_set_midside, then scvs_mesh_set_bc, then scvs_assemble. Moving
 * midside nodes after scvs_mesh_set_bc clears the boundary conditions (their
 * traction loads and lumped outlets were integrated on the old facets) and the
 * assembly, so both must be done again.
 * Errors: SCVS_E_INVALID if a pair is not an edge. */
int scvs_mesh_set_midside(scvs_mesh mesh, int64_t n, const int32_t* edge_vertices,
                          const double* xyz);

/* Boundary conditions: kind per tag (SCVS_BC_*); tags not listed are FREE.
 * Computes the Dirichlet node sets and, per TRACTION tag (in ascending tag
 * order), n^tau_A = int_{Gamma_tau} M_A n dGamma. May be called again. */
int scvs_mesh_set_bc(scvs_mesh mesh, int n, const int32_t* tags, const int32_t* kinds);

/* Lumped (Windkessel) outlets, as on the outflow faces of the Glenn case
 * (section 3.5, which names the model without its form). Each listed tag must
 * already be a TRACTION tag; its pressure becomes P = Z(w) Q + P0, where
 * Q = int u.n over the tag (outward flow), P0 is the tag's traction coefficient
 * of the system, and Z(w) = rp + rd / (1 + j w rd c) is the three-element model
 * (rp in series with c parallel to rd; c = 0 or rd = 0 gives a resistance). The
 * momentum rows gain Z b b^T with b = n^tau_A, one rank-one term per outlet,
 * in every solve, residual and scvs_spmv; a distal pressure Pd behind rd enters
 * as P0 = Pd / (1 + j w rd c). The preconditioner does not include these terms.
 * tags, rp, c, rd: host arrays of n (n <= 64); n = 0 removes every lumped
 * outlet; scvs_mesh_set_bc removes them too. Errors: SCVS_E_STATE before
 * scvs_mesh_set_bc, SCVS_E_INVALID for a tag that is not TRACTION, a repeated
 * tag, or a negative or non-finite parameter. */
int scvs_mesh_set_windkessel(scvs_mesh mesh, int n, const int32_t* tags, const double* rp,
                             const double* c, const double* rd);

/* ---- a2: element assembly (section 2.3, Eq. LS_construction) ----
 * Assembles the mode-independent matrices
 *   Ks_AB = int grad M_A . grad M_B,  M_AB = int M_A M_B   (S2 order)
 *   G^c_Av = -int d_c M_A N_v                              (C21 order)
 * by degree-5 Grundmann-Moeller quadrature on (possibly curved, quadratic)
 * cells, the dense element contraction on FP64 matrix cores, and a
 * deterministic per-slot sum in ascending cell order. rho, mu > 0 are stored
 * for the solves. Requires set_bc first (the preconditioner diagonals use the
 * Dirichlet set). */
int scvs_assemble(scvs_mesh mesh, double rho, double mu);

/* Host copies of mesh data for tests. Sizes from scvs_mesh_info:
 *  SCVS_X_EDGES    int32[ne][2]      SCVS_X_C2N     int32[nc][nn]
 *  SCVS_X_ROWPTR   int64[n2+1]       SCVS_X_COL     int32[nnz_s2]
 *  SCVS_X_KS       double[nnz_s2]    SCVS_X_M       double[nnz_s2]
 *  SCVS_X_G        double[dim][nnz_c21]  (C21 = vertex-column prefix of S2 rows)
 *  SCVS_X_MP       double[nv]        lumped pressure mass int N_v
 *  SCVS_X_DIRNODES int32[ndir]       ascending DIRICHLET node ids
 *  SCVS_X_DMASK    int32[n2]         0 free, 1 wall, 2 Dirichlet
 *  SCVS_X_LOADS    double[ntraction][n2][dim]
 *  SCVS_X_NODEXYZ  double[n2][dim]   node coordinates (vertices, then midside)
 *  SCVS_X_C21PTR   int64[n2+1]       C21 row pointers (quadratic node -> vertex
 *                                    columns of the cells containing it)
 *  SCVS_X_C21COL   int32[nnz_c21]    C21 columns, ascending per row (the S2 row's
 *                                    vertex-column prefix; section 2.3, Eq. shape_fun) */
#define SCVS_X_EDGES 0
#define SCVS_X_C2N 1
#define SCVS_X_ROWPTR 2
#define SCVS_X_COL 3
#define SCVS_X_KS 4
#define SCVS_X_M 5
#define SCVS_X_G 6
#define SCVS_X_MP 7
#define SCVS_X_DIRNODES 8
#define SCVS_X_DMASK 9
#define SCVS_X_LOADS 10
#define SCVS_X_NODEXYZ 11
#define SCVS_X_C21PTR 12
#define SCVS_X_C21COL 13
int scvs_mesh_export(scvs_mesh mesh, int which, void* out_host);

/* ---- a4: multi-system complex SpMV (section 2.3, Eq. linear_sys_def) ----
 * y_s = A(w_s) x_s for nsys systems sharing the mesh, with A the constrained
 * system matrix (Dirichlet rows identity, Dirichlet columns dropped).
 * omega: host double[nsys]; x, y: device c128[nsys][ndof]. */
int scvs_spmv(scvs_mesh mesh, int64_t nsys, const double* omega, const void* x, void* y);

/* ---- a3: right-hand sides (section 2.3, Eq. LS_construction, B_A) ----
 * f_s = [sum_tau (-P_s,tau) n^tau - A_FC g_s ; g_s on Dirichlet rows ; -G^T g_s]
 * traction: host c128[nsys][ntraction]; g: device c128[nsys][ndir][dim] (may be
 * NULL when ndir == 0); f: device c128[nsys][ndof]. */
int scvs_rhs(scvs_mesh mesh, int64_t nsys, const double* omega, const double* traction,
             const void* g, void* f);

/* ---- a5/a6: block-preconditioned restarted GMRES (section 2.3; section 3.1) ----
 * Right-preconditioned GMRES(m) with classical Gram-Schmidt applied twice,
 * complex Givens rotations and restarts on the true residual. Preconditioner:
 * block upper-triangular [[A_v, G], [0, -S]] with A_v^-1 a Chebyshev-Jacobi
 * polynomial of the real-shifted velocity block mu Ks + |w| rho M and
 * S^-1 = mu Mp^-1 + j w rho L^-1 (L^-1 a Chebyshev-Jacobi polynomial of
 * G^T diag(M)^-1 G on the free velocity rows). */
typedef struct {
  double rtol;        /* stop when ||f - A x||_2 <= rtol ||f||_2 (true residual) */
  int32_t restart;    /* Krylov dimension m per cycle, 1..256 (shortened, not below 30, when
                         memory would hold fewer than min(nsys, 8) systems' workspaces) */
  int32_t max_iters;  /* cap on Arnoldi steps per system, applied at restart boundaries: a system
                         stops (status 1) after the first cycle that reaches it */
  int32_t cheb_vel;   /* Chebyshev degree of the velocity block, >= 1 */
  int32_t cheb_pres;  /* Chebyshev degree of the pressure Laplacian, >= 1; 0 drops the j w rho L^-1
                         term (Schur block = mu Mp^-1, the pressure mass alone) */
  double cheb_ratio;  /* the polynomials target [lambda_max / cheb_ratio, lambda_max] of the
                         Jacobi-scaled blocks (lambda_max from a Gershgorin bound) */
  int32_t max_batch;  /* systems solved together (0 = as many as fit) */
  int32_t use_graph;  /* replay the steps of each cycle, in chunks of 30, from captured hipGraphs */
  int32_t verbose;    /* print per-cycle residuals to stderr */
  int32_t precision;  /* 0: all FP64. 1: mixed -- inside each restart cycle the operator
                         product, the velocity-block polynomial and the pressure-Laplacian
                         recurrence run on FP32 matrix copies and FP32 vectors with FP32
                         accumulation; the true residual f - A x recomputed at every restart
                         (iterative refinement), the Arnoldi orthogonalization,
                         Givens/least-squares, the pressure-mass Schur scaling and the
                         solution update stay FP64. 2: as 1, with the Krylov basis stored as
                         FP32 pairs (its arithmetic stays FP64; needs orth = 1) */
  int32_t orth;       /* 0: classical Gram-Schmidt, second pass when the first loses more than
                         30% of the norm (three passes over the basis per step). 1: the second
                         pass of each vector lagged into the next step's single reduction
                         (DCGS2, Swirydowicz et al. 2020; two passes per step, one extra
                         closing reduction per cycle) */
  double cheb_ratio_pres; /* interval ratio of the pressure-Laplacian polynomial (0: cheb_ratio) */
  double penalty;     /* epsilon >= 0: solve the penalized system whose continuity block is
                         -(epsilon / mu) Mp (lumped pressure mass) instead of 0; 0 = the
                         unstabilized method */
  double inner_rtol;  /* mixed precision only: a restart cycle also ends once its own residual
                         estimate has fallen by this factor (the FP32 operator cannot take the
                         true residual much further within one cycle); 0 = only at rtol or m */
  int32_t vel_block;  /* velocity block of the preconditioner. 0: Chebyshev polynomial of degree
                         cheb_vel in the Jacobi-scaled real shift mu Ks + |w| rho M. 1: one
                         V-cycle of aggregation multigrid on the complex block mu Ks + j w rho M
                         (levels: the quadratic nodes, the linear space of the same mesh, then
                         smoothed aggregates down to at most 256 rows, whose operator is
                         inverted densely per system; built once per assembly and boundary
                         conditions) */
  int32_t pres_block; /* pressure Laplacian inverse in the Schur block (when cheb_pres > 0).
                         0: Chebyshev polynomial of degree cheb_pres. 1: one multigrid V-cycle */
  int32_t mg_smooth;  /* multigrid: Chebyshev smoothing steps before and after each coarse
                         correction, >= 1 */
  double mg_ratio;    /* multigrid: smoothers target [lambda / mg_ratio, lambda] of the level
                         operator scaled by its complex diagonal, > 1 (default 4: wider
                         intervals smooth less of the complex spectrum, and at some middle
                         frequencies the cycle then stalls) */
  double steady_schur_omega; /* >= 0: for steady systems (w = 0) the Schur block uses this
                         w in its Laplacian term, mu Mp^-1 + j w_s rho L^-1, instead of the
                         pressure mass alone. The preconditioner acts from the right, so the
                         solution is unchanged; pressure modes that the velocity controls only
                         weakly (corners whose velocity nodes are all prescribed) then no
                         longer stall the steady solve. 0 = off */
  int32_t mg_post0;   /* multigrid: Chebyshev steps after the coarse correction on the
                         velocity's level 0 (the quadratic level, the costliest to smooth);
                         0 = mg_smooth; 0..16 */
} scvs_solve_opts;

/* Fill `o` with the defaults (rtol 1e-10, m 200, 20000 iterations, degrees 12/50,
 * ratios 300 (velocity) / 1000 (pressure), batch 0, graphs on, FP64, lagged
 * orthogonalization, inner_rtol 3e-5, polynomial blocks (vel_block = pres_block = 0),
 * multigrid smoothing 2 steps, ratio 4, steady_schur_omega 0, mg_post0 0). */
void scvs_solve_opts_default(scvs_solve_opts* o);

typedef struct {
  int32_t status;       /* 0 converged, 1 iteration cap, 2 breakdown without convergence, 3 non-finite */
  int32_t iterations;   /* Arnoldi steps */
  int32_t restarts;     /* completed cycles */
  double rel_residual;  /* final ||f - A x|| / ||f|| */
  int32_t warm;         /* 1 if the supplied x0 was kept, 0 if zero guess (none given or fallback) */
} scvs_report;

/* Solve nsys mode systems on one mesh (section 2.4, step 3).
 *   omega     host double[nsys]            w_s (any sign; 0 = steady Stokes)
 *   traction  host c128[nsys][ntraction]   normal pressure per traction tag
 *   g         device c128[nsys][ndir][dim] Dirichlet data (NULL if ndir == 0)
 *   x0        device c128[nsys][ndof] initial guesses, or NULL for zero (the
 *             Dirichlet entries are overwritten with g)
 *   u_out     device c128[nsys][n2][dim]; p_out device c128[nsys][nv]
 *   rep       host scvs_report[nsys] (may be NULL)
 * Non-convergence is reported per system, not as a call error. */
int scvs_solve(scvs_mesh mesh, int64_t nsys, const double* omega, const double* traction,
               const void* g, const void* x0, void* u_out, void* p_out,
               const scvs_solve_opts* opts, scvs_report* rep);

/* ---- a5: the multigrid hierarchies of the preconditioner ----
 * Builds them if needed (as the first solve with vel_block or pres_block = 1
 * does: once per assembly and boundary-condition set) and reports, for
 * hierarchy `which` (0: velocity block, whose level 0 is the quadratic pattern;
 * 1: pressure Laplacian), the rows and nonzeros of each level and the nonzeros
 * of its transfer to the next coarser level (0 on the coarsest, which is
 * inverted densely), for up to `maxlev` levels (host int64_t[maxlev] each);
 * *nlev = the number of levels. Errors: SCVS_E_STATE before assembly,
 * SCVS_E_CAPACITY if coarsening stalls. */
int scvs_mesh_mg_info(scvs_mesh mesh, int which, int maxlev, int64_t* rows, int64_t* nnz, int64_t* pnnz,
                      int* nlev);

/* ---- a8: several meshes at once ----
 * Solves n groups of systems, each on its own mesh, concurrently: every group
 * runs scvs_solve (same arguments, same results) from its own host thread on
 * its own context's stream, so the GPU overlaps the groups' kernels -- a small
 * mesh's launches fill the gaps and tails of a large one's. The groups must use
 * distinct contexts (create each with its own stream); 1 <= n <= 64. The call
 * returns when every group is done; on failure it returns the first failing
 * group's status, its message prefixed with "group k: ", and the other groups'
 * results are still written. */
typedef struct {
  scvs_mesh mesh;
  int64_t nsys;
  const double* omega;
  const double* traction;
  const void* g;
  const void* x0;
  void* u_out;
  void* p_out;
  const scvs_solve_opts* opts;
  scvs_report* rep;
} scvs_solve_group;
int scvs_solve_groups(int n, const scvs_solve_group* groups);

/* ---- a8: autotuner ----
 * Times candidate solver settings on the caller's own systems (the same
 * arguments as scvs_solve, no initial guesses) and returns the fastest in
 * `best` (and its solve time in *best_ms, may be NULL). With the Chebyshev
 * velocity block (vel_block = 0) the candidates vary the restart length (160,
 * 220) and the pressure and velocity Chebyshev degrees (30/50, 10/12); with the
 * multigrid velocity block (vel_block = 1) they vary the restart length (30,
 * 40, 60), the smoothing steps (1, 2) and the smoother interval ratio (4, 10).
 * Every other field, including the precision, the tolerance and the
 * orthogonalization, comes from `base` (NULL: the defaults). A candidate counts
 * only if all systems converge. Each candidate is one full solve, so a call
 * costs 8 or 12 solves; the choice is cached in the context per (mesh,
 * assembly, number of systems, every option that is not tuned) and later calls
 * return it at once, the tuned fields over the caller's other options.
 * Reassembly or new boundary conditions start a new entry. */
int scvs_autotune(scvs_mesh mesh, int64_t nsys, const double* omega, const double* traction, const void* g,
                  const scvs_solve_opts* base, scvs_solve_opts* best, double* best_ms);

/* ---- f2: mode selection (section 2.4, step 2, Eq. mode_error, and its closing remarks) ----
 * For real periodic data given by two-sided coefficients, Parseval turns the
 * L2(Gamma x T) norms of Eq. mode_error into mode sums with weight 1 for
 * omega = 0 and 2 otherwise.
 *   scvs_boundary_norms  per system: hn2 = int |h|^2 over the traction facets
 *       (h = -P n per traction tag) and gn2 = int |g_h|^2 over the Dirichlet
 *       facets (g_h the quadratic interpolant of the nodal data, walls zero);
 *       arguments as scvs_solve; host outputs double[nsys].
 *   scvs_mode_norms  per solved mode: un2 = u^H (I_d (x) M) u and pn2 = p^H Mp p
 *       (lumped pressure mass); u, p device as written by scvs_solve.
 *   scvs_select_modes  host only (needs no GPU): the fewest modes whose relative
 *       truncation error e_M (the square root of Eq. mode_error's left side)
 *       is below eps. Modes enter in the given order (consecutive = 1) or by
 *       their share of the data energy (consecutive = 0, the non-consecutive
 *       choice the paper suggests). Outputs: order[nk] (a permutation), *count,
 *       *err = e_M of the chosen set.
 *   scvs_mode_increments  host only: inc[k] = relative L2(Omega x T) change of
 *       the reconstruction when mode k is added to modes 0..k-1 (the
 *       a-posteriori stopping quantity). */
int scvs_boundary_norms(scvs_mesh mesh, int64_t nsys, const double* traction, const void* g, double* hn2,
                        double* gn2);
int scvs_mode_norms(scvs_mesh mesh, int64_t nsys, const void* u, const void* p, double* un2, double* pn2);

/* ---- scvs_mode_norms without allocation ----
 * For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same arguments and
 * the same results, bit for bit, as scvs_mode_norms, with its partial sums in a
 * file-scope device array of SCVS_NOALLOC_MAX_SYSTEMS * 514 doubles (1.05 MB
 * per GPU, held from the first context created on that GPU until the process
 * ends) instead of a per-call buffer. The call makes no hipMalloc or hipFree.
 * Errors: as scvs_mode_norms, plus SCVS_E_CAPACITY when nsys exceeds
 * SCVS_NOALLOC_MAX_SYSTEMS. Every call on one GPU uses that GPU's array and
 * leaves its contents there; calls that overlap on one GPU (from several host
 * threads or streams) race on it, so the caller must serialize them. */
#define SCVS_NOALLOC_MAX_SYSTEMS 256
int scvs_mode_norms_noalloc(scvs_mesh mesh, int64_t nsys, const void* u, const void* p, double* un2,
                            double* pn2);
int scvs_select_modes(int64_t nk, const double* omega, const double* hn2, const double* gn2, double eps,
                      int consecutive, int64_t* order, int64_t* count, double* err);
int scvs_mode_increments(int64_t n, const double* omega, const double* un2, double* inc);

/* ---- a10: time synthesis (section 2.4, step 4, Eq. sol_reconstruct) ----
 * out[n][i] = sum_k c_k Re(modes[k][i] exp(j omega_k t_n)), c_k = 1 if
 * omega_k == 0 else 2 (real fields from the one-sided coefficients of
 * Eq. SCVS_bc). omega: host double[nk] (>= 0); modes: device c128[nk][nvals];
 * times: host double[nt]; out: device double[nt][nvals]. nk <= 256. With nt = 0 or
 * nvals = 0 nothing is written and modes/out may be NULL. */
int scvs_synthesize(scvs_ctx ctx, int64_t nk, const double* omega, const void* modes,
                    int64_t nvals, int64_t nt, const double* times, void* out);

/* ---- a9: learned warm start (no counterpart in the paper) ----
 * A model built from the method's own solutions: POD of `nsnap` snapshot
 * systems (device c128 [nsnap][ndof], each the solution for a unit-amplitude
 * boundary datum at frequency omega[s]), truncated to `rank` <= nsnap <= 128
 * modes, and an MLP with `layers` layers of width `width` (tanh hidden
 * layers) from the features (w, sqrt w, w^2) of w = omega/max|omega| to the
 * rank complex POD coefficients. With the Gram eigenpairs (sigma_i^2, W_i)
 * of the snapshots, snapshot s equals sum_i sigma_i conj(W_si) phi_i, so its
 * coefficients relative to sigma_0 are t_si = sigma_i conj(W_si) / sigma_0
 * (real parts, then imaginary parts). Each of these 2*rank outputs is
 * standardized over the snapshots: the network's targets are
 * (t_so - tmean_o) / tscale_o, with tmean_o the mean and tscale_o the RMS
 * deviation (1 for an output that does not vary), so every coefficient is
 * fitted to the same relative accuracy. Matrix products of the MLP run on BF16 matrix cores
 * with FP32 accumulation and FP32 master weights. The model keeps its own
 * copy of the basis.
 *   scvs_ws_train    epochs of full-batch Adam (lr; beta 0.9/0.999, eps 1e-8);
 *                    *loss = mean-squared error before the last epoch's update
 *                    (epochs == 0: the current loss, no update)
 *   scvs_ws_predict  x0[s] = amp[s] sigma_0 sum_i t_i(omega[s]) phi_i   (device c128 [n][ndof]),
 *                    t_o = tmean_o + tscale_o * (network output o)
 * Pass the predictions as x0 to scvs_solve; it falls back to the zero guess
 * for any system whose initial residual is not below ||f||.
 *   scvs_ws_refine   optional correction of guesses x0 (device c128 [n][ndof],
 *                    updated in place): x0 += Phi d, d minimizing
 *                    ||f - A(omega)(x0 + Phi d)|| over unconstrained rows, with
 *                    f built from (traction, g) exactly as scvs_solve builds it.
 *                    A(omega) Phi is affine in omega, so A(0) Phi and its slope
 *                    (2*rank*ndof complex values) are formed on the first call
 *                    after each assembly or boundary-condition change; each
 *                    call then costs one residual, one projection and a host
 *                    rank x rank solve per system. The result is the best
 *                    residual in x0 + span(Phi), whatever the network said. */
typedef struct scvs_ws_s* scvs_ws;
int scvs_ws_create(scvs_mesh mesh, int64_t nsnap, const double* omega, const void* snaps, int rank,
                   int width, int layers, uint64_t seed, scvs_ws* out);
int scvs_ws_train(scvs_ws ws, int epochs, double lr, double* loss);
int scvs_ws_predict(scvs_ws ws, int64_t n, const double* omega, const double* amp, void* x0);
int scvs_ws_refine(scvs_ws ws, int64_t n, const double* omega, const double* traction, const void* g,
                   void* x0);
int scvs_ws_destroy(scvs_ws ws);
/* Test/inspection hooks (host buffers unless stated):
 *  SCVS_WS_SIGMA double[rank]; SCVS_WS_BASIS device c128[rank][ndof];
 *  SCVS_WS_PARAMS float[nparam] (per layer W [out][in] row-major, then b);
 *  SCVS_WS_TARGETS float[nsnap][2*rank] (standardized); SCVS_WS_NPARAM int64;
 *  SCVS_WS_TMEAN, SCVS_WS_TSCALE double[2*rank] */
#define SCVS_WS_SIGMA 0
#define SCVS_WS_BASIS 1
#define SCVS_WS_PARAMS 2
#define SCVS_WS_TARGETS 3
#define SCVS_WS_NPARAM 4
#define SCVS_WS_TMEAN 5
#define SCVS_WS_TSCALE 6
int scvs_ws_export(scvs_ws ws, int which, void* out);
int scvs_ws_set_params(scvs_ws ws, const float* params);
/* Loss and gradients of the MLP on given inputs x[n][3] and targets t[n][2*rank] (host). */
int scvs_ws_loss_grad(scvs_ws ws, int64_t n, const float* x, const float* t, double* loss, float* grads);
/* Host eigen-decomposition used by the POD (complex Hermitian, cyclic Jacobi):
 * a c128[n][n] -> w double[n] descending, v c128[n][n] (columns). Needs no GPU. */
int scvs_herm_eig(int n, const double* a, double* w, double* v);

/* ---- measurement ----
 * When profiling is on, solves run without graph replay and every kernel
 * launch is bracketed by HIP events recorded on the context stream (the
 * stream the kernels run on). Per kernel class the library accumulates the
 * number of launches, the summed event time and the algorithmic bytes that
 * class moves per launch by construction (matrix arrays read once, each
 * vector element read or written once; formulas in the source of each
 * launcher). scvs_profile_read copies up to `max` entries to `out` (host),
 * sets *n, and clears the statistics. */
typedef struct {
  char name[40];
  int64_t launches;
  double total_ms;  /* summed launch durations */
  double bytes;     /* summed algorithmic bytes */
} scvs_kernel_stat;
int scvs_profile_enable(scvs_ctx ctx, int on);
int scvs_profile_read(scvs_ctx ctx, int max, scvs_kernel_stat* out, int* n);

/* Test hook: runs one FP64 16x16x4 matrix-core instruction on A[i][k] = a[i*4+k],
 * B[k][j] = b[k*16+j] (host double[64] each) and returns D = A B (host
 * double[256], row-major) as laid out by the library's lane mapping. */
int scvs_probe_mfma(scvs_ctx ctx, const double* a, const double* b, double* d);
/* Same for one BF16 16x16x16 instruction (operands rounded to bfloat16, FP32
 * accumulate): a float[16][16], b float[16][16], d float[16][16]. */
int scvs_probe_mfma_bf16(scvs_ctx ctx, const float* a, const float* b, float* d);

#ifdef __cplusplus
}
#endif
#endif /* SCVS_H */
