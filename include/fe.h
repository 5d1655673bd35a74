/*
 * fe.h -- C ABI of the MI355X element-level finite-element hot path.
 *
 * The library computes, for a two-phase (or multi-phase) micromechanics RVE on
 * a structured n x n x n mesh of 8-node bricks covering the unit cube, or on any
 * conforming mesh of 8-node bricks (fe_problem_create_hex8), the pieces of the
 * paper's Newton method for R(u) = 0 (Sec. II-A):
 *   - element residuals assembled into R(u)            (fe_residual)
 *   - element Jacobians assembled into a sparse K(u)   (fe_csr_indices, fe_tangent_csr;
 *     the sorted, duplicate-combined sparse tuple of Sec. III-B)
 *   - the matrix-free action y = K(u) x                 (fe_apply_matfree; Sec. III-A)
 *   - the sparse mat-vec with the explicit matrix       (fe_apply_csr; Fig. 3)
 *   - a Jacobi-preconditioned CG solve in FP64 scalars  (fe_pcg; Fig. 4)
 *   - Newton load stepping around them                  (fe_newton; Sec. II-A, Sec. V-A)
 *   - the vector-Jacobian product of the residual with respect to a per-element
 *     modulus scale, for adjoint gradients               (fe_vjp)
 *
 * Mesh conventions of the structured problem: node (i,j,k) has id
 * i + (n+1)(j + (n+1)k) at x = (i,j,k)/n; element (a,b,c) has id a + n(b + nc).
 * Both kinds: dof = 3*node + comp; 2x2x2 Gauss points, point q = qx + 2 qy + 4 qz
 * at reference coordinates (+-1/sqrt 3) with weight 1.
 *
 * Conventions of every call:
 *   - Array arguments are DEVICE pointers unless the name ends in _host.  The
 *     caller owns them; the library only borrows them for the duration of the
 *     call (and of the work it enqueues).
 *   - Floating-point arrays are double when the problem was created with
 *     FE_F64 and float with FE_F32 ("real" below).  Solver scalars and
 *     reductions are always double.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Work is
 *     enqueued on it; outputs are valid once the stream has reached that point.
 *     Calls that return host values (fe_csr_nnz, fe_pcg, fe_newton,
 *     fe_read_flags) synchronise the stream.
 *   - Every call returns an fe_status; arguments are validated before anything
 *     is enqueued; a failing HIP call maps to FE_ERR_HIP and fe_last_error()
 *     (thread-local) holds the message.  Nothing aborts.
 *   - Plastic state arrays are SoA with 7 components [eps_p xx,yy,zz,yz,xz,xy
 *     (engineering shears), alpha], each laid out [q][element]: entry
 *     (comp, q, e) is at ((comp*8 + q) * n_el + e).
 */
#ifndef FE_H
#define FE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FE_OK = 0,
  FE_ERR_ARG = 1,           /* invalid argument or unsupported combination */
  FE_ERR_HIP = 2,           /* a HIP runtime call failed */
  FE_ERR_OOM = 3,           /* device allocation failed */
  FE_ERR_NOT_CONVERGED = 4, /* iteration limit reached */
  FE_ERR_BREAKDOWN = 5,     /* CG found p.Ap <= 0 (operator not SPD) */
  FE_ERR_NONFINITE = 6,     /* NaN or Inf met in a solver scalar */
  FE_ERR_INVERTED = 7,      /* an element has det F <= 0 (finite strain) */
  FE_ERR_STATE = 8          /* call made before the state it needs exists */
} fe_status;

enum { FE_F64 = 0, FE_F32 = 1 };                      /* precision of real arrays */
enum { FE_LINEAR = 0, FE_J2 = 1, FE_NEOHOOKE = 2 };    /* constitutive model per phase */
enum { FE_OP_CSR = 0, FE_OP_MATFREE = 1 };             /* operator used by fe_pcg / fe_newton */
enum { FE_PC_JACOBI = 0, FE_PC_BLOCK_JACOBI = 1, FE_PC_ILU0 = 2 };  /* preconditioner (fe_set_preconditioner) */
enum { FE_SOLVER_CG = 0, FE_SOLVER_BICGSTAB = 1, FE_SOLVER_GMRES = 2 };  /* Krylov method of fe_newton's inner solves */
enum { FE_APPLY_BC = 1, FE_STORE_TANGENT = 2 };        /* fe_residual flags */
enum { FE_MAX_PHASES = 8 };

typedef struct fe_problem fe_problem;

typedef struct {
  int iterations;        /* CG iterations performed */
  int status;            /* fe_status of the solve */
  double relres;         /* recursive ||r|| / ||b|| at exit */
  double bnorm;          /* ||b||_2 */
} fe_pcg_info;

typedef struct {
  int op;                /* FE_OP_CSR or FE_OP_MATFREE: operator used inside CG */
  int assemble_csr;      /* with FE_OP_MATFREE: 1 = also assemble the CSR tangent every
                            iteration (matrix-explicit Jacobian, Sec. III-B) and take the
                            Jacobi diagonal from it; 0 = diagonal from the element kernel */
  int max_newton;        /* Newton iterations per load step (e.g. 20) */
  double newton_rtol;    /* stop when ||P_f R|| <= newton_rtol * ||P_f R||_first (e.g. 1e-8) */
  double pcg_rtol;       /* inner CG tolerance (e.g. 1e-10) */
  int pcg_max_it;        /* inner CG iteration limit */
  int solver;            /* FE_SOLVER_CG (symmetric tangents), FE_SOLVER_BICGSTAB or FE_SOLVER_GMRES */
  int restart;           /* GMRES restart length (1..64; 0 = 30) */
  int predictor;         /* start of load step k >= 2: FE_PREDICT_BOUNDARY moves only the boundary values
                            to the new macro strain; FE_PREDICT_EXTRAPOLATE first adds
                            (|E_k - E_{k-1}| / |E_{k-1} - E_{k-2}|) (u_{k-1} - u_{k-2}) to the free
                            values (linear extrapolation of the converged path, Frobenius norms of
                            the macro-strain increments) */
  int* step_log_host;    /* NULL, or [n_steps][3] host ints: per load step the Newton iterations,
                            line-search halvings and inner Krylov iterations (filled as steps end) */
} fe_newton_opts;

enum { FE_PREDICT_BOUNDARY = 0, FE_PREDICT_EXTRAPOLATE = 1 };

typedef struct {
  int newton_iterations; /* summed over load steps */
  int pcg_iterations;    /* summed over all linear solves */
  int operator_applies;  /* K*x applications (one per CG iteration plus one per solve) */
  int steps_done;        /* load steps that converged */
  int line_search_halvings; /* step halvings taken by the line search, summed */
  int status;            /* fe_status of the whole run */
  double last_residual;  /* ||P_f R|| at the end of the last step */
} fe_newton_info;

/* Create the structured problem: n elements per side of [0,1]^3 (1 <= n <= 1024,
 * with 3(n+1)^3 dofs and 9(3n+1)^3 matrix entries both below 2^31), precision
 * FE_F64 or FE_F32, on the current HIP device.  *out receives an opaque handle
 * owned by the library (free with fe_problem_destroy).  This is the problem
 * structure of the paper's construction phase (Fig. 1: mesh, element information,
 * Dirichlet data; Sec. IV) for the regular RVE meshes of Sec. V-A, whose numbering
 * (above) lets the element kernels stage bricks of elements and the sparse pattern
 * be written in closed form. */
int fe_problem_create(fe_problem** out, int n, int precision);

/* Create a problem on a general mesh of 8-node bricks (the element information and
 * problem structure of Fig. 1 given explicitly; Sec. III-B builds the Jacobian of
 * such a mesh by sorting and combining the element pairs, Sec. IV).
 *   coords: double, DEVICE, [3][n_nodes] (x of all nodes, then y, then z);
 *   conn:   int32, DEVICE, [8][n_el]: conn[p * n_el + e] = node of local node p of
 *           element e, local order (-1,-1,-1) (1,-1,-1) (1,1,-1) (-1,1,-1) (-1,-1,1)
 *           (1,-1,1) (1,1,1) (-1,1,1) in reference coordinates (any right-handed
 *           numbering of the brick, e.g. a rotation of this one).
 * Both are copied (the caller keeps ownership; coordinates are stored in the
 * problem's precision).  The library checks every node id (FE_ERR_ARG outside
 * [0, n_nodes)) and det J > 0 at every Gauss point (FE_ERR_ARG otherwise), then builds
 * the node-pair pattern on the device: every element's 64 (row node, column node)
 * pairs are bucketed by row and sorted by (column, element), duplicates combined;
 * the sorted element list of each pair drives the deterministic gather of
 * fe_tangent_csr.  Limits: 3 n_nodes < 2^31, 64 n_el < 2^31, 9 (node pairs) < 2^31,
 * at most 128 elements per node (FE_ERR_ARG otherwise).  Every other call works as on
 * the structured problem (dofs 3 node + c, Gauss point q of element e at index
 * q n_el + e of state arrays, fe_lift from the stored coordinates, fe_mean_stress
 * divided by the mesh volume), except: FE_PC_ILU0, the learned surrogate and its
 * sample capture, and fe_vjp_path are structured-only (FE_ERR_ARG); CG runs one
 * operator, one update and one direction launch per iteration.  Synchronises the
 * stream.  Needs device memory of 64 n_el + 12 (node pairs) + 3 n_nodes int32 and,
 * once fe_tangent_csr runs, 576 n_el reals for the element Jacobians. */
int fe_problem_create_hex8(fe_problem** out, int64_t n_nodes, int64_t n_el, const double* coords,
                           const int32_t* conn, int precision, void* stream);
void fe_problem_destroy(fe_problem* p);

/* Sizes: out_host[0..5] = n (0 for a general mesh), n_el, n_nodes, n_dof,
 * n_qp (= 8 n_el), nnz.
 * Sizes of the discretisation of Sec. II-A and of its sparse matrix (Sec. III-B). */
int fe_problem_sizes(const fe_problem* p, int64_t* out_host);

/* Materials (the phase-dependent laws of Sec. V-A).  phase: uint8 [n_el] with
 * values < n_phases; models_host: [n_phases] FE_LINEAR / FE_J2 / FE_NEOHOOKE;
 * params_host: [n_phases][4] = {E, nu, sigma_y, H} (the last two used by J2
 * only); scale: real [n_el] multiplying the elastic moduli of each element, or
 * NULL for 1.  Phase and scale are copied into library memory. */
int fe_set_materials(fe_problem* p, const uint8_t* phase, int n_phases, const int* models_host,
                     const double* params_host, const void* scale, void* stream);

/* Dirichlet dofs (the boundary treatment that Sec. II-B applies before the solve):
 * uint8 [n_dof], 1 = constrained (copied into library memory).  Default: none.
 * mask = NULL removes them. */
int fe_set_dirichlet(fe_problem* p, const uint8_t* mask, void* stream);

/* Affine boundary values of a macro strain (the RVE loading of Sec. V-A):
 * u[d] = (eps_bar . x)_comp on constrained dofs d; free dofs keep their value
 * (zero_free = 0) or are set to 0 (zero_free = 1).  eps_bar_host: 3x3 row-major. */
int fe_lift(fe_problem* p, const double* eps_bar_host, void* u, int zero_free, void* stream);

/* Residual R(u) = sum_e A_e^T r_e (Sec. II-A).  u, r: real [n_dof].
 * state_in: plastic state at the last converged step (NULL = zero); state_out:
 * trial state written for J2 points (NULL = not written).  flags: FE_APPLY_BC
 * zeroes r on constrained dofs; FE_STORE_TANGENT records the linearisation at u
 * (J2 consistent tangent per point, Neo-Hookean deformation per point) for
 * fe_apply_matfree / fe_diagonal / fe_pcg. */
int fe_residual(fe_problem* p, const void* u, const void* state_in, void* state_out, void* r,
                int flags, void* stream);

/* Number of stored entries of the sparse Jacobian, known before any value is
 * computed (the pre-computed non-zero count of the assembly listing in Sec. III-B;
 * structural pattern: every pair of dofs that share an element, explicit zeros
 * kept): 9(3n+1)^3 on the structured mesh, 9 x (node pairs) on a general one. */
int fe_csr_nnz(const fe_problem* p, int64_t* nnz_host);

/* CSR pattern, rows = dofs, columns ascending: row_ptr int32 [n_dof+1],
 * col_idx int32 [nnz]; identical to sorting all element (row, col) pairs and
 * combining duplicates (Sec. III-B). */
int fe_csr_indices(fe_problem* p, int32_t* row_ptr, int32_t* col_idx, void* stream);

/* Jacobian values K(u) in the pattern of fe_csr_indices: vals real [nnz],
 * duplicates summed.  Linearises at (u, state_in) first (as FE_STORE_TANGENT).
 * apply_bc = 1 zeroes constrained rows and columns and puts 1 on their diagonal.
 * The Jacobian of Sec. II-A as the sparse matrix of Sec. III-B. */
int fe_tangent_csr(fe_problem* p, const void* u, const void* state_in, void* vals, int apply_bc,
                   void* stream);

/* Matrix-free y = K x at the stored linearisation (the elastic K when the
 * problem has only linear phases).  apply_bc = 1 gives P_f K P_f x + P_b x.
 * The matrix-free operator of Sec. III-A. */
int fe_apply_matfree(fe_problem* p, const void* x, void* y, int apply_bc, void* stream);

/* CSR y = A x for any CSR matrix with n_dof rows (row_ptr, col_idx int32).
 * The explicit-matrix mat-vec timed in Fig. 3. */
int fe_apply_csr(fe_problem* p, const int32_t* row_ptr, const int32_t* col_idx, const void* vals,
                 const void* x, void* y, void* stream);

/* CSR y = A x for a matrix in the node-structured pattern of fe_csr_indices
 * (rows 3a, 3a+1, 3a+2 have identical column lists): the column indices and the
 * gathered x of a node's first row serve all three rows, so index traffic is a
 * third of fe_apply_csr's.  Results equal fe_apply_csr's (same products and sums,
 * possibly in another order).  The pattern is not checked.
 * The explicit-matrix mat-vec of Fig. 3 for this pattern. */
int fe_apply_csr_nodal(fe_problem* p, const int32_t* row_ptr, const int32_t* col_idx, const void* vals,
                       const void* x, void* y, void* stream);

/* Diagonal of the (masked, if apply_bc) matrix-free operator, the Jacobi
 * preconditioner of the Krylov solves compared in Fig. 4: d real [n_dof]
 * (constrained dofs get 1 when apply_bc). */
int fe_diagonal(fe_problem* p, void* d, int apply_bc, void* stream);

/* Preconditioner of fe_pcg and fe_newton's inner solves (default FE_PC_JACOBI).
 * FE_PC_JACOBI: M = diag(A) (Fig. 4).  FE_PC_BLOCK_JACOBI: M = the 3x3 blocks of
 * A that couple the three components of one node, the first step towards the
 * stronger preconditioning of the assembled matrix compared in Fig. 7; taken
 * from the CSR values with FE_OP_CSR (and with fe_newton's assemble_csr), from
 * the stored linearisation otherwise.  The blocks are inverted once per solve
 * (workspace of 6 reals per node, allocated on first use; FE_ERR_OOM if that
 * fails).  A block with determinant <= 0 sets bit 1 of fe_read_flags; a
 * singular one makes the solve end with FE_ERR_NONFINITE.  FE_PC_ILU0: node-block
 * incomplete LU without fill (3x3 blocks of node pairs that share an element),
 * nodes taken in 8 colours by the parities of their grid indices so that each
 * colour is one data-parallel level of the factorisation and of the two
 * triangular sweeps (Fig. 7 compares ILU with Jacobi on the assembled matrix);
 * it needs the CSR values (FE_OP_CSR, or fe_newton with assemble_csr), is
 * factored once per solve into 243 reals per node (allocated here; FE_ERR_OOM if
 * that fails) and is applied by fe_gmres, fe_bicgstab and fe_pcg (CG then runs
 * unfused: the operator, the step, the two sweeps and the new direction as
 * separate launches; for symmetric A the factors satisfy U = D L^T, so M is
 * symmetric); a singular pivot block sets bit 2 of fe_read_flags and ends the
 * solve with FE_ERR_NONFINITE.  FE_ERR_ARG for any other kind. */
int fe_set_preconditioner(fe_problem* p, int kind);

/* z = M^-1 r for the preconditioner chosen by fe_set_preconditioner, set up as the
 * solvers set it up: from the CSR matrix when row_ptr, col_idx and vals are given
 * (already eliminated; required for FE_PC_ILU0), else from the stored
 * linearisation (FE_ERR_STATE without one).  r, z: real [n_dof], distinct.
 * Preconditioners of the Krylov solves compared in Sec. V-B (Fig. 7). */
int fe_apply_preconditioner(fe_problem* p, const int32_t* row_ptr, const int32_t* col_idx,
                            const void* vals, const void* r, void* z, void* stream);

/* Preconditioned CG on A x = b (Fig. 4): A is the masked operator
 * P_f K P_f + P_b, matrix-free (op = FE_OP_MATFREE, CSR arguments ignored) or the
 * CSR matrix given (op = FE_OP_CSR, already eliminated).  x0 = 0; stops when
 * ||r||_2 <= rtol ||b||_2.  x: real [n_dof] output.  info_host may be NULL.
 * Returns FE_OK, FE_ERR_NOT_CONVERGED, FE_ERR_BREAKDOWN or FE_ERR_NONFINITE. */
int fe_pcg(fe_problem* p, int op, const int32_t* row_ptr, const int32_t* col_idx,
           const void* vals, const void* b, void* x, double rtol, int max_it,
           fe_pcg_info* info_host, void* stream);

/* Preconditioned BiCGStab on A x = b for nonsymmetric operators (the paper's
 * Fig. 4 compares CG, GMRES and BiCGStab): same operators, arguments,
 * preconditioner (fe_set_preconditioner) and stopping rule as fe_pcg; one
 * iteration applies A twice.  Returns FE_OK, FE_ERR_NOT_CONVERGED,
 * FE_ERR_BREAKDOWN (rho or (r_hat, v) vanished) or FE_ERR_NONFINITE.  Workspace of
 * 8 vectors allocated on first use (FE_ERR_OOM if that fails). */
int fe_bicgstab(fe_problem* p, int op, const int32_t* row_ptr, const int32_t* col_idx,
                const void* vals, const void* b, void* x, double rtol, int max_it,
                fe_pcg_info* info_host, void* stream);

/* Restarted GMRES(m) on A x = b (Saad & Schultz 1986; Fig. 4 of the paper compares
 * it with CG and BiCGStab), right-preconditioned by the preconditioner of
 * fe_set_preconditioner: same operators and arguments as fe_pcg, x0 = 0, stops
 * when the least-squares residual estimate |g_k| <= rtol ||b||_2 (info relres is
 * that estimate over ||b||); after `restart` Arnoldi steps (1..64, else
 * FE_ERR_ARG) x is updated and the next cycle starts from b - A x.  One iteration
 * = one Arnoldi step = one application of A.  Returns FE_OK,
 * FE_ERR_NOT_CONVERGED (max_it steps; x holds the last least-squares iterate),
 * FE_ERR_BREAKDOWN (singular Hessenberg block) or FE_ERR_NONFINITE.  Workspace of
 * restart + 3 vectors allocated on first use or when a longer restart is asked
 * for (FE_ERR_OOM if that fails). */
int fe_gmres(fe_problem* p, int op, const int32_t* row_ptr, const int32_t* col_idx,
             const void* vals, const void* b, void* x, double rtol, int max_it, int restart,
             fe_pcg_info* info_host, void* stream);

/* Vector-Jacobian product with respect to the per-element modulus scale s_e:
 * out[e] = lambda_e^T d r_e / d s_e, real [n_el].  Supported for linear and
 * Neo-Hookean phases (r_e is proportional to s_e); FE_ERR_ARG with J2 phases.
 * Adjoint gradients for the differentiable-simulation use of Sec. I. */
int fe_vjp(fe_problem* p, const void* u, const void* lambda, void* out, void* stream);

/* One backward step of the discrete adjoint through a J2 load path (history
 * checkpointing, Sec. I's differentiable simulation through the path-dependent
 * material).  FE_F64 problems with linear and J2 phases.  The step maps
 * (u_n, h_{n-1}, s) to the residual R_n and the trial state h_n = Phi(u_n, h_{n-1}, s);
 * given the linearisation point u (real [n_dof]) and the state at the start of
 * the step state_in ([7][8][n_el], NULL = zero), and cotangents c on R_n (real
 * [n_dof], NULL = 0) and mu_in on h_n ([7][8][n_el], NULL = 0), it writes
 *   mu_out[7][8][n_el] = d(c.R_n + mu_in.h_n)/d h_{n-1}
 * and accumulates (both optional, caller-zeroed)
 *   u_bar[n_dof] += d(mu_in.h_n)/d u      (history part only: the adjoint right-hand side)
 *   s_bar[n_el]  += d(c.R_n + mu_in.h_n)/d s_e.
 * s is the per-element modulus scale of fe_set_materials (sigma_y, H unscaled).
 * FE_ERR_ARG for FE_F32 problems or Neo-Hookean phases. */
int fe_vjp_path(fe_problem* p, const void* u, const void* state_in, const void* c, const void* mu_in,
                void* mu_out, void* u_bar, void* s_bar, void* stream);

/* Newton load stepping: for each of n_steps macro strains (load_path_host:
 * [n_steps][3][3] row-major) lift the boundary, iterate Newton with the chosen
 * operator until the opts tolerance, then commit the plastic state.  Each
 * Newton update w is taken as u += s w with s = 1 halved (at most 5 times)
 * while ||P_f R(u + s w)|| >= ||P_f R(u)||.
 * u: real [n_dof] in/out (the starting field); state: real [7][8][n_el] in/out
 * (NULL for problems without J2 phases); sigma_bar_host: [n_steps][6] volume
 * averaged stress after each step, or NULL.
 * Newton's method for R(u) = 0 (Sec. II-A) over the load ramps of Sec. V-A. */
int fe_newton(fe_problem* p, const double* load_path_host, int n_steps, const fe_newton_opts* opts,
              void* u, void* state, double* sigma_bar_host, fe_newton_info* info_host,
              void* stream);

/* Resume the load stepping of fe_newton at step first_step (0 <= first_step <= n_steps)
 * of the same load_path_host, e.g. from a snapshot taken after step first_step - 1
 * (the load-step history of Sec. II-A / V-A: converged field and committed plastic state).
 * u: in, the converged field of step first_step - 1 (out: of the last step); state: in,
 * the committed state after that step; u_prev: the converged field of step first_step - 2,
 * read only by FE_PREDICT_EXTRAPOLATE when first_step >= 2 (required there, else may be
 * NULL).  sigma_bar_host and opts->step_log_host keep the [n_steps] layout; rows before
 * first_step are not written.  info counts the resumed steps only.  With the same inputs
 * the steps run exactly the arithmetic of an uninterrupted fe_newton call (bit-identical
 * results in deterministic mode). fe_newton(...) is fe_newton_resume with first_step = 0. */
int fe_newton_resume(fe_problem* p, const double* load_path_host, int n_steps, int first_step,
                     const fe_newton_opts* opts, void* u, const void* u_prev, void* state,
                     double* sigma_bar_host, fe_newton_info* info_host, void* stream);

/* Deterministic mode (on = 1) of a structured problem: the residual, the matrix-free operator
 * and the Jacobi diagonal (R(u), K x and diag K of Sec. II-A) sum element contributions in a
 * fixed order instead of with floating-point atomics -- each element writes its 24 nodal
 * values to a library buffer (24 n_el reals, allocated here; FE_ERR_OOM if that fails) and
 * one pass sums, per dof, the (up to 8) elements around its node in element order -- the
 * volume-averaged stress sums per-workgroup partials in order, and matrix-free CG runs its
 * unfused form (operator, update and direction launches; the fused launch's atomic slot sums
 * are not used).  Results are then bit-identical from run to run on one GPU (same inputs,
 * launch configuration and library build), so Newton and Krylov iteration counts become
 * reproducible; they equal the default mode's up to rounding order.  Not covered: node-block
 * Jacobi built from the stored linearisation (use it with the assembled matrix), the learned
 * surrogate's sample lists (their slot order varies; values do not).  General meshes:
 * FE_ERR_ARG.  on = 0 returns to the default (faster) mode. */
int fe_set_deterministic(fe_problem* p, int on);

/* FP32 accumulation (on = 1) of an FP32 structured problem (an extension: the paper computes
 * in FP64).  By default FP32 problems store and compute in FP32 but sum each node's element
 * forces (residual R(u), K x of Sec. II-A) in FP64 inside the workgroup; with on = 1 those
 * sums run in FP32 as well, so every nodal value is formed in FP32.  Reductions that decide
 * convergence (PCG dots, residual norms, the Newton test) stay FP64 either way.  FP64
 * problems and general meshes: FE_ERR_ARG.  on = 0 returns to FP64 nodal sums. */
int fe_set_fp32_accumulation(fe_problem* p, int on);

/* Commit the plastic history of a converged load step (the state update that ends
 * each Newton solve of Sec. II-A / V-A): state = state_trial, both real [7][8][n_el]
 * (the trial state written by fe_residual's state_out).  For callers that drive
 * their own Newton loop; fe_newton commits by itself.  No-op for problems without
 * J2 phases.  Enqueued on the stream (a copy kernel, no allocation). */
int fe_commit_state(fe_problem* p, const void* state_trial, void* state, void* stream);

/* Volume-averaged stress (1/V) sum_q w_q detJ_q sigma_q at (u, state_in),
 * written to sigma_host[6] in Voigt order [xx,yy,zz,yz,xz,xy].
 * The homogenised (effective) response of the RVE, Sec. V-A. */
int fe_mean_stress(fe_problem* p, const void* u, const void* state_in, double* sigma_host,
                   void* stream);

/* Kernel timing for measurement.  While enabled, the library records a HIP
 * event pair inside the dispatch of each launch of: class 0 the matrix-free
 * operator kernel (fe_apply_matfree and inside CG), class 1 the CSR mat-vec
 * (fe_apply_csr and inside CG), class 2 the residual / return-map element
 * kernel, class 3 the CSR tangent kernel, class 4 the node-structured CSR
 * mat-vec (fe_apply_csr_nodal).  enable = 1 clears previous records; enable = 0
 * stops recording; enable = k > 1 is enable = 1 except that inside a CG solve
 * only operator launches 0, k, 2k, ... are timed (an event pair costs several
 * microseconds of issue time per launch); enable < 0 is FE_ERR_ARG.
 * fe_profile_read synchronises the device and writes, for
 * c = 0..4, out_host[3*c] = launches, out_host[3*c+1] = summed milliseconds,
 * out_host[3*c+2] = summed algorithmic bytes of those launches for classes 0, 1
 * and 4 (compulsory traffic: x read and y written once, phase ids, the stored
 * tangent values the kernel must read at the current linearisation; CSR:
 * values, column indices (one list per node for class 4), row pointers, x and
 * y once), 0 for classes 2 and 3; then clears the records.  out_host: 15 doubles.
 * Per-operation timing as in the measurements of Sec. V-B. */
int fe_profile(fe_problem* p, int enable);
int fe_profile_read(fe_problem* p, double* out_host);

/* Statistics of the stored linearisation: out_host[0] = Gauss points of J2
 * phases, out_host[1] = those that were plastic (synchronises).
 * Of the J2 phase's constitutive update (Sec. V-A). */
int fe_linearization_stats(fe_problem* p, int64_t* out_host, void* stream);

/* Device-side error flags raised by element kernels since the last read
 * (bit 0: inverted element; bit 1: a node block of the block-Jacobi
 * preconditioner with determinant <= 0; bit 2: a singular ILU(0) pivot block).
 * Synchronises and clears.
 * Failures of the element computations of Sec. II-A. */
int fe_read_flags(fe_problem* p, int* flags_host, void* stream);

/* ---- learned constitutive surrogate (Sec. III-B: a surrogate may replace the
 * designed stress-strain function, its Jacobian serving as the tangent) ----
 * Network: dense 13 -> 128 -> 128 -> 128 -> 6, SiLU after the hidden layers,
 * linear output.  Parameters are FP32 on the device, FE_MLP_PARAMS floats: for
 * layers l = 1..4 in order, the weights input-major Wt_l[in][out] followed by
 * the bias b_l[out].  Inputs/outputs are the normalised quantities. */
enum { FE_MLP_IN = 13, FE_MLP_HIDDEN = 128, FE_MLP_OUT = 6, FE_MLP_PARAMS = 35590, FE_MLP_STATIC_MAX = 8192 };

/* y = net(x): x float [n][13], y float [n][6].  jac (float [n][6][6], may be
 * NULL): jac[s][o][j] = dy_o/dx_j for the first six inputs (forward-mode
 * tangents carried through FP32 matrix cores).  cache (float [n][3][128], may
 * be NULL): hidden pre-activations, for fe_mlp_backward.
 * Learned constitutive surrogate (the surrogate-model remark of Sec. III-B). */
int fe_mlp_forward(const float* W, const float* x, float* y, float* jac, float* cache, int64_t n, void* stream);

/* Gradients of L = mean_s sum_o (y - target)^2 over the n samples of one batch:
 * dW (float [FE_MLP_PARAMS]) is overwritten; loss_dev (double [1]) receives L;
 * work is scratch of float [n][3*128+6] (per-sample pre-activation gradients).
 * Training of the learned surrogate of Sec. III-B. */
int fe_mlp_backward(const float* W, const float* x, const float* cache, const float* y, const float* target,
                    float* dW, double* loss_dev, float* work, int64_t n, void* stream);

/* fe_mlp_backward without the workspace argument and without any device allocation, for
 * callers that cannot allocate (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  The per-sample gradients go to a library-owned device array sized for
 * FE_MLP_STATIC_MAX samples (12.8 MB, one copy per GPU the library runs on, held until the
 * process ends).  n > FE_MLP_STATIC_MAX is FE_ERR_ARG.  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (concurrent streams, threads) race and must be
 * ordered by the caller.  Results equal fe_mlp_backward's up to the order of the FP32 atomic
 * additions of the weight gradients. */
int fe_mlp_backward_static(const float* W, const float* x, const float* cache, const float* y, const float* target,
                           float* dW, double* loss_dev, int64_t n, void* stream);

/* One Adam step (Kingma & Ba), t >= 1: m, v are the first/second moment buffers.
 * Training of the learned surrogate of Sec. III-B. */
int fe_adam_step(float* W, const float* dW, float* m, float* v, int64_t n_param, double lr, double beta1,
                 double beta2, double eps, int t, void* stream);

/* Use the network as the constitutive law at J2 points whose elastic trial is
 * plastic (elsewhere, and in other phases, the exact laws apply).  The network
 * interface is normalised by the first J2 phase: inputs
 * [eps - eps_p_n, eps_p_n] in Mandel form (shears times sqrt 2 of the tensor
 * components) and alpha_n, divided by sigma_y / E; output stress in Mandel
 * form divided by sigma_y.  From the predicted stress the point's plastic
 * strain is eps - C^-1 sigma and alpha grows by sqrt(2/3) |d eps_p|; where the
 * prediction's local check max(|q - sigma_y - H alpha| / sigma_y,
 * |dev s / |dev s| - N_trial|) exceeds fallback_tol the exact radial return is
 * used instead.  The tangent of accepted points is the symmetric part of the
 * network Jacobian (the linear solver is CG).  W (float [FE_MLP_PARAMS],
 * device) is borrowed until the next call; NULL switches the surrogate off.
 * Every fe_residual then runs three launches (list plastic-trial points,
 * network, residual) and synchronises once.
 * The learned surrogate of Sec. III-B in place of the return map. */
int fe_set_surrogate(fe_problem* p, const float* W, double fallback_tol);

/* Tangent handed to the linear solver at accepted surrogate points: 0 (default)
 * the symmetric part of the network Jacobian (for CG), 1 the Jacobian itself,
 * which makes the operator nonsymmetric (solve with FE_SOLVER_BICGSTAB /
 * fe_bicgstab).  Takes effect at the next residual evaluation.
 * Linearisation of the learned surrogate of Sec. III-B. */
int fe_set_surrogate_tangent(fe_problem* p, int full);

/* After fe_residual with a surrogate: out_host = {points given to the network,
 * accepted, fallbacks} (synchronises).
 * Of the learned surrogate of Sec. III-B. */
int fe_surrogate_stats(fe_problem* p, int64_t* out_host, void* stream);

/* Training-sample capture: while set (x != NULL), every fe_residual appends,
 * at J2 points whose elastic trial is plastic and whose hashed point index
 * passes a 1-in-stride thinning, the normalised network input x [13] and the
 * exact return-map stress y [6] (same normalisation as fe_set_surrogate) to the
 * caller's buffers (float [capacity][13], [capacity][6]) at slot *count_dev
 * (device unsigned, incremented; slots beyond capacity are dropped).
 * Training data of the learned surrogate of Sec. III-B. */
int fe_set_capture(fe_problem* p, float* x, float* y, int64_t capacity, unsigned int* count_dev, int stride);

const char* fe_status_string(int status);
const char* fe_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FE_H */
