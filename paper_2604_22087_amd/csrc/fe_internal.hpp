// Internal declarations shared by the host API and the HIP kernels of libfe.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/fe.h"

namespace fe {

// Per-phase material constants, already converted to the forms kernels use.
struct PhaseConst {
  int model;        // FE_LINEAR / FE_J2 / FE_NEOHOOKE
  double lam, mu;   // Lame parameters (before the per-element scale)
  double K, G;      // bulk and shear moduli (J2)
  double sy, H;     // yield stress and linear hardening modulus (J2)
};

struct Phases {
  PhaseConst ph[FE_MAX_PHASES];
  int n;
};

// Which constitutive models a launch has to handle (selects a kernel instance).
enum ModelSet { MS_LINEAR = 0, MS_J2 = 1, MS_NH = 2 };

enum SurMode { SUR_OFF = 0, SUR_CAPTURE = 1, SUR_CLASSIFY = 2, SUR_CONSUME = 3 };
constexpr float SUR_FLAG = -2.0f;  // first stored-tangent word of a point whose tangent comes from the surrogate

// Element-kernel operations.
enum ElemOp {
  OP_RESID = 0,   // r = sum_e A_e^T r_e(u)        (+ state / linearisation side outputs)
  OP_APPLY = 1,   // y = K_lin x                   (matrix-free)
  OP_VJP = 2,     // out_e = lambda_e . d r_e / d s_e
  OP_CG_APPLY = 3 // single-reduction CG launch: vector updates, u = M^-1 r, w = A u, three dot partials
};

// CG status word: kernels stop on any non-zero value, so "converged" must differ from 0.
constexpr int CG_RUNNING = 0;
constexpr int CG_CONVERGED = -1;
constexpr int CG_UGRID = 512;        // workgroups of the CG vector kernels (= update partial slots)
constexpr int SPMV_MAXGRID = 2048;   // workgroups of the CG mat-vec (grid-stride over rows)

// Device scalar block used by CG (one per problem).
// restarted GMRES (fe_krylov.hip)
constexpr int GM_MAXM = 64;   // longest restart cycle
constexpr int GM_GRID = 512;  // workgroups of the GMRES vector kernels (= partial slots per vector)

struct GmresCtrl {
  double rtol, tol;  // tol = rtol ||b|| (set at the first cycle start)
  double bb;         // ||b||^2 (-1 until the first cycle start)
  double res_est;    // |g_k|: residual norm of the current least-squares iterate
  double inv_norm;   // 1 / ||w|| for the next basis vector
  int status;        // CG_RUNNING, CG_CONVERGED or an fe_status error code
  int iters;         // Arnoldi steps over all cycles
  int max_it;
  int k;             // finished columns of the running cycle
  int m;             // restart length
  int cycles;
};

struct GmresDev {
  GmresCtrl ctrl;
  double H[GM_MAXM][GM_MAXM + 1];  // Hessenberg matrix by columns (rotated to triangular form)
  double cs[GM_MAXM], sn[GM_MAXM];
  double g[GM_MAXM + 1];
  double y[GM_MAXM];
  double c[2][GM_MAXM + 1];        // Gram-Schmidt coefficients of the two passes
};

// CG with a separately applied preconditioner (ILU(0)), fe_krylov.hip
struct IpcgCtrl {
  double rzs[2];     // (r_k, z_k) of iteration k in slot k & 1
  double alpha, pq;  // last step length and (p, A p)
  double rtol, bb, tol2, rr;
  int status, iters, max_it, pad;
};

enum IpcgStage { IPCG_INIT = 1, IPCG_CHECK_FIRST, IPCG_FIRST_DIRECTION, IPCG_UPDATE, IPCG_CHECK, IPCG_DIRECTION };

enum GmStage { GM_START = 1, GM_BASIS, GM_ORTHO, GM_FINISH, GM_RESIDUAL, GM_ADD_Z };

// single-reduction CG: slots per reduced quantity that the workgroups of a launch add into
constexpr int CGS_SLOTS = 256;
// general meshes: workgroups (= partial slots) of the pass that completes the CG operator
constexpr int GEN_CG_GRID = 512;

struct CgCtrl {
  double rz[2];     // r.M^-1 r after update k-1, slot k&1 (written by the direction step of iteration k)
  double pq;        // p.Ap of the last operator
  double alpha, beta;
  double rr;        // ||r||^2 at the last direction step
  double bb;        // ||b||^2
  double tol2;      // rtol^2 ||b||^2
  double rtol2;     // rtol^2
  int iters;        // completed updates
  int status;       // CG_RUNNING, CG_CONVERGED or an fe_status error code
  int max_it;
  int pad;
  double ghist[2], ahist[2];  // single-reduction CG: (r, M^-1 r) and alpha of iterate i in slot i & 1
};

// Device scalar block of BiCGStab (one per problem).
struct BicgCtrl {
  double rho, rho_old, alpha, omega, beta;
  double rr;        // ||r||^2 at the last check
  double bb, tol2, rtol2;
  int iters, status, max_it;
  int finish;       // set by the update that met the tolerance; the next direction step stops
};
constexpr int BICG_GRID = 512;       // workgroups of the BiCGStab vector kernels (= partial slots)

struct ElemArgs {
  int n;
  double h;
  int64_t n_el;
  const uint8_t* phase;
  const void* scale;      // real [n_el] or null
  const uint8_t* mask;    // [n_dof] or null
  const void* x;          // gathered field (u for RESID/VJP, x for APPLY)
  const void* xlin;       // lambda (VJP)
  void* y;                // scattered output (may be null for RESID = linearise only)
  const void* state_in;   // J2 state [7][8][n_el] or null
  void* state_out;        // J2 trial state or null
  void* tangent;          // J2 compact tangent [6][8][n_el] (written in RESID, read in APPLY)
  void* out_el;           // VJP output [n_el]
  double* stress_sum;     // [6] volume-integrated stress accumulator or null
  int* flags;             // device error flags
  int apply_bc;
  int store_tangent;
  Phases mat;
  // learned surrogate at J2 points whose elastic trial is plastic
  int sur_mode;           // SUR_OFF / SUR_CAPTURE / SUR_CLASSIFY / SUR_CONSUME
  int* sur_map;           // [8][n_el] list slot of each point, -1 if none
  unsigned int* sur_count;
  int64_t sur_cap;
  float* sur_x;           // [cap][13] normalised network inputs
  float* sur_y;           // [cap][6] capture: normalised stress; consume: network output
  const float* sur_jac;   // [cap][6][6] network Jacobian (consume)
  void* sur_D;            // [cap][36] float: Voigt tangent of accepted points (symmetrised unless sur_full)
  unsigned int* sur_stats;// [2] accepted, fallback
  float sur_sin, sur_sout;
  double sur_tol;
  int sur_full;           // 1: the network Jacobian as tangent (nonsymmetric), 0: its symmetric part
  unsigned int sur_stride, sur_salt;
  // OP_CG_APPLY only (single-reduction CG, one operator launch per iteration; see the kernel)
  long cg_j;              // launch index j; launch 0 makes no update, only u_0 = M^-1 b and w_0 = A u_0
  const void* cg_rold;    // r_{j-1}
  void* cg_rnew;          // r_j (written by owners)
  const void* cg_wold;    // w_{j-1} = A u_{j-1}
  void* cg_wzero;         // the w buffer of launch j+1 (zeroed by owners)
  const void* cg_sold;    // s_{j-2}
  void* cg_snew;          // s_{j-1} (written by owners)
  void* cg_pvec;          // p (updated in place by owners)
  void* cg_x;             // x (updated in place by owners)
  const void* cg_dinv;    // preconditioner: inverse diagonal [n_dof] or inverse node blocks [n_nodes][6]
  int cg_block;           // 1: node-block Jacobi
  CgCtrl* ctrl;           // scalars and status (workgroup 0 writes those of launch j)
  const double* cg_acc_in;// [3][CGS_SLOTS] sums of launch j-1: (u, A u), (r, u), ||r||^2
  double* cg_acc_out;     // [3][CGS_SLOTS] sums of launch j (atomics; zeroed by launch j-1)
  double* cg_acc_zero;    // [3][CGS_SLOTS] slots of launch j+1 (zeroed by workgroup 0)
  // deterministic mode (fe_set_deterministic; RESID and APPLY only): element nodal forces go to
  // elf [24][n_el] (corner-major, corner = i + 2 j + 4 k, then component) instead of being summed
  // with atomics; the stress integral goes to per-workgroup partials stress_part [grid][6]
  void* elf;
  double* stress_part;
};

template <typename T> struct Buf { T* p = nullptr; };

}  // namespace fe

struct fe_problem {
  int n = 0;
  int prec = FE_F64;
  int64_t n_el = 0, n_nodes = 0, n_dof = 0, nnz = 0;
  double h = 0;
  int device = 0;
  fe::Phases mat{};
  int model_set = fe::MS_LINEAR;
  bool materials_set = false;
  uint8_t* phase = nullptr;   // [n_el]
  void* scale = nullptr;      // real [n_el] or null
  uint8_t* mask = nullptr;    // [n_dof] or null
  void* tangent = nullptr;    // J2 compact tangent [6][8][n_el]
  bool lin_valid = false;
  // solver workspace
  void* w_r = nullptr;
  void* w_p = nullptr;
  void* w_q = nullptr;
  void* w_d = nullptr;        // inverse diagonal
  int precond = FE_PC_JACOBI; // FE_PC_JACOBI or FE_PC_BLOCK_JACOBI
  void* w_blk = nullptr;      // inverse node blocks [n_nodes][6] (allocated on first use)
  int csr_nodal = 0;          // solver in progress: the CSR matrix given has the node-triple structure
  int* nodal_flag = nullptr;  // device flag of the structure check
  void* w_ilu = nullptr;      // ILU(0) factors [27][9][n_nodes] (allocated by fe_set_preconditioner)
  void* w_ipcg = nullptr;     // CG with ILU(0): r, p, q, z [n_dof] each
  fe::IpcgCtrl* ipcg = nullptr;
  void* w_gm = nullptr;       // GMRES: basis [gm_cap + 1][n_dof], then w and z [n_dof] each
  int gm_cap = 0;             // restart length w_gm was sized for
  fe::GmresDev* gm_dev = nullptr; // GMRES scalars (device)
  double* gm_part = nullptr;  // [GM_MAXM + 1][GM_GRID] partial sums
  void* w_cg = nullptr;       // single-reduction CG vectors r_1, s_0, s_1, w_0, w_1, w_2 (allocated on first use)
  void* w_bicg = nullptr;     // BiCGStab vectors r, r_hat, p, v, s, t, p_hat, s_hat (allocated on first use)
  double* bicg_part = nullptr;  // BiCGStab partial sums [8][BICG_GRID]
  fe::BicgCtrl* bicg_ctrl = nullptr;
  void* w_v = nullptr;        // scratch vector (Newton)
  void* w_v2 = nullptr;       // scratch vector (Newton)
  void* w_uprev = nullptr;    // Newton with the extrapolating predictor: the converged u two steps back
  int deterministic = 0;      // fe_set_deterministic: fixed summation orders, no floating-point atomics
  int acc32 = 0;              // fe_set_fp32_accumulation: FP32 problems sum element forces in FP32
  void* w_elf = nullptr;      // deterministic mode: element nodal forces [24][n_el]
  double* stress_part = nullptr;  // deterministic mode: per-workgroup stress partials [elem grid][6]
  void* w_state = nullptr;    // J2 trial state (Newton)
  double* partials = nullptr; // block partial sums (double)
  unsigned int* counter = nullptr;
  fe::CgCtrl* ctrl = nullptr;
  double* stress_sum = nullptr;
  int* flags = nullptr;
  int32_t* csr_rp = nullptr;  // Newton's own CSR (matrix-explicit path)
  int32_t* csr_ci = nullptr;
  void* csr_v = nullptr;
  fe::CgCtrl* host_ctrl = nullptr;  // pinned
  double* host_buf = nullptr;       // pinned scratch
  // learned surrogate (fe_set_surrogate) and sample capture (fe_set_capture)
  int64_t n_j2_el = 0;              // elements of J2 phases
  int64_t n_nh_el = 0;              // elements of Neo-Hookean phases
  const float* sur_W = nullptr;     // network parameters (caller-owned)
  double sur_tol = 0;
  int sur_full = 0;                 // fe_set_surrogate_tangent
  int64_t sur_cap = 0;
  int* sur_map = nullptr;
  float* sur_x = nullptr;
  float* sur_y = nullptr;
  float* sur_jac = nullptr;
  void* sur_D = nullptr;
  unsigned int* sur_count = nullptr;   // [0] list length, [1] accepted, [2] fallback
  float* cap_x = nullptr;              // capture: caller buffers
  float* cap_y = nullptr;
  int64_t cap_n = 0;
  unsigned int* cap_count = nullptr;
  unsigned int cap_stride = 1, cap_salt = 0;
  // kernel timing (fe_profile): event pairs around selected launches
  bool prof = false;
  int prof_stride = 1;  // inside CG: time operator launches 0, k, 2k, ... of each solve
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, size_t>> prof_recs;  // (kernel class, index of the start event)
  size_t ev_used = 0;
  double prof_bytes[5] = {0, 0, 0, 0, 0};         // algorithmic bytes of the recorded launches
  // general hex8 mesh (fe_problem_create_hex8; n = 0 there)
  bool general = false;
  double volume = 1.0;             // sum over Gauss points of w detJ (the unit cube: 1)
  void* coords = nullptr;          // real [3][n_nodes]
  int32_t* conn = nullptr;         // [8][n_el]
  int64_t n_pairs = 0;             // node pairs that share an element (nnz = 9 n_pairs)
  int32_t* adj_ptr = nullptr;      // [n_nodes + 1] first pair of each row node
  int32_t* adj = nullptr;          // [n_pairs] column node of each pair, ascending within a row
  int32_t* pair_row = nullptr;     // [n_pairs] row node of each pair
  int32_t* pair_src_ptr = nullptr; // [n_pairs + 1] run of each pair in pair_src
  int32_t* pair_src = nullptr;     // [64 n_el] element codes e*64 + a*8 + b sorted by (row, column, code)
  int32_t* gen_col = nullptr;      // [64 n_el] sorted column nodes (work array of the symbolic step)
  void* ke = nullptr;              // element Jacobians [n_el][576] (allocated on the first tangent)
};

namespace fe {

size_t real_size(const fe_problem* p);
void set_error(const std::string& msg);
int hip_fail(hipError_t e, const char* what);

// Kernel timing: when armed, the next timed launch records `start` and `stop` inside its own
// dispatch (hipExtLaunchKernelGGL), so the interval is the kernel alone, without separate
// marker packets on the stream.  One per host thread.
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
  bool armed = false, used = false;
};
LaunchEvents& launch_events();

template <typename F, typename... Args>
inline void timed_launch(F kernel, dim3 grid, dim3 block, uint32_t shmem, hipStream_t s, Args... args) {
  LaunchEvents& ev = launch_events();
  if (ev.armed && !ev.used) {
    ev.used = true;
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, ev.start, ev.stop, 0u, args...);
  } else {
    hipLaunchKernelGGL(kernel, grid, block, shmem, s, args...);
  }
}

// kernel launchers (fe_kernels.hip); each returns hipError_t of the launch
hipError_t launch_elem(const fe_problem* p, int op, const ElemArgs& a, hipStream_t s);
hipError_t launch_diag(const fe_problem* p, void* d, int apply_bc, hipStream_t s);
hipError_t launch_csr_pattern(const fe_problem* p, int32_t* row_ptr, int32_t* col_idx, hipStream_t s);
hipError_t launch_tangent_csr(const fe_problem* p, void* vals, int apply_bc, hipStream_t s);
hipError_t launch_spmv(const fe_problem* p, const int32_t* rp, const int32_t* ci, const void* v,
                       const void* x, void* y, hipStream_t s);
hipError_t launch_fill(const fe_problem* p, void* x, int64_t n, double v, hipStream_t s);
hipError_t launch_spmv_nodal(const fe_problem* p, const int32_t* rp, const int32_t* ci, const void* v, const void* x,
                             void* y, hipStream_t s);
hipError_t launch_lift(const fe_problem* p, const double* eps, void* u, int zero_free, hipStream_t s);
hipError_t launch_axpby(const fe_problem* p, int64_t n, double a, const void* x, double b, void* y,
                        hipStream_t s);
hipError_t launch_mask_zero(const fe_problem* p, void* x, hipStream_t s);
hipError_t launch_dot(const fe_problem* p, const void* a, const void* b, int64_t n, double* out,
                      hipStream_t s);
hipError_t launch_csr_diag(const fe_problem* p, const int32_t* rp, const int32_t* ci, const void* v, void* d,
                           hipStream_t s);
hipError_t launch_copy_cvt(const fe_problem* p, const void* src, void* dst, int64_t n, hipStream_t s);
// inverse node blocks of the CSR matrix (rp != null) or of the matrix-free operator, Dirichlet-eliminated
hipError_t launch_block_jacobi(const fe_problem* p, const int32_t* rp, const int32_t* ci, const void* v, void* blk,
                               hipStream_t s);
// buffer the CG kernels read M^-1 from
inline void* pc_buffer(const fe_problem* p) { return p->precond == FE_PC_BLOCK_JACOBI ? p->w_blk : p->w_d; }

hipError_t launch_lin_stats(const fe_problem* p, unsigned long long* out, hipStream_t s);
// element / CSR operator launches that return at once while *stop is set (BiCGStab)
hipError_t launch_elem_stop(const fe_problem* p, int op, const ElemArgs& a, const int* stop, hipStream_t s);
// *flag <- 1 unless rows 3a, 3a+1, 3a+2 of every node share one column list (the flag is
// cleared by the caller); with it, solvers use the node-structured mat-vec
hipError_t launch_csr_nodal_check(const fe_problem* p, const int32_t* rp, const int32_t* ci, int* flag,
                                  hipStream_t s);
// solver mat-vec: node-structured when p->csr_nodal, else one row per LPR lanes
hipError_t launch_spmv_stop(const fe_problem* p, const int32_t* rp, const int32_t* ci, const void* v,
                            const void* x, void* y, const int* stop, hipStream_t s);
// BiCGStab pieces (see the kernels): init, then per iteration
//   bicg_dir, A p_hat -> v, bicg_half, A s_hat -> t, bicg_dots, bicg_update
hipError_t bicg_init(const fe_problem* p, const void* b, void* x, double rtol, int max_it, hipStream_t s);
hipError_t bicg_step(const fe_problem* p, int stage, void* x, hipStream_t s);
// path adjoint through the return map (FP64 problems): see fe_vjp_path
hipError_t launch_path_vjp(const fe_problem* p, const void* u, const void* hist, const void* c, const void* mu_in,
                           void* mu_out, void* u_bar, void* s_bar, hipStream_t s);
// network forward + Jacobian over a device-counted list (blocks beyond *count return)
hipError_t launch_mlp_forward_counted(const float* W, const float* x, float* y, float* jac, int64_t cap,
                                      const unsigned int* count, hipStream_t s);

// CSR CG pieces: one iteration = cg_pre (direction), cg_operator (q = A p, p.Ap partials),
// cg_vectors (scalars and updates)
hipError_t cg_init(const fe_problem* p, const void* b, void* x, double rtol, int max_it, hipStream_t s);
hipError_t cg_operator(const fe_problem* p, int op, const int32_t* rp, const int32_t* ci, const void* vals, long k,
                       hipStream_t s);
hipError_t cg_vectors(const fe_problem* p, int op, void* x, long k, hipStream_t s);
hipError_t cg_pre(const fe_problem* p, int op, long k, hipStream_t s);  // CSR: direction kernel before the mat-vec
// restarted GMRES pieces (fe_krylov.hip): setup (x = 0, w = b, preconditioner inverted),
// then per cycle GM_START, per Arnoldi step j GM_BASIS + operator (z -> w) + GM_ORTHO,
// GM_FINISH at the cycle end, and A x -> w + GM_RESIDUAL before the next cycle
hipError_t gm_setup(const fe_problem* p, const void* b, void* x, double rtol, int max_it, int m, hipStream_t s);
hipError_t gm_step(const fe_problem* p, int stage, int j, const void* b, void* x, hipStream_t s);
void* gm_work_w(const fe_problem* p);
void* gm_work_z(const fe_problem* p);
// z = M^-1 r with the point (diagonal in w_d, not inverted) or node-block (inverted
// blocks in w_blk) preconditioner as set up last (fe_krylov.hip)
hipError_t pc_apply(const fe_problem* p, const void* r, void* z, hipStream_t s);
// CG with ILU(0) (fe_krylov.hip): one stage per call (IpcgStage); k = iteration index;
// vector v of the workspace: 0 r, 1 p, 2 q, 3 z
hipError_t ipcg_step(const fe_problem* p, int stage, long k, const void* b, void* x, double rtol, int max_it,
                     hipStream_t s);
void* ipcg_vec(const fe_problem* p, int v);
// node-block ILU(0) in 8-colour order (fe_ilu.hip): factor from the CSR matrix, apply
// z = (L U)^-1 r (r may equal z; 16 launches, which return at once when *stop is set)
size_t ilu_words(const fe_problem* p);
hipError_t ilu_setup(const fe_problem* p, const int32_t* rp, const int32_t* ci, const void* v, hipStream_t s);
hipError_t ilu_apply(const fe_problem* p, const void* r, void* z, const int* stop, hipStream_t s);
// matrix-free single-reduction CG: init, then one fused operator launch j = 0, 1, ... per
// iteration (its last workgroup computes the scalars of the next launch)
hipError_t cgs_init(const fe_problem* p, const void* b, void* x, double rtol, int max_it, hipStream_t s);
hipError_t cgs_operator(const fe_problem* p, void* x, long j, hipStream_t s);
int elem_grid_size(int n);  // workgroups of an element-kernel launch (also the partial-sum slots it needs)

// general hex8 meshes (fe_general.hip); TanArgs is defined in fe_device.hpp
struct TanArgs;
hipError_t gen_setup(fe_problem* p, const double* coords, const int32_t* conn, hipStream_t s);
hipError_t gen_check_geometry(const fe_problem* p, double* vol_dev, int* bad, hipStream_t s);
hipError_t gen_symbolic(fe_problem* p, int32_t* cnt, int32_t* coo_ptr, int32_t* cursor, int32_t* tmp, hipStream_t s,
                        int64_t* n_pairs, int* max_row);
int64_t gen_scan_tmp_words(int64_t n);
hipError_t gen_pairs(fe_problem* p, const int32_t* coo_ptr, hipStream_t s);
hipError_t gen_csr_pattern(const fe_problem* p, int32_t* row_ptr, int32_t* col_idx, hipStream_t s);
hipError_t gen_launch_elem(const fe_problem* p, int op, const ElemArgs& a, const int* stop, hipStream_t s);
hipError_t gen_cg_operator(const fe_problem* p, hipStream_t s);
hipError_t gen_diag(const fe_problem* p, void* d, int nb, int apply_bc, const TanArgs& ta, hipStream_t s);
hipError_t gen_tangent(const fe_problem* p, void* vals, int apply_bc, const TanArgs& ta, hipStream_t s);
hipError_t gen_lift(const fe_problem* p, const double* E, void* u, int zero_free, hipStream_t s);
hipError_t gen_copy_state(const fe_problem* p, const void* src, void* dst, int64_t n, hipStream_t s);
// deterministic mode, structured problems: sum per-element nodal values (elf [24][n_el]) into y
// in fixed element order; mode 0 residual (constrained dofs 0 when apply_bc), 1 operator
// (constrained dofs y = x when apply_bc), 2 diagonal (constrained dofs 1 when apply_bc); with
// pa, per-workgroup partials of x.y (GEN_CG_GRID workgroups) for CG
hipError_t det_gather(const fe_problem* p, const void* elf, int mode, int apply_bc, const void* x, void* y,
                      const int* stop, double* pa, hipStream_t s);
hipError_t det_stress_reduce(const fe_problem* p, hipStream_t s);
// partial-sum slots of a CG operator launch; the update partials (2 * CG_UGRID) follow them
inline int64_t cg_pa_size(const fe_problem* p) { return std::max<int64_t>(elem_grid_size(p->n), SPMV_MAXGRID); }

}  // namespace fe
