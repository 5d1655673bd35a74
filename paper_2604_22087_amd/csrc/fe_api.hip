// Host side of libfe: the extern "C" entry points declared in include/fe.h.
// Argument checks happen before anything is enqueued; HIP failures become
// FE_ERR_HIP with the runtime's message kept in a thread-local string.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "fe_internal.hpp"

namespace fe {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? FE_ERR_OOM : FE_ERR_HIP;
}

size_t real_size(const fe_problem* p) { return p->prec == FE_F64 ? sizeof(double) : sizeof(float); }

static int arg_error(const char* msg) {
  set_error(msg);
  return FE_ERR_ARG;
}

}  // namespace fe

using namespace fe;

#define HIPCHK(x)                                  \
  do {                                             \
    hipError_t _e = (x);                           \
    if (_e != hipSuccess) return hip_fail(_e, #x); \
  } while (0)

#define CHKP(p)                                           \
  do {                                                    \
    if (!(p)) return arg_error("null problem handle");    \
  } while (0)

static hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }

static int alloc(void** ptr, size_t bytes) {
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    *ptr = nullptr;
    return hip_fail(e, "hipMalloc");
  }
  return FE_OK;
}

static void free_dev(void* p) {
  if (p) (void)hipFree(p);
}

// Kernel timing: an event pair recorded by the timed launch itself (see timed_launch).
static int prof_begin(fe_problem* p, hipStream_t s, long* idx) {
  (void)s;
  *idx = -1;
  if (!p->prof) return FE_OK;
  while (p->ev_used + 2 > p->ev_pool.size()) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    p->ev_pool.push_back(e);
  }
  *idx = (long)p->ev_used;
  LaunchEvents& ev = launch_events();
  ev.start = p->ev_pool[*idx];
  ev.stop = p->ev_pool[*idx + 1];
  ev.armed = true;
  ev.used = false;
  return FE_OK;
}

static int prof_end(fe_problem* p, hipStream_t s, long idx, int cls) {
  (void)s;
  if (idx < 0) return FE_OK;
  LaunchEvents& ev = launch_events();
  const bool used = ev.used;
  ev.armed = false;
  ev.used = false;
  if (!used) return FE_OK;  // nothing was launched (the pair stays free)
  p->ev_used += 2;
  p->prof_recs.push_back({cls, (size_t)idx});
  return FE_OK;
}

static int operator_bytes(fe_problem* p, int op, hipStream_t s, double* bytes);

#define PROF(p, s, cls, launch_expr)                    \
  do {                                                  \
    long _pi;                                           \
    if (int _st = prof_begin(p, s, &_pi)) return _st;   \
    const hipError_t _le = (launch_expr);               \
    const int _pe = prof_end(p, s, _pi, cls);           \
    HIPCHK(_le);                                        \
    if (_pe) return _pe;                                \
  } while (0)

extern "C" {

const char* fe_status_string(int status) {
  switch (status) {
    case FE_OK: return "ok";
    case FE_ERR_ARG: return "invalid argument";
    case FE_ERR_HIP: return "HIP runtime error";
    case FE_ERR_OOM: return "out of device memory";
    case FE_ERR_NOT_CONVERGED: return "iteration limit reached";
    case FE_ERR_BREAKDOWN: return "CG breakdown (p.Ap <= 0)";
    case FE_ERR_NONFINITE: return "non-finite value";
    case FE_ERR_INVERTED: return "inverted element (det F <= 0)";
    case FE_ERR_STATE: return "required state missing";
    default: return "unknown status";
  }
}

const char* fe_last_error(void) { return g_last_error.c_str(); }

void fe_problem_destroy(fe_problem* p) {
  if (!p) return;
  free_dev(p->phase);
  free_dev(p->scale);
  free_dev(p->mask);
  free_dev(p->tangent);
  free_dev(p->w_r);
  free_dev(p->w_p);
  free_dev(p->w_q);
  free_dev(p->w_d);
  free_dev(p->w_blk);
  free_dev(p->w_bicg);
  free_dev(p->w_cg);
  free_dev(p->w_gm);
  free_dev(p->w_ilu);
  free_dev(p->w_ipcg);
  free_dev(p->nodal_flag);
  free_dev(p->ipcg);
  free_dev(p->gm_dev);
  free_dev(p->gm_part);
  free_dev(p->bicg_part);
  free_dev(p->bicg_ctrl);
  free_dev(p->w_v);
  free_dev(p->w_v2);
  free_dev(p->w_uprev);
  free_dev(p->w_elf);
  free_dev(p->stress_part);
  free_dev(p->w_state);
  free_dev(p->partials);
  free_dev(p->counter);
  free_dev(p->ctrl);
  free_dev(p->stress_sum);
  free_dev(p->flags);
  free_dev(p->csr_rp);
  free_dev(p->csr_ci);
  free_dev(p->csr_v);
  free_dev(p->sur_map);
  free_dev(p->sur_x);
  free_dev(p->sur_y);
  free_dev(p->sur_jac);
  free_dev(p->sur_D);
  free_dev(p->sur_count);
  free_dev(p->coords);
  free_dev(p->conn);
  free_dev(p->adj_ptr);
  free_dev(p->adj);
  free_dev(p->pair_row);
  free_dev(p->pair_src_ptr);
  free_dev(p->pair_src);
  free_dev(p->gen_col);
  free_dev(p->ke);
  for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
  if (p->host_ctrl) (void)hipHostFree(p->host_ctrl);
  if (p->host_buf) (void)hipHostFree(p->host_buf);
  delete p;
}

// Library memory every problem needs (vectors, partial sums, scalars, flags); destroys p on failure.
static int alloc_common(fe_problem* p) {
  if (hipError_t e0 = hipGetDevice(&p->device)) {
    fe_problem_destroy(p);
    return hip_fail(e0, "hipGetDevice");
  }
  const int n = p->n;
  const size_t rs = real_size(p), vec = rs * p->n_dof;
  int st = FE_OK;
  const size_t n_part =
      std::max<size_t>({(size_t)2 * 1024, (size_t)std::max<int64_t>(elem_grid_size(n), SPMV_MAXGRID) + 2 * CG_UGRID,
                        (size_t)9 * CGS_SLOTS});
  if ((st = alloc((void**)&p->phase, p->n_el)) || (st = alloc(&p->w_r, vec)) || (st = alloc(&p->w_p, vec)) ||
      (st = alloc(&p->w_q, vec)) || (st = alloc(&p->w_d, vec)) ||
      (st = alloc((void**)&p->partials, n_part * sizeof(double))) ||
      (st = alloc((void**)&p->counter, sizeof(unsigned int))) || (st = alloc((void**)&p->ctrl, sizeof(CgCtrl))) ||
      (st = alloc((void**)&p->stress_sum, 8 * sizeof(double))) || (st = alloc((void**)&p->flags, sizeof(int)))) {
    fe_problem_destroy(p);
    return st;
  }
  hipError_t e;
  if ((e = hipMemset(p->phase, 0, p->n_el)) != hipSuccess || (e = hipMemset(p->counter, 0, sizeof(unsigned int))) ||
      (e = hipMemset(p->flags, 0, sizeof(int))) || (e = hipMemset(p->ctrl, 0, sizeof(CgCtrl))) ||
      (e = hipHostMalloc((void**)&p->host_ctrl, sizeof(CgCtrl), hipHostMallocDefault)) ||
      (e = hipHostMalloc((void**)&p->host_buf, 64 * sizeof(double), hipHostMallocDefault))) {
    fe_problem_destroy(p);
    return hip_fail(e, "fe_problem_create");
  }
  // default material: one linear phase with E = 1, nu = 0.3
  p->mat.n = 1;
  p->mat.ph[0] = PhaseConst{FE_LINEAR, 1.0 * 0.3 / (1.3 * 0.4), 1.0 / 2.6, 1.0 / 1.2, 1.0 / 2.6, 0, 0};
  return FE_OK;
}

int fe_problem_create(fe_problem** out, int n, int precision) {
  if (!out) return arg_error("out is null");
  *out = nullptr;
  if (n < 1 || n > 1024) return arg_error("n must be in [1, 1024]");
  if (precision != FE_F64 && precision != FE_F32) return arg_error("precision must be FE_F64 or FE_F32");
  const int64_t np1 = n + 1;
  if (3 * np1 * np1 * np1 >= (int64_t(1) << 31)) return arg_error("too many dofs for 32-bit indexing");
  fe_problem* p = new fe_problem();
  p->n = n;
  p->prec = precision;
  p->n_el = (int64_t)n * n * n;
  p->n_nodes = np1 * np1 * np1;
  p->n_dof = 3 * p->n_nodes;
  const int64_t t = 3 * (int64_t)n + 1;
  p->nnz = 9 * t * t * t;
  p->h = 1.0 / n;
  if (int st = alloc_common(p)) return st;
  *out = p;
  return FE_OK;
}

int fe_problem_create_hex8(fe_problem** out, int64_t n_nodes, int64_t n_el, const double* coords,
                           const int32_t* conn, int precision, void* stream) {
  if (!out) return arg_error("out is null");
  *out = nullptr;
  if (!coords || !conn) return arg_error("coords and conn are required");
  if (n_nodes < 8 || n_el < 1) return arg_error("a mesh needs at least 8 nodes and one element");
  if (precision != FE_F64 && precision != FE_F32) return arg_error("precision must be FE_F64 or FE_F32");
  if (3 * n_nodes >= (int64_t(1) << 31)) return arg_error("too many dofs for 32-bit indexing");
  if (64 * n_el >= (int64_t(1) << 31)) return arg_error("too many elements for 32-bit element-pair codes");
  hipStream_t s = S(stream);
  fe_problem* p = new fe_problem();
  p->general = true;
  p->n = 0;
  p->prec = precision;
  p->n_el = n_el;
  p->n_nodes = n_nodes;
  p->n_dof = 3 * n_nodes;
  p->h = 0.0;
  if (int st = alloc_common(p)) return st;
  const size_t rs = real_size(p);
  int32_t *cnt = nullptr, *coo_ptr = nullptr, *cursor = nullptr, *tmp = nullptr;
  auto fail = [&](int st) {
    free_dev(cnt);
    free_dev(coo_ptr);
    free_dev(cursor);
    free_dev(tmp);
    fe_problem_destroy(p);
    return st;
  };
  const int64_t tmp_words = gen_scan_tmp_words(n_nodes);
  int st;
  if ((st = alloc(&p->coords, rs * 3 * n_nodes)) || (st = alloc((void**)&p->conn, sizeof(int32_t) * 8 * n_el)) ||
      (st = alloc((void**)&p->adj_ptr, sizeof(int32_t) * (n_nodes + 1))) ||
      (st = alloc((void**)&p->pair_src, sizeof(int32_t) * 64 * n_el)) ||
      (st = alloc((void**)&p->gen_col, sizeof(int32_t) * 64 * n_el)) ||
      (st = alloc((void**)&cnt, sizeof(int32_t) * n_nodes)) ||
      (st = alloc((void**)&coo_ptr, sizeof(int32_t) * (n_nodes + 1))) ||
      (st = alloc((void**)&cursor, sizeof(int32_t) * n_nodes)) ||
      (st = alloc((void**)&tmp, sizeof(int32_t) * tmp_words)))
    return fail(st);
  hipError_t e;
  int bad = 0;
  // copies, node ids in range
  if ((e = gen_setup(p, coords, conn, s)) != hipSuccess ||
      (e = hipMemcpyAsync(&bad, p->flags, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return fail(hip_fail(e, "fe_problem_create_hex8"));
  if (bad) {
    fail(FE_OK);
    return arg_error("connectivity holds a node id outside [0, n_nodes)");
  }
  // every Gauss point of every element must have det J > 0 (right-handed, not degenerate)
  double vol = 0;
  if ((e = hipMemsetAsync(p->stress_sum, 0, sizeof(double), s)) != hipSuccess ||
      (e = gen_check_geometry(p, p->stress_sum, p->flags, s)) != hipSuccess ||
      (e = hipMemcpyAsync(&vol, p->stress_sum, sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipMemcpyAsync(&bad, p->flags, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipMemsetAsync(p->flags, 0, sizeof(int), s)) != hipSuccess || (e = hipStreamSynchronize(s)) != hipSuccess)
    return fail(hip_fail(e, "fe_problem_create_hex8"));
  if (bad) {
    fail(FE_OK);
    return arg_error("an element has det J <= 0 at a Gauss point (inverted, degenerate or left-handed node order)");
  }
  p->volume = vol;
  // sorted node-pair pattern
  int64_t n_pairs = 0;
  int max_row = 0;
  if ((e = gen_symbolic(p, cnt, coo_ptr, cursor, tmp, s, &n_pairs, &max_row)) != hipSuccess)
    return fail(hip_fail(e, "fe_problem_create_hex8 (symbolic)"));
  if (max_row > 1024) {
    fail(FE_OK);
    return arg_error("a node is shared by more than 128 elements");
  }
  if (9 * n_pairs >= (int64_t(1) << 31)) {
    fail(FE_OK);
    return arg_error("matrix too large for int32 CSR indices");
  }
  p->n_pairs = n_pairs;
  p->nnz = 9 * n_pairs;
  if ((st = alloc((void**)&p->adj, sizeof(int32_t) * n_pairs)) ||
      (st = alloc((void**)&p->pair_row, sizeof(int32_t) * n_pairs)) ||
      (st = alloc((void**)&p->pair_src_ptr, sizeof(int32_t) * (n_pairs + 1))))
    return fail(st);
  if ((e = gen_pairs(p, coo_ptr, s)) != hipSuccess || (e = hipStreamSynchronize(s)) != hipSuccess)
    return fail(hip_fail(e, "fe_problem_create_hex8 (pairs)"));
  free_dev(cnt);
  free_dev(coo_ptr);
  free_dev(cursor);
  free_dev(tmp);
  free_dev(p->gen_col);
  p->gen_col = nullptr;
  *out = p;
  return FE_OK;
}

int fe_problem_sizes(const fe_problem* p, int64_t* out) {
  CHKP(p);
  if (!out) return arg_error("out is null");
  out[0] = p->n;
  out[1] = p->n_el;
  out[2] = p->n_nodes;
  out[3] = p->n_dof;
  out[4] = 8 * p->n_el;
  out[5] = p->nnz;
  return FE_OK;
}

int fe_set_materials(fe_problem* p, const uint8_t* phase, int n_phases, const int* models, const double* params,
                     const void* scale, void* stream) {
  CHKP(p);
  if (!phase || !models || !params) return arg_error("phase, models and params are required");
  if (n_phases < 1 || n_phases > FE_MAX_PHASES) return arg_error("n_phases out of range");
  Phases m{};
  m.n = n_phases;
  bool j2 = false, nh = false;
  for (int i = 0; i < n_phases; ++i) {
    const double E = params[4 * i], nu = params[4 * i + 1], sy = params[4 * i + 2], H = params[4 * i + 3];
    if (models[i] < FE_LINEAR || models[i] > FE_NEOHOOKE) return arg_error("unknown model");
    if (!(nu > -1.0 && nu < 0.5) || !std::isfinite(E)) return arg_error("invalid E or nu");
    if (models[i] == FE_J2 && !(sy > 0 && H >= 0)) return arg_error("J2 needs sigma_y > 0 and H >= 0");
    PhaseConst c;
    c.model = models[i];
    c.lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    c.mu = E / (2.0 * (1.0 + nu));
    c.K = E / (3.0 * (1.0 - 2.0 * nu));
    c.G = c.mu;
    c.sy = sy;
    c.H = H;
    m.ph[i] = c;
    j2 |= models[i] == FE_J2;
    nh |= models[i] == FE_NEOHOOKE;
  }
  if (j2 && nh) return arg_error("J2 and Neo-Hookean phases cannot be mixed in one problem");
  const size_t rs = real_size(p);
  {  // every phase id must index the table: checked on the host before any kernel reads it
    std::vector<uint8_t> h(p->n_el);
    HIPCHK(hipMemcpyAsync(h.data(), phase, p->n_el, hipMemcpyDeviceToHost, S(stream)));
    HIPCHK(hipStreamSynchronize(S(stream)));
    int64_t n_j2 = 0, n_nh = 0;
    for (uint8_t v : h) {
      if (v >= n_phases) return arg_error("phase id >= n_phases");
      n_j2 += models[v] == FE_J2;
      n_nh += models[v] == FE_NEOHOOKE;
    }
    p->n_j2_el = n_j2;
    p->n_nh_el = n_nh;
  }
  HIPCHK(hipMemcpyAsync(p->phase, phase, p->n_el, hipMemcpyDeviceToDevice, S(stream)));
  if (scale) {
    if (!p->scale) {
      int st = alloc(&p->scale, rs * p->n_el);
      if (st) return st;
    }
    HIPCHK(hipMemcpyAsync(p->scale, scale, rs * p->n_el, hipMemcpyDeviceToDevice, S(stream)));
  } else if (p->scale) {
    free_dev(p->scale);
    p->scale = nullptr;
  }
  const int comps = nh ? 10 : (j2 ? 6 : 0);
  if (comps) {
    free_dev(p->tangent);
    p->tangent = nullptr;
    int st = alloc(&p->tangent, rs * comps * 8 * p->n_el);
    if (st) return st;
  }
  p->mat = m;
  p->model_set = j2 ? MS_J2 : (nh ? MS_NH : MS_LINEAR);
  p->materials_set = true;
  p->lin_valid = !(j2 || nh);
  return FE_OK;
}

int fe_set_dirichlet(fe_problem* p, const uint8_t* mask, void* stream) {
  CHKP(p);
  if (!mask) {
    free_dev(p->mask);
    p->mask = nullptr;
    return FE_OK;
  }
  if (!p->mask) {
    int st = alloc((void**)&p->mask, p->n_dof);
    if (st) return st;
  }
  HIPCHK(hipMemcpyAsync(p->mask, mask, p->n_dof, hipMemcpyDeviceToDevice, S(stream)));
  return FE_OK;
}

int fe_lift(fe_problem* p, const double* eps_bar, void* u, int zero_free, void* stream) {
  CHKP(p);
  if (!eps_bar || !u) return arg_error("eps_bar and u are required");
  HIPCHK(launch_lift(p, eps_bar, u, zero_free, S(stream)));
  return FE_OK;
}

static ElemArgs base_args(const fe_problem* p) {
  ElemArgs a{};
  a.n = p->n;
  a.h = p->h;
  a.n_el = p->n_el;
  a.phase = p->phase;
  a.scale = p->scale;
  a.mask = p->mask;
  a.tangent = p->tangent;
  a.flags = p->flags;
  a.mat = p->mat;
  a.sur_map = p->sur_map;
  a.sur_D = p->sur_D;
  return a;
}

static int residual_impl(fe_problem* p, const void* u, const void* state_in, void* state_out, void* r, int flags,
                         double* stress_sum, hipStream_t s) {
  if (r) HIPCHK(launch_fill(p, r, p->n_dof, 0.0, s));
  ElemArgs a = base_args(p);
  a.x = u;
  a.y = r;
  a.state_in = state_in;
  a.state_out = state_out;
  a.store_tangent = (flags & FE_STORE_TANGENT) ? 1 : 0;
  a.apply_bc = (flags & FE_APPLY_BC) ? 1 : 0;
  a.stress_sum = stress_sum;
  const bool j2 = p->model_set == MS_J2;
  if (j2 && (p->sur_W || p->cap_x)) {
    // normalisation of the network interface by the first J2 phase: strains by sigma_y / E, stress by sigma_y
    for (int i = 0; i < p->mat.n; ++i)
      if (p->mat.ph[i].model == FE_J2) {
        const double E = 9.0 * p->mat.ph[i].K * p->mat.ph[i].G / (3.0 * p->mat.ph[i].K + p->mat.ph[i].G);
        a.sur_sin = (float)(p->mat.ph[i].sy / E);
        a.sur_sout = (float)p->mat.ph[i].sy;
        break;
      }
  }
  if (j2 && p->sur_W) {
    // 1) list the points whose elastic trial is plastic, with their network inputs
    HIPCHK(hipMemsetAsync(p->sur_count, 0, 3 * sizeof(unsigned int), s));
    ElemArgs c = a;
    c.y = nullptr;
    c.state_out = nullptr;
    c.store_tangent = 0;
    c.stress_sum = nullptr;
    c.sur_mode = SUR_CLASSIFY;
    c.sur_map = p->sur_map;
    c.sur_count = p->sur_count;
    c.sur_cap = p->sur_cap;
    c.sur_x = p->sur_x;
    HIPCHK(launch_elem(p, OP_RESID, c, s));
    HIPCHK(hipMemcpyAsync(p->host_buf, p->sur_count, sizeof(unsigned int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const int64_t listed = std::min<int64_t>(*reinterpret_cast<unsigned int*>(p->host_buf), p->sur_cap);
    // 2) network value and Jacobian for the listed points
    if (int st = fe_mlp_forward(p->sur_W, p->sur_x, p->sur_y, p->sur_jac, nullptr, listed, s)) return st;
    // 3) residual with the network's stresses where the local check passes
    a.sur_mode = SUR_CONSUME;
    a.sur_map = p->sur_map;
    a.sur_y = p->sur_y;
    a.sur_jac = p->sur_jac;
    a.sur_D = p->sur_D;
    a.sur_stats = p->sur_count + 1;
    a.sur_tol = p->sur_tol;
    a.sur_full = p->sur_full;
  } else if (j2 && p->cap_x) {
    a.sur_mode = SUR_CAPTURE;
    a.sur_count = p->cap_count;
    a.sur_cap = p->cap_n;
    a.sur_x = p->cap_x;
    a.sur_y = p->cap_y;
    a.sur_stride = p->cap_stride;
    a.sur_salt = p->cap_salt++ * 0x9E3779B9u;
  }
  PROF(p, s, 2, launch_elem(p, OP_RESID, a, s));
  if (a.store_tangent) p->lin_valid = true;
  return FE_OK;
}

int fe_residual(fe_problem* p, const void* u, const void* state_in, void* state_out, void* r, int flags,
                void* stream) {
  CHKP(p);
  if (!u || !r) return arg_error("u and r are required");
  if (state_out && p->model_set != MS_J2) state_out = nullptr;
  return residual_impl(p, u, state_in, state_out, r, flags, nullptr, S(stream));
}

int fe_mean_stress(fe_problem* p, const void* u, const void* state_in, double* sigma, void* stream) {
  CHKP(p);
  if (!u || !sigma) return arg_error("u and sigma are required");
  HIPCHK(hipMemsetAsync(p->stress_sum, 0, 6 * sizeof(double), S(stream)));
  int st = residual_impl(p, u, state_in, nullptr, nullptr, 0, p->stress_sum, S(stream));
  if (st) return st;
  HIPCHK(hipMemcpyAsync(p->host_buf, p->stress_sum, 6 * sizeof(double), hipMemcpyDeviceToHost, S(stream)));
  HIPCHK(hipStreamSynchronize(S(stream)));
  for (int k = 0; k < 6; ++k) sigma[k] = p->host_buf[k] / p->volume;
  return FE_OK;
}

int fe_set_deterministic(fe_problem* p, int on) {
  CHKP(p);
  if (on && p->general) return arg_error("deterministic mode is available on structured problems");
  if (on) {
    if (!p->w_elf && alloc(&p->w_elf, real_size(p) * 24 * (size_t)p->n_el)) return FE_ERR_OOM;
    if (!p->stress_part && alloc((void**)&p->stress_part, sizeof(double) * 6 * (size_t)elem_grid_size(p->n)))
      return FE_ERR_OOM;
  }
  p->deterministic = on ? 1 : 0;
  return FE_OK;
}

int fe_set_fp32_accumulation(fe_problem* p, int on) {
  CHKP(p);
  if (on && p->prec != FE_F32) return arg_error("FP32 accumulation applies to FP32 problems");
  if (on && p->general) return arg_error("FP32 accumulation is available on structured problems");
  p->acc32 = on ? 1 : 0;
  return FE_OK;
}

int fe_commit_state(fe_problem* p, const void* state_trial, void* state, void* stream) {
  CHKP(p);
  if (!state_trial || !state) return arg_error("state_trial and state are required");
  if (p->model_set != MS_J2) return FE_OK;  // only J2 points carry history
  HIPCHK(gen_copy_state(p, state_trial, state, 7 * 8 * p->n_el, S(stream)));
  return FE_OK;
}

int fe_csr_nnz(const fe_problem* p, int64_t* nnz) {
  CHKP(p);
  if (!nnz) return arg_error("nnz is null");
  *nnz = p->nnz;
  return FE_OK;
}

static int check_csr_size(const fe_problem* p) {
  if (p->nnz >= (int64_t(1) << 31)) return arg_error("matrix too large for int32 CSR indices");
  return FE_OK;
}

int fe_csr_indices(fe_problem* p, int32_t* row_ptr, int32_t* col_idx, void* stream) {
  CHKP(p);
  if (!row_ptr || !col_idx) return arg_error("row_ptr and col_idx are required");
  if (int st = check_csr_size(p)) return st;
  HIPCHK(launch_csr_pattern(p, row_ptr, col_idx, S(stream)));
  return FE_OK;
}

// General meshes keep every element's dense Jacobian between the matrix-core kernel and the
// sorted gather into the CSR values: n_el x 576 reals, allocated on the first tangent.
static int ensure_ke(fe_problem* p) {
  if (!p->general || p->ke) return FE_OK;
  return alloc(&p->ke, real_size(p) * 576 * (size_t)p->n_el);
}

int fe_tangent_csr(fe_problem* p, const void* u, const void* state_in, void* vals, int apply_bc, void* stream) {
  CHKP(p);
  if (!u || !vals) return arg_error("u and vals are required");
  if (int st = check_csr_size(p)) return st;
  if (int st = ensure_ke(p)) return st;
  if (p->model_set != MS_LINEAR) {
    int st = residual_impl(p, u, state_in, nullptr, nullptr, FE_STORE_TANGENT, nullptr, S(stream));
    if (st) return st;
  }
  PROF(p, S(stream), 3, launch_tangent_csr(p, vals, apply_bc, S(stream)));
  return FE_OK;
}

int fe_apply_matfree(fe_problem* p, const void* x, void* y, int apply_bc, void* stream) {
  CHKP(p);
  if (!x || !y) return arg_error("x and y are required");
  if (!p->lin_valid) {
    set_error("no linearisation stored: call fe_residual with FE_STORE_TANGENT or fe_tangent_csr first");
    return FE_ERR_STATE;
  }
  HIPCHK(launch_fill(p, y, p->n_dof, 0.0, S(stream)));
  ElemArgs a = base_args(p);
  a.x = x;
  a.y = y;
  a.apply_bc = apply_bc ? 1 : 0;
  PROF(p, S(stream), 0, launch_elem(p, OP_APPLY, a, S(stream)));
  if (p->prof) {
    double b = 0;
    if (int e = operator_bytes(p, FE_OP_MATFREE, S(stream), &b)) return e;
    p->prof_bytes[0] += b;
  }
  return FE_OK;
}

int fe_apply_csr(fe_problem* p, const int32_t* row_ptr, const int32_t* col_idx, const void* vals, const void* x,
                 void* y, void* stream) {
  CHKP(p);
  if (!row_ptr || !col_idx || !vals || !x || !y) return arg_error("all CSR arrays and vectors are required");
  PROF(p, S(stream), 1, launch_spmv(p, row_ptr, col_idx, vals, x, y, S(stream)));
  if (p->prof) {
    double b = 0;
    if (int e = operator_bytes(p, FE_OP_CSR, S(stream), &b)) return e;
    p->prof_bytes[1] += b;
  }
  return FE_OK;
}

int fe_apply_csr_nodal(fe_problem* p, const int32_t* row_ptr, const int32_t* col_idx, const void* vals,
                       const void* x, void* y, void* stream) {
  CHKP(p);
  if (!row_ptr || !col_idx || !vals || !x || !y) return arg_error("all CSR arrays and vectors are required");
  PROF(p, S(stream), 4, launch_spmv_nodal(p, row_ptr, col_idx, vals, x, y, S(stream)));
  if (p->prof) {  // one column list per node triple
    const double w = (double)real_size(p);
    p->prof_bytes[4] += (w + 4.0 / 3.0) * (double)p->nnz + 4.0 * (double)(p->n_dof + 1) + 2.0 * w * (double)p->n_dof;
  }
  return FE_OK;
}

int fe_diagonal(fe_problem* p, void* d, int apply_bc, void* stream) {
  CHKP(p);
  if (!d) return arg_error("d is required");
  if (!p->lin_valid) {
    set_error("no linearisation stored");
    return FE_ERR_STATE;
  }
  HIPCHK(launch_diag(p, d, apply_bc, S(stream)));
  return FE_OK;
}

int fe_set_surrogate_tangent(fe_problem* p, int full) {
  CHKP(p);
  if (full != 0 && full != 1) return arg_error("full must be 0 or 1");
  p->sur_full = full;
  return FE_OK;
}

int fe_set_preconditioner(fe_problem* p, int kind) {
  CHKP(p);
  if (kind != FE_PC_JACOBI && kind != FE_PC_BLOCK_JACOBI && kind != FE_PC_ILU0)
    return arg_error("kind must be FE_PC_JACOBI, FE_PC_BLOCK_JACOBI or FE_PC_ILU0");
  if (kind == FE_PC_ILU0 && p->general)
    return arg_error("FE_PC_ILU0 orders nodes by the parities of structured grid indices: not on a general mesh");
  if (kind == FE_PC_BLOCK_JACOBI && !p->w_blk) {
    if (int st = alloc(&p->w_blk, 6 * real_size(p) * (size_t)p->n_nodes)) return st;
  }
  if (kind == FE_PC_ILU0 && !p->w_ilu) {
    if (int st = alloc(&p->w_ilu, ilu_words(p) * real_size(p))) return st;
  }
  p->precond = kind;
  return FE_OK;
}

}  // extern "C"

// CG driver: kernels run with device-side scalars; the host checks the status
// word every `chunk` iterations (iterations after convergence are no-ops).
// The Jacobi diagonal comes from the CSR matrix when one is given (rp != null),
// else from the element kernel; `op` selects the operator inside the iteration.
// Solvers on a CSR operator use the node-structured mat-vec when rows 3a..3a+2 of the
// matrix share their column list (always so for fe_csr_indices' pattern); one check per solve.
static int detect_csr_structure(fe_problem* p, int op, const int32_t* rp, const int32_t* ci, hipStream_t s) {
  p->csr_nodal = 0;
  if (op != FE_OP_CSR || !rp) return FE_OK;
  if (!p->nodal_flag && alloc((void**)&p->nodal_flag, sizeof(int))) return FE_ERR_OOM;
  HIPCHK(hipMemsetAsync(p->nodal_flag, 0, sizeof(int), s));
  HIPCHK(launch_csr_nodal_check(p, rp, ci, p->nodal_flag, s));
  int* h = reinterpret_cast<int*>(p->host_buf);
  HIPCHK(hipMemcpyAsync(h, p->nodal_flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  p->csr_nodal = *h == 0 ? 1 : 0;
  return FE_OK;
}

// CG with the ILU(0) preconditioner (applied by its own sweeps, so not fused into the
// operator launch): per iteration q = A p, step, test, z = (L U)^-1 r, new direction.
static int ipcg_run(fe_problem* p, int op, const int32_t* rp, const int32_t* ci, const void* vals, const void* b,
                    void* x, double rtol, int max_it, fe_pcg_info* info, hipStream_t s, int* applies) {
  if (!rp) return arg_error("FE_PC_ILU0 needs the assembled CSR matrix");
  if (int e = detect_csr_structure(p, op, rp, ci, s)) return e;
  if (!p->w_ipcg && alloc(&p->w_ipcg, 4 * real_size(p) * (size_t)p->n_dof)) return FE_ERR_OOM;
  if (!p->ipcg && alloc((void**)&p->ipcg, sizeof(IpcgCtrl))) return FE_ERR_OOM;
  if (!p->gm_part && alloc((void**)&p->gm_part, (size_t)(GM_MAXM + 1) * GM_GRID * sizeof(double)))
    return FE_ERR_OOM;
  HIPCHK(ilu_setup(p, rp, ci, vals, s));
  const int* stop = &p->ipcg->status;
  void* r = ipcg_vec(p, 0);
  void* pv = ipcg_vec(p, 1);
  void* q = ipcg_vec(p, 2);
  void* z = ipcg_vec(p, 3);
  auto apply = [&]() -> hipError_t {
    if (op == FE_OP_CSR) return launch_spmv_stop(p, rp, ci, vals, pv, q, stop, s);
    ElemArgs a = base_args(p);
    a.x = pv;
    a.y = q;
    a.apply_bc = 1;
    return launch_elem_stop(p, OP_APPLY, a, stop, s);
  };
  HIPCHK(ipcg_step(p, IPCG_INIT, 0, b, x, rtol, max_it, s));
  HIPCHK(ipcg_step(p, IPCG_CHECK_FIRST, 0, b, x, rtol, max_it, s));
  HIPCHK(ilu_apply(p, r, z, stop, s));
  HIPCHK(ipcg_step(p, IPCG_FIRST_DIRECTION, 0, b, x, rtol, max_it, s));
  IpcgCtrl* hc = reinterpret_cast<IpcgCtrl*>(p->host_buf);
  static_assert(sizeof(IpcgCtrl) <= 64 * sizeof(double), "host scratch too small");
  int launched = 0, chunk = 4;
  long k = 0;
  for (;;) {
    HIPCHK(hipMemcpyAsync(hc, p->ipcg, sizeof(IpcgCtrl), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hc->status != CG_RUNNING || launched > max_it + 16) break;
    for (int c = 0; c < chunk; ++c, ++k) {
      HIPCHK(apply());
      HIPCHK(ipcg_step(p, IPCG_UPDATE, k, b, x, rtol, max_it, s));
      HIPCHK(ipcg_step(p, IPCG_CHECK, k, b, x, rtol, max_it, s));
      HIPCHK(ilu_apply(p, r, z, stop, s));
      HIPCHK(ipcg_step(p, IPCG_DIRECTION, k + 1, b, x, rtol, max_it, s));
    }
    launched += chunk;
    if (chunk < 16) chunk *= 2;
  }
  const int status = hc->status == CG_RUNNING ? FE_ERR_NOT_CONVERGED
                     : (hc->status == CG_CONVERGED ? FE_OK : hc->status);
  if (info) {
    info->iterations = hc->iters;
    info->status = status;
    info->bnorm = std::sqrt(hc->bb);
    info->relres = hc->bb > 0 ? std::sqrt(hc->rr / hc->bb) : 0.0;
  }
  if (applies) *applies += hc->iters + (status == FE_ERR_BREAKDOWN || status == FE_ERR_NONFINITE ? 1 : 0);
  if (status != FE_OK) set_error(fe_status_string(status));
  return status;
}

static int pcg_run(fe_problem* p, int op, const int32_t* rp, const int32_t* ci, const void* vals, const void* b,
                   void* x, double rtol, int max_it, fe_pcg_info* info, hipStream_t s, int* applies) {
  if (p->precond == FE_PC_ILU0) return ipcg_run(p, op, rp, ci, vals, b, x, rtol, max_it, info, s, applies);
  if (int e = detect_csr_structure(p, op, rp, ci, s)) return e;
  if (p->precond == FE_PC_BLOCK_JACOBI) {
    HIPCHK(launch_block_jacobi(p, rp, ci, vals, p->w_blk, s));
  } else if (rp) {
    HIPCHK(launch_csr_diag(p, rp, ci, vals, p->w_d, s));
  } else {
    HIPCHK(launch_diag(p, p->w_d, 1, s));
  }
  const bool fused = op == FE_OP_MATFREE && !p->general && !p->deterministic;
  if (fused) {
    if (!p->w_cg && alloc(&p->w_cg, 6 * real_size(p) * (size_t)p->n_dof)) return FE_ERR_OOM;
    HIPCHK(cgs_init(p, b, x, rtol, max_it, s));
  } else {
    HIPCHK(cg_init(p, b, x, rtol, max_it, s));
  }
  const size_t rec0 = p->prof_recs.size();
  const int cls = op == FE_OP_CSR ? 1 : 0;
  const long stride = p->prof ? p->prof_stride : 1;
  long n_op = 0;  // operator launches of this solve; every stride-th one is timed
#define CG_OPERATOR(expr)                \
  do {                                   \
    if (n_op++ % stride == 0)            \
      PROF(p, s, cls, expr);             \
    else                                 \
      HIPCHK(expr);                      \
  } while (0)
  int launched = 0, chunk = 8;
  long k = 0;
  if (fused) CG_OPERATOR(cgs_operator(p, x, 0, s));
  for (;;) {
    for (int c = 0; c < chunk; ++c, ++k) {
      if (fused) {
        CG_OPERATOR(cgs_operator(p, x, k + 1, s));
        continue;
      }
      HIPCHK(cg_pre(p, op, k, s));
      CG_OPERATOR(cg_operator(p, op, rp, ci, vals, k, s));
      HIPCHK(cg_vectors(p, op, x, k, s));
    }
    launched += chunk;
    HIPCHK(hipMemcpyAsync(p->host_ctrl, p->ctrl, sizeof(CgCtrl), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (p->host_ctrl->status != CG_RUNNING || launched > max_it + 64) break;
    if (chunk < 32) chunk *= 2;
  }
  const CgCtrl& c = *p->host_ctrl;
  const int status = c.status == CG_RUNNING ? FE_ERR_NOT_CONVERGED : (c.status == CG_CONVERGED ? FE_OK : c.status);
  // operator launches after the stopping iteration returned at once: drop their timings
  // (the fused form runs one launch more than iterations: launch j forms u_j = M^-1 r_j)
  const size_t executed = (size_t)c.iters + (fused ? 1 : 0) +
                          (!fused && (status == FE_ERR_BREAKDOWN || status == FE_ERR_NONFINITE) ? 1 : 0);
#undef CG_OPERATOR
  if (p->prof) {  // timed launches among the executed ones: 0, stride, 2 stride, ...
    const size_t kept = (executed + (size_t)stride - 1) / (size_t)stride;
    if (p->prof_recs.size() > rec0 + kept) p->prof_recs.resize(rec0 + kept);
    const size_t timed = p->prof_recs.size() - rec0;
    double b = 0;
    if (int e = operator_bytes(p, op, s, &b)) return e;
    // the fused matrix-free CG launch reads r, w, s, p, x and M^-1 (1 or 2 reals per dof)
    // and writes r, s, p, x and the zeroed w instead of reading x
    if (fused) b += (p->precond == FE_PC_BLOCK_JACOBI ? 11.0 : 10.0) * (double)real_size(p) * (double)p->n_dof;
    p->prof_bytes[cls] += b * (double)timed;
  }
  if (info) {
    info->iterations = c.iters;
    info->status = status;
    info->bnorm = std::sqrt(c.bb);
    info->relres = c.bb > 0 ? std::sqrt(c.rr / c.bb) : 0.0;
  }
  if (applies) *applies += (int)executed;
  if (status != FE_OK) set_error(fe_status_string(status));
  return status;
}

// Preconditioned BiCGStab driver (same preconditioner set-up and polling as pcg_run).
static int bicg_run(fe_problem* p, int op, const int32_t* rp, const int32_t* ci, const void* vals, const void* b,
                    void* x, double rtol, int max_it, fe_pcg_info* info, hipStream_t s, int* applies) {
  if (int e = detect_csr_structure(p, op, rp, ci, s)) return e;
  const bool ilu = p->precond == FE_PC_ILU0;
  if (ilu && !rp) return arg_error("FE_PC_ILU0 needs the assembled CSR matrix");
  const size_t rs = real_size(p);
  if (!p->w_bicg && alloc(&p->w_bicg, 8 * rs * (size_t)p->n_dof)) return FE_ERR_OOM;
  if (!p->bicg_part && alloc((void**)&p->bicg_part, 6 * BICG_GRID * sizeof(double))) return FE_ERR_OOM;
  if (!p->bicg_ctrl && alloc((void**)&p->bicg_ctrl, sizeof(BicgCtrl))) return FE_ERR_OOM;
  if (ilu) {
    HIPCHK(ilu_setup(p, rp, ci, vals, s));
  } else if (p->precond == FE_PC_BLOCK_JACOBI) {
    HIPCHK(launch_block_jacobi(p, rp, ci, vals, p->w_blk, s));
  } else if (rp) {
    HIPCHK(launch_csr_diag(p, rp, ci, vals, p->w_d, s));
  } else {
    HIPCHK(launch_diag(p, p->w_d, 1, s));
  }
  HIPCHK(bicg_init(p, b, x, rtol, max_it, s));
  const int* stop = &p->bicg_ctrl->status;
  char* base = static_cast<char*>(p->w_bicg);
  void* v = base + 3 * rs * p->n_dof;
  void* t = base + 5 * rs * p->n_dof;
  void* ph = base + 6 * rs * p->n_dof;
  void* sh = base + 7 * rs * p->n_dof;
  auto apply = [&](const void* in, void* out) -> hipError_t {
    if (op == FE_OP_CSR) return launch_spmv_stop(p, rp, ci, vals, in, out, stop, s);
    ElemArgs a = base_args(p);
    a.x = in;
    a.y = out;
    a.apply_bc = 1;
    return launch_elem_stop(p, OP_APPLY, a, stop, s);
  };
  BicgCtrl* hc = reinterpret_cast<BicgCtrl*>(p->host_buf);
  static_assert(sizeof(BicgCtrl) <= 64 * sizeof(double), "host scratch too small");
  int launched = 0, chunk = 4;
  for (;;) {
    for (int c = 0; c < chunk; ++c) {
      HIPCHK(bicg_step(p, 0, x, s));  // direction
      if (ilu) HIPCHK(ilu_apply(p, ph, ph, stop, s));
      HIPCHK(apply(ph, v));
      HIPCHK(bicg_step(p, 4, x, s));  // (r_hat, v)
      HIPCHK(bicg_step(p, 1, x, s));  // half step
      if (ilu) HIPCHK(ilu_apply(p, sh, sh, stop, s));
      HIPCHK(apply(sh, t));
      HIPCHK(bicg_step(p, 2, x, s));  // (t, s), (t, t)
      HIPCHK(bicg_step(p, 3, x, s));  // update
    }
    launched += chunk;
    HIPCHK(hipMemcpyAsync(hc, p->bicg_ctrl, sizeof(BicgCtrl), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hc->status != CG_RUNNING || hc->finish || launched > max_it + 16) break;
    if (chunk < 16) chunk *= 2;
  }
  const int status = hc->finish ? FE_OK
                     : (hc->status == CG_RUNNING ? FE_ERR_NOT_CONVERGED
                                                 : (hc->status == CG_CONVERGED ? FE_OK : hc->status));
  if (info) {
    info->iterations = hc->iters;
    info->status = status;
    info->bnorm = std::sqrt(hc->bb);
    info->relres = hc->bb > 0 ? std::sqrt(hc->rr / hc->bb) : 0.0;
  }
  if (applies) *applies += 2 * hc->iters;
  if (status != FE_OK) set_error(fe_status_string(status));
  return status;
}

// Restarted GMRES(m) driver: the host enqueues Arnoldi steps in chunks and polls the
// device status between chunks; a cycle ends after m steps or at a stop, then
// x += M^-1 V y runs and, unless stopped, the next cycle starts from b - A x.
static int gmres_run(fe_problem* p, int op, const int32_t* rp, const int32_t* ci, const void* vals, const void* b,
                     void* x, double rtol, int max_it, int m, fe_pcg_info* info, hipStream_t s, int* applies) {
  if (int e = detect_csr_structure(p, op, rp, ci, s)) return e;
  const size_t rs = real_size(p);
  if (p->w_gm && p->gm_cap < m) {
    free_dev(p->w_gm);
    p->w_gm = nullptr;
  }
  if (!p->w_gm) {
    if (int st = alloc(&p->w_gm, (size_t)(m + 3) * rs * (size_t)p->n_dof)) return st;
    p->gm_cap = m;
  }
  if (!p->gm_dev && alloc((void**)&p->gm_dev, sizeof(GmresDev))) return FE_ERR_OOM;
  if (!p->gm_part && alloc((void**)&p->gm_part, (size_t)(GM_MAXM + 1) * GM_GRID * sizeof(double)))
    return FE_ERR_OOM;
  if (p->precond == FE_PC_ILU0) {
    if (!rp) return arg_error("FE_PC_ILU0 needs the assembled CSR matrix");
    HIPCHK(ilu_setup(p, rp, ci, vals, s));
  } else if (p->precond == FE_PC_BLOCK_JACOBI) {
    HIPCHK(launch_block_jacobi(p, rp, ci, vals, p->w_blk, s));
  } else if (rp) {
    HIPCHK(launch_csr_diag(p, rp, ci, vals, p->w_d, s));
  } else {
    HIPCHK(launch_diag(p, p->w_d, 1, s));
  }
  const bool ilu = p->precond == FE_PC_ILU0;
  const int* stop = &p->gm_dev->ctrl.status;
  auto apply = [&](const void* in, void* out, const int* stp) -> hipError_t {
    if (op == FE_OP_CSR) return launch_spmv_stop(p, rp, ci, vals, in, out, stp, s);
    ElemArgs a = base_args(p);
    a.x = in;
    a.y = out;
    a.apply_bc = 1;
    return launch_elem_stop(p, OP_APPLY, a, stp, s);
  };
  GmresCtrl* hc = reinterpret_cast<GmresCtrl*>(p->host_buf);
  static_assert(sizeof(GmresCtrl) <= 64 * sizeof(double), "host scratch too small");
  auto poll = [&]() -> int {
    HIPCHK(hipMemcpyAsync(hc, &p->gm_dev->ctrl, sizeof(GmresCtrl), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return FE_OK;
  };
  HIPCHK(gm_setup(p, b, x, rtol, max_it, m, s));
  HIPCHK(gm_step(p, GM_START, 0, b, x, s));
  int restarts = 0;
  for (;;) {
    if (int e = poll()) return e;
    if (hc->status != CG_RUNNING) break;
    int j = 0, chunk = 4;
    while (j < m) {
      for (int c = 0; c < chunk && j < m; ++c, ++j) {
        HIPCHK(gm_step(p, GM_BASIS, j, b, x, s));
        if (ilu) HIPCHK(ilu_apply(p, gm_work_z(p), gm_work_z(p), stop, s));
        HIPCHK(apply(gm_work_z(p), gm_work_w(p), stop));
        HIPCHK(gm_step(p, GM_ORTHO, j, b, x, s));
      }
      if (int e = poll()) return e;
      if (hc->status != CG_RUNNING) break;
      if (chunk < 16) chunk *= 2;
    }
    HIPCHK(gm_step(p, GM_FINISH, 0, b, x, s));
    if (ilu) {  // x += (L U)^-1 V y
      HIPCHK(ilu_apply(p, gm_work_z(p), gm_work_z(p), nullptr, s));
      HIPCHK(gm_step(p, GM_ADD_Z, 0, b, x, s));
    }
    if (int e = poll()) return e;
    if (hc->status != CG_RUNNING) break;
    HIPCHK(apply(x, gm_work_w(p), nullptr));  // next cycle: w = b - A x
    HIPCHK(gm_step(p, GM_RESIDUAL, 0, b, x, s));
    ++restarts;
  }
  const int status = hc->status == CG_CONVERGED ? FE_OK : hc->status;
  if (info) {
    info->iterations = hc->iters;
    info->status = status;
    info->bnorm = hc->bb > 0 ? std::sqrt(hc->bb) : 0.0;
    info->relres = hc->bb > 0 ? hc->res_est / std::sqrt(hc->bb) : 0.0;
  }
  if (applies) *applies += hc->iters + restarts;
  if (status != FE_OK) set_error(fe_status_string(status));
  return status;
}

extern "C" int fe_apply_preconditioner(fe_problem* p, const int32_t* row_ptr, const int32_t* col_idx,
                                       const void* vals, const void* r, void* z, void* stream) {
  CHKP(p);
  if (!r || !z) return arg_error("r and z are required");
  if ((row_ptr || col_idx || vals) && !(row_ptr && col_idx && vals))
    return arg_error("give all of row_ptr, col_idx and vals, or none");
  if (!row_ptr && p->precond == FE_PC_ILU0) return arg_error("FE_PC_ILU0 needs the assembled CSR matrix");
  if (!row_ptr && !p->lin_valid) {
    set_error("no linearisation stored");
    return FE_ERR_STATE;
  }
  hipStream_t s = S(stream);
  if (p->precond == FE_PC_ILU0) {
    HIPCHK(ilu_setup(p, row_ptr, col_idx, vals, s));
    HIPCHK(ilu_apply(p, r, z, nullptr, s));
    return FE_OK;
  }
  if (p->precond == FE_PC_BLOCK_JACOBI) {
    HIPCHK(launch_block_jacobi(p, row_ptr, col_idx, vals, p->w_blk, s));
  } else if (row_ptr) {
    HIPCHK(launch_csr_diag(p, row_ptr, col_idx, vals, p->w_d, s));
  } else {
    HIPCHK(launch_diag(p, p->w_d, 1, s));
  }
  HIPCHK(pc_apply(p, r, z, s));
  return FE_OK;
}

extern "C" int fe_gmres(fe_problem* p, int op, const int32_t* row_ptr, const int32_t* col_idx, const void* vals,
                        const void* b, void* x, double rtol, int max_it, int restart, fe_pcg_info* info,
                        void* stream) {
  CHKP(p);
  if (!b || !x) return arg_error("b and x are required");
  if (op != FE_OP_CSR && op != FE_OP_MATFREE) return arg_error("op must be FE_OP_CSR or FE_OP_MATFREE");
  if (op == FE_OP_CSR && (!row_ptr || !col_idx || !vals)) return arg_error("CSR operator needs row_ptr, col_idx, vals");
  if (op == FE_OP_MATFREE && !p->lin_valid) {
    set_error("no linearisation stored");
    return FE_ERR_STATE;
  }
  if (!(rtol >= 0) || max_it < 0) return arg_error("rtol must be >= 0 and max_it >= 0");
  if (restart < 1 || restart > GM_MAXM) return arg_error("restart must be in [1, 64]");
  if (op == FE_OP_MATFREE) row_ptr = nullptr, col_idx = nullptr, vals = nullptr;
  return gmres_run(p, op, row_ptr, col_idx, vals, b, x, rtol, max_it, restart, info, S(stream), nullptr);
}

extern "C" int fe_bicgstab(fe_problem* p, int op, const int32_t* row_ptr, const int32_t* col_idx, const void* vals,
                           const void* b, void* x, double rtol, int max_it, fe_pcg_info* info, void* stream) {
  CHKP(p);
  if (!b || !x) return arg_error("b and x are required");
  if (op != FE_OP_CSR && op != FE_OP_MATFREE) return arg_error("op must be FE_OP_CSR or FE_OP_MATFREE");
  if (op == FE_OP_CSR && (!row_ptr || !col_idx || !vals)) return arg_error("CSR operator needs row_ptr, col_idx, vals");
  if (op == FE_OP_MATFREE && !p->lin_valid) {
    set_error("no linearisation stored");
    return FE_ERR_STATE;
  }
  if (!(rtol >= 0) || max_it < 0) return arg_error("rtol must be >= 0 and max_it >= 0");
  if (op == FE_OP_MATFREE) row_ptr = nullptr, col_idx = nullptr, vals = nullptr;
  return bicg_run(p, op, row_ptr, col_idx, vals, b, x, rtol, max_it, info, S(stream), nullptr);
}

extern "C" int fe_pcg(fe_problem* p, int op, const int32_t* row_ptr, const int32_t* col_idx, const void* vals,
                      const void* b, void* x, double rtol, int max_it, fe_pcg_info* info, void* stream) {
  CHKP(p);
  if (!b || !x) return arg_error("b and x are required");
  if (op != FE_OP_CSR && op != FE_OP_MATFREE) return arg_error("op must be FE_OP_CSR or FE_OP_MATFREE");
  if (op == FE_OP_CSR && (!row_ptr || !col_idx || !vals)) return arg_error("CSR operator needs row_ptr, col_idx, vals");
  if (op == FE_OP_MATFREE && !p->lin_valid) {
    set_error("no linearisation stored");
    return FE_ERR_STATE;
  }
  if (!(rtol >= 0) || max_it < 0) return arg_error("rtol must be >= 0 and max_it >= 0");
  if (op == FE_OP_MATFREE) row_ptr = nullptr, col_idx = nullptr, vals = nullptr;
  return pcg_run(p, op, row_ptr, col_idx, vals, b, x, rtol, max_it, info, S(stream), nullptr);
}

extern "C" int fe_vjp(fe_problem* p, const void* u, const void* lambda, void* out, void* stream) {
  CHKP(p);
  if (!u || !lambda || !out) return arg_error("u, lambda and out are required");
  if (p->model_set == MS_J2) return arg_error("fe_vjp supports linear and Neo-Hookean phases only");
  ElemArgs a = base_args(p);
  a.x = u;
  a.xlin = lambda;
  a.out_el = out;
  HIPCHK(launch_elem(p, OP_VJP, a, S(stream)));
  return FE_OK;
}

extern "C" int fe_vjp_path(fe_problem* p, const void* u, const void* state_in, const void* c, const void* mu_in,
                           void* mu_out, void* u_bar, void* s_bar, void* stream) {
  CHKP(p);
  if (p->prec != FE_F64) return arg_error("fe_vjp_path needs an FE_F64 problem");
  if (p->general) return arg_error("fe_vjp_path runs on structured problems only");
  if (!p->materials_set) return arg_error("materials not set");
  if (p->model_set == MS_NH) return arg_error("fe_vjp_path supports linear and J2 phases only");
  if (!u || !mu_out) return arg_error("u and mu_out are required");
  HIPCHK(launch_path_vjp(p, u, state_in, c, mu_in, mu_out, u_bar, s_bar, S(stream)));
  return FE_OK;
}

extern "C" int fe_read_flags(fe_problem* p, int* flags, void* stream) {
  CHKP(p);
  if (!flags) return arg_error("flags is null");
  int* hb = reinterpret_cast<int*>(p->host_buf);
  HIPCHK(hipMemcpyAsync(hb, p->flags, sizeof(int), hipMemcpyDeviceToHost, S(stream)));
  HIPCHK(hipMemsetAsync(p->flags, 0, sizeof(int), S(stream)));
  HIPCHK(hipStreamSynchronize(S(stream)));
  *flags = *hb;
  return FE_OK;
}

static int read_norm(fe_problem* p, const void* v, hipStream_t s, double* out) {
  HIPCHK(launch_dot(p, v, v, p->n_dof, p->stress_sum + 6, s));
  HIPCHK(hipMemcpyAsync(p->host_buf, p->stress_sum + 6, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  *out = std::sqrt(p->host_buf[0]);
  return FE_OK;
}

// Load steps first_step .. n_steps-1 of path; u enters as the converged field of step
// first_step - 1 (or the starting field), u_prev as that of step first_step - 2 (read only by
// the extrapolating predictor when first_step >= 2).
static int newton_run(fe_problem* p, const double* path, int n_steps, int first_step, const fe_newton_opts* o,
                      void* u, const void* u_prev, void* state, double* sigma_bar, fe_newton_info* info,
                      void* stream) {
  CHKP(p);
  if (!path || !o || !u || n_steps < 0) return arg_error("path, opts and u are required");
  if (first_step < 0 || first_step > n_steps) return arg_error("first_step must be in [0, n_steps]");
  if (o->op != FE_OP_CSR && o->op != FE_OP_MATFREE) return arg_error("opts.op must be FE_OP_CSR or FE_OP_MATFREE");
  if (o->max_newton < 1 || !(o->newton_rtol >= 0) || !(o->pcg_rtol >= 0) || o->pcg_max_it < 1)
    return arg_error("invalid Newton options");
  if (o->solver < FE_SOLVER_CG || o->solver > FE_SOLVER_GMRES) return arg_error("opts.solver is not a solver");
  if (o->restart < 0 || o->restart > GM_MAXM) return arg_error("opts.restart must be in [0, 64]");
  if (o->predictor != FE_PREDICT_BOUNDARY && o->predictor != FE_PREDICT_EXTRAPOLATE)
    return arg_error("opts.predictor must be FE_PREDICT_BOUNDARY or FE_PREDICT_EXTRAPOLATE");
  if (p->model_set == MS_J2 && !state) return arg_error("J2 problems need a state array");
  hipStream_t s = S(stream);
  const size_t rs = real_size(p), vec = rs * p->n_dof;
  if (!p->w_v && alloc(&p->w_v, vec)) return FE_ERR_OOM;
  if (!p->w_v2 && alloc(&p->w_v2, vec)) return FE_ERR_OOM;
  if (p->model_set == MS_J2 && !p->w_state && alloc(&p->w_state, rs * 7 * 8 * p->n_el)) return FE_ERR_OOM;
  const bool extrapolate = o->predictor == FE_PREDICT_EXTRAPOLATE && n_steps > 2;
  if (extrapolate && first_step >= 2 && first_step < n_steps && !u_prev)
    return arg_error("the extrapolating predictor resumed at step >= 2 needs u_prev");
  if (extrapolate && !p->w_uprev && alloc(&p->w_uprev, vec)) return FE_ERR_OOM;
  const bool use_csr = o->op == FE_OP_CSR || o->assemble_csr;
  if (use_csr) {
    if (int st = check_csr_size(p)) return st;
    if (!p->csr_rp) {
      if (alloc((void**)&p->csr_rp, sizeof(int32_t) * (p->n_dof + 1)) ||
          alloc((void**)&p->csr_ci, sizeof(int32_t) * p->nnz) || alloc(&p->csr_v, rs * p->nnz))
        return FE_ERR_OOM;
      HIPCHK(launch_csr_pattern(p, p->csr_rp, p->csr_ci, s));
    }
    if (int st = ensure_ke(p)) return st;
  }
  fe_newton_info inf{};
  inf.status = FE_OK;
  void* r = p->w_v;
  void* w = p->w_v2;
  void* trial = p->model_set == MS_J2 ? p->w_state : nullptr;
  // residual, its norm and the linearisation at u (state: last committed)
  auto evaluate = [&](double* norm) -> int {
    int st = residual_impl(p, u, state, trial, r, FE_APPLY_BC | FE_STORE_TANGENT, nullptr, s);
    if (st) return st;
    if ((st = read_norm(p, r, s, norm))) return st;
    int fl = 0;
    if ((st = fe_read_flags(p, &fl, stream))) return st;
    if (fl & 1) {
      set_error("inverted element");
      return FE_ERR_INVERTED;
    }
    if (!std::isfinite(*norm)) {
      set_error("non-finite residual");
      return FE_ERR_NONFINITE;
    }
    return FE_OK;
  };
  const int max_halvings = 5;
  auto frob_step = [&](int k) {  // |E_k - E_{k-1}| (E_{-1} = 0)
    double a = 0;
    for (int i = 0; i < 9; ++i) {
      const double d = path[9 * k + i] - (k > 0 ? path[9 * (k - 1) + i] : 0.0);
      a += d * d;
    }
    return std::sqrt(a);
  };
  for (int step = first_step; step < n_steps; ++step) {
    const fe_newton_info at_start = inf;
    if (extrapolate) {
      // w_uprev holds u_{k-2} from step 2 on; u += ratio (u - w_uprev), then w_uprev <- the old u
      if (step >= 2) {
        if (step == first_step) HIPCHK(launch_axpby(p, p->n_dof, 1.0, u_prev, 0.0, p->w_uprev, s));
        const double d0 = frob_step(step - 1);
        const double ratio = d0 > 0 ? frob_step(step) / d0 : 0.0;
        HIPCHK(launch_axpby(p, p->n_dof, 1.0, u, 0.0, w, s));                // w = u_{k-1}
        HIPCHK(launch_axpby(p, p->n_dof, -ratio, p->w_uprev, 1.0 + ratio, u, s));  // u = u + ratio (u - u_{k-2})
        HIPCHK(launch_axpby(p, p->n_dof, 1.0, w, 0.0, p->w_uprev, s));       // u_{k-2} <- u_{k-1}
      } else {
        HIPCHK(launch_axpby(p, p->n_dof, 1.0, u, 0.0, p->w_uprev, s));
      }
    }
    HIPCHK(launch_lift(p, path + 9 * step, u, 0, s));
    double r0 = -1.0, rn = 0.0;
    bool converged = false;
    int est = evaluate(&rn);
    if (est == FE_ERR_HIP || est == FE_ERR_OOM) return est;
    if (est) inf.status = est;
    for (int it = 0; inf.status == FE_OK && it <= o->max_newton; ++it) {
      int st = FE_OK;
      if (r0 < 0) r0 = rn;
      if (rn <= o->newton_rtol * r0 || rn == 0.0) {
        converged = true;
        break;
      }
      if (it == o->max_newton) break;
      inf.newton_iterations += 1;
      HIPCHK(launch_axpby(p, p->n_dof, -1.0, r, 0.0, r, s));  // b = -P_f R
      const int32_t *rp = nullptr, *ci = nullptr;
      const void* vals = nullptr;
      if (use_csr) {
        PROF(p, s, 3, launch_tangent_csr(p, p->csr_v, 1, s));
        rp = p->csr_rp;
        ci = p->csr_ci;
        vals = p->csr_v;
      }
      fe_pcg_info pi{};
      st = o->solver == FE_SOLVER_GMRES
               ? gmres_run(p, o->op, rp, ci, vals, r, w, o->pcg_rtol, o->pcg_max_it,
                           o->restart > 0 ? o->restart : 30, &pi, s, &inf.operator_applies)
           : o->solver == FE_SOLVER_BICGSTAB
               ? bicg_run(p, o->op, rp, ci, vals, r, w, o->pcg_rtol, o->pcg_max_it, &pi, s, &inf.operator_applies)
               : pcg_run(p, o->op, rp, ci, vals, r, w, o->pcg_rtol, o->pcg_max_it, &pi, s, &inf.operator_applies);
      inf.pcg_iterations += pi.iterations;
      if (st) {
        inf.status = st;
        break;
      }
      // halving line search on ||P_f R||: u += s w with s = 1, 1/2, ... while the norm does not drop
      const double r_prev = rn;
      double sc = 1.0;
      HIPCHK(launch_axpby(p, p->n_dof, sc, w, 1.0, u, s));
      for (int hv = 0;; ++hv) {
        st = evaluate(&rn);
        if (st == FE_ERR_HIP || st == FE_ERR_OOM) return st;
        if ((st == FE_OK && rn < r_prev) || hv == max_halvings) break;
        HIPCHK(launch_axpby(p, p->n_dof, -0.5 * sc, w, 1.0, u, s));  // back to u_old + (sc/2) w
        sc *= 0.5;
      }
      inf.line_search_halvings += (int)std::lround(-std::log2(sc));
      if (st) {
        inf.status = st;
        break;
      }
    }
    inf.last_residual = rn;
    if (inf.status != FE_OK) break;
    if (!converged) {
      inf.status = FE_ERR_NOT_CONVERGED;
      set_error("Newton did not converge");
      break;
    }
    if (sigma_bar) {  // stress of the converged iterate, from the state the step started from
      int st = fe_mean_stress(p, u, state, sigma_bar + 6 * step, stream);
      if (st) return st;
    }
    if (trial) HIPCHK(gen_copy_state(p, trial, state, 7 * 8 * p->n_el, s));
    inf.steps_done += 1;
    if (o->step_log_host) {
      o->step_log_host[3 * step] = inf.newton_iterations - at_start.newton_iterations;
      o->step_log_host[3 * step + 1] = inf.line_search_halvings - at_start.line_search_halvings;
      o->step_log_host[3 * step + 2] = inf.pcg_iterations - at_start.pcg_iterations;
    }
  }
  HIPCHK(hipStreamSynchronize(s));
  if (info) *info = inf;
  return inf.status;
}

extern "C" int fe_newton(fe_problem* p, const double* path, int n_steps, const fe_newton_opts* o, void* u,
                         void* state, double* sigma_bar, fe_newton_info* info, void* stream) {
  return newton_run(p, path, n_steps, 0, o, u, nullptr, state, sigma_bar, info, stream);
}

extern "C" int fe_newton_resume(fe_problem* p, const double* path, int n_steps, int first_step,
                                const fe_newton_opts* o, void* u, const void* u_prev, void* state,
                                double* sigma_bar, fe_newton_info* info, void* stream) {
  return newton_run(p, path, n_steps, first_step, o, u, u_prev, state, sigma_bar, info, stream);
}

extern "C" int fe_profile(fe_problem* p, int enable) {
  CHKP(p);
  if (enable < 0) return arg_error("enable must be >= 0");
  if (enable) {
    p->prof_recs.clear();
    p->ev_used = 0;
    p->prof_stride = enable;
  }
  p->prof = enable != 0;
  return FE_OK;
}

extern "C" int fe_profile_read(fe_problem* p, double* out) {
  CHKP(p);
  if (!out) return arg_error("out is null");
  for (int k = 0; k < 15; ++k) out[k] = 0;
  HIPCHK(hipDeviceSynchronize());
  for (const auto& r : p->prof_recs) {
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, p->ev_pool[r.second], p->ev_pool[r.second + 1]));
    out[3 * r.first] += 1;
    out[3 * r.first + 1] += ms;
  }
  for (int c = 0; c < 5; ++c) {
    out[3 * c + 2] = p->prof_bytes[c];
    p->prof_bytes[c] = 0;
  }
  p->prof_recs.clear();
  p->ev_used = 0;
  return FE_OK;
}

// Algorithmic bytes of one operator launch at the current linearisation.
static int operator_bytes(fe_problem* p, int op, hipStream_t s, double* bytes) {
  const double w = (double)real_size(p);
  if (op == FE_OP_CSR) {  // one column list per node triple in the node-structured mat-vec
    *bytes = (w + (p->csr_nodal ? 4.0 / 3.0 : 4.0)) * (double)p->nnz + 4.0 * (double)(p->n_dof + 1) +
             2.0 * w * (double)p->n_dof;
    return FE_OK;
  }
  int64_t st[2] = {0, 0};
  if (p->model_set == MS_J2) {
    if (int e = fe_linearization_stats(p, st, s)) return e;
  }
  // x in, y out, phase ids, and per J2 point the plastic flag word plus 5 more values if plastic
  double b = 2.0 * w * (double)p->n_dof + (double)p->n_el + w * ((double)st[0] + 5.0 * (double)st[1]);
  if (p->general)  // connectivity and coordinates; all six tangent words of every J2 point
    b = 2.0 * w * (double)p->n_dof + 33.0 * (double)p->n_el + 3.0 * w * (double)p->n_nodes + 6.0 * w * (double)st[0];
  if (p->model_set == MS_NH) b += 80.0 * w * (double)p->n_nh_el;  // stored F^-T and ln J of every point
  if (p->scale) b += w * (double)p->n_el;  // per-element modulus scale
  *bytes = b;
  return FE_OK;
}

extern "C" int fe_linearization_stats(fe_problem* p, int64_t* out, void* stream) {
  CHKP(p);
  if (!out) return arg_error("out is null");
  out[0] = out[1] = 0;
  if (p->model_set != MS_J2 || !p->lin_valid) return FE_OK;
  unsigned long long* d = reinterpret_cast<unsigned long long*>(p->stress_sum);
  HIPCHK(hipMemsetAsync(d, 0, 2 * sizeof(unsigned long long), S(stream)));
  HIPCHK(launch_lin_stats(p, d, S(stream)));
  HIPCHK(hipMemcpyAsync(p->host_buf, d, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, S(stream)));
  HIPCHK(hipStreamSynchronize(S(stream)));
  const unsigned long long* h = reinterpret_cast<const unsigned long long*>(p->host_buf);
  out[0] = (int64_t)h[0];
  out[1] = (int64_t)h[1];
  return FE_OK;
}

extern "C" int fe_set_surrogate(fe_problem* p, const float* W, double tol) {
  CHKP(p);
  if (W && p->general) return arg_error("the surrogate runs on structured problems only");
  if (!W) {
    p->sur_W = nullptr;
    return FE_OK;
  }
  if (p->model_set != MS_J2) return arg_error("the surrogate replaces a J2 phase: set J2 materials first");
  if (!(tol >= 0)) return arg_error("fallback_tol must be >= 0");
  const int64_t cap = 8 * p->n_j2_el;
  if (cap >= (int64_t(1) << 31)) return arg_error("too many J2 points for the surrogate list");
  if (p->sur_cap < cap) {
    free_dev(p->sur_x);
    free_dev(p->sur_y);
    free_dev(p->sur_jac);
    free_dev(p->sur_D);
    p->sur_x = p->sur_y = p->sur_jac = nullptr;
    p->sur_D = nullptr;
    p->sur_cap = 0;
    const int64_t c = std::max<int64_t>(cap, 1);
    if (alloc((void**)&p->sur_x, sizeof(float) * 13 * c) || alloc((void**)&p->sur_y, sizeof(float) * 6 * c) ||
        alloc((void**)&p->sur_jac, sizeof(float) * 36 * c) || alloc(&p->sur_D, sizeof(float) * 36 * c))
      return FE_ERR_OOM;
    p->sur_cap = c;
  }
  if (!p->sur_map && alloc((void**)&p->sur_map, sizeof(int) * 8 * p->n_el)) return FE_ERR_OOM;
  if (!p->sur_count && alloc((void**)&p->sur_count, 4 * sizeof(unsigned int))) return FE_ERR_OOM;
  p->sur_W = W;
  p->sur_tol = tol;
  p->lin_valid = false;  // stored tangents of an earlier law no longer apply
  return FE_OK;
}

extern "C" int fe_surrogate_stats(fe_problem* p, int64_t* out, void* stream) {
  CHKP(p);
  if (!out) return arg_error("out is null");
  out[0] = out[1] = out[2] = 0;
  if (!p->sur_count) return FE_OK;
  unsigned int* h = reinterpret_cast<unsigned int*>(p->host_buf);
  HIPCHK(hipMemcpyAsync(h, p->sur_count, 3 * sizeof(unsigned int), hipMemcpyDeviceToHost, S(stream)));
  HIPCHK(hipStreamSynchronize(S(stream)));
  out[0] = std::min<int64_t>(h[0], p->sur_cap);
  out[1] = h[1];
  out[2] = h[2];
  return FE_OK;
}

extern "C" int fe_set_capture(fe_problem* p, float* x, float* y, int64_t capacity, unsigned int* count, int stride) {
  CHKP(p);
  if (x && p->general) return arg_error("sample capture runs on structured problems only");
  if (!x) {
    p->cap_x = nullptr;
    return FE_OK;
  }
  if (!y || !count || capacity < 1 || stride < 1) return arg_error("capture needs y, count, capacity >= 1, stride >= 1");
  if (p->model_set != MS_J2) return arg_error("capture records J2 return-map samples: set J2 materials first");
  p->cap_x = x;
  p->cap_y = y;
  p->cap_n = capacity;
  p->cap_count = count;
  p->cap_stride = (unsigned)stride;
  return FE_OK;
}
