// Restarted GMRES(m) on the device (right preconditioning), for nonsymmetric operators.
//
// Fig. 4 compares GMRES with CG and BiCGStab on the assembled system.  One Arnoldi
// step here: v_j = w / h_{j,j-1} and z = M^-1 v_j (one launch), w = A z (the library's
// operator), classical Gram-Schmidt run twice (dots, reduce, update; dots, reduce,
// update + ||w||^2; the second pass restores the orthogonality that one classical pass
// loses in floating point), then one workgroup applies the Givens rotations to the new
// Hessenberg column and tests |g_{j+1}| <= rtol ||b||.  All dot products are FP64 and
// summed in a fixed order (per-workgroup partials, then one workgroup per vector).
// Iteration kernels return at once after a stop; the cycle-end kernels (triangular solve,
// x += M^-1 V y) always run.

#include <cmath>

#include "fe_internal.hpp"

namespace fe {

namespace {

constexpr int KB = 256;  // threads per workgroup of every GMRES kernel

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Sum of part[0..np) by the whole workgroup, in fixed order; valid in every lane.
__device__ double group_sum(const double* part, int np, double* sh) {
  double v = 0;
  for (int i = threadIdx.x; i < np; i += KB) v += part[i];
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0;
#pragma unroll
  for (int w = 0; w < KB / 64; ++w) t += sh[w];
  __syncthreads();
  return t;
}

__device__ __forceinline__ bool is_finite(double v) { return v == v && v - v == 0.0; }

// z = M^-1 r for the three dofs of one node: node-block inverse (blk = 1; 6 words per
// node: xx, yy, zz, yz, xz, xy) or inverted point diagonal (blk = 0); blk = 2 (ILU(0),
// applied by its own sweeps afterwards) copies r.
template <typename T>
__device__ __forceinline__ void precond_node(const T* M, int blk, int64_t node, const T r[3], T z[3]) {
  if (blk == 2) {
#pragma unroll
    for (int c = 0; c < 3; ++c) z[c] = r[c];
  } else if (blk) {
    const T* m = M + 6 * node;
    z[0] = m[0] * r[0] + m[5] * r[1] + m[4] * r[2];
    z[1] = m[5] * r[0] + m[1] * r[1] + m[3] * r[2];
    z[2] = m[4] * r[0] + m[3] * r[1] + m[2] * r[2];
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) z[c] = M[3 * node + c] * r[c];
  }
}

// x = 0, w = b, point diagonal inverted in place; controls reset.
template <typename T>
__global__ __launch_bounds__(KB) void gm_setup_kernel(int64_t n, const T* b, T* x, T* w, T* dinv, int blk,
                                                      GmresDev* dev, double rtol, int max_it, int m) {
  for (int64_t i = (int64_t)blockIdx.x * KB + threadIdx.x; i < n; i += (int64_t)gridDim.x * KB) {
    x[i] = 0;
    w[i] = b[i];
    if (!blk) dinv[i] = T(1) / dinv[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    GmresCtrl& c = dev->ctrl;
    c.rtol = rtol;
    c.tol = 0;
    c.bb = -1;  // set by the first cycle start
    c.res_est = 0;
    c.status = CG_RUNNING;
    c.iters = 0;
    c.max_it = max_it;
    c.k = 0;
    c.m = m;
    c.cycles = 0;
  }
}

// part[i][blockIdx] = (V_i, w) for i < nv (V_i = V + i n).  Tiles of 8 vectors keep the
// accumulators in registers; w is re-read once per tile.
template <typename T>
__global__ __launch_bounds__(KB) void gm_dots_kernel(int64_t n, const T* V, int nv, const T* w, double* part,
                                                     const int* stop) {
  if (stop && *stop) return;
  __shared__ double sh[8][KB / 64];
  for (int i0 = 0; i0 < nv; i0 += 8) {
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t d = (int64_t)blockIdx.x * KB + threadIdx.x; d < n; d += (int64_t)gridDim.x * KB) {
      const double wd = (double)w[d];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (i0 + u < nv) acc[u] += (double)V[(int64_t)(i0 + u) * n + d] * wd;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double t = wave_sum(acc[u]);
      if ((threadIdx.x & 63) == 0) sh[u][threadIdx.x >> 6] = t;
    }
    __syncthreads();
    if (threadIdx.x < 8 && i0 + (int)threadIdx.x < nv) {
      double t = 0;
#pragma unroll
      for (int q = 0; q < KB / 64; ++q) t += sh[threadIdx.x][q];
      part[(int64_t)(i0 + threadIdx.x) * gridDim.x + blockIdx.x] = t;
    }
    __syncthreads();
  }
}

// One workgroup per vector i < nv: c_i = sum of its partials; pass 0 sets the Hessenberg
// entries H[j][i] = c_i, pass 1 adds the re-orthogonalisation coefficients to them.
__global__ __launch_bounds__(KB) void gm_reduce_kernel(const double* part, int np, GmresDev* dev, int j, int pass,
                                                       const int* stop) {
  if (stop && *stop) return;
  __shared__ double sh[KB / 64];
  const int i = blockIdx.x;
  const double c = group_sum(part + (int64_t)i * np, np, sh);
  if (threadIdx.x == 0) {
    dev->c[pass][i] = c;
    dev->H[j][i] = pass == 0 ? c : dev->H[j][i] + c;
  }
}

// w -= sum_{i<nv} c_i V_i with c = dev->c[pass]; with_norm: part[blockIdx] = partial ||w||^2.
template <typename T>
__global__ __launch_bounds__(KB) void gm_update_kernel(int64_t n, const T* V, int nv, T* w, const GmresDev* dev,
                                                       int pass, int with_norm, double* part, const int* stop) {
  if (stop && *stop) return;
  __shared__ double cs[GM_MAXM + 1];
  __shared__ double sh[KB / 64];
  for (int i = threadIdx.x; i < nv; i += KB) cs[i] = dev->c[pass][i];
  __syncthreads();
  double nrm = 0;
  for (int64_t d = (int64_t)blockIdx.x * KB + threadIdx.x; d < n; d += (int64_t)gridDim.x * KB) {
    double t = (double)w[d];
    for (int i = 0; i < nv; ++i) t -= cs[i] * (double)V[(int64_t)i * n + d];
    const T tv = T(t);
    w[d] = tv;
    nrm += (double)tv * (double)tv;
  }
  if (!with_norm) return;
  nrm = wave_sum(nrm);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = nrm;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
#pragma unroll
    for (int q = 0; q < KB / 64; ++q) t += sh[q];
    part[blockIdx.x] = t;
  }
}

// Start of a cycle (one workgroup): beta = ||r|| from the partials of the residual in w;
// g = beta e_1; the first cycle also sets ||b|| and the tolerance.
__global__ __launch_bounds__(KB) void gm_beta_kernel(const double* part, int np, GmresDev* dev) {
  __shared__ double sh[KB / 64];
  GmresCtrl& c = dev->ctrl;
  if (c.status) return;
  const double beta = std::sqrt(group_sum(part, np, sh));
  if (threadIdx.x != 0) return;
  if (c.bb < 0) {
    c.bb = beta * beta;
    c.tol = c.rtol * beta;
  }
  c.k = 0;
  c.cycles += 1;
  c.res_est = beta;
  for (int i = 0; i <= c.m; ++i) dev->g[i] = 0;
  dev->g[0] = beta;
  if (!is_finite(beta)) {
    c.status = FE_ERR_NONFINITE;
  } else if (beta <= c.tol) {
    c.status = CG_CONVERGED;
  } else if (c.iters >= c.max_it) {
    c.status = FE_ERR_NOT_CONVERGED;
  } else {
    c.inv_norm = 1.0 / beta;
  }
}

// v_j = w / ||w|| (stored as basis vector j) and z = M^-1 v_j, one node per lane; w is
// cleared for the operator, which adds its face contributions atomically.
template <typename T>
__global__ __launch_bounds__(KB) void gm_basis_kernel(int64_t n_nodes, T* w, T* vj, T* z, const T* M, int blk,
                                                      const GmresDev* dev, const int* stop) {
  if (stop && *stop) return;
  const T s = T(dev->ctrl.inv_norm);
  for (int64_t nd = (int64_t)blockIdx.x * KB + threadIdx.x; nd < n_nodes; nd += (int64_t)gridDim.x * KB) {
    T v[3], zz[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      v[c] = w[3 * nd + c] * s;
      vj[3 * nd + c] = v[c];
      w[3 * nd + c] = 0;
    }
    precond_node(M, blk, nd, v, zz);
#pragma unroll
    for (int c = 0; c < 3; ++c) z[3 * nd + c] = zz[c];
  }
}

// End of Arnoldi step j (one workgroup): h_{j+1,j} = ||w||, rotations on column j,
// new rotation, g update, stopping tests.
__global__ __launch_bounds__(KB) void gm_givens_kernel(const double* part, int np, GmresDev* dev, int j,
                                                       const int* stop) {
  if (stop && *stop) return;
  __shared__ double sh[KB / 64];
  const double hn = std::sqrt(group_sum(part, np, sh));
  if (threadIdx.x != 0) return;
  GmresCtrl& c = dev->ctrl;
  double* h = dev->H[j];
  h[j + 1] = hn;
  if (!is_finite(hn)) {
    c.status = FE_ERR_NONFINITE;
    return;
  }
  for (int i = 0; i < j; ++i) {
    const double t = dev->cs[i] * h[i] + dev->sn[i] * h[i + 1];
    h[i + 1] = -dev->sn[i] * h[i] + dev->cs[i] * h[i + 1];
    h[i] = t;
  }
  const double rho = std::hypot(h[j], h[j + 1]);
  if (rho == 0.0) {
    c.status = FE_ERR_BREAKDOWN;
    return;
  }
  dev->cs[j] = h[j] / rho;
  dev->sn[j] = h[j + 1] / rho;
  h[j] = rho;
  h[j + 1] = 0.0;
  dev->g[j + 1] = -dev->sn[j] * dev->g[j];
  dev->g[j] = dev->cs[j] * dev->g[j];
  c.iters += 1;
  c.k = j + 1;
  c.res_est = std::fabs(dev->g[j + 1]);
  if (c.res_est <= c.tol) c.status = CG_CONVERGED;
  else if (c.iters >= c.max_it) c.status = FE_ERR_NOT_CONVERGED;
  else c.inv_norm = 1.0 / hn;
}

// y = R^-1 g over the k finished columns (one lane; k <= GM_MAXM).
__global__ void gm_solve_kernel(GmresDev* dev) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const int k = dev->ctrl.k;
  for (int i = k - 1; i >= 0; --i) {
    double t = dev->g[i];
    for (int q = i + 1; q < k; ++q) t -= dev->H[q][i] * dev->y[q];
    dev->y[i] = t / dev->H[i][i];
  }
}

// x += M^-1 (sum_{i<k} y_i V_i), one node per lane (blk = 2: t = sum_i y_i V_i goes to
// tz instead, for the ILU sweeps and GM_ADD_Z); w is cleared for the operator application
// that starts the next cycle.
template <typename T>
__global__ __launch_bounds__(KB) void gm_combine_kernel(int64_t n_nodes, const T* V, int64_t n, T* x, T* w,
                                                        T* tz, const T* M, int blk, const GmresDev* dev) {
  __shared__ double ys[GM_MAXM];
  const int k = dev->ctrl.k;
  for (int i = threadIdx.x; i < k; i += KB) ys[i] = dev->y[i];
  __syncthreads();
  for (int64_t nd = (int64_t)blockIdx.x * KB + threadIdx.x; nd < n_nodes; nd += (int64_t)gridDim.x * KB) {
    T t[3], z[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) w[3 * nd + c] = 0;
    if (k == 0) continue;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double a = 0;
      for (int i = 0; i < k; ++i) a += ys[i] * (double)V[(int64_t)i * n + 3 * nd + c];
      t[c] = T(a);
    }
    if (blk == 2) {
#pragma unroll
      for (int c = 0; c < 3; ++c) tz[3 * nd + c] = t[c];
      continue;
    }
    precond_node(M, blk, nd, t, z);
#pragma unroll
    for (int c = 0; c < 3; ++c) x[3 * nd + c] += z[c];
  }
}

// x += z
template <typename T>
__global__ __launch_bounds__(KB) void gm_add_kernel(int64_t n, const T* z, T* x) {
  for (int64_t d = (int64_t)blockIdx.x * KB + threadIdx.x; d < n; d += (int64_t)gridDim.x * KB) x[d] += z[d];
}

// w = b - w (w holds A x) and partial ||w||^2 for the next cycle start.
template <typename T>
__global__ __launch_bounds__(KB) void gm_residual_kernel(int64_t n, const T* b, T* w, double* part) {
  __shared__ double sh[KB / 64];
  double nrm = 0;
  for (int64_t d = (int64_t)blockIdx.x * KB + threadIdx.x; d < n; d += (int64_t)gridDim.x * KB) {
    const T t = b[d] - w[d];
    w[d] = t;
    nrm += (double)t * (double)t;
  }
  nrm = wave_sum(nrm);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = nrm;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
#pragma unroll
    for (int q = 0; q < KB / 64; ++q) t += sh[q];
    part[blockIdx.x] = t;
  }
}

template <typename T> T* basis(const fe_problem* p, int i) { return static_cast<T*>(p->w_gm) + (int64_t)i * p->n_dof; }
template <typename T> T* work_w(const fe_problem* p) { return basis<T>(p, p->gm_cap + 1); }
template <typename T> T* work_z(const fe_problem* p) { return basis<T>(p, p->gm_cap + 2); }

int node_grid(const fe_problem* p) {
  return (int)std::min<int64_t>((p->n_nodes + KB - 1) / KB, 4 * GM_GRID);
}

template <typename T>
hipError_t gm_step_t(const fe_problem* p, int stage, int j, const void* b, void* x, hipStream_t s) {
  const int64_t n = p->n_dof;
  const int* stop = &p->gm_dev->ctrl.status;
  const T* M = static_cast<const T*>(pc_buffer(p));
  switch (stage) {
    case GM_BASIS:
      hipLaunchKernelGGL(gm_basis_kernel<T>, dim3(node_grid(p)), dim3(KB), 0, s, p->n_nodes, work_w<T>(p),
                         basis<T>(p, j), work_z<T>(p), M, p->precond, p->gm_dev, stop);
      break;
    case GM_ORTHO: {  // two classical Gram-Schmidt passes, then ||w||
      for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(gm_dots_kernel<T>, dim3(GM_GRID), dim3(KB), 0, s, n, basis<T>(p, 0), j + 1, work_w<T>(p),
                           p->gm_part, stop);
        hipLaunchKernelGGL(gm_reduce_kernel, dim3(j + 1), dim3(KB), 0, s, p->gm_part, GM_GRID, p->gm_dev, j, pass,
                           stop);
        hipLaunchKernelGGL(gm_update_kernel<T>, dim3(GM_GRID), dim3(KB), 0, s, n, basis<T>(p, 0), j + 1,
                           work_w<T>(p), p->gm_dev, pass, pass == 1 ? 1 : 0, p->gm_part, stop);
      }
      hipLaunchKernelGGL(gm_givens_kernel, dim3(1), dim3(KB), 0, s, p->gm_part, GM_GRID, p->gm_dev, j, stop);
      break;
    }
    case GM_START:  // w holds the residual: ||w|| -> beta, g = beta e_1
      hipLaunchKernelGGL(gm_dots_kernel<T>, dim3(GM_GRID), dim3(KB), 0, s, n, work_w<T>(p), 1, work_w<T>(p),
                         p->gm_part, nullptr);
      hipLaunchKernelGGL(gm_beta_kernel, dim3(1), dim3(KB), 0, s, p->gm_part, GM_GRID, p->gm_dev);
      break;
    case GM_FINISH:  // cycle end: y = R^-1 g, x += M^-1 V y
      hipLaunchKernelGGL(gm_solve_kernel, dim3(1), dim3(64), 0, s, p->gm_dev);
      hipLaunchKernelGGL(gm_combine_kernel<T>, dim3(node_grid(p)), dim3(KB), 0, s, p->n_nodes, basis<T>(p, 0), n,
                         static_cast<T*>(x), work_w<T>(p), work_z<T>(p), M, p->precond, p->gm_dev);
      break;
    case GM_ADD_Z:  // x += z (after the ILU sweeps of the cycle-end combination)
      hipLaunchKernelGGL(gm_add_kernel<T>, dim3(GM_GRID), dim3(KB), 0, s, n, work_z<T>(p), static_cast<T*>(x));
      break;
    case GM_RESIDUAL:  // w = b - w (w = A x), then ||w||
      hipLaunchKernelGGL(gm_residual_kernel<T>, dim3(GM_GRID), dim3(KB), 0, s, n, static_cast<const T*>(b),
                         work_w<T>(p), p->gm_part);
      hipLaunchKernelGGL(gm_beta_kernel, dim3(1), dim3(KB), 0, s, p->gm_part, GM_GRID, p->gm_dev);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// z = M^-1 r with the point diagonal d (not inverted; blk = 0) or the inverted node blocks
// (blk = 1), one node per lane.
template <typename T>
__global__ __launch_bounds__(KB) void pc_apply_kernel(int64_t n_nodes, const T* M, int blk, const T* r, T* z) {
  for (int64_t nd = (int64_t)blockIdx.x * KB + threadIdx.x; nd < n_nodes; nd += (int64_t)gridDim.x * KB) {
    T v[3], w[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = r[3 * nd + c];
    if (blk) {
      precond_node(M, 1, nd, v, w);
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) w[c] = v[c] / M[3 * nd + c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) z[3 * nd + c] = w[c];
  }
}

template <typename T>
hipError_t pc_apply_t(const fe_problem* p, const void* r, void* z, hipStream_t s) {
  hipLaunchKernelGGL(pc_apply_kernel<T>, dim3(node_grid(p)), dim3(KB), 0, s, p->n_nodes,
                     static_cast<const T*>(pc_buffer(p)), p->precond == FE_PC_BLOCK_JACOBI ? 1 : 0,
                     static_cast<const T*>(r), static_cast<T*>(z));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// CG with a preconditioner applied by separate launches (ILU(0)): Hestenes & Stiefel
// recursion with z = M^-1 r, FP64 dots in fixed order, device-resident scalars.

template <typename T>
__global__ __launch_bounds__(KB) void ipcg_init_kernel(int64_t n, const T* b, T* x, T* r, T* q, double* part,
                                                       IpcgCtrl* c, double rtol, int max_it) {
  __shared__ double sh[KB / 64];
  double v = 0;
  for (int64_t d = (int64_t)blockIdx.x * KB + threadIdx.x; d < n; d += (int64_t)gridDim.x * KB) {
    x[d] = 0;
    q[d] = 0;
    const T t = b[d];
    r[d] = t;
    v += (double)t * (double)t;
  }
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
#pragma unroll
    for (int q = 0; q < KB / 64; ++q) t += sh[q];
    part[blockIdx.x] = t;
    if (blockIdx.x == 0) {
      c->rtol = rtol;
      c->max_it = max_it;
      c->iters = 0;
      c->status = CG_RUNNING;
      c->alpha = c->pq = 0;
      c->rzs[0] = c->rzs[1] = 0;
    }
  }
}

// ||r||^2 from the partials; the first call sets ||b|| and the tolerance, later calls
// count the finished iteration and test it.
__global__ __launch_bounds__(KB) void ipcg_check_kernel(const double* part, int np, IpcgCtrl* c, int first) {
  __shared__ double sh[KB / 64];
  if (c->status) return;
  const double rr = group_sum(part, np, sh);
  if (threadIdx.x != 0) return;
  c->rr = rr;
  if (!is_finite(rr)) {
    c->status = FE_ERR_NONFINITE;
    return;
  }
  if (first) {
    c->bb = rr;
    c->tol2 = c->rtol * c->rtol * rr;
    if (rr == 0.0) c->status = CG_CONVERGED;
    else if (c->max_it <= 0) c->status = FE_ERR_NOT_CONVERGED;
    return;
  }
  c->iters += 1;
  if (rr <= c->tol2) c->status = CG_CONVERGED;
  else if (c->iters >= c->max_it) c->status = FE_ERR_NOT_CONVERGED;
}

// p = z + beta p with beta = (r, z)_k / (r, z)_{k-1} (k = 0: p = z); every workgroup sums the
// (r, z) partials itself, workgroup 0 records them in slot k & 1.  q is cleared for the
// next operator application (the matrix-free operator adds into it).
template <typename T>
__global__ __launch_bounds__(KB) void ipcg_direction_kernel(int64_t n, const T* z, T* p, T* q, const double* part,
                                                            int np, IpcgCtrl* c, long k) {
  __shared__ double sh[KB / 64];
  if (c->status) return;
  const double rz = group_sum(part, np, sh);
  const double beta = k == 0 ? 0.0 : rz / c->rzs[(k - 1) & 1];
  if (!is_finite(rz) || !is_finite(beta)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) c->status = FE_ERR_NONFINITE;
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) c->rzs[k & 1] = rz;
  const T bt = T(beta);
  for (int64_t d = (int64_t)blockIdx.x * KB + threadIdx.x; d < n; d += (int64_t)gridDim.x * KB) {
    p[d] = k == 0 ? z[d] : z[d] + bt * p[d];
    q[d] = 0;
  }
}

// alpha = (r, z)_k / (p, A p) (every workgroup sums the partials itself), x += alpha p,
// r -= alpha q, partials of ||r||^2.
template <typename T>
__global__ __launch_bounds__(KB) void ipcg_update_kernel(int64_t n, const T* p, const T* q, T* x, T* r,
                                                         const double* part_pq, int np, IpcgCtrl* c, long k,
                                                         double* part_rr) {
  __shared__ double sh[KB / 64];
  if (c->status) return;
  const double pq = group_sum(part_pq, np, sh);
  if (!(pq > 0.0) || !is_finite(pq)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) c->status = is_finite(pq) ? FE_ERR_BREAKDOWN : FE_ERR_NONFINITE;
    return;
  }
  const double alpha = c->rzs[k & 1] / pq;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    c->alpha = alpha;
    c->pq = pq;
  }
  const T a = T(alpha);
  double v = 0;
  for (int64_t d = (int64_t)blockIdx.x * KB + threadIdx.x; d < n; d += (int64_t)gridDim.x * KB) {
    x[d] += a * p[d];
    const T t = r[d] - a * q[d];
    r[d] = t;
    v += (double)t * (double)t;
  }
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
#pragma unroll
    for (int w = 0; w < KB / 64; ++w) t += sh[w];
    part_rr[blockIdx.x] = t;
  }
}

template <typename T> T* ipcg_v(const fe_problem* p, int v) {
  return static_cast<T*>(p->w_ipcg) + (int64_t)v * p->n_dof;
}

template <typename T>
hipError_t ipcg_step_t(const fe_problem* p, int stage, long k, const void* b, void* x, double rtol, int max_it,
                       hipStream_t s) {
  const int64_t n = p->n_dof;
  double* part_pq = p->gm_part;
  double* part_rr = p->gm_part + GM_GRID;
  double* part_rz = p->gm_part + 2 * GM_GRID;
  const int* stop = &p->ipcg->status;
  T* r = ipcg_v<T>(p, 0);
  T* pp = ipcg_v<T>(p, 1);
  T* q = ipcg_v<T>(p, 2);
  T* z = ipcg_v<T>(p, 3);
  switch (stage) {
    case IPCG_INIT:
      hipLaunchKernelGGL(ipcg_init_kernel<T>, dim3(GM_GRID), dim3(KB), 0, s, n, static_cast<const T*>(b),
                         static_cast<T*>(x), r, q, part_rr, p->ipcg, rtol, max_it);
      break;
    case IPCG_CHECK_FIRST:
    case IPCG_CHECK:
      hipLaunchKernelGGL(ipcg_check_kernel, dim3(1), dim3(KB), 0, s, part_rr, GM_GRID, p->ipcg,
                         stage == IPCG_CHECK_FIRST ? 1 : 0);
      break;
    case IPCG_FIRST_DIRECTION:  // (r, z) partials, then p = z
    case IPCG_DIRECTION:
      hipLaunchKernelGGL(gm_dots_kernel<T>, dim3(GM_GRID), dim3(KB), 0, s, n, r, 1, z, part_rz, stop);
      hipLaunchKernelGGL(ipcg_direction_kernel<T>, dim3(GM_GRID), dim3(KB), 0, s, n, z, pp, q, part_rz, GM_GRID,
                         p->ipcg, stage == IPCG_FIRST_DIRECTION ? 0L : k);
      break;
    case IPCG_UPDATE:  // (p, q) partials, then the step
      hipLaunchKernelGGL(gm_dots_kernel<T>, dim3(GM_GRID), dim3(KB), 0, s, n, pp, 1, q, part_pq, stop);
      hipLaunchKernelGGL(ipcg_update_kernel<T>, dim3(GM_GRID), dim3(KB), 0, s, n, pp, q, static_cast<T*>(x), r,
                         part_pq, GM_GRID, p->ipcg, k, part_rr);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t gm_setup_t(const fe_problem* p, const void* b, void* x, double rtol, int max_it, int m, hipStream_t s) {
  hipLaunchKernelGGL(gm_setup_kernel<T>, dim3(GM_GRID), dim3(KB), 0, s, p->n_dof, static_cast<const T*>(b),
                     static_cast<T*>(x), work_w<T>(p), static_cast<T*>(pc_buffer(p)), p->precond, p->gm_dev, rtol,
                     max_it, m);
  return hipGetLastError();
}

}  // namespace

hipError_t gm_setup(const fe_problem* p, const void* b, void* x, double rtol, int max_it, int m, hipStream_t s) {
  return p->prec == FE_F64 ? gm_setup_t<double>(p, b, x, rtol, max_it, m, s)
                           : gm_setup_t<float>(p, b, x, rtol, max_it, m, s);
}

hipError_t ipcg_step(const fe_problem* p, int stage, long k, const void* b, void* x, double rtol, int max_it,
                     hipStream_t s) {
  return p->prec == FE_F64 ? ipcg_step_t<double>(p, stage, k, b, x, rtol, max_it, s)
                           : ipcg_step_t<float>(p, stage, k, b, x, rtol, max_it, s);
}

void* ipcg_vec(const fe_problem* p, int v) {
  return static_cast<char*>(p->w_ipcg) + (size_t)v * p->n_dof * (p->prec == FE_F64 ? 8 : 4);
}

hipError_t pc_apply(const fe_problem* p, const void* r, void* z, hipStream_t s) {
  return p->prec == FE_F64 ? pc_apply_t<double>(p, r, z, s) : pc_apply_t<float>(p, r, z, s);
}

hipError_t gm_step(const fe_problem* p, int stage, int j, const void* b, void* x, hipStream_t s) {
  return p->prec == FE_F64 ? gm_step_t<double>(p, stage, j, b, x, s) : gm_step_t<float>(p, stage, j, b, x, s);
}

void* gm_work_w(const fe_problem* p) {
  return static_cast<char*>(p->w_gm) + (size_t)(p->gm_cap + 1) * p->n_dof * (p->prec == FE_F64 ? 8 : 4);
}

void* gm_work_z(const fe_problem* p) {
  return static_cast<char*>(p->w_gm) + (size_t)(p->gm_cap + 2) * p->n_dof * (p->prec == FE_F64 ? 8 : 4);
}

}  // namespace fe
