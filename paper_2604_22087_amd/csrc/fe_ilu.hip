// Node-block ILU(0) preconditioner in an 8-colour node order (needs the assembled CSR).
//
// Sec. V-B (Fig. 7) compares Jacobi with ILU preconditioning of the assembled matrix.
// A natural-order ILU(0) on this mesh has ~7n dependency levels per triangular solve,
// one launch (or grid barrier) each; colouring the nodes by the parities of their grid
// indices leaves 8 levels: no two nodes of one colour share an element, so every colour
// is factored and solved in one data-parallel launch.  Blocks are the 3x3 couplings of
// node pairs; no fill outside the block pattern (node pairs sharing an element).
//
// Factor storage F[27 slots][9 entries][n_nodes], nodes by position in the colour order
// (so the lanes of one colour's launch touch consecutive words).  Slot s of node i holds
// the block of neighbour i + (di, dj, dk), s = (di+1) + 3 (dj+1) + 9 (dk+1): L_ij when j's
// colour is lower, U_ij when higher, and the inverse of the pivot block U_ii in slot 13.
// The colour of i + (di, dj, dk) is colour(i) XOR m with m = [di != 0] + 2 [dj != 0] +
// 4 [dk != 0].

#include <cmath>

#include "fe_internal.hpp"

namespace fe {

namespace {

constexpr int IB = 128;  // lanes per workgroup of the ILU kernels

struct Colouring {
  int n;
  int cnt[2];     // grid indices in [0, n] of parity 0 and 1
  int64_t off[9]; // first position of each colour (off[8] = n_nodes)
};

Colouring colouring(int n) {
  Colouring c{};
  c.n = n;
  c.cnt[0] = (n + 2) / 2;
  c.cnt[1] = (n + 1) / 2;
  c.off[0] = 0;
  for (int col = 0; col < 8; ++col)
    c.off[col + 1] = c.off[col] + (int64_t)c.cnt[col & 1] * c.cnt[(col >> 1) & 1] * c.cnt[(col >> 2) & 1];
  return c;
}

// grid indices of the t-th node of colour col
__device__ __forceinline__ void colour_node(const Colouring& c, int col, int64_t t, int& i, int& j, int& k) {
  const int cx = c.cnt[col & 1], cy = c.cnt[(col >> 1) & 1];
  i = 2 * (int)(t % cx) + (col & 1);
  j = 2 * (int)((t / cx) % cy) + ((col >> 1) & 1);
  k = 2 * (int)(t / ((int64_t)cx * cy)) + ((col >> 2) & 1);
}

// position of node (i, j, k) in the colour order
__device__ __forceinline__ int64_t colour_pos(const Colouring& c, int i, int j, int k) {
  const int col = (i & 1) + 2 * (j & 1) + 4 * (k & 1);
  const int cx = c.cnt[col & 1], cy = c.cnt[(col >> 1) & 1];
  return c.off[col] + (i >> 1) + (int64_t)cx * ((j >> 1) + (int64_t)cy * (k >> 1));
}

__device__ __forceinline__ int slot_mask(int s) {
  return (s % 3 != 1 ? 1 : 0) | ((s / 3) % 3 != 1 ? 2 : 0) | (s / 9 != 1 ? 4 : 0);
}

template <typename T>
__device__ __forceinline__ void load_block(const T* F, int64_t nn, int s, int64_t p, double b[9]) {
#pragma unroll
  for (int e = 0; e < 9; ++e) b[e] = (double)F[((int64_t)s * 9 + e) * nn + p];
}

template <typename T>
__device__ __forceinline__ void store_block(T* F, int64_t nn, int s, int64_t p, const double b[9]) {
#pragma unroll
  for (int e = 0; e < 9; ++e) F[((int64_t)s * 9 + e) * nn + p] = T(b[e]);
}

// 3x3 inverse by the adjugate; false when singular or not finite
__device__ bool inverse3(const double a[9], double r[9]) {
  const double c00 = a[4] * a[8] - a[5] * a[7], c01 = a[5] * a[6] - a[3] * a[8], c02 = a[3] * a[7] - a[4] * a[6];
  const double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
  if (!(det != 0.0) || !(det - det == 0.0)) return false;
  const double id = 1.0 / det;
  r[0] = c00 * id;
  r[1] = (a[2] * a[7] - a[1] * a[8]) * id;
  r[2] = (a[1] * a[5] - a[2] * a[4]) * id;
  r[3] = c01 * id;
  r[4] = (a[0] * a[8] - a[2] * a[6]) * id;
  r[5] = (a[2] * a[3] - a[0] * a[5]) * id;
  r[6] = c02 * id;
  r[7] = (a[1] * a[6] - a[0] * a[7]) * id;
  r[8] = (a[0] * a[4] - a[1] * a[3]) * id;
  return true;
}

// F <- the CSR blocks of every node (one lane per node position).
template <typename T>
__global__ __launch_bounds__(IB) void ilu_load_kernel(Colouring c, const int32_t* rp, const int32_t* ci, const T* v,
                                                      T* F) {
  const int n = c.n;
  const int64_t nn = c.off[8];
  const int64_t p = (int64_t)blockIdx.x * IB + threadIdx.x;
  if (p >= nn) return;
  int col = 0;
  while (p >= c.off[col + 1]) ++col;
  int i, j, k;
  colour_node(c, col, p - c.off[col], i, j, k);
  const int64_t node = i + (int64_t)(n + 1) * (j + (int64_t)(n + 1) * k);
  for (int s = 0; s < 27; ++s) {
    const int a = i + s % 3 - 1, b = j + (s / 3) % 3 - 1, d = k + s / 9 - 1;
    double blk[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (a >= 0 && a <= n && b >= 0 && b <= n && d >= 0 && d <= n) {
      const int64_t nb = a + (int64_t)(n + 1) * (b + (int64_t)(n + 1) * d);
      for (int r = 0; r < 3; ++r) {
        const int64_t row = 3 * node + r;
        int lo = rp[row], hi = rp[row + 1] - 1;
        const int32_t want = (int32_t)(3 * nb);
        while (lo < hi) {  // first column >= 3 nb (sorted row)
          const int mid = (lo + hi) >> 1;
          if (ci[mid] < want) lo = mid + 1;
          else hi = mid;
        }
        for (int q = lo; q < rp[row + 1] && ci[q] < want + 3; ++q)
          if (ci[q] >= want) blk[3 * r + (ci[q] - want)] = (double)v[q];
      }
    }
    store_block(F, nn, s, p, blk);
  }
}

// Factor the rows of colour col (all lower colours are final): for each lower neighbour k in
// colour order, L_ik = A_ik U_kk^-1 and A_ij -= L_ik U_kj for the later j of both patterns;
// then slot 13 <- U_ii^-1.
template <typename T>
__global__ __launch_bounds__(IB) void ilu_factor_kernel(Colouring c, int col, T* F, unsigned int* flags) {
  const int n = c.n;
  const int64_t nn = c.off[8];
  const int64_t t = (int64_t)blockIdx.x * IB + threadIdx.x;
  if (t >= c.off[col + 1] - c.off[col]) return;
  const int64_t p = c.off[col] + t;
  int i, j, k;
  colour_node(c, col, t, i, j, k);
  for (int kc = 0; kc < col; ++kc) {
    const int m = col ^ kc;
    for (int s = 0; s < 27; ++s) {
      if (slot_mask(s) != m) continue;
      const int ox = s % 3 - 1, oy = (s / 3) % 3 - 1, oz = s / 9 - 1;
      const int ka = i + ox, kb = j + oy, kd = k + oz;
      if (ka < 0 || ka > n || kb < 0 || kb > n || kd < 0 || kd > n) continue;
      const int64_t pk = colour_pos(c, ka, kb, kd);
      double a[9], ui[9], l[9];
      load_block(F, nn, s, p, a);
      load_block(F, nn, 13, pk, ui);
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) l[3 * r + q] = a[3 * r] * ui[q] + a[3 * r + 1] * ui[3 + q] + a[3 * r + 2] * ui[6 + q];
      store_block(F, nn, s, p, l);
      for (int sj = 0; sj < 27; ++sj) {
        if ((col ^ slot_mask(sj)) <= kc) continue;  // j must come after k
        const int dx = sj % 3 - 1 - ox, dy = (sj / 3) % 3 - 1 - oy, dz = sj / 9 - 1 - oz;
        if (dx < -1 || dx > 1 || dy < -1 || dy > 1 || dz < -1 || dz > 1) continue;  // j not adjacent to k
        const int ja = i + sj % 3 - 1, jb = j + (sj / 3) % 3 - 1, jd = k + sj / 9 - 1;
        if (ja < 0 || ja > n || jb < 0 || jb > n || jd < 0 || jd > n) continue;
        const int skj = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
        double u[9], aij[9];
        load_block(F, nn, skj, pk, u);
        load_block(F, nn, sj, p, aij);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int q = 0; q < 3; ++q)
            aij[3 * r + q] -= l[3 * r] * u[q] + l[3 * r + 1] * u[3 + q] + l[3 * r + 2] * u[6 + q];
        store_block(F, nn, sj, p, aij);
      }
    }
  }
  double d[9], di[9];
  load_block(F, nn, 13, p, d);
  if (!inverse3(d, di)) {
    atomicOr(flags, 4u);
    for (int e = 0; e < 9; ++e) di[e] = NAN;
  }
  store_block(F, nn, 13, p, di);
}

// Forward sweep of colour col: z_i = r_i - sum_{k lower} L_ik z_k.
template <typename T>
__global__ __launch_bounds__(IB) void ilu_forward_kernel(Colouring c, int col, const T* F, const T* r, T* z,
                                                         const int* stop) {
  if (stop && *stop) return;
  const int n = c.n;
  const int64_t nn = c.off[8];
  const int64_t t = (int64_t)blockIdx.x * IB + threadIdx.x;
  if (t >= c.off[col + 1] - c.off[col]) return;
  const int64_t p = c.off[col] + t;
  int i, j, k;
  colour_node(c, col, t, i, j, k);
  const int64_t node = i + (int64_t)(n + 1) * (j + (int64_t)(n + 1) * k);
  double y[3] = {(double)r[3 * node], (double)r[3 * node + 1], (double)r[3 * node + 2]};
  for (int s = 0; s < 27; ++s) {
    if ((col ^ slot_mask(s)) >= col) continue;
    const int a = i + s % 3 - 1, b = j + (s / 3) % 3 - 1, d = k + s / 9 - 1;
    if (a < 0 || a > n || b < 0 || b > n || d < 0 || d > n) continue;
    const int64_t nb = a + (int64_t)(n + 1) * (b + (int64_t)(n + 1) * d);
    const double x0 = (double)z[3 * nb], x1 = (double)z[3 * nb + 1], x2 = (double)z[3 * nb + 2];
    double l[9];
    load_block(F, nn, s, p, l);
#pragma unroll
    for (int q = 0; q < 3; ++q) y[q] -= l[3 * q] * x0 + l[3 * q + 1] * x1 + l[3 * q + 2] * x2;
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) z[3 * node + q] = T(y[q]);
}

// Backward sweep of colour col: z_i = U_ii^-1 (z_i - sum_{j higher} U_ij z_j).
template <typename T>
__global__ __launch_bounds__(IB) void ilu_backward_kernel(Colouring c, int col, const T* F, T* z, const int* stop) {
  if (stop && *stop) return;
  const int n = c.n;
  const int64_t nn = c.off[8];
  const int64_t t = (int64_t)blockIdx.x * IB + threadIdx.x;
  if (t >= c.off[col + 1] - c.off[col]) return;
  const int64_t p = c.off[col] + t;
  int i, j, k;
  colour_node(c, col, t, i, j, k);
  const int64_t node = i + (int64_t)(n + 1) * (j + (int64_t)(n + 1) * k);
  double y[3] = {(double)z[3 * node], (double)z[3 * node + 1], (double)z[3 * node + 2]};
  for (int s = 0; s < 27; ++s) {
    if ((col ^ slot_mask(s)) <= col) continue;
    const int a = i + s % 3 - 1, b = j + (s / 3) % 3 - 1, d = k + s / 9 - 1;
    if (a < 0 || a > n || b < 0 || b > n || d < 0 || d > n) continue;
    const int64_t nb = a + (int64_t)(n + 1) * (b + (int64_t)(n + 1) * d);
    const double x0 = (double)z[3 * nb], x1 = (double)z[3 * nb + 1], x2 = (double)z[3 * nb + 2];
    double u[9];
    load_block(F, nn, s, p, u);
#pragma unroll
    for (int q = 0; q < 3; ++q) y[q] -= u[3 * q] * x0 + u[3 * q + 1] * x1 + u[3 * q + 2] * x2;
  }
  double ui[9];
  load_block(F, nn, 13, p, ui);
#pragma unroll
  for (int q = 0; q < 3; ++q) z[3 * node + q] = T(ui[3 * q] * y[0] + ui[3 * q + 1] * y[1] + ui[3 * q + 2] * y[2]);
}

int grid_for(int64_t count) { return (int)std::max<int64_t>(1, (count + IB - 1) / IB); }

template <typename T>
hipError_t ilu_setup_t(const fe_problem* p, const int32_t* rp, const int32_t* ci, const T* v, hipStream_t s) {
  const Colouring c = colouring(p->n);
  T* F = static_cast<T*>(p->w_ilu);
  hipLaunchKernelGGL(ilu_load_kernel<T>, dim3(grid_for(c.off[8])), dim3(IB), 0, s, c, rp, ci, v, F);
  for (int col = 0; col < 8; ++col)
    hipLaunchKernelGGL(ilu_factor_kernel<T>, dim3(grid_for(c.off[col + 1] - c.off[col])), dim3(IB), 0, s, c, col, F,
                       reinterpret_cast<unsigned int*>(p->flags));
  return hipGetLastError();
}

template <typename T>
hipError_t ilu_apply_t(const fe_problem* p, const T* r, T* z, const int* stop, hipStream_t s) {
  const Colouring c = colouring(p->n);
  const T* F = static_cast<const T*>(p->w_ilu);
  for (int col = 0; col < 8; ++col)
    hipLaunchKernelGGL(ilu_forward_kernel<T>, dim3(grid_for(c.off[col + 1] - c.off[col])), dim3(IB), 0, s, c, col, F,
                       r, z, stop);
  for (int col = 7; col >= 0; --col)
    hipLaunchKernelGGL(ilu_backward_kernel<T>, dim3(grid_for(c.off[col + 1] - c.off[col])), dim3(IB), 0, s, c, col,
                       F, z, stop);
  return hipGetLastError();
}

}  // namespace

size_t ilu_words(const fe_problem* p) { return (size_t)27 * 9 * (size_t)p->n_nodes; }

hipError_t ilu_setup(const fe_problem* p, const int32_t* rp, const int32_t* ci, const void* v, hipStream_t s) {
  return p->prec == FE_F64 ? ilu_setup_t(p, rp, ci, static_cast<const double*>(v), s)
                           : ilu_setup_t(p, rp, ci, static_cast<const float*>(v), s);
}

hipError_t ilu_apply(const fe_problem* p, const void* r, void* z, const int* stop, hipStream_t s) {
  return p->prec == FE_F64 ? ilu_apply_t(p, static_cast<const double*>(r), static_cast<double*>(z), stop, s)
                           : ilu_apply_t(p, static_cast<const float*>(r), static_cast<float*>(z), stop, s);
}

}  // namespace fe
