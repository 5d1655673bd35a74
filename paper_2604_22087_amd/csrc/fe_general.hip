// HIP kernels of libfe for general hex8 meshes (fe_problem_create_hex8): any conforming mesh
// of 8-node bricks given by device coordinates [3][n_nodes] and connectivity [8][n_el].
//
// Element kernels run one lane per (element, Gauss point): a 256-lane workgroup holds 32
// elements x 8 points, the 8 lanes of an element sit side by side in one wave.
//   1. lane (e, p) stages node p of element e (coordinates and the gathered field) in LDS;
//   2. each lane forms the isoparametric Jacobian of its point from the 8 nodal positions,
//      its inverse, the physical basis gradients and the displacement gradient;
//   3. the constitutive law gives the stress, pushed back to the 8 nodes (w detJ B^T sigma);
//   4. the 8 lanes of an element sum their nodal forces by recursive halving (three lane
//      exchanges of 12, 6 and 3 values, no atomics), after which lane p holds node p's total
//      and adds it to the global vector with one hardware FP atomic per component.
//
// The sparse Jacobian follows the sort-and-combine assembly of the paper (Sec. III-B):
//   symbolic (once per mesh): every element contributes its 64 node pairs; pairs are
//   bucketed by row node (counting sort) and each row is sorted by (column node, element
//   code), so the whole list is ordered by the int64 key (row, column); runs of equal keys
//   are the duplicates, their first positions give the node-pair pattern, and the sorted
//   element codes of each run say which element blocks sum into that pair;
//   numeric (per tangent): each element's dense 24 x 24 Jacobian K_e = sum_q B_q^T D_q B_q
//   w detJ is one batched contraction on the FP64 / FP32 matrix cores (v_mfma_*_16x16x4),
//   written to a per-element buffer; a gather then sums every pair's run in sorted order
//   into the CSR values (deterministic: the same bits on every run).
#include <type_traits>

#include "fe_internal.hpp"
#include "fe_device.hpp"

namespace fe {

constexpr int GBLOCK = 256;
constexpr int GEL = GBLOCK / 8;  // elements per element-kernel workgroup
constexpr double GAUSS = 0.57735026918962576451;  // 1/sqrt(3)

// Reference coordinates of local node a: (-1,-1,-1) (1,-1,-1) (1,1,-1) (-1,1,-1), then z = +1.
__device__ __forceinline__ int ref_sx(int a) { return (((a + 1) >> 1) & 1) ? 1 : -1; }
__device__ __forceinline__ int ref_sy(int a) { return (a & 2) ? 1 : -1; }
__device__ __forceinline__ int ref_sz(int a) { return (a & 4) ? 1 : -1; }

// dN_a / dxi_k of the trilinear basis at Gauss point q = qx + 2 qy + 4 qz (xi = +-1/sqrt 3).
template <typename T> __device__ __forceinline__ void ref_grad(int q, T dn[8][3]) {
  const T g = T(GAUSS);
  const T xi = (q & 1) ? g : -g, eta = (q & 2) ? g : -g, zeta = (q & 4) ? g : -g;
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const T sx = T(ref_sx(a)), sy = T(ref_sy(a)), sz = T(ref_sz(a));
    const T fx = 1 + sx * xi, fy = 1 + sy * eta, fz = 1 + sz * zeta;
    dn[a][0] = T(0.125) * sx * fy * fz;
    dn[a][1] = T(0.125) * fx * sy * fz;
    dn[a][2] = T(0.125) * fx * fy * sz;
  }
}

// Physical basis gradients g[a][j] = dN_a/dx_j at Gauss point q of the element with nodal
// positions xe[a][i]; returns det J (J_ik = dx_i/dxi_k).
template <typename T> __device__ __forceinline__ T phys_grad(const T (*xe)[3], int q, T g[8][3]) {
  T dn[8][3];
  ref_grad<T>(q, dn);
  T J[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      T s = 0;
#pragma unroll
      for (int a = 0; a < 8; ++a) s += xe[a][i] * dn[a][k];
      J[i][k] = s;
    }
  const T c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1], c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2],
          c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  const T det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
  const T id = T(1) / det;
  // (J^-1)_kj = cof(J)_jk / det
  T Ji[3][3];
  Ji[0][0] = c00 * id;
  Ji[1][0] = c01 * id;
  Ji[2][0] = c02 * id;
  Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
  Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
  Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
  Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
  Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
  Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int j = 0; j < 3; ++j) g[a][j] = dn[a][0] * Ji[0][j] + dn[a][1] * Ji[1][j] + dn[a][2] * Ji[2][j];
  return det;
}

// Displacement gradient H[c][j] = sum_a u[a][c] g[a][j].
template <typename T> __device__ __forceinline__ void field_grad(const T (*ue)[3], const T g[8][3], T H[3][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      T s = 0;
#pragma unroll
      for (int a = 0; a < 8; ++a) s += ue[a][c] * g[a][j];
      H[c][j] = s;
    }
}

// Sum of per-lane values v[8][NV] (node, component) over the 8 lanes of an element (lanes q =
// lane % 8); afterwards lane q holds node q's total in out[NV].  Recursive halving: each step
// sends the half the partner keeps and adds the received half to its own.
template <typename T, int NV> __device__ __forceinline__ void reduce_scatter8(const T v[8][NV], int q, T out[NV]) {
  T h1[4][NV], h2[2][NV];
  const bool b4 = q & 4, b2 = q & 2, b1 = q & 1;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      const T send = b4 ? v[a][c] : v[a + 4][c];
      const T keep = b4 ? v[a + 4][c] : v[a][c];
      h1[a][c] = keep + __shfl_xor(send, 4, 64);
    }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      const T send = b2 ? h1[a][c] : h1[a + 2][c];
      const T keep = b2 ? h1[a + 2][c] : h1[a][c];
      h2[a][c] = keep + __shfl_xor(send, 2, 64);
    }
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    const T send = b1 ? h2[0][c] : h2[1][c];
    const T keep = b1 ? h2[1][c] : h2[0][c];
    out[c] = keep + __shfl_xor(send, 1, 64);
  }
}

// Sum of one value over the 8 lanes of an element (every lane gets it).
__device__ __forceinline__ double sum8(double v) {
  v += __shfl_xor(v, 4, 64);
  v += __shfl_xor(v, 2, 64);
  v += __shfl_xor(v, 1, 64);
  return v;
}

struct GenArgs {
  const void* coords;     // real [3][n_nodes]
  const int32_t* conn;    // [8][n_el]
  int64_t n_nodes;
};

static GenArgs gen_args(const fe_problem* p) {
  GenArgs g;
  g.coords = p->coords;
  g.conn = p->conn;
  g.n_nodes = p->n_nodes;
  return g;
}

// ---------------------------------------------------------------------------
// element kernel: OP_RESID, OP_APPLY, OP_VJP (ElemArgs as for the structured kernels; y
// zeroed by the caller; constrained dofs receive nothing, see gen_bc_kernel)

template <typename T, int OP, int MS>
__global__ __launch_bounds__(GBLOCK) void gen_elem_kernel(GenArgs g, ElemArgs a, const int* stop) {
  constexpr bool APPLY = OP == OP_APPLY;
  constexpr bool NEED_L = OP == OP_VJP;
  __shared__ T s_c[GEL][8][3];
  __shared__ T s_x[GEL][8][3];
  __shared__ T s_l[NEED_L ? GEL : 1][8][3];
  __shared__ double s_red[6][GBLOCK / 64];
  if (stop && *stop) return;
  const int tid = threadIdx.x, el = tid >> 3, q = tid & 7;
  const int64_t ne = a.n_el;
  const int64_t e = (int64_t)blockIdx.x * GEL + el;
  const bool valid = e < ne;
  const T* X = static_cast<const T*>(a.x);
  const T* XL = static_cast<const T*>(a.xlin);
  const T* C = static_cast<const T*>(g.coords);
  const bool bc = a.apply_bc && a.mask;
  // stage node q of element e
  int node = 0;
  if (valid) node = g.conn[(int64_t)q * ne + e];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int64_t dof = 3 * (int64_t)node + c;
    s_c[el][q][c] = valid ? C[(int64_t)c * g.n_nodes + node] : T(0);
    T v = valid ? X[dof] : T(0);
    if (APPLY && bc && valid && a.mask[dof]) v = T(0);
    s_x[el][q][c] = v;
    if (NEED_L) s_l[NEED_L ? el : 0][q][c] = valid ? XL[dof] : T(0);
  }
  __syncthreads();

  T f[8][3];
#pragma unroll
  for (int b = 0; b < 8; ++b)
#pragma unroll
    for (int c = 0; c < 3; ++c) f[b][c] = 0;
  double ssum[6] = {0, 0, 0, 0, 0, 0};
  if (valid) {
    T gr[8][3];
    const T wdet = phys_grad<T>(s_c[el], q, gr);  // Gauss weight 1
    T H[3][3], S[3][3];
    field_grad<T>(s_x[el], gr, H);
    const PhaseConst pc = a.mat.ph[a.phase[e]];
    const T sc = (a.scale && OP != OP_VJP) ? static_cast<const T*>(a.scale)[e] : T(1);
    const T lam = T(pc.lam) * sc, mu = T(pc.mu) * sc;
    const T Kb = T(pc.K) * sc, Gs = T(pc.G) * sc, sy = T(pc.sy), Hh = T(pc.H);
    const int64_t pidx = (int64_t)q * ne + e;  // Gauss-point index in [8][n_el] arrays
    const T* st_in = static_cast<const T*>(a.state_in);
    T* st_out = static_cast<T*>(a.state_out);
    T* tang = static_cast<T*>(a.tangent);
    bool done = false;
    if (MS == MS_J2 && pc.model == FE_J2) {
      if (OP == OP_RESID) {
        T epn[6], an = 0, ep[6], al, tn[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) epn[k] = st_in ? st_in[(int64_t)k * 8 * ne + pidx] : T(0);
        if (st_in) an = st_in[(int64_t)6 * 8 * ne + pidx];
        j2_update(H, epn, an, Kb, Gs, sy, Hh, S, ep, al, tn);
        if (st_out) {
#pragma unroll
          for (int k = 0; k < 6; ++k) st_out[(int64_t)k * 8 * ne + pidx] = ep[k];
          st_out[(int64_t)6 * 8 * ne + pidx] = al;
        }
        if (a.store_tangent) {
#pragma unroll
          for (int k = 0; k < 6; ++k) tang[(int64_t)k * 8 * ne + pidx] = tn[k];
        }
        done = true;
      } else if (APPLY) {
        T tn[6], lp, mp, beta, N[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) tn[k] = tang[(int64_t)k * 8 * ne + pidx];
        j2_tangent_coeffs(tn, Kb, Gs, Hh, lp, mp, beta, N);
        j2_apply(H, lp, mp, beta, N, S);
        done = true;
      }
    }
    if (MS == MS_NH && pc.model == FE_NEOHOOKE) {
      if (APPLY) {  // F^-T and ln J of the linearisation, as the residual stored them
        T FiT[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) FiT[i][j] = tang[(int64_t)(3 * i + j) * 8 * ne + pidx];
        nh_apply(H, FiT, tang[(int64_t)9 * 8 * ne + pidx], lam, mu, S);
      } else {
        T FiT[3][3], lnJ;
        if (!nh_kin(H, FiT, lnJ) && a.flags) atomicOr(a.flags, 1);
        nh_stress(H, FiT, lnJ, lam, mu, S);
        if (OP == OP_RESID && a.store_tangent) {
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) tang[(int64_t)(3 * i + j) * 8 * ne + pidx] = FiT[i][j];
          tang[(int64_t)9 * 8 * ne + pidx] = lnJ;
        }
      }
      done = true;
    }
    if (!done) {
      hooke(H, lam, mu, S);
      if (MS == MS_J2 && OP == OP_RESID && st_out) {  // non-J2 phase: state passes through
#pragma unroll
        for (int k = 0; k < 7; ++k) st_out[(int64_t)k * 8 * ne + pidx] = st_in ? st_in[(int64_t)k * 8 * ne + pidx] : T(0);
      }
    }
    // nodal forces of this point: w detJ S g_b
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
      for (int c = 0; c < 3; ++c) f[b][c] = wdet * (S[c][0] * gr[b][0] + S[c][1] * gr[b][1] + S[c][2] * gr[b][2]);
    if (OP == OP_RESID && a.stress_sum) {
      const double w = (double)wdet;
      ssum[0] = w * S[0][0];
      ssum[1] = w * S[1][1];
      ssum[2] = w * S[2][2];
      ssum[3] = w * S[1][2];
      ssum[4] = w * S[0][2];
      ssum[5] = w * S[0][1];
    }
  }
  T fn[3];
  reduce_scatter8<T, 3>(f, q, fn);  // all lanes take part (invalid ones with zeros)

  if (OP == OP_VJP) {
    // out_e = sum_b f_b . (lambda_b - mean lambda): exact (the element's nodal forces sum to
    // zero) and free of the cancellation of a large rigid part of lambda
    double lm[3] = {0, 0, 0};
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
      for (int c = 0; c < 3; ++c) lm[c] += (double)s_l[NEED_L ? el : 0][b][c];
    double d = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) d += (double)fn[c] * ((double)s_l[NEED_L ? el : 0][q][c] - 0.125 * lm[c]);
    d = sum8(d);
    if (valid && q == 0) static_cast<T*>(a.out_el)[e] = T(d);
    return;
  }

  if (OP == OP_RESID && a.stress_sum) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      double v = ssum[k];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if ((tid & 63) == 0) s_red[k][tid >> 6] = v;
    }
    __syncthreads();
    if (tid < 6) {
      double v = 0;
      for (int w = 0; w < GBLOCK / 64; ++w) v += s_red[tid][w];
      atomic_add(a.stress_sum + tid, v);
    }
  }

  T* Y = static_cast<T*>(a.y);
  if (!Y || !valid) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int64_t dof = 3 * (int64_t)node + c;
    if (a.apply_bc && a.mask && a.mask[dof]) continue;
    atomic_add(Y + dof, fn[c]);
  }
}

// Constrained dofs of a masked operator: y = x there (A = P_f K P_f + P_b).  With pa, also the
// per-workgroup partials of x.y over all dofs (CG: p.Ap); x, y complete (kernel boundary).
template <typename T>
__global__ __launch_bounds__(VBLOCK) void gen_bc_kernel(int64_t n, const uint8_t* mask, const T* x, T* y,
                                                        const int* stop, double* pa) {
  __shared__ double sh[VBLOCK / 64];
  if (stop && *stop) return;
  double v = 0;
  for (int64_t i = (int64_t)blockIdx.x * VBLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * VBLOCK) {
    T yi;
    if (mask && mask[i]) {
      yi = x[i];
      y[i] = yi;
    } else {
      yi = y[i];
    }
    if (pa) v += (double)x[i] * (double)yi;
  }
  if (pa) {
    v = block_sum(v, sh);
    if (threadIdx.x == 0) pa[blockIdx.x] = v;
  }
}

// ---------------------------------------------------------------------------
// diagonal (NB = 3) or symmetric 3x3 node blocks (NB = 6: xx yy zz yz xz xy) of K at the
// stored linearisation, summed over elements (d zeroed before; constrained dofs skipped)

template <typename T, int MS, int NB>
__global__ __launch_bounds__(GBLOCK) void gen_diag_kernel(GenArgs g, TanArgs ta, T* d, int skip_bc) {
  __shared__ T s_c[GEL][8][3];
  const int tid = threadIdx.x, el = tid >> 3, q = tid & 7;
  const int64_t ne = ta.n_el;
  const int64_t e = (int64_t)blockIdx.x * GEL + el;
  const bool valid = e < ne;
  const T* C = static_cast<const T*>(g.coords);
  int node = 0;
  if (valid) node = g.conn[(int64_t)q * ne + e];
#pragma unroll
  for (int c = 0; c < 3; ++c) s_c[el][q][c] = valid ? C[(int64_t)c * g.n_nodes + node] : T(0);
  __syncthreads();
  T v[8][NB];
#pragma unroll
  for (int b = 0; b < 8; ++b)
#pragma unroll
    for (int k = 0; k < NB; ++k) v[b][k] = 0;
  if (valid) {
    T gr[8][3];
    const T wdet = phys_grad<T>(s_c[el], q, gr);
    QpTangent<T> t;
    load_qp_tangent<T, MS>(ta, e, q, t);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      T B[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
      block_add(t, gr[b], gr[b], wdet, B);
      v[b][0] = B[0][0];
      v[b][1] = B[1][1];
      v[b][2] = B[2][2];
      if (NB == 6) {
        v[b][NB == 6 ? 3 : 0] = B[1][2];
        v[b][NB == 6 ? 4 : 0] = B[0][2];
        v[b][NB == 6 ? 5 : 0] = B[0][1];
      }
    }
  }
  T out[NB];
  reduce_scatter8<T, NB>(v, q, out);
  if (!valid) return;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    if (NB == 3 && skip_bc && ta.mask && ta.mask[3 * (int64_t)node + k]) continue;
    atomic_add(d + (int64_t)NB * node + k, out[k]);
  }
}

template <typename T> __global__ void gen_mask_one_kernel(int64_t n, const uint8_t* mask, T* d) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (mask[i]) d[i] = T(1);
}

// ---------------------------------------------------------------------------
// element Jacobians on the matrix cores
//
// K_e = G^T (D G) with the Gauss points stacked along the contraction: for small strain
// G = [B_0; ...; B_7] (48 x 24, the Voigt strain-displacement rows) and D = blockdiag(w detJ
// D_q) (6 x 6 blocks); for finite strain G stacks the 9 x 24 gradient operators
// (row (i, J) of node b's column (b, k) is delta_ik dN_b/dX_J) and D holds w detJ times the
// 9 x 9 tangent moduli A_iJkL.  The 24 x 24 result is padded to 32 x 32 = 2 x 2 tiles of the
// 16 x 16 x 4 MFMA; K_e is symmetric, so the lower-left tile is the transpose of the upper-right
// one and only three tiles are computed.  Lane layout (16 x 16 x 4, both precisions): lane l
// holds A[l % 16][l / 16] and B[l / 16][l % 16]; result entry r of lane l sits in column l % 16
// and row 4 (l / 16) + r for FP32, row l / 16 + 4 r for FP64 (measured on gfx950).
// One wave per workgroup, one element at a time; the element's basis gradients and scaled
// moduli are staged in LDS by its 64 lanes (lane = 8 * point + node).
// Output: ke[e][a][b][i][k] = K_e[(a, i), (b, k)] (a 3 x 3 block per node pair, 576 reals).

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f_t mfma16(float a, float b, v4f_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename T> struct Acc4;
template <> struct Acc4<double> { typedef v4d type; };
template <> struct Acc4<float> { typedef v4f_t type; };

// Calls f(std::integral_constant<int, i>) for i = 0 .. N-1 (compile-time loop index).
template <int I, int N, typename F> __device__ __forceinline__ void static_for_impl(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for_impl<I + 1, N>(f);
  }
}
template <int N, typename F> __device__ __forceinline__ void static_for(F&& f) { static_for_impl<0, N>(f); }

// Row of result entry r of lane l (16 x 16 x 4 MFMA).
template <typename T> __device__ __forceinline__ int mfma_row(int l, int r);
template <> __device__ __forceinline__ int mfma_row<double>(int l, int r) { return (l >> 4) + 4 * r; }
template <> __device__ __forceinline__ int mfma_row<float>(int l, int r) { return 4 * (l >> 4) + r; }

// Entry (m, (b, k)) of the stacked gradient operator at one point: Voigt rows
// [xx yy zz yz xz xy] (DIM 6) or gradient rows (i, J) = 3 i + J (DIM 9).  m is a compile-time
// row of the unrolled contraction loop and k the lane's component, so this is a pair of selects.
template <typename T, int DIM, int M> __device__ __forceinline__ T g_entry(int k, const T* gb) {
  if (DIM == 9) return k == M / 3 ? gb[M % 3] : T(0);
  if (M < 3) return k == M ? gb[M] : T(0);
  constexpr int ka = M == 3 ? 1 : 0, da = M == 3 ? 2 : (M == 4 ? 2 : 1);   // shear rows: two components
  constexpr int kb = M == 5 ? 1 : 2, db = M == 3 ? 1 : 0;
  return k == ka ? gb[da] : (k == kb ? gb[db] : T(0));
}

// Rows of B's column (b, k) that are non-zero (Voigt): row k (d/dx_k) and two shear rows n1, n2
// with the derivative directions g1, g2 -- per lane constants.
struct VoigtCol {
  int n1, g1, n2, g2;
};
__device__ __forceinline__ VoigtCol voigt_col(int k) {
  VoigtCol c;
  c.n1 = k == 0 ? 4 : 3;
  c.g1 = k == 2 ? 1 : 2;
  c.n2 = k == 2 ? 4 : 5;
  c.g2 = k == 0 ? 1 : 0;
  return c;
}

// (D G)[m][(b, k)] at one point.
template <typename T, int DIM, int M>
__device__ __forceinline__ T dg_entry(const T* D, int k, const VoigtCol& vc, const T* gb) {
  const T* Dm = D + M * DIM;
  if (DIM == 9) return Dm[3 * k] * gb[0] + Dm[3 * k + 1] * gb[1] + Dm[3 * k + 2] * gb[2];
  return Dm[k] * gb[k] + Dm[vc.n1] * gb[vc.g1] + Dm[vc.n2] * gb[vc.g2];
}

template <typename T, int MS>
__global__ __launch_bounds__(64) void gen_tangent_kernel(GenArgs g, TanArgs ta, T* ke) {
  constexpr int DIM = MS == MS_NH ? 9 : 6;
  typedef typename Acc4<T>::type acc_t;
  __shared__ T s_xe[8][3];
  __shared__ T s_g[8][8][3];          // [point][node][direction]
  __shared__ T s_D[8][DIM * DIM];     // w detJ times the tangent moduli of each point
  const int l = threadIdx.x;
  const int pq = l >> 3, pa = l & 7;  // staging role: point, node
  const int64_t ne = ta.n_el;
  for (int64_t e = blockIdx.x; e < ne; e += gridDim.x) {
    if (l < 24) {
      const int a = l / 3, i = l % 3;
      const int node = g.conn[(int64_t)a * ne + e];
      s_xe[a][i] = static_cast<const T*>(g.coords)[(int64_t)i * g.n_nodes + node];
    }
    __syncthreads();
    {
      T gr[8][3];
      const T wdet = phys_grad<T>(s_xe, pq, gr);
#pragma unroll
      for (int a = 0; a < 8; ++a)  // (compile-time register index; lane pa keeps node pa)
        if (a == pa)
#pragma unroll
          for (int j = 0; j < 3; ++j) s_g[pq][a][j] = gr[a][j];
      QpTangent<T> t;
      load_qp_tangent<T, MS>(ta, e, pq, t);
      // every lane forms all entries of its point's moduli with compile-time indices (no
      // dynamic indexing of the per-point data) and stores every 8th one
      if (DIM == 6) {
        // D = lp 1 x 1 + 2 mp I_sym - beta N x N, engineering shear strains, tensor stress
#pragma unroll
        for (int m = 0; m < 36; ++m) {
          const int r = m / 6, c = m % 6;
          const T v = (r < 3 && c < 3 ? t.lp : T(0)) + (r == c ? (r < 3 ? 2 * t.mp : t.mp) : T(0)) -
                      t.beta * t.N[r] * t.N[c];
          if ((m & 7) == pa) s_D[pq][m] = wdet * v;
        }
      } else if (t.kind == 1) {
        // A_iJkL = mu d_ik d_JL + (mu - lam ln J) F^-1_Jk F^-1_Li + lam F^-1_Ji F^-1_Lk, F^-1_Jk = FiT[k][J]
        const T cc = t.mu - t.lam * t.lnJ;
#pragma unroll
        for (int m = 0; m < 81; ++m) {
          const int r = m / 9, c = m % 9;
          const int i = r / 3, J = r % 3, k = c / 3, L = c % 3;
          const T v = (i == k && J == L ? t.mu : T(0)) + cc * t.FiT[k][J] * t.FiT[i][L] +
                      t.lam * t.FiT[i][J] * t.FiT[k][L];
          if ((m & 7) == pa) s_D[pq][m] = wdet * v;
        }
      } else {
        // small-strain phase of a finite-strain problem, in gradient form:
        // A_iJkL = lp d_iJ d_kL + mp (d_ik d_JL + d_iL d_Jk) - beta N_iJ N_kL
        const T Nt[3][3] = {{t.N[0], t.N[5], t.N[4]}, {t.N[5], t.N[1], t.N[3]}, {t.N[4], t.N[3], t.N[2]}};
#pragma unroll
        for (int m = 0; m < 81; ++m) {
          const int r = m / 9, c = m % 9;
          const int i = r / 3, J = r % 3, k = c / 3, L = c % 3;
          const T v = (i == J && k == L ? t.lp : T(0)) +
                      t.mp * ((i == k && J == L ? T(1) : T(0)) + (i == L && J == k ? T(1) : T(0))) -
                      t.beta * Nt[i][J] * Nt[k][L];
          if ((m & 7) == pa) s_D[pq][m] = wdet * v;
        }
      }
    }
    __syncthreads();
    acc_t c00 = {0, 0, 0, 0}, c01 = {0, 0, 0, 0}, c11 = {0, 0, 0, 0};
    const int r16 = l & 15;
    const int ra = r16 / 3, ri = r16 % 3;                 // tile 0 row / column (node, component)
    const int rb = (16 + r16) / 3, rk = (16 + r16) % 3;   // tile 1 (valid for r16 < 8)
    const bool t1 = r16 < 8;
    const VoigtCol va = voigt_col(ri), vb = voigt_col(rk);
    // contraction index ordered row-major over (m, point): k-step s covers row m = s / 2 of the
    // points 4 (s % 2) + l / 16, so m is the same on every lane of a step (compile time)
    auto step = [&](auto mc, int half) {
      constexpr int M = decltype(mc)::value;
      const int qp = 4 * half + (l >> 4);
      const T* Dq = s_D[qp];
      const T a0 = g_entry<T, DIM, M>(ri, s_g[qp][ra]);
      const T a1 = t1 ? g_entry<T, DIM, M>(rk, s_g[qp][rb]) : T(0);
      const T b0 = dg_entry<T, DIM, M>(Dq, ri, va, s_g[qp][ra]);
      const T b1 = t1 ? dg_entry<T, DIM, M>(Dq, rk, vb, s_g[qp][rb]) : T(0);
      c00 = mfma16(a0, b0, c00);
      c01 = mfma16(a0, b1, c01);
      c11 = mfma16(a1, b1, c11);
    };
    static_for<DIM>([&](auto mc) {
      step(mc, 0);
      step(mc, 1);
    });
    T* K = ke + e * 576;
    const int col = l & 15;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = mfma_row<T>(l, r);
      // tile (0,0): rows / columns 0..15
      {
        const int ar = row / 3, ir = row % 3, bc = col / 3, kc = col % 3;
        K[(ar * 8 + bc) * 9 + ir * 3 + kc] = c00[r];
      }
      // tile (0,1): rows 0..15, columns 16..23, and its mirror
      if (col < 8) {
        const int ar = row / 3, ir = row % 3, bc = (16 + col) / 3, kc = (16 + col) % 3;
        K[(ar * 8 + bc) * 9 + ir * 3 + kc] = c01[r];
        K[(bc * 8 + ar) * 9 + kc * 3 + ir] = c01[r];
      }
      // tile (1,1): rows / columns 16..23
      if (row < 8 && col < 8) {
        const int ar = (16 + row) / 3, ir = (16 + row) % 3, bc = (16 + col) / 3, kc = (16 + col) % 3;
        K[(ar * 8 + bc) * 9 + ir * 3 + kc] = c11[r];
      }
    }
    __syncthreads();  // LDS reused by the next element
  }
}

// CSR values: one lane per node pair, its run of element blocks summed in sorted order.
// Row (a, i) of the pair (a, b) at position k of a's row: value index 9 ptr[a] + 3 i deg(a) + 3 k + c.
template <typename T>
__global__ __launch_bounds__(VBLOCK) void gen_assemble_kernel(int64_t n_pairs, const int32_t* __restrict__ adj_ptr,
                                                              const int32_t* __restrict__ adj,
                                                              const int32_t* __restrict__ pair_row,
                                                              const int32_t* __restrict__ src_ptr,
                                                              const int32_t* __restrict__ src,
                                                              const T* __restrict__ ke, const uint8_t* mask,
                                                              int apply_bc, T* __restrict__ vals) {
  for (int64_t p = (int64_t)blockIdx.x * VBLOCK + threadIdx.x; p < n_pairs; p += (int64_t)gridDim.x * VBLOCK) {
    T acc[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) acc[j] = 0;
    const int s0 = src_ptr[p], s1 = src_ptr[p + 1];
    for (int s = s0; s < s1; ++s) {
      const int code = src[s];  // element * 64 + local row node * 8 + local column node
      const T* blk = ke + (int64_t)(code >> 6) * 576 + (code & 63) * 9;
#pragma unroll
      for (int j = 0; j < 9; ++j) acc[j] += blk[j];
    }
    const int a = pair_row[p], b = adj[p];
    const int base = adj_ptr[a], deg = adj_ptr[a + 1] - base;
    const int64_t k = p - base;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int64_t rdof = 3 * (int64_t)a + i;
      const int64_t pos = 9 * (int64_t)base + 3 * (int64_t)i * deg + 3 * k;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int64_t cdof = 3 * (int64_t)b + c;
        T v = acc[3 * i + c];
        if (apply_bc && mask && (mask[rdof] || mask[cdof])) v = (rdof == cdof) ? T(1) : T(0);
        vals[pos + c] = v;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// symbolic assembly: node-pair pattern by sorting the element pairs

// COO entries per row node: 8 per element that contains it.
__global__ void sym_count_kernel(int64_t ne, const int32_t* conn, int32_t* cnt) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 8 * ne; i += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(cnt + conn[i], 8);
}

// Exclusive scan of int32 in tiles of 2048 (8 per lane); tile totals to sums.
constexpr int SCAN_TILE = 2048;
__global__ __launch_bounds__(256) void scan_tile_kernel(const int32_t* in, int32_t* out, int64_t n, int32_t* sums) {
  __shared__ int32_t sh[256];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + 8 * threadIdx.x;
  int32_t v[8], run = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    v[j] = base + j < n ? in[base + j] : 0;
    run += v[j];
  }
  sh[threadIdx.x] = run;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {  // inclusive Hillis-Steele scan of the lane totals
    const int32_t t = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  int32_t acc = sh[threadIdx.x] - run;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    if (base + j < n) out[base + j] = acc;
    acc += v[j];
  }
  if (threadIdx.x == 255) sums[blockIdx.x] = sh[255];
}

__global__ void scan_add_kernel(int32_t* out, int64_t n, const int32_t* offs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += offs[i / SCAN_TILE];
}

__global__ void scan_total_kernel(int32_t* dst, const int32_t* src) { *dst = *src; }

// out[0..n) = exclusive scan of in, out[n] = total; tmp holds at least gen_scan_tmp_words(n) int32.
int64_t gen_scan_tmp_words(int64_t n) {
  int64_t w = 0;
  for (int64_t m = n; m > 1;) {
    m = (m + SCAN_TILE - 1) / SCAN_TILE;
    w += 2 * (m + 1);
  }
  return w + 2;
}

static hipError_t scan_exclusive(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp, hipStream_t s) {
  const int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
  int32_t* sums = tmp;
  int32_t* offs = tmp + tiles + 1;
  hipLaunchKernelGGL(scan_tile_kernel, dim3((unsigned)std::max<int64_t>(tiles, 1)), dim3(256), 0, s, in, out, n, sums);
  if (tiles > 1) {
    hipError_t e = scan_exclusive(sums, offs, tiles, offs + tiles + 1, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_add_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n, offs);
    // total = offs[tiles] (the scan of the tile totals, one past its end)
    hipLaunchKernelGGL(scan_total_kernel, dim3(1), dim3(1), 0, s, out + n, offs + tiles);
  } else {
    hipLaunchKernelGGL(scan_total_kernel, dim3(1), dim3(1), 0, s, out + n, sums);
  }
  return hipGetLastError();
}

// Scatter every element's 64 node pairs into its row node's bucket: column node and the
// element code e * 64 + a * 8 + b (order inside a bucket is arbitrary; the row sort fixes it).
__global__ void sym_fill_kernel(int64_t ne, const int32_t* conn, int32_t* cursor, int32_t* col, int32_t* code) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 8 * ne; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i % ne;
    const int a = (int)(i / ne);
    const int pos = atomicAdd(cursor + conn[i], 8);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      col[pos + b] = conn[(int64_t)b * ne + e];
      code[pos + b] = (int32_t)(e * 64 + a * 8 + b);
    }
  }
}

// One wave per row: sort the row's bucket by the key (column, code) (all keys distinct: the
// code names the entry) by ranking, write it back in order and count the distinct columns.
constexpr int SYM_MAXROW = 1024;  // COO entries per row node (128 elements sharing a node)
__global__ __launch_bounds__(64) void sym_row_sort_kernel(int64_t n_nodes, const int32_t* ptr, int32_t* col,
                                                          int32_t* code, int32_t* deg) {
  __shared__ long long key[SYM_MAXROW];
  const int l = threadIdx.x;
  for (int64_t r = blockIdx.x; r < n_nodes; r += gridDim.x) {
    const int b = ptr[r], len = ptr[r + 1] - b;
    for (int j = l; j < len; j += 64) key[j] = ((long long)col[b + j] << 32) | (unsigned)code[b + j];
    __syncthreads();
    for (int j = l; j < len; j += 64) {
      const long long kj = key[j];
      int rank = 0;
      for (int i = 0; i < len; ++i) rank += key[i] < kj;
      col[b + rank] = (int32_t)(kj >> 32);
      code[b + rank] = (int32_t)(kj & 0xffffffffll);
    }
    __syncthreads();
    // distinct columns: count run heads of the sorted keys (sorted order = rank order)
    int heads = 0;
    for (int j = l; j < len; j += 64) {
      const long long kj = key[j];
      // kj is a run head when no key with the same column sorts before it
      bool head = true;
      for (int i = 0; i < len; ++i)
        if ((key[i] >> 32) == (kj >> 32) && key[i] < kj) {
          head = false;
          break;
        }
      heads += head;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) heads += __shfl_down(heads, off, 64);
    if (l == 0) deg[r] = heads;
    __syncthreads();
  }
}

// Pair arrays from the sorted buckets: for each run head at sorted position j of row r, its pair
// index is adj_ptr[r] + (heads before j); it records the column node, the row node and where
// its run starts in the sorted code list.
__global__ __launch_bounds__(64) void sym_pairs_kernel(int64_t n_nodes, const int32_t* ptr, const int32_t* col,
                                                       const int32_t* adj_ptr, int32_t* adj, int32_t* pair_row,
                                                       int32_t* src_ptr) {
  const int l = threadIdx.x;
  for (int64_t r = blockIdx.x; r < n_nodes; r += gridDim.x) {
    const int b = ptr[r], len = ptr[r + 1] - b;
    int run = adj_ptr[r];
    for (int j0 = 0; j0 < len; j0 += 64) {
      const int j = j0 + l;
      const bool head = j < len && (j == 0 || col[b + j] != col[b + j - 1]);
      const unsigned long long m = __ballot(head);
      const int before = __popcll(m & ((1ull << l) - 1ull));
      if (head) {
        const int pidx = run + before;
        adj[pidx] = col[b + j];
        pair_row[pidx] = (int32_t)r;
        src_ptr[pidx] = b + j;
      }
      run += __popcll(m);
    }
  }
}

__global__ void sym_last_kernel(int32_t* src_ptr, int64_t n_pairs, int32_t total) { src_ptr[n_pairs] = total; }

// CSR indices of the dof-level matrix: 3 x 3 entries per node pair.
__global__ void gen_csr_pattern_kernel(int64_t n_pairs, int64_t n_nodes, const int32_t* adj_ptr, const int32_t* adj,
                                       const int32_t* pair_row, int32_t* row_ptr, int32_t* col_idx) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n_pairs; p += (int64_t)gridDim.x * blockDim.x) {
    const int a = pair_row[p], b = adj[p];
    const int base = adj_ptr[a], deg = adj_ptr[a + 1] - base;
    const int64_t k = p - base;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int64_t pos = 9 * (int64_t)base + 3 * (int64_t)i * deg;
      if (k == 0) row_ptr[3 * (int64_t)a + i] = (int32_t)pos;
#pragma unroll
      for (int c = 0; c < 3; ++c) col_idx[pos + 3 * k + c] = 3 * b + c;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) row_ptr[3 * n_nodes] = (int32_t)(9 * n_pairs);
}

// ---------------------------------------------------------------------------
// geometry check (every Gauss point det J > 0) and the mesh volume sum_q w detJ

template <typename T>
__global__ __launch_bounds__(GBLOCK) void gen_volume_kernel(GenArgs g, int64_t ne, double* vol, int* bad) {
  __shared__ T s_c[GEL][8][3];
  __shared__ double sh[GBLOCK / 64];
  const int tid = threadIdx.x, el = tid >> 3, q = tid & 7;
  const int64_t e = (int64_t)blockIdx.x * GEL + el;
  const bool valid = e < ne;
  int node = 0;
  if (valid) node = g.conn[(int64_t)q * ne + e];
#pragma unroll
  for (int c = 0; c < 3; ++c) s_c[el][q][c] = valid ? static_cast<const T*>(g.coords)[(int64_t)c * g.n_nodes + node] : T(0);
  __syncthreads();
  double v = 0;
  if (valid) {
    T gr[8][3];
    const T det = phys_grad<T>(s_c[el], q, gr);
    if (!(det > T(0))) atomicOr(bad, 1);
    v = (double)det;
  }
  v = block_sum(v, sh);
  if (threadIdx.x == 0) atomic_add(vol, v);
}

// u[3 node + c] = (eps . x_node)_c on constrained dofs; free dofs kept or zeroed.
template <typename T>
__global__ void gen_lift_kernel(int64_t n_nodes, const T* coords, const uint8_t* mask, T* u, int zero_free, double e00,
                                double e01, double e02, double e10, double e11, double e12, double e20, double e21,
                                double e22) {
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < 3 * n_nodes; d += (int64_t)gridDim.x * blockDim.x) {
    if (mask && mask[d]) {
      const int64_t P = d / 3;
      const int c = (int)(d % 3);
      const double x = coords[P], y = coords[n_nodes + P], z = coords[2 * n_nodes + P];
      const double v = c == 0 ? e00 * x + e01 * y + e02 * z : (c == 1 ? e10 * x + e11 * y + e12 * z : e20 * x + e21 * y + e22 * z);
      u[d] = T(v);
    } else if (zero_free) {
      u[d] = T(0);
    }
  }
}

// int32 node ids in range?  (bad |= 1 otherwise)
__global__ void gen_conn_check_kernel(int64_t n, const int32_t* conn, int64_t n_nodes, int* bad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (conn[i] < 0 || conn[i] >= n_nodes) atomicOr(bad, 1);
}

template <typename T> __global__ void gen_fill_kernel(T* x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = T(0);
}

template <typename S, typename D> __global__ void gen_cvt_kernel(const S* a, D* b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = D(a[i]);
}

template <typename T> __global__ void gen_copy_kernel(const T* a, T* b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

// ---------------------------------------------------------------------------
// launchers

static unsigned vblocks(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)); }
static unsigned eblocks(int64_t ne) { return (unsigned)std::max<int64_t>(1, (ne + GEL - 1) / GEL); }

hipError_t gen_setup(fe_problem* p, const double* coords, const int32_t* conn, hipStream_t s) {
  const int64_t ne = p->n_el, nn = p->n_nodes;
  int* bad = p->flags;
  hipError_t e;
  if ((e = hipMemsetAsync(bad, 0, sizeof(int), s)) != hipSuccess) return e;
  hipLaunchKernelGGL(gen_conn_check_kernel, dim3(vblocks(8 * ne)), dim3(256), 0, s, 8 * ne, conn, nn, bad);
  if (p->prec == FE_F64)
    hipLaunchKernelGGL((gen_cvt_kernel<double, double>), dim3(vblocks(3 * nn)), dim3(256), 0, s, coords,
                       (double*)p->coords, 3 * nn);
  else
    hipLaunchKernelGGL((gen_cvt_kernel<double, float>), dim3(vblocks(3 * nn)), dim3(256), 0, s, coords,
                       (float*)p->coords, 3 * nn);
  hipLaunchKernelGGL(gen_copy_kernel<int32_t>, dim3(vblocks(8 * ne)), dim3(256), 0, s, conn, p->conn, 8 * ne);
  return hipGetLastError();
}

hipError_t gen_check_geometry(const fe_problem* p, double* vol_dev, int* bad, hipStream_t s) {
  const GenArgs g = gen_args(p);
  if (p->prec == FE_F64)
    hipLaunchKernelGGL(gen_volume_kernel<double>, dim3(eblocks(p->n_el)), dim3(GBLOCK), 0, s, g, p->n_el, vol_dev, bad);
  else
    hipLaunchKernelGGL(gen_volume_kernel<float>, dim3(eblocks(p->n_el)), dim3(GBLOCK), 0, s, g, p->n_el, vol_dev, bad);
  return hipGetLastError();
}

// Node-pair pattern: counts, bucket offsets, buckets, row sorts, degrees, pair arrays.
// Returns the number of pairs in *n_pairs (synchronises).  tmp: gen_scan_tmp_words(n_nodes) words.
hipError_t gen_symbolic(fe_problem* p, int32_t* cnt, int32_t* coo_ptr, int32_t* cursor, int32_t* tmp, hipStream_t s,
                        int64_t* n_pairs, int* max_row) {
  const int64_t ne = p->n_el, nn = p->n_nodes;
  hipError_t e;
  if ((e = hipMemsetAsync(cnt, 0, sizeof(int32_t) * nn, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(sym_count_kernel, dim3(vblocks(8 * ne)), dim3(256), 0, s, ne, p->conn, cnt);
  if ((e = scan_exclusive(cnt, coo_ptr, nn, tmp, s)) != hipSuccess) return e;
  // longest bucket (host check against the row-sort capacity)
  std::vector<int32_t> h(nn + 1);
  if ((e = hipMemcpyAsync(h.data(), coo_ptr, sizeof(int32_t) * (nn + 1), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  int mx = 0;
  for (int64_t i = 0; i < nn; ++i) mx = std::max(mx, h[i + 1] - h[i]);
  *max_row = mx;
  if (mx > SYM_MAXROW) return hipSuccess;  // caller reports
  if ((e = hipMemcpyAsync(cursor, coo_ptr, sizeof(int32_t) * nn, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(sym_fill_kernel, dim3(vblocks(8 * ne)), dim3(256), 0, s, ne, p->conn, cursor, p->gen_col,
                     p->pair_src);
  const unsigned rows_grid = (unsigned)std::min<int64_t>(nn, 65536);
  hipLaunchKernelGGL(sym_row_sort_kernel, dim3(rows_grid), dim3(64), 0, s, nn, coo_ptr, p->gen_col, p->pair_src, cnt);
  if ((e = scan_exclusive(cnt, p->adj_ptr, nn, tmp, s)) != hipSuccess) return e;
  int32_t np = 0;
  if ((e = hipMemcpyAsync(&np, p->adj_ptr + nn, sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  *n_pairs = np;
  return hipSuccess;
}

hipError_t gen_pairs(fe_problem* p, const int32_t* coo_ptr, hipStream_t s) {
  const int64_t nn = p->n_nodes;
  const unsigned rows_grid = (unsigned)std::min<int64_t>(nn, 65536);
  hipLaunchKernelGGL(sym_pairs_kernel, dim3(rows_grid), dim3(64), 0, s, nn, coo_ptr, p->gen_col, p->adj_ptr, p->adj,
                     p->pair_row, p->pair_src_ptr);
  hipLaunchKernelGGL(sym_last_kernel, dim3(1), dim3(1), 0, s, p->pair_src_ptr, p->n_pairs, (int32_t)(64 * p->n_el));
  return hipGetLastError();
}

hipError_t gen_csr_pattern(const fe_problem* p, int32_t* row_ptr, int32_t* col_idx, hipStream_t s) {
  hipLaunchKernelGGL(gen_csr_pattern_kernel, dim3(vblocks(p->n_pairs)), dim3(256), 0, s, p->n_pairs, p->n_nodes,
                     p->adj_ptr, p->adj, p->pair_row, row_ptr, col_idx);
  return hipGetLastError();
}

template <typename T, int OP>
static hipError_t gen_elem_t(const fe_problem* p, const ElemArgs& a, const int* stop, hipStream_t s) {
  const GenArgs g = gen_args(p);
  const dim3 grid(eblocks(p->n_el)), block(GBLOCK);
  switch (p->model_set) {
    case MS_J2: timed_launch((gen_elem_kernel<T, OP, MS_J2>), grid, block, 0, s, g, a, stop); break;
    case MS_NH: timed_launch((gen_elem_kernel<T, OP, MS_NH>), grid, block, 0, s, g, a, stop); break;
    default: timed_launch((gen_elem_kernel<T, OP, MS_LINEAR>), grid, block, 0, s, g, a, stop);
  }
  if (OP == OP_APPLY && a.apply_bc && p->mask && a.y)
    hipLaunchKernelGGL(gen_bc_kernel<T>, dim3(vblocks(p->n_dof)), dim3(VBLOCK), 0, s, p->n_dof, p->mask,
                       (const T*)a.x, (T*)a.y, stop, (double*)nullptr);
  return hipGetLastError();
}

hipError_t gen_launch_elem(const fe_problem* p, int op, const ElemArgs& a, const int* stop, hipStream_t s) {
  if (op == OP_CG_APPLY) return hipErrorInvalidValue;  // general meshes run the unfused CG
  if (p->prec == FE_F64) {
    if (op == OP_RESID) return gen_elem_t<double, OP_RESID>(p, a, stop, s);
    if (op == OP_APPLY) return gen_elem_t<double, OP_APPLY>(p, a, stop, s);
    return gen_elem_t<double, OP_VJP>(p, a, stop, s);
  }
  if (op == OP_RESID) return gen_elem_t<float, OP_RESID>(p, a, stop, s);
  if (op == OP_APPLY) return gen_elem_t<float, OP_APPLY>(p, a, stop, s);
  return gen_elem_t<float, OP_VJP>(p, a, stop, s);
}

// CG operator on a general mesh: q = A p (q zeroed by the previous update), then the
// constrained rows and the per-workgroup partials of p.q.
hipError_t gen_cg_operator(const fe_problem* p, hipStream_t s) {
  ElemArgs a{};
  a.n_el = p->n_el;
  a.phase = p->phase;
  a.scale = p->scale;
  a.mask = p->mask;
  a.tangent = p->tangent;
  a.flags = p->flags;
  a.mat = p->mat;
  a.x = p->w_p;
  a.y = p->w_q;
  a.apply_bc = 1;
  const int* stop = &p->ctrl->status;
  const GenArgs g = gen_args(p);
  const dim3 grid(eblocks(p->n_el)), block(GBLOCK);
  if (p->prec == FE_F64) {
    switch (p->model_set) {
      case MS_J2: timed_launch((gen_elem_kernel<double, OP_APPLY, MS_J2>), grid, block, 0, s, g, a, stop); break;
      case MS_NH: timed_launch((gen_elem_kernel<double, OP_APPLY, MS_NH>), grid, block, 0, s, g, a, stop); break;
      default: timed_launch((gen_elem_kernel<double, OP_APPLY, MS_LINEAR>), grid, block, 0, s, g, a, stop);
    }
    hipLaunchKernelGGL(gen_bc_kernel<double>, dim3(GEN_CG_GRID), dim3(VBLOCK), 0, s, p->n_dof, p->mask,
                       (const double*)p->w_p, (double*)p->w_q, stop, p->partials);
  } else {
    switch (p->model_set) {
      case MS_J2: timed_launch((gen_elem_kernel<float, OP_APPLY, MS_J2>), grid, block, 0, s, g, a, stop); break;
      case MS_NH: timed_launch((gen_elem_kernel<float, OP_APPLY, MS_NH>), grid, block, 0, s, g, a, stop); break;
      default: timed_launch((gen_elem_kernel<float, OP_APPLY, MS_LINEAR>), grid, block, 0, s, g, a, stop);
    }
    hipLaunchKernelGGL(gen_bc_kernel<float>, dim3(GEN_CG_GRID), dim3(VBLOCK), 0, s, p->n_dof, p->mask,
                       (const float*)p->w_p, (float*)p->w_q, stop, p->partials);
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t gen_diag_t(const fe_problem* p, T* d, int nb, int apply_bc, const TanArgs& ta, hipStream_t s) {
  const GenArgs g = gen_args(p);
  const int64_t n = nb == 3 ? p->n_dof : 6 * p->n_nodes;
  hipLaunchKernelGGL(gen_fill_kernel<T>, dim3(vblocks(n)), dim3(256), 0, s, d, n);
  const dim3 grid(eblocks(p->n_el)), block(GBLOCK);
  const int skip = apply_bc && p->mask ? 1 : 0;
  if (nb == 3) {
    switch (p->model_set) {
      case MS_J2: hipLaunchKernelGGL((gen_diag_kernel<T, MS_J2, 3>), grid, block, 0, s, g, ta, d, skip); break;
      case MS_NH: hipLaunchKernelGGL((gen_diag_kernel<T, MS_NH, 3>), grid, block, 0, s, g, ta, d, skip); break;
      default: hipLaunchKernelGGL((gen_diag_kernel<T, MS_LINEAR, 3>), grid, block, 0, s, g, ta, d, skip);
    }
    if (skip) hipLaunchKernelGGL(gen_mask_one_kernel<T>, dim3(vblocks(p->n_dof)), dim3(256), 0, s, p->n_dof, p->mask, d);
  } else {
    switch (p->model_set) {
      case MS_J2: hipLaunchKernelGGL((gen_diag_kernel<T, MS_J2, 6>), grid, block, 0, s, g, ta, d, 0); break;
      case MS_NH: hipLaunchKernelGGL((gen_diag_kernel<T, MS_NH, 6>), grid, block, 0, s, g, ta, d, 0); break;
      default: hipLaunchKernelGGL((gen_diag_kernel<T, MS_LINEAR, 6>), grid, block, 0, s, g, ta, d, 0);
    }
  }
  return hipGetLastError();
}

hipError_t gen_diag(const fe_problem* p, void* d, int nb, int apply_bc, const TanArgs& ta, hipStream_t s) {
  return p->prec == FE_F64 ? gen_diag_t(p, (double*)d, nb, apply_bc, ta, s) : gen_diag_t(p, (float*)d, nb, apply_bc, ta, s);
}

template <typename T>
static hipError_t gen_tangent_t(const fe_problem* p, T* vals, int apply_bc, const TanArgs& ta, hipStream_t s) {
  const GenArgs g = gen_args(p);
  T* ke = static_cast<T*>(p->ke);
  const unsigned grid = (unsigned)std::min<int64_t>(p->n_el, 8192);
  switch (p->model_set) {
    case MS_J2: timed_launch((gen_tangent_kernel<T, MS_J2>), dim3(grid), dim3(64), 0, s, g, ta, ke); break;
    case MS_NH: timed_launch((gen_tangent_kernel<T, MS_NH>), dim3(grid), dim3(64), 0, s, g, ta, ke); break;
    default: timed_launch((gen_tangent_kernel<T, MS_LINEAR>), dim3(grid), dim3(64), 0, s, g, ta, ke);
  }
  hipLaunchKernelGGL(gen_assemble_kernel<T>, dim3(vblocks(p->n_pairs)), dim3(VBLOCK), 0, s, p->n_pairs, p->adj_ptr,
                     p->adj, p->pair_row, p->pair_src_ptr, p->pair_src, (const T*)ke, p->mask, apply_bc, vals);
  return hipGetLastError();
}

hipError_t gen_tangent(const fe_problem* p, void* vals, int apply_bc, const TanArgs& ta, hipStream_t s) {
  return p->prec == FE_F64 ? gen_tangent_t(p, (double*)vals, apply_bc, ta, s)
                           : gen_tangent_t(p, (float*)vals, apply_bc, ta, s);
}

hipError_t gen_lift(const fe_problem* p, const double* E, void* u, int zero_free, hipStream_t s) {
  const dim3 gr(vblocks(p->n_dof)), b(256);
  if (p->prec == FE_F64)
    hipLaunchKernelGGL(gen_lift_kernel<double>, gr, b, 0, s, p->n_nodes, (const double*)p->coords, p->mask, (double*)u,
                       zero_free, E[0], E[1], E[2], E[3], E[4], E[5], E[6], E[7], E[8]);
  else
    hipLaunchKernelGGL(gen_lift_kernel<float>, gr, b, 0, s, p->n_nodes, (const float*)p->coords, p->mask, (float*)u,
                       zero_free, E[0], E[1], E[2], E[3], E[4], E[5], E[6], E[7], E[8]);
  return hipGetLastError();
}

hipError_t gen_copy_state(const fe_problem* p, const void* src, void* dst, int64_t n, hipStream_t s) {
  if (p->prec == FE_F64)
    hipLaunchKernelGGL(gen_copy_kernel<double>, dim3(vblocks(n)), dim3(256), 0, s, (const double*)src, (double*)dst, n);
  else
    hipLaunchKernelGGL(gen_copy_kernel<float>, dim3(vblocks(n)), dim3(256), 0, s, (const float*)src, (float*)dst, n);
  return hipGetLastError();
}

}  // namespace fe
