// HIP kernels of libfe for gfx950 (MI355X).
//
// Element kernels work on bricks of TX x TY x TZ = 16 x 4 x 4 elements, one
// element per lane, 256 lanes per workgroup:
//   1. the brick's (TX+1)(TY+1)(TZ+1) nodal values are staged in LDS with
//      coalesced row loads (each node is then read from LDS by up to 8 lanes);
//   2. each lane forms the displacement gradient at its 8 Gauss points by sum
//      factorisation of the trilinear basis (the x-derivative at a Gauss point
//      only depends on its (y,z) position, so 9 bilinear interpolations of
//      nodal differences give all 72 gradient entries);
//   3. the constitutive law turns each gradient into a stress, which is pushed
//      back to the nodes by the transposed factorisation;
//   4. nodal forces are summed into LDS in 8 colour passes (elements of equal
//      index parity share no node, so a pass has no conflicts and the LDS sum is
//      deterministic); nodes owned by the brick alone are stored, nodes on the
//      brick's faces are added with hardware FP atomics.
// Bricks are numbered so that consecutive bricks land on one XCD (workgroups
// are dealt round-robin over the 8 XCDs), keeping shared face nodes in one L2.
#include "fe_internal.hpp"

namespace fe {

constexpr int TX = 16, TY = 4, TZ = 4;
constexpr int NX = TX + 1, NY = TY + 1, NZ = TZ + 1, NN = NX * NY * NZ;
constexpr int EBLOCK = TX * TY * TZ;
static_assert(EBLOCK == 256, "one element per lane");

// Linear 1-D basis at the Gauss points +-1/sqrt(3): phi_i(g_p) = GA if i == p else GB.
constexpr double GA = 0.78867513459481288225;
constexpr double GB = 0.21132486540518711775;
constexpr double SQRT1_5 = 1.22474487139158904910;

constexpr int VBLOCK = 256;     // vector kernels
constexpr int VGRID_MAX = 1024; // vector kernels: blocks (== partial-sum slots)

// ---------------------------------------------------------------------------
// small helpers

template <typename T> __device__ __forceinline__ void atomic_add(T* p, T v) { unsafeAtomicAdd(p, v); }

// Block sum of a double over 256 lanes; the result is valid in lane 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < VBLOCK / 64; ++i) r += sh[i];
  return r;
}

// Last-block-done: every block publishes partials, the last one to arrive
// reduces them in block order (deterministic) and resets the counter.
__device__ __forceinline__ bool arrive_last(unsigned int* counter) {
  __shared__ bool last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = (atomicAdd(counter, 1u) == gridDim.x - 1);
  __syncthreads();
  if (last) __threadfence();
  return last;
}

__device__ __forceinline__ double load_coherent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum of partials[0..nb) in fixed order by the whole block; valid in lane 0.
__device__ __forceinline__ double reduce_partials(const double* partials, int nb, double* sh) {
  double v = 0;
  for (int i = threadIdx.x; i < nb; i += VBLOCK) v += load_coherent(partials + i);
  return block_sum(v, sh);
}

__device__ __forceinline__ bool finite(double v) { return v == v && v - v == 0.0; }

// CG step length from the block partials of p.Ap (last block): alpha = rz / pAp.
__device__ __forceinline__ void cg_alpha_arrive(double v, CgCtrl* ctrl, double* partials, unsigned int* counter,
                                                double* sh) {
  v = block_sum(v, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = v;
  if (arrive_last(counter)) {
    const double pq = reduce_partials(partials, gridDim.x, sh);
    if (threadIdx.x == 0) {
      ctrl->pq = pq;
      if (!finite(pq))
        ctrl->status = FE_ERR_NONFINITE;
      else if (pq <= 0.0)
        ctrl->status = FE_ERR_BREAKDOWN;
      else
        ctrl->alpha = ctrl->rz / pq;
      *counter = 0;
    }
  }
}

// G[r][q] = sum_{k,j} M[r][k] M[q][j] D[k][j] with M = [[GA,GB],[GB,GA]] (M symmetric,
// so the same map also pushes Gauss-point values back to the nodes).
template <typename T> __device__ __forceinline__ void interp2(const T D[2][2], T G[2][2]) {
  const T a = T(GA), b = T(GB);
  const T t00 = a * D[0][0] + b * D[0][1];
  const T t01 = b * D[0][0] + a * D[0][1];
  const T t10 = a * D[1][0] + b * D[1][1];
  const T t11 = b * D[1][0] + a * D[1][1];
  G[0][0] = a * t00 + b * t10;
  G[0][1] = a * t01 + b * t11;
  G[1][0] = b * t00 + a * t10;
  G[1][1] = b * t01 + a * t11;
}

// Gradient tables of a nodal field U[k][j][i][c] (node (i,j,k) of the brick element):
// du_c/dx at Gauss point (p,q,r) = Gx[r][q][c], du_c/dy = Gy[r][p][c], du_c/dz = Gz[q][p][c].
template <typename T>
__device__ __forceinline__ void gradients(const T U[2][2][2][3], T inv_h, T Gx[2][2][3], T Gy[2][2][3],
                                          T Gz[2][2][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    T D[2][2], G[2][2];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int j = 0; j < 2; ++j) D[k][j] = U[k][j][1][c] - U[k][j][0][c];
    interp2(D, G);
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int q = 0; q < 2; ++q) Gx[r][q][c] = G[r][q] * inv_h;
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int i = 0; i < 2; ++i) D[k][i] = U[k][1][i][c] - U[k][0][i][c];
    interp2(D, G);
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int p = 0; p < 2; ++p) Gy[r][p][c] = G[r][p] * inv_h;
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < 2; ++i) D[j][i] = U[1][j][i][c] - U[0][j][i][c];
    interp2(D, G);
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int p = 0; p < 2; ++p) Gz[q][p][c] = G[q][p] * inv_h;
  }
}

// Nodal forces F[k][j][i][c] += f * sum over Gauss points of S_cJ dN/dx_J, from the
// per-direction Gauss-point sums Px[r][q][c] (summed over p), Py[r][p][c], Pz[q][p][c].
template <typename T>
__device__ __forceinline__ void push_back(const T Px[2][2][3], const T Py[2][2][3], const T Pz[2][2][3],
                                          T f, T F[2][2][2][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    T D[2][2], G[2][2];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int q = 0; q < 2; ++q) D[r][q] = Px[r][q][c];
    interp2(D, G);  // -> [k][j]
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        F[k][j][1][c] += f * G[k][j];
        F[k][j][0][c] -= f * G[k][j];
      }
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int p = 0; p < 2; ++p) D[r][p] = Py[r][p][c];
    interp2(D, G);  // -> [k][i]
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        F[k][1][i][c] += f * G[k][i];
        F[k][0][i][c] -= f * G[k][i];
      }
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int p = 0; p < 2; ++p) D[q][p] = Pz[q][p][c];
    interp2(D, G);  // -> [j][i]
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        F[1][j][i][c] += f * G[j][i];
        F[0][j][i][c] -= f * G[j][i];
      }
  }
}

// ---------------------------------------------------------------------------
// constitutive laws at one Gauss point; H = displacement gradient H[c][J] = du_c/dx_J,
// S = stress-like tensor S[c][J] whose divergence is the internal force.

// Hooke: S = lam tr(eps) I + 2 mu eps.
template <typename T> __device__ __forceinline__ void hooke(const T H[3][3], T lam, T mu, T S[3][3]) {
  const T tr = H[0][0] + H[1][1] + H[2][2];
  S[0][0] = lam * tr + 2 * mu * H[0][0];
  S[1][1] = lam * tr + 2 * mu * H[1][1];
  S[2][2] = lam * tr + 2 * mu * H[2][2];
  S[1][2] = S[2][1] = mu * (H[1][2] + H[2][1]);
  S[0][2] = S[2][0] = mu * (H[0][2] + H[2][0]);
  S[0][1] = S[1][0] = mu * (H[0][1] + H[1][0]);
}

// J2 radial return (von Mises, linear isotropic hardening) from the converged state
// epn (engineering Voigt) / an.  Writes the stress, the trial state and the compact
// consistent tangent {dgamma/q_trial (-1 when elastic), N_xx, N_yy, N_yz, N_xz, N_xy}.
template <typename T>
__device__ __forceinline__ void j2_update(const T H[3][3], const T epn[6], T an, T K, T G, T sy, T Hh,
                                          T S[3][3], T ep[6], T& al, T tan[6]) {
  const T e00 = H[0][0] - epn[0], e11 = H[1][1] - epn[1], e22 = H[2][2] - epn[2];
  const T e12 = T(0.5) * (H[1][2] + H[2][1] - epn[3]);
  const T e02 = T(0.5) * (H[0][2] + H[2][0] - epn[4]);
  const T e01 = T(0.5) * (H[0][1] + H[1][0] - epn[5]);
  const T tr = e00 + e11 + e22;
  const T p = K * tr;
  const T m = tr / T(3);
  const T g2 = 2 * G;
  T s00 = g2 * (e00 - m), s11 = g2 * (e11 - m), s22 = g2 * (e22 - m);
  T s12 = g2 * e12, s02 = g2 * e02, s01 = g2 * e01;
  const T sn = sqrt(s00 * s00 + s11 * s11 + s22 * s22 + 2 * (s12 * s12 + s02 * s02 + s01 * s01));
  const T q = T(SQRT1_5) * sn;
  const T f = q - (sy + Hh * an);
#pragma unroll
  for (int i = 0; i < 6; ++i) ep[i] = epn[i];
  al = an;
  tan[0] = T(-1);
  tan[1] = tan[2] = tan[3] = tan[4] = tan[5] = 0;
  T theta = 1;
  if (f > 0) {
    const T dg = f / (3 * G + Hh);
    theta = 1 - 3 * G * dg / q;
    const T inv = 1 / sn;
    const T n00 = s00 * inv, n11 = s11 * inv, n22 = s22 * inv, n12 = s12 * inv, n02 = s02 * inv,
            n01 = s01 * inv;
    const T c = T(SQRT1_5) * dg;
    ep[0] += c * n00;
    ep[1] += c * n11;
    ep[2] += c * n22;
    ep[3] += 2 * c * n12;
    ep[4] += 2 * c * n02;
    ep[5] += 2 * c * n01;
    al = an + dg;
    tan[0] = dg / q;
    tan[1] = n00;
    tan[2] = n11;
    tan[3] = n12;
    tan[4] = n02;
    tan[5] = n01;
  }
  S[0][0] = theta * s00 + p;
  S[1][1] = theta * s11 + p;
  S[2][2] = theta * s22 + p;
  S[1][2] = S[2][1] = theta * s12;
  S[0][2] = S[2][0] = theta * s02;
  S[0][1] = S[1][0] = theta * s01;
}

// Compact J2 tangent -> (lam', mu', beta, N): D = lam' 1x1 + 2 mu' I_sym - beta N x N.
template <typename T>
__device__ __forceinline__ void j2_tangent_coeffs(const T tan[6], T K, T G, T Hh, T& lp, T& mp, T& beta,
                                                  T N[6]) {
  const T r = tan[0];
  if (r < 0) {
    mp = G;
    beta = 0;
  } else {
    mp = G * (1 - 3 * G * r);
    beta = 6 * G * G * (1 / (3 * G + Hh) - r);
  }
  lp = K - T(2.0 / 3.0) * mp;
  N[0] = tan[1];
  N[1] = tan[2];
  N[2] = -(tan[1] + tan[2]);
  N[3] = tan[3];
  N[4] = tan[4];
  N[5] = tan[5];
}

// Linearised J2 stress  D : sym(H).
template <typename T>
__device__ __forceinline__ void j2_apply(const T H[3][3], T lp, T mp, T beta, const T N[6], T S[3][3]) {
  const T e12 = T(0.5) * (H[1][2] + H[2][1]);
  const T e02 = T(0.5) * (H[0][2] + H[2][0]);
  const T e01 = T(0.5) * (H[0][1] + H[1][0]);
  const T tr = H[0][0] + H[1][1] + H[2][2];
  const T ne = N[0] * H[0][0] + N[1] * H[1][1] + N[2] * H[2][2] + 2 * (N[3] * e12 + N[4] * e02 + N[5] * e01);
  const T bn = beta * ne;
  S[0][0] = lp * tr + 2 * mp * H[0][0] - bn * N[0];
  S[1][1] = lp * tr + 2 * mp * H[1][1] - bn * N[1];
  S[2][2] = lp * tr + 2 * mp * H[2][2] - bn * N[2];
  S[1][2] = S[2][1] = 2 * mp * e12 - bn * N[3];
  S[0][2] = S[2][0] = 2 * mp * e02 - bn * N[4];
  S[0][1] = S[1][0] = 2 * mp * e01 - bn * N[5];
}

// Neo-Hookean kinematics: F = I + H, J - 1 without cancellation, ln J, F^-T.
// Returns false when J <= 0.
template <typename T>
__device__ __forceinline__ bool nh_kin(const T H[3][3], T FiT[3][3], T& lnJ) {
  const T trH = H[0][0] + H[1][1] + H[2][2];
  T trH2 = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) trH2 += H[i][j] * H[j][i];
  const T detH = H[0][0] * (H[1][1] * H[2][2] - H[1][2] * H[2][1]) -
                 H[0][1] * (H[1][0] * H[2][2] - H[1][2] * H[2][0]) +
                 H[0][2] * (H[1][0] * H[2][1] - H[1][1] * H[2][0]);
  const T jm1 = trH + T(0.5) * (trH * trH - trH2) + detH;
  const T J = 1 + jm1;
  T F[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) F[i][j] = H[i][j] + (i == j ? T(1) : T(0));
  // F^-T = cof(F) / J
  const T ij = 1 / J;
  FiT[0][0] = (F[1][1] * F[2][2] - F[1][2] * F[2][1]) * ij;
  FiT[0][1] = (F[1][2] * F[2][0] - F[1][0] * F[2][2]) * ij;
  FiT[0][2] = (F[1][0] * F[2][1] - F[1][1] * F[2][0]) * ij;
  FiT[1][0] = (F[0][2] * F[2][1] - F[0][1] * F[2][2]) * ij;
  FiT[1][1] = (F[0][0] * F[2][2] - F[0][2] * F[2][0]) * ij;
  FiT[1][2] = (F[0][1] * F[2][0] - F[0][0] * F[2][1]) * ij;
  FiT[2][0] = (F[0][1] * F[1][2] - F[0][2] * F[1][1]) * ij;
  FiT[2][1] = (F[0][2] * F[1][0] - F[0][0] * F[1][2]) * ij;
  FiT[2][2] = (F[0][0] * F[1][1] - F[0][1] * F[1][0]) * ij;
  lnJ = log1p(jm1);
  return J > 0;
}

// First Piola-Kirchhoff stress P = mu (F - F^-T) + lam ln J F^-T.
template <typename T>
__device__ __forceinline__ void nh_stress(const T H[3][3], const T FiT[3][3], T lnJ, T lam, T mu, T S[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) S[i][j] = mu * (H[i][j] + (i == j ? T(1) : T(0)) - FiT[i][j]) + lam * lnJ * FiT[i][j];
}

// dP = mu dH + (mu - lam ln J) (F^-1 dH F^-1)^T + lam tr(F^-1 dH) F^-T.
template <typename T>
__device__ __forceinline__ void nh_apply(const T dH[3][3], const T FiT[3][3], T lnJ, T lam, T mu, T S[3][3]) {
  // A = F^-1 dH  (F^-1[i][k] = FiT[k][i])
  T A[3][3];
  T tr = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      T s = 0;
#pragma unroll
      for (int k = 0; k < 3; ++k) s += FiT[k][i] * dH[k][j];
      A[i][j] = s;
    }
  tr = A[0][0] + A[1][1] + A[2][2];
  const T c = mu - lam * lnJ;
  // (A F^-1)^T [i][j] = (A F^-1)[j][i] = sum_k A[j][k] F^-1[k][i] = sum_k A[j][k] FiT[i][k]
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      T s = 0;
#pragma unroll
      for (int k = 0; k < 3; ++k) s += A[j][k] * FiT[i][k];
      S[i][j] = mu * dH[i][j] + c * s + lam * tr * FiT[i][j];
    }
}

// ---------------------------------------------------------------------------
// element brick kernel

template <typename T, int OP, int MS>
__global__ __launch_bounds__(EBLOCK) void elem_kernel(ElemArgs a, const int* stop) {
  constexpr bool APPLY_LIKE = (OP == OP_APPLY) || (OP == OP_CG_APPLY);
  constexpr bool NEED_L = (OP == OP_VJP) || (APPLY_LIKE && MS == MS_NH);
  __shared__ T s_x[NN * 3];
  __shared__ T s_y[OP == OP_VJP ? 1 : NN * 3];
  __shared__ T s_l[NEED_L ? NN * 3 : 1];
  __shared__ double s_red[6][EBLOCK / 64];

  if (stop && *stop) return;
  const int n = a.n;
  const int ntx = (n + TX - 1) / TX, nty = (n + TY - 1) / TY, ntz = (n + TZ - 1) / TZ;
  const int nb = ntx * nty * ntz;
  const int per = (nb + 7) >> 3;
  const int tile = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (tile >= nb) {
    // padding block of the XCD-aware numbering: still takes part in the p.Ap reduction
    if (OP == OP_CG_APPLY) cg_alpha_arrive(0.0, a.ctrl, a.partials, a.counter, &s_red[0][0]);
    return;
  }
  const int a0 = (tile % ntx) * TX, b0 = ((tile / ntx) % nty) * TY, c0 = (tile / (ntx * nty)) * TZ;
  const int tid = threadIdx.x;
  const T* X = static_cast<const T*>(a.x);
  const T* XL = static_cast<const T*>(a.xlin);
  const T* CR = static_cast<const T*>(a.cg_r);
  const T* CD = static_cast<const T*>(a.cg_dinv);
  const T* CP = static_cast<const T*>(a.cg_pold);
  T* CPN = static_cast<T*>(a.cg_pnew);
  const T cg_beta = (OP == OP_CG_APPLY) ? T(a.ctrl->beta) : T(0);
  const int64_t np1 = n + 1;

  for (int i = tid; i < NN * 3; i += EBLOCK) {
    const int c = i % 3, nd = i / 3;
    const int li = nd % NX, lj = (nd / NX) % NY, lk = nd / (NX * NY);
    const int gi = a0 + li, gj = b0 + lj, gk = c0 + lk;
    T v = 0, vl = 0;
    if (gi <= n && gj <= n && gk <= n) {
      const int64_t dof = 3 * (gi + np1 * (gj + np1 * gk)) + c;
      if (OP == OP_CG_APPLY) {
        // new search direction, formed identically by every brick that touches the node
        v = CD[dof] * CR[dof] + cg_beta * CP[dof];
        if ((min(gi, n - 1) - a0 < TX) && (min(gj, n - 1) - b0 < TY) && (min(gk, n - 1) - c0 < TZ)) CPN[dof] = v;
      } else {
        v = X[dof];
      }
      if (APPLY_LIKE && a.apply_bc && a.mask && a.mask[dof]) v = 0;
      if (NEED_L) vl = XL[dof];
    }
    s_x[i] = v;
    if (OP != OP_VJP) s_y[i] = 0;
    if (NEED_L) s_l[i] = vl;
  }
  __syncthreads();

  const int ex = tid % TX, ey = (tid / TX) % TY, ez = tid / (TX * TY);
  const int ga = a0 + ex, gb = b0 + ey, gc = c0 + ez;
  const bool valid = ga < n && gb < n && gc < n;
  const int64_t e = valid ? (ga + (int64_t)n * (gb + (int64_t)n * gc)) : 0;
  const int64_t ne = a.n_el;
  const T h = T(a.h), inv_h = T(1.0 / a.h);

  T Fo[2][2][2][3];
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) Fo[k][j][i][c] = 0;
  double ssum[6] = {0, 0, 0, 0, 0, 0};

  if (valid) {
    const int ph = a.phase[e];
    const PhaseConst pc = a.mat.ph[ph];
    const T sc = (a.scale && OP != OP_VJP) ? static_cast<const T*>(a.scale)[e] : T(1);
    const T lam = T(pc.lam) * sc, mu = T(pc.mu) * sc;
    const T Kb = T(pc.K) * sc, Gs = T(pc.G) * sc, sy = T(pc.sy), Hh = T(pc.H);

    T U[2][2][2][3];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int c = 0; c < 3; ++c) U[k][j][i][c] = s_x[3 * ((ex + i) + NX * ((ey + j) + NY * (ez + k))) + c];
    T Gx[2][2][3], Gy[2][2][3], Gz[2][2][3];
    gradients(U, inv_h, Gx, Gy, Gz);

    // Neo-Hookean APPLY also needs the gradient at the linearisation point
    T Lx[2][2][3], Ly[2][2][3], Lz[2][2][3];
    if (APPLY_LIKE && MS == MS_NH) {
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int c = 0; c < 3; ++c)
              U[k][j][i][c] = s_l[3 * ((ex + i) + NX * ((ey + j) + NY * (ez + k))) + c];
      gradients(U, inv_h, Lx, Ly, Lz);
    }

    T Px[2][2][3], Py[2][2][3], Pz[2][2][3];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int c = 0; c < 3; ++c) Px[x][y][c] = Py[x][y][c] = Pz[x][y][c] = 0;

    const T* st_in = static_cast<const T*>(a.state_in);
    T* st_out = static_cast<T*>(a.state_out);
    T* tang = static_cast<T*>(a.tangent);

#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          const int qp = p + 2 * q + 4 * r;
          T H[3][3], S[3][3];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            H[c][0] = Gx[r][q][c];
            H[c][1] = Gy[r][p][c];
            H[c][2] = Gz[q][p][c];
          }
          bool done = false;
          if (MS == MS_J2 && pc.model == FE_J2) {
            if (OP == OP_RESID) {
              T epn[6], an = 0, ep[6], al, tn[6];
#pragma unroll
              for (int k = 0; k < 6; ++k) epn[k] = st_in ? st_in[(int64_t)(k * 8 + qp) * ne + e] : T(0);
              if (st_in) an = st_in[(int64_t)(6 * 8 + qp) * ne + e];
              j2_update(H, epn, an, Kb, Gs, sy, Hh, S, ep, al, tn);
              if (st_out) {
#pragma unroll
                for (int k = 0; k < 6; ++k) st_out[(int64_t)(k * 8 + qp) * ne + e] = ep[k];
                st_out[(int64_t)(6 * 8 + qp) * ne + e] = al;
              }
              if (a.store_tangent) {
#pragma unroll
                for (int k = 0; k < 6; ++k) tang[(int64_t)(k * 8 + qp) * ne + e] = tn[k];
              }
              done = true;
            } else if (APPLY_LIKE) {
              T tn[6], lp, mp, beta, N[6];
              tn[0] = tang[(int64_t)qp * ne + e];
              if (tn[0] >= 0) {
#pragma unroll
                for (int k = 1; k < 6; ++k) tn[k] = tang[(int64_t)(k * 8 + qp) * ne + e];
              } else {
#pragma unroll
                for (int k = 1; k < 6; ++k) tn[k] = 0;
              }
              j2_tangent_coeffs(tn, Kb, Gs, Hh, lp, mp, beta, N);
              j2_apply(H, lp, mp, beta, N, S);
              done = true;
            }
          }
          if (MS == MS_NH && pc.model == FE_NEOHOOKE) {
            if (APPLY_LIKE) {
              T H0[3][3], FiT[3][3], lnJ;
#pragma unroll
              for (int c = 0; c < 3; ++c) {
                H0[c][0] = Lx[r][q][c];
                H0[c][1] = Ly[r][p][c];
                H0[c][2] = Lz[q][p][c];
              }
              nh_kin(H0, FiT, lnJ);
              nh_apply(H, FiT, lnJ, lam, mu, S);
            } else {
              T FiT[3][3], lnJ;
              if (!nh_kin(H, FiT, lnJ) && a.flags) atomicOr(a.flags, 1);
              nh_stress(H, FiT, lnJ, lam, mu, S);
              if (OP == OP_RESID && a.store_tangent) {
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                  for (int j = 0; j < 3; ++j) tang[(int64_t)((3 * i + j) * 8 + qp) * ne + e] = FiT[i][j];
                tang[(int64_t)(9 * 8 + qp) * ne + e] = lnJ;
              }
            }
            done = true;
          }
          if (!done) {
            hooke(H, lam, mu, S);
            if (MS == MS_J2 && OP == OP_RESID && st_out) {  // non-J2 phase: state passes through
#pragma unroll
              for (int k = 0; k < 7; ++k)
                st_out[(int64_t)(k * 8 + qp) * ne + e] = st_in ? st_in[(int64_t)(k * 8 + qp) * ne + e] : T(0);
            }
          }
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            Px[r][q][c] += S[c][0];
            Py[r][p][c] += S[c][1];
            Pz[q][p][c] += S[c][2];
          }
          if (OP == OP_RESID && a.stress_sum) {
            ssum[0] += S[0][0];
            ssum[1] += S[1][1];
            ssum[2] += S[2][2];
            ssum[3] += S[1][2];
            ssum[4] += S[0][2];
            ssum[5] += S[0][1];
          }
        }
    // w_q detJ = h^3/8, physical derivative factor 1/h
    push_back(Px, Py, Pz, T(0.125) * h * h, Fo);
  }

  if (OP == OP_RESID && a.stress_sum) {
    const double w = a.h * a.h * a.h * 0.125;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      double v = ssum[k] * w;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if ((tid & 63) == 0) s_red[k][tid >> 6] = v;
    }
  }

  if (OP == OP_VJP) {
    if (valid) {
      double d = 0;
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int c = 0; c < 3; ++c)
              d += (double)Fo[k][j][i][c] * (double)s_l[3 * ((ex + i) + NX * ((ey + j) + NY * (ez + k))) + c];
      static_cast<T*>(a.out_el)[e] = T(d);
    }
    return;
  }

  // CG: element part of p.Ap = sum_e p_e . K_e p_e (p masked on constrained dofs)
  double pq = 0;
  if (OP == OP_CG_APPLY && valid) {
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int c = 0; c < 3; ++c)
            pq += (double)Fo[k][j][i][c] * (double)s_x[3 * ((ex + i) + NX * ((ey + j) + NY * (ez + k))) + c];
  }

  // colour passes: equal index parity => no shared node
  const int color = (ex & 1) | ((ey & 1) << 1) | ((ez & 1) << 2);
  for (int col = 0; col < 8; ++col) {
    if (valid && color == col) {
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int c = 0; c < 3; ++c) s_y[3 * ((ex + i) + NX * ((ey + j) + NY * (ez + k))) + c] += Fo[k][j][i][c];
    }
    __syncthreads();
  }

  if (OP == OP_RESID && a.stress_sum && tid < 6) {
    double v = 0;
    for (int w = 0; w < EBLOCK / 64; ++w) v += s_red[tid][w];
    atomic_add(a.stress_sum + tid, v);
  }

  T* Y = static_cast<T*>(a.y);
  if (!Y) return;
  for (int i = tid; i < NN * 3; i += EBLOCK) {
    const int c = i % 3, nd = i / 3;
    const int li = nd % NX, lj = (nd / NX) % NY, lk = nd / (NX * NY);
    const int gi = a0 + li, gj = b0 + lj, gk = c0 + lk;
    if (gi > n || gj > n || gk > n) continue;
    const int64_t dof = 3 * (gi + np1 * (gj + np1 * gk)) + c;
    const bool own = (min(gi, n - 1) - a0 < TX) && (min(gj, n - 1) - b0 < TY) && (min(gk, n - 1) - c0 < TZ);
    const bool priv = (gi == 0 || li >= 1) && (gi == n || li < TX) && (gj == 0 || lj >= 1) && (gj == n || lj < TY) &&
                      (gk == 0 || lk >= 1) && (gk == n || lk < TZ);
    if (a.apply_bc && a.mask && a.mask[dof]) {
      if (own) {
        if (OP == OP_CG_APPLY) {  // A p = p on constrained dofs; their p.Ap share is p^2
          const T v = CD[dof] * CR[dof] + cg_beta * CP[dof];
          Y[dof] = v;
          pq += (double)v * (double)v;
        } else {
          Y[dof] = (OP == OP_APPLY) ? X[dof] : T(0);
        }
      }
      continue;
    }
    if (priv)
      Y[dof] = s_y[i];
    else
      atomic_add(Y + dof, s_y[i]);
  }
  if (OP == OP_CG_APPLY) cg_alpha_arrive(pq, a.ctrl, a.partials, a.counter, &s_red[0][0]);
}

static int elem_grid(int n) {
  const int nb = ((n + TX - 1) / TX) * ((n + TY - 1) / TY) * ((n + TZ - 1) / TZ);
  return 8 * ((nb + 7) / 8);
}

template <typename T, int OP>
static hipError_t launch_elem_t(const fe_problem* p, const ElemArgs& a, const int* stop, hipStream_t s) {
  const dim3 grid(elem_grid(p->n)), block(EBLOCK);
  switch (p->model_set) {
    case MS_J2:
      hipLaunchKernelGGL((elem_kernel<T, OP, MS_J2>), grid, block, 0, s, a, stop);
      break;
    case MS_NH:
      hipLaunchKernelGGL((elem_kernel<T, OP, MS_NH>), grid, block, 0, s, a, stop);
      break;
    default:
      hipLaunchKernelGGL((elem_kernel<T, OP, MS_LINEAR>), grid, block, 0, s, a, stop);
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_elem_op(const fe_problem* p, int op, const ElemArgs& a, const int* stop, hipStream_t s) {
  if (op == OP_RESID) return launch_elem_t<T, OP_RESID>(p, a, stop, s);
  if (op == OP_APPLY) return launch_elem_t<T, OP_APPLY>(p, a, stop, s);
  return launch_elem_t<T, OP_VJP>(p, a, stop, s);
}

hipError_t launch_elem(const fe_problem* p, int op, const ElemArgs& a, hipStream_t s) {
  return p->prec == FE_F64 ? launch_elem_op<double>(p, op, a, nullptr, s) : launch_elem_op<float>(p, op, a, nullptr, s);
}

// ---------------------------------------------------------------------------
// Per-(element, Gauss point) tangent data used by the diagonal and CSR kernels.

// Gradient of the basis function of brick-local node (i,j,k) at Gauss point (p,q,r).
template <typename T>
__device__ __forceinline__ void basis_grad(int i, int j, int k, int p, int q, int r, T inv_h, T g[3]) {
  const T mi = (i == p) ? T(GA) : T(GB), mj = (j == q) ? T(GA) : T(GB), mk = (k == r) ? T(GA) : T(GB);
  const T si = i ? inv_h : -inv_h, sj = j ? inv_h : -inv_h, sk = k ? inv_h : -inv_h;
  g[0] = si * mj * mk;
  g[1] = mi * sj * mk;
  g[2] = mi * mj * sk;
}

struct TanArgs {
  int n;
  double h;
  int64_t n_el;
  const uint8_t* phase;
  const void* scale;
  const void* tangent;
  const uint8_t* mask;
  Phases mat;
};

template <typename T> struct QpTangent {
  int kind;  // 0: small strain D = lp 1x1 + 2 mp I_sym - beta N x N; 1: Neo-Hookean at F
  T lp, mp, beta, N[6];
  T mu, lam, lnJ, FiT[3][3];
};

template <typename T, int MS>
__device__ __forceinline__ void load_qp_tangent(const TanArgs& a, int64_t e, int qp, QpTangent<T>& t) {
  const PhaseConst pc = a.mat.ph[a.phase[e]];
  const T sc = a.scale ? static_cast<const T*>(a.scale)[e] : T(1);
  const T* tg = static_cast<const T*>(a.tangent);
  const int64_t ne = a.n_el;
  t.kind = 0;
  t.lp = T(pc.lam) * sc;
  t.mp = T(pc.mu) * sc;
  t.beta = 0;
#pragma unroll
  for (int k = 0; k < 6; ++k) t.N[k] = 0;
  if (MS == MS_J2 && pc.model == FE_J2) {
    T tn[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) tn[k] = tg[(int64_t)(k * 8 + qp) * ne + e];
    j2_tangent_coeffs(tn, T(pc.K) * sc, T(pc.G) * sc, T(pc.H), t.lp, t.mp, t.beta, t.N);
  }
  if (MS == MS_NH && pc.model == FE_NEOHOOKE) {
    t.kind = 1;
    t.mu = T(pc.mu) * sc;
    t.lam = T(pc.lam) * sc;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) t.FiT[i][j] = tg[(int64_t)((3 * i + j) * 8 + qp) * ne + e];
    t.lnJ = tg[(int64_t)(9 * 8 + qp) * ne + e];
  }
}

// B[i][k] += w * (dN_a/dx_J) C_iJkL (dN_b/dx_L): the 3x3 block of nodes a, b at one point.
template <typename T>
__device__ __forceinline__ void block_add(const QpTangent<T>& t, const T ga[3], const T gb[3], T w, T B[3][3]) {
  const T dot = ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2];
  if (t.kind == 0) {
    const T* N = t.N;  // xx yy zz yz xz xy
    const T na[3] = {N[0] * ga[0] + N[5] * ga[1] + N[4] * ga[2], N[5] * ga[0] + N[1] * ga[1] + N[3] * ga[2],
                     N[4] * ga[0] + N[3] * ga[1] + N[2] * ga[2]};
    const T nb[3] = {N[0] * gb[0] + N[5] * gb[1] + N[4] * gb[2], N[5] * gb[0] + N[1] * gb[1] + N[3] * gb[2],
                     N[4] * gb[0] + N[3] * gb[1] + N[2] * gb[2]};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        B[i][k] += w * (t.lp * ga[i] * gb[k] + t.mp * ((i == k ? dot : T(0)) + ga[k] * gb[i]) - t.beta * na[i] * nb[k]);
  } else {
    T va[3], vb[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      va[i] = t.FiT[i][0] * ga[0] + t.FiT[i][1] * ga[1] + t.FiT[i][2] * ga[2];
      vb[i] = t.FiT[i][0] * gb[0] + t.FiT[i][1] * gb[1] + t.FiT[i][2] * gb[2];
    }
    const T c = t.mu - t.lam * t.lnJ;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        B[i][k] += w * ((i == k ? t.mu * dot : T(0)) + c * vb[i] * va[k] + t.lam * va[i] * vb[k]);
  }
}

static TanArgs tan_args(const fe_problem* p) {
  TanArgs a;
  a.n = p->n;
  a.h = p->h;
  a.n_el = p->n_el;
  a.phase = p->phase;
  a.scale = p->scale;
  a.tangent = p->tangent;
  a.mask = p->mask;
  a.mat = p->mat;
  return a;
}

// Diagonal of K: one lane per element, 24 entries added atomically (d zeroed before).
template <typename T, int MS>
__global__ __launch_bounds__(256) void diag_kernel(TanArgs a, T* d) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= a.n_el) return;
  const int n = a.n;
  const int ea = (int)(e % n), eb = (int)((e / n) % n), ec = (int)(e / ((int64_t)n * n));
  const T inv_h = T(1.0 / a.h), w = T(0.125 * a.h * a.h * a.h);
  T acc[2][2][2][3] = {};
  for (int qp = 0; qp < 8; ++qp) {
    const int p = qp & 1, q = (qp >> 1) & 1, r = qp >> 2;
    QpTangent<T> t;
    load_qp_tangent<T, MS>(a, e, qp, t);
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          T g[3], B[3][3] = {};
          basis_grad(i, j, k, p, q, r, inv_h, g);
          block_add(t, g, g, w, B);
#pragma unroll
          for (int c = 0; c < 3; ++c) acc[k][j][i][c] += B[c][c];
        }
  }
  const int64_t np1 = n + 1;
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c)
          atomic_add(d + 3 * ((ea + i) + np1 * ((eb + j) + np1 * (ec + k))) + c, acc[k][j][i][c]);
}

template <typename T> __global__ void mask_set_kernel(T* x, const uint8_t* mask, int64_t n, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (mask[i]) x[i] = v;
}

static int vgrid(int64_t n) {
  const int64_t b = (n + VBLOCK - 1) / VBLOCK;
  return (int)(b < VGRID_MAX ? (b > 0 ? b : 1) : VGRID_MAX);
}

template <typename T> __global__ void fill_kernel(T* x, int64_t n, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) x[i] = v;
}

hipError_t launch_fill(const fe_problem* p, void* x, int64_t n, double v, hipStream_t s) {
  if (p->prec == FE_F64)
    hipLaunchKernelGGL(fill_kernel<double>, dim3(vgrid(n)), dim3(VBLOCK), 0, s, (double*)x, n, v);
  else
    hipLaunchKernelGGL(fill_kernel<float>, dim3(vgrid(n)), dim3(VBLOCK), 0, s, (float*)x, n, (float)v);
  return hipGetLastError();
}

template <typename T> static hipError_t launch_diag_t(const fe_problem* p, T* d, int apply_bc, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel<T>, dim3(vgrid(p->n_dof)), dim3(VBLOCK), 0, s, d, p->n_dof, T(0));
  const TanArgs a = tan_args(p);
  const dim3 grid((unsigned)((p->n_el + 255) / 256));
  switch (p->model_set) {
    case MS_J2: hipLaunchKernelGGL((diag_kernel<T, MS_J2>), grid, dim3(256), 0, s, a, d); break;
    case MS_NH: hipLaunchKernelGGL((diag_kernel<T, MS_NH>), grid, dim3(256), 0, s, a, d); break;
    default: hipLaunchKernelGGL((diag_kernel<T, MS_LINEAR>), grid, dim3(256), 0, s, a, d);
  }
  if (apply_bc && p->mask)
    hipLaunchKernelGGL(mask_set_kernel<T>, dim3(vgrid(p->n_dof)), dim3(VBLOCK), 0, s, d, p->mask, p->n_dof, T(1));
  return hipGetLastError();
}

hipError_t launch_diag(const fe_problem* p, void* d, int apply_bc, hipStream_t s) {
  return p->prec == FE_F64 ? launch_diag_t(p, (double*)d, apply_bc, s) : launch_diag_t(p, (float*)d, apply_bc, s);
}

// ---------------------------------------------------------------------------
// Structured CSR pattern in closed form.  Along an axis a node has cnt = 2 (face)
// or 3 (inside) neighbours (itself included) and cum(i) = sum_{i' < i} cnt(i').
// Row 3P+c starts at 9 [cum(k) T^2 + cnt(k) cum(j) T + cnt(k) cnt(j) cum(i)] +
// 3 c cnt(i) cnt(j) cnt(k), T = 3n + 1; columns are the neighbour nodes in
// ascending id order, three dofs each.  This equals sorting all element
// (row, col) pairs and keeping each once.

__device__ __forceinline__ int axis_cnt(int i, int n) { return (i == 0 || i == n) ? 2 : 3; }
__device__ __forceinline__ int64_t axis_cum(int i) { return i == 0 ? 0 : 2 + 3 * (int64_t)(i - 1); }
__device__ __forceinline__ int axis_rank(int i, int d) { return i == 0 ? d : d + 1; }  // d in {-1,0,1}

__device__ __forceinline__ int64_t node_row_start(int i, int j, int k, int n) {
  const int64_t T = 3 * (int64_t)n + 1;
  return 9 * (axis_cum(k) * T * T + axis_cnt(k, n) * axis_cum(j) * T + (int64_t)axis_cnt(k, n) * axis_cnt(j, n) * axis_cum(i));
}

__global__ void csr_pattern_kernel(int n, int32_t* row_ptr, int32_t* col_idx) {
  const int64_t np1 = n + 1;
  const int64_t n_nodes = np1 * np1 * np1;
  const int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (P >= n_nodes) return;
  const int i = (int)(P % np1), j = (int)((P / np1) % np1), k = (int)(P / (np1 * np1));
  const int cx = axis_cnt(i, n), cy = axis_cnt(j, n), cz = axis_cnt(k, n);
  const int len = 3 * cx * cy * cz;
  const int64_t start = node_row_start(i, j, k, n);
  for (int c = 0; c < 3; ++c) {
    const int64_t rs = start + (int64_t)c * len;
    row_ptr[3 * P + c] = (int32_t)rs;
    int pos = 0;
    for (int dk = -1; dk <= 1; ++dk) {
      const int qk = k + dk;
      if (qk < 0 || qk > n) continue;
      for (int dj = -1; dj <= 1; ++dj) {
        const int qj = j + dj;
        if (qj < 0 || qj > n) continue;
        for (int di = -1; di <= 1; ++di) {
          const int qi = i + di;
          if (qi < 0 || qi > n) continue;
          const int64_t Q = qi + np1 * (qj + np1 * qk);
          for (int d = 0; d < 3; ++d) col_idx[rs + pos++] = (int32_t)(3 * Q + d);
        }
      }
    }
  }
  if (P == n_nodes - 1) row_ptr[3 * n_nodes] = (int32_t)(start + 3 * (int64_t)len);
}

hipError_t launch_csr_pattern(const fe_problem* p, int32_t* row_ptr, int32_t* col_idx, hipStream_t s) {
  hipLaunchKernelGGL(csr_pattern_kernel, dim3((unsigned)((p->n_nodes + 255) / 256)), dim3(256), 0, s, p->n, row_ptr,
                     col_idx);
  return hipGetLastError();
}

// CSR values: one lane per (row node P, neighbour Q) 3x3 block, summed over the
// elements that contain both nodes and their Gauss points (no atomics, deterministic).
template <typename T, int MS>
__global__ __launch_bounds__(256) void tangent_csr_kernel(TanArgs a, T* vals, int apply_bc) {
  const int n = a.n;
  const int64_t np1 = n + 1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= np1 * np1 * np1 * 27) return;
  const int64_t P = t / 27;
  const int s = (int)(t % 27);
  const int di = s % 3 - 1, dj = (s / 3) % 3 - 1, dk = s / 9 - 1;
  const int i = (int)(P % np1), j = (int)((P / np1) % np1), k = (int)(P / (np1 * np1));
  const int qi = i + di, qj = j + dj, qk = k + dk;
  if (qi < 0 || qi > n || qj < 0 || qj > n || qk < 0 || qk > n) return;
  const T inv_h = T(1.0 / a.h), w = T(0.125 * a.h * a.h * a.h);
  T B[3][3] = {};
  const int ea0 = max(max(i, qi) - 1, 0), ea1 = min(min(i, qi), n - 1);
  const int eb0 = max(max(j, qj) - 1, 0), eb1 = min(min(j, qj), n - 1);
  const int ec0 = max(max(k, qk) - 1, 0), ec1 = min(min(k, qk), n - 1);
  for (int ec = ec0; ec <= ec1; ++ec)
    for (int eb = eb0; eb <= eb1; ++eb)
      for (int ea = ea0; ea <= ea1; ++ea) {
        const int64_t e = ea + (int64_t)n * (eb + (int64_t)n * ec);
        for (int qp = 0; qp < 8; ++qp) {
          const int p = qp & 1, q = (qp >> 1) & 1, r = qp >> 2;
          QpTangent<T> tq;
          load_qp_tangent<T, MS>(a, e, qp, tq);
          T gP[3], gQ[3];
          basis_grad(i - ea, j - eb, k - ec, p, q, r, inv_h, gP);
          basis_grad(qi - ea, qj - eb, qk - ec, p, q, r, inv_h, gQ);
          block_add(tq, gP, gQ, w, B);
        }
      }
  const int cx = axis_cnt(i, n), cy = axis_cnt(j, n), cz = axis_cnt(k, n);
  const int len = 3 * cx * cy * cz;
  const int rank = axis_rank(k, dk) * cx * cy + axis_rank(j, dj) * cx + axis_rank(i, di);
  const int64_t start = node_row_start(i, j, k, n);
  const int64_t Q = qi + np1 * (qj + np1 * qk);
  for (int c = 0; c < 3; ++c) {
    const int64_t base = start + (int64_t)c * len + 3 * rank;
    const bool rc = apply_bc && a.mask && a.mask[3 * P + c];
    for (int d = 0; d < 3; ++d) {
      T v = B[c][d];
      if (apply_bc && a.mask && (rc || a.mask[3 * Q + d])) v = (P == Q && c == d) ? T(1) : T(0);
      vals[base + d] = v;
    }
  }
}

hipError_t launch_tangent_csr(const fe_problem* p, void* vals, int apply_bc, hipStream_t s) {
  const TanArgs a = tan_args(p);
  const dim3 grid((unsigned)((p->n_nodes * 27 + 255) / 256));
  if (p->prec == FE_F64) {
    double* v = (double*)vals;
    switch (p->model_set) {
      case MS_J2: hipLaunchKernelGGL((tangent_csr_kernel<double, MS_J2>), grid, dim3(256), 0, s, a, v, apply_bc); break;
      case MS_NH: hipLaunchKernelGGL((tangent_csr_kernel<double, MS_NH>), grid, dim3(256), 0, s, a, v, apply_bc); break;
      default: hipLaunchKernelGGL((tangent_csr_kernel<double, MS_LINEAR>), grid, dim3(256), 0, s, a, v, apply_bc);
    }
  } else {
    float* v = (float*)vals;
    switch (p->model_set) {
      case MS_J2: hipLaunchKernelGGL((tangent_csr_kernel<float, MS_J2>), grid, dim3(256), 0, s, a, v, apply_bc); break;
      case MS_NH: hipLaunchKernelGGL((tangent_csr_kernel<float, MS_NH>), grid, dim3(256), 0, s, a, v, apply_bc); break;
      default: hipLaunchKernelGGL((tangent_csr_kernel<float, MS_LINEAR>), grid, dim3(256), 0, s, a, v, apply_bc);
    }
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// CSR sparse mat-vec: LPR lanes per row, contiguous row segments (coalesced),
// butterfly reduction inside the lane group.

template <typename T, int LPR>
__global__ __launch_bounds__(256) void spmv_kernel(int64_t n_rows, const int32_t* __restrict__ rp,
                                                   const int32_t* __restrict__ ci, const T* __restrict__ v,
                                                   const T* __restrict__ x, T* __restrict__ y, const int* stop) {
  if (stop && *stop) return;
  const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / LPR;
  const int lane = threadIdx.x % LPR;
  T acc = 0;
  if (row < n_rows) {
    const int b = rp[row], e = rp[row + 1];
    for (int k = b + lane; k < e; k += LPR) acc += v[k] * x[ci[k]];
  }
#pragma unroll
  for (int off = LPR / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, LPR);
  if (row < n_rows && lane == 0) y[row] = acc;
}

constexpr int SPMV_LPR = 16;

template <typename T>
static hipError_t launch_spmv_t(const fe_problem* p, const int32_t* rp, const int32_t* ci, const T* v, const T* x,
                                T* y, const int* stop, hipStream_t s) {
  const int64_t threads = p->n_dof * SPMV_LPR;
  hipLaunchKernelGGL((spmv_kernel<T, SPMV_LPR>), dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, p->n_dof,
                     rp, ci, v, x, y, stop);
  return hipGetLastError();
}

hipError_t launch_spmv(const fe_problem* p, const int32_t* rp, const int32_t* ci, const void* v, const void* x,
                       void* y, hipStream_t s) {
  return p->prec == FE_F64 ? launch_spmv_t(p, rp, ci, (const double*)v, (const double*)x, (double*)y, nullptr, s)
                           : launch_spmv_t(p, rp, ci, (const float*)v, (const float*)x, (float*)y, nullptr, s);
}

// Diagonal of a CSR matrix with sorted columns (binary search per row).
template <typename T>
__global__ void csr_diag_kernel(int64_t n, const int32_t* rp, const int32_t* ci, const T* v, T* d) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    int lo = rp[r], hi = rp[r + 1] - 1;
    T val = 0;
    while (lo <= hi) {
      const int mid = (lo + hi) >> 1;
      const int64_t c = ci[mid];
      if (c == r) {
        val = v[mid];
        break;
      }
      if (c < r)
        lo = mid + 1;
      else
        hi = mid - 1;
    }
    d[r] = val;
  }
}

hipError_t launch_csr_diag(const fe_problem* p, const int32_t* rp, const int32_t* ci, const void* v, void* d,
                           hipStream_t s) {
  if (p->prec == FE_F64)
    hipLaunchKernelGGL(csr_diag_kernel<double>, dim3(vgrid(p->n_dof)), dim3(VBLOCK), 0, s, p->n_dof, rp, ci,
                       (const double*)v, (double*)d);
  else
    hipLaunchKernelGGL(csr_diag_kernel<float>, dim3(vgrid(p->n_dof)), dim3(VBLOCK), 0, s, p->n_dof, rp, ci,
                       (const float*)v, (float*)d);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// vector kernels

template <typename T> __global__ void lift_kernel(int n, double h, const uint8_t* mask, T* u, int zero_free,
                                                  double e00, double e01, double e02, double e10, double e11,
                                                  double e12, double e20, double e21, double e22) {
  const int64_t np1 = n + 1, n_dof = 3 * np1 * np1 * np1;
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < n_dof; d += (int64_t)gridDim.x * blockDim.x) {
    if (mask && mask[d]) {
      const int64_t P = d / 3;
      const int c = (int)(d % 3);
      const double x = (P % np1) * h, y = ((P / np1) % np1) * h, z = (P / (np1 * np1)) * h;
      const double v = c == 0 ? e00 * x + e01 * y + e02 * z : (c == 1 ? e10 * x + e11 * y + e12 * z : e20 * x + e21 * y + e22 * z);
      u[d] = T(v);
    } else if (zero_free) {
      u[d] = T(0);
    }
  }
}

hipError_t launch_lift(const fe_problem* p, const double* E, void* u, int zero_free, hipStream_t s) {
  const dim3 g(vgrid(p->n_dof)), b(VBLOCK);
  if (p->prec == FE_F64)
    hipLaunchKernelGGL(lift_kernel<double>, g, b, 0, s, p->n, p->h, p->mask, (double*)u, zero_free, E[0], E[1], E[2],
                       E[3], E[4], E[5], E[6], E[7], E[8]);
  else
    hipLaunchKernelGGL(lift_kernel<float>, g, b, 0, s, p->n, p->h, p->mask, (float*)u, zero_free, E[0], E[1], E[2],
                       E[3], E[4], E[5], E[6], E[7], E[8]);
  return hipGetLastError();
}

template <typename T> __global__ void axpby_kernel(int64_t n, double a, const T* x, double b, T* y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = b == 0.0 ? T(a) * x[i] : T(a) * x[i] + T(b) * y[i];
}

hipError_t launch_axpby(const fe_problem* p, int64_t n, double a, const void* x, double b, void* y, hipStream_t s) {
  if (p->prec == FE_F64)
    hipLaunchKernelGGL(axpby_kernel<double>, dim3(vgrid(n)), dim3(VBLOCK), 0, s, n, a, (const double*)x, b, (double*)y);
  else
    hipLaunchKernelGGL(axpby_kernel<float>, dim3(vgrid(n)), dim3(VBLOCK), 0, s, n, a, (const float*)x, b, (float*)y);
  return hipGetLastError();
}

hipError_t launch_mask_zero(const fe_problem* p, void* x, hipStream_t s) {
  if (!p->mask) return hipSuccess;
  if (p->prec == FE_F64)
    hipLaunchKernelGGL(mask_set_kernel<double>, dim3(vgrid(p->n_dof)), dim3(VBLOCK), 0, s, (double*)x, p->mask,
                       p->n_dof, 0.0);
  else
    hipLaunchKernelGGL(mask_set_kernel<float>, dim3(vgrid(p->n_dof)), dim3(VBLOCK), 0, s, (float*)x, p->mask,
                       p->n_dof, 0.0f);
  return hipGetLastError();
}

template <typename S, typename D> __global__ void copy_cvt_kernel(const S* a, D* b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = D(a[i]);
}

hipError_t launch_copy_cvt(const fe_problem* p, const void* src, void* dst, int64_t n, hipStream_t s) {
  if (p->prec == FE_F64)
    hipLaunchKernelGGL((copy_cvt_kernel<double, double>), dim3(vgrid(n)), dim3(VBLOCK), 0, s, (const double*)src,
                       (double*)dst, n);
  else
    hipLaunchKernelGGL((copy_cvt_kernel<float, float>), dim3(vgrid(n)), dim3(VBLOCK), 0, s, (const float*)src,
                       (float*)dst, n);
  return hipGetLastError();
}


template <typename T> __global__ __launch_bounds__(VBLOCK) void dot_kernel(const T* a, const T* b, int64_t n,
                                                                            double* partials, unsigned int* counter,
                                                                            double* out) {
  __shared__ double sh[VBLOCK / 64];
  double v = 0;
  for (int64_t i = (int64_t)blockIdx.x * VBLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * VBLOCK)
    v += (double)a[i] * (double)b[i];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = v;
  if (arrive_last(counter)) {
    const double t = reduce_partials(partials, gridDim.x, sh);
    if (threadIdx.x == 0) {
      *out = t;
      *counter = 0;
    }
  }
}

hipError_t launch_dot(const fe_problem* p, const void* a, const void* b, int64_t n, double* out, hipStream_t s) {
  if (p->prec == FE_F64)
    hipLaunchKernelGGL(dot_kernel<double>, dim3(vgrid(n)), dim3(VBLOCK), 0, s, (const double*)a, (const double*)b, n,
                       p->partials, p->counter, out);
  else
    hipLaunchKernelGGL(dot_kernel<float>, dim3(vgrid(n)), dim3(VBLOCK), 0, s, (const float*)a, (const float*)b, n,
                       p->partials, p->counter, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Jacobi-preconditioned CG with device-resident scalars.  Kernels of an
// iteration return at once when ctrl->status is set, so the host can enqueue
// several iterations between convergence checks without changing the result.

// x = 0, r = b, d = 1/d, p = d r, q = 0; rz = r.p, bb = b.b
template <typename T> __global__ __launch_bounds__(VBLOCK) void cg_init_kernel(
    int64_t n, const T* b, T* x, T* r, T* p, T* q, T* dinv, CgCtrl* ctrl, double rtol, int max_it, double* partials,
    unsigned int* counter) {
  __shared__ double sh[VBLOCK / 64];
  double rz = 0, bb = 0;
  for (int64_t i = (int64_t)blockIdx.x * VBLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * VBLOCK) {
    const T bi = b[i];
    const T di = T(1) / dinv[i];
    dinv[i] = di;
    x[i] = 0;
    r[i] = bi;
    q[i] = 0;
    const T zi = di * bi;
    p[i] = zi;
    rz += (double)bi * (double)zi;
    bb += (double)bi * (double)bi;
  }
  rz = block_sum(rz, sh);
  bb = block_sum(bb, sh);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = rz;
    partials[VGRID_MAX + blockIdx.x] = bb;
  }
  if (arrive_last(counter)) {
    const double trz = reduce_partials(partials, gridDim.x, sh);
    const double tbb = reduce_partials(partials + VGRID_MAX, gridDim.x, sh);
    if (threadIdx.x == 0) {
      ctrl->rz = trz;
      ctrl->bb = tbb;
      ctrl->rr = tbb;
      ctrl->tol2 = rtol * rtol * tbb;
      ctrl->iters = 0;
      ctrl->max_it = max_it;
      ctrl->alpha = ctrl->beta = ctrl->pq = 0;
      ctrl->status = !finite(trz) || !finite(tbb)
                         ? FE_ERR_NONFINITE
                         : (tbb == 0.0 ? CG_CONVERGED : (max_it <= 0 ? FE_ERR_NOT_CONVERGED : CG_RUNNING));
      *counter = 0;
    }
  }
}

// pq = p.q  -> alpha = rz / pq (breakdown / non-finite checks)
template <typename T> __global__ __launch_bounds__(VBLOCK) void cg_alpha_kernel(int64_t n, const T* p, const T* q,
                                                                                 CgCtrl* ctrl, double* partials,
                                                                                 unsigned int* counter) {
  __shared__ double sh[VBLOCK / 64];
  if (ctrl->status) return;
  double v = 0;
  for (int64_t i = (int64_t)blockIdx.x * VBLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * VBLOCK)
    v += (double)p[i] * (double)q[i];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = v;
  if (arrive_last(counter)) {
    const double pq = reduce_partials(partials, gridDim.x, sh);
    if (threadIdx.x == 0) {
      ctrl->pq = pq;
      if (!finite(pq))
        ctrl->status = FE_ERR_NONFINITE;
      else if (pq <= 0.0)
        ctrl->status = FE_ERR_BREAKDOWN;
      else
        ctrl->alpha = ctrl->rz / pq;
      *counter = 0;
    }
  }
}

// x += alpha p; r -= alpha q; q = 0; rr = r.r; rz' = r.(dinv r) -> convergence test, beta
template <typename T> __global__ __launch_bounds__(VBLOCK) void cg_update_kernel(int64_t n, T* x, T* r, const T* p,
                                                                                  T* q, const T* dinv, CgCtrl* ctrl,
                                                                                  double* partials,
                                                                                  unsigned int* counter) {
  __shared__ double sh[VBLOCK / 64];
  if (ctrl->status) return;
  const T alpha = T(ctrl->alpha);
  double rr = 0, rz = 0;
  for (int64_t i = (int64_t)blockIdx.x * VBLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * VBLOCK) {
    x[i] += alpha * p[i];
    const T ri = r[i] - alpha * q[i];
    r[i] = ri;
    q[i] = 0;
    rr += (double)ri * (double)ri;
    rz += (double)ri * (double)(dinv[i] * ri);
  }
  rr = block_sum(rr, sh);
  rz = block_sum(rz, sh);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = rr;
    partials[VGRID_MAX + blockIdx.x] = rz;
  }
  if (arrive_last(counter)) {
    const double trr = reduce_partials(partials, gridDim.x, sh);
    const double trz = reduce_partials(partials + VGRID_MAX, gridDim.x, sh);
    if (threadIdx.x == 0) {
      ctrl->iters += 1;
      ctrl->rr = trr;
      if (!finite(trr) || !finite(trz))
        ctrl->status = FE_ERR_NONFINITE;
      else if (trr <= ctrl->tol2)
        ctrl->status = CG_CONVERGED;
      else if (ctrl->iters >= ctrl->max_it)
        ctrl->status = FE_ERR_NOT_CONVERGED;
      else {
        ctrl->beta = trz / ctrl->rz;
        ctrl->rz = trz;
      }
      *counter = 0;
    }
  }
}

// p = dinv r + beta p
template <typename T> __global__ __launch_bounds__(VBLOCK) void cg_direction_kernel(int64_t n, const T* r,
                                                                                     const T* dinv, T* p,
                                                                                     const CgCtrl* ctrl) {
  if (ctrl->status) return;
  const T beta = T(ctrl->beta);
  for (int64_t i = (int64_t)blockIdx.x * VBLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * VBLOCK)
    p[i] = dinv[i] * r[i] + beta * p[i];
}

template <typename T>
static hipError_t cg_init_t(const fe_problem* p, const T* b, T* x, double rtol, int max_it, hipStream_t s) {
  const int64_t n = p->n_dof;
  hipLaunchKernelGGL(cg_init_kernel<T>, dim3(vgrid(n)), dim3(VBLOCK), 0, s, n, b, x, (T*)p->w_r, (T*)p->w_p,
                     (T*)p->w_q, (T*)p->w_d, p->ctrl, rtol, max_it, p->partials, p->counter);
  return hipGetLastError();
}

hipError_t cg_init(const fe_problem* p, const void* b, void* x, double rtol, int max_it, hipStream_t s) {
  return p->prec == FE_F64 ? cg_init_t(p, (const double*)b, (double*)x, rtol, max_it, s)
                           : cg_init_t(p, (const float*)b, (float*)x, rtol, max_it, s);
}

int elem_grid_size(int n) { return elem_grid(n); }

// Search-direction buffers of CG iteration k: the fused matrix-free iteration reads
// p_old and writes p_new, alternating between w_p and w_p2; the CSR iteration keeps p in w_p.
static void* cg_p_new(const fe_problem* p, int op, long k) {
  return (op == FE_OP_CSR || (k & 1)) ? p->w_p : p->w_p2;
}

template <typename T>
static hipError_t cg_operator_t(const fe_problem* p, int op, const int32_t* rp, const int32_t* ci, const T* vals,
                                long k, hipStream_t s) {
  const int* stop = &p->ctrl->status;
  T* Q = (T*)p->w_q;
  if (op == FE_OP_CSR) return launch_spmv_t(p, rp, ci, vals, (const T*)p->w_p, Q, stop, s);
  ElemArgs a{};
  a.n = p->n;
  a.h = p->h;
  a.n_el = p->n_el;
  a.phase = p->phase;
  a.scale = p->scale;
  a.mask = p->mask;
  a.xlin = p->u_lin;
  a.y = Q;
  a.tangent = p->tangent;
  a.apply_bc = 1;
  a.mat = p->mat;
  a.cg_r = p->w_r;
  a.cg_dinv = p->w_d;
  a.cg_pnew = cg_p_new(p, op, k);
  a.cg_pold = (a.cg_pnew == p->w_p) ? p->w_p2 : p->w_p;
  a.ctrl = p->ctrl;
  a.partials = p->partials;
  a.counter = p->counter;
  return launch_elem_t<T, OP_CG_APPLY>(p, a, stop, s);
}

hipError_t cg_operator(const fe_problem* p, int op, const int32_t* rp, const int32_t* ci, const void* vals, long k,
                       hipStream_t s) {
  return p->prec == FE_F64 ? cg_operator_t(p, op, rp, ci, (const double*)vals, k, s)
                           : cg_operator_t(p, op, rp, ci, (const float*)vals, k, s);
}

template <typename T> static hipError_t cg_vectors_t(const fe_problem* p, int op, T* x, long k, hipStream_t s) {
  const int64_t n = p->n_dof;
  T* P = (T*)cg_p_new(p, op, k);
  T* Q = (T*)p->w_q;
  const dim3 g(vgrid(n)), b(VBLOCK);
  if (op == FE_OP_CSR)
    hipLaunchKernelGGL(cg_alpha_kernel<T>, g, b, 0, s, n, (const T*)P, (const T*)Q, p->ctrl, p->partials, p->counter);
  hipLaunchKernelGGL(cg_update_kernel<T>, g, b, 0, s, n, x, (T*)p->w_r, (const T*)P, Q, (const T*)p->w_d, p->ctrl,
                     p->partials, p->counter);
  if (op == FE_OP_CSR)
    hipLaunchKernelGGL(cg_direction_kernel<T>, g, b, 0, s, n, (const T*)p->w_r, (const T*)p->w_d, P, p->ctrl);
  return hipGetLastError();
}

hipError_t cg_vectors(const fe_problem* p, int op, void* x, long k, hipStream_t s) {
  return p->prec == FE_F64 ? cg_vectors_t(p, op, (double*)x, k, s) : cg_vectors_t(p, op, (float*)x, k, s);
}

// Gauss points of J2 phases and how many of them were plastic at the stored linearisation.
template <typename T>
__global__ void lin_stats_kernel(int64_t ne, const uint8_t* phase, Phases mat, const T* tangent,
                                 unsigned long long* out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne || mat.ph[phase[e]].model != FE_J2) return;
  unsigned long long pl = 0;
  for (int q = 0; q < 8; ++q) pl += tangent[(int64_t)q * ne + e] >= T(0) ? 1 : 0;
  atomicAdd(out, 8ull);
  atomicAdd(out + 1, pl);
}

hipError_t launch_lin_stats(const fe_problem* p, unsigned long long* out, hipStream_t s) {
  const dim3 g((unsigned)((p->n_el + 255) / 256)), b(256);
  if (p->prec == FE_F64)
    hipLaunchKernelGGL(lin_stats_kernel<double>, g, b, 0, s, p->n_el, p->phase, p->mat, (const double*)p->tangent, out);
  else
    hipLaunchKernelGGL(lin_stats_kernel<float>, g, b, 0, s, p->n_el, p->phase, p->mat, (const float*)p->tangent, out);
  return hipGetLastError();
}

}  // namespace fe
