// Device-side building blocks shared by the structured-brick kernels (fe_kernels.hip) and
// the general-mesh kernels (fe_general.hip): reduction helpers, the constitutive laws at
// one Gauss point and the per-point tangent data of the diagonal / CSR kernels.
#pragma once

#include "fe_internal.hpp"

namespace fe {

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

// Wavefront-aggregated append: lanes with pred set get consecutive slots of *counter
// (one atomic per wave).  Valid for any set of active lanes.
__device__ __forceinline__ unsigned wave_append(unsigned int* counter, bool pred) {
  const unsigned long long m = __ballot(pred);
  if (m == 0) return 0;
  const int lane = __lane_id();
  const int leader = __ffsll((long long)m) - 1;
  unsigned base = 0;
  if (lane == leader) base = atomicAdd(counter, (unsigned)__popcll(m));
  base = __shfl(base, leader, 64);
  return base + (unsigned)__popcll(m & ((1ull << lane) - 1ull));
}

__device__ __forceinline__ void wave_count(unsigned int* counter, bool pred) {
  const unsigned long long m = __ballot(pred);
  if (m != 0 && __lane_id() == __ffsll((long long)m) - 1) atomicAdd(counter, (unsigned)__popcll(m));
}

// Block-wide sum of partials[0..nb), returned to every thread.
__device__ __forceinline__ double sum_partials_all(const double* partials, int nb, double* sh, double* bc) {
  double v = 0;
  for (int i = threadIdx.x; i < nb; i += 256) v += partials[i];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) *bc = v;
  __syncthreads();
  return *bc;
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

// ---- learned surrogate at a plastic-trial J2 point ----------------------------------
constexpr double RSQ2 = 0.70710678118654752440;  // 1/sqrt(2)

// Normalised network inputs [eps - eps_p_n, eps_p_n] (Mandel: shear = gamma / sqrt 2), alpha_n; / s_in.
template <typename T>
__device__ __forceinline__ void sur_inputs(const T H[3][3], const T epn[6], T an, float s_in, float* x) {
  const T e[6] = {H[0][0], H[1][1], H[2][2], H[1][2] + H[2][1], H[0][2] + H[2][0], H[0][1] + H[1][0]};
  const T inv = T(1) / T(s_in);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const T c = k < 3 ? T(1) : T(RSQ2);
    x[k] = float((e[k] - epn[k]) * c * inv);
    x[6 + k] = float(epn[k] * c * inv);
  }
  x[12] = float(an * inv);
}

// Stress, history and symmetrised Voigt tangent from the network output y (normalised
// Mandel stress) and Jacobian J = dy/dx[:, :6]; false when the local check exceeds tol.
template <typename T>
__device__ __forceinline__ bool sur_consume(const T H[3][3], const T epn[6], T an, T K, T G, T sy, T Hh,
                                            const float* y, const float* J, float s_in, float s_out, double tol,
                                            const T tn[6], T S[3][3], T ep[6], T& al, float* Dsym, int full) {
  const T c[6] = {T(1), T(1), T(1), T(RSQ2), T(RSQ2), T(RSQ2)};
  T sig[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) sig[i] = T(s_out) * T(y[i]) * c[i];
  // elastic strain C^-1 sigma (engineering shear) -> plastic strain and hardening variable
  const T lam = K - T(2.0 / 3.0) * G;
  const T trs = sig[0] + sig[1] + sig[2];
  const T a = lam / (2 * G + 3 * lam);
  const T e[6] = {H[0][0], H[1][1], H[2][2], H[1][2] + H[2][1], H[0][2] + H[2][0], H[0][1] + H[1][0]};
  T dsq = 0;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const T ee = k < 3 ? (sig[k] - a * trs) / (2 * G) : sig[k] / G;
    ep[k] = e[k] - ee;
    const T d = ep[k] - epn[k];
    dsq += k < 3 ? d * d : T(0.5) * d * d;
  }
  al = an + sqrt(T(2.0 / 3.0) * dsq);
  // local check: yield condition and flow direction of the prediction
  const T m = trs / T(3);
  const T d0 = sig[0] - m, d1 = sig[1] - m, d2 = sig[2] - m;
  const T dn = sqrt(d0 * d0 + d1 * d1 + d2 * d2 + 2 * (sig[3] * sig[3] + sig[4] * sig[4] + sig[5] * sig[5]));
  const T q = T(SQRT1_5) * dn;
  const T r1 = fabs(q - sy - Hh * al) / sy;
  const T idn = dn > 0 ? T(1) / dn : T(1);
  const T nzz = -(tn[1] + tn[2]);
  const T f0 = d0 * idn - tn[1], f1 = d1 * idn - tn[2], f2 = d2 * idn - nzz;
  const T f3 = sig[3] * idn - tn[3], f4 = sig[4] * idn - tn[4], f5 = sig[5] * idn - tn[5];
  const T r2 = sqrt(f0 * f0 + f1 * f1 + f2 * f2 + 2 * (f3 * f3 + f4 * f4 + f5 * f5));
  if (!(fmax(r1, r2) <= T(tol))) return false;
  S[0][0] = sig[0];
  S[1][1] = sig[1];
  S[2][2] = sig[2];
  S[1][2] = S[2][1] = sig[3];
  S[0][2] = S[2][0] = sig[4];
  S[0][1] = S[1][0] = sig[5];
  const T f = T(s_out) / T(s_in);
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j)
      Dsym[i * 6 + j] = float(full ? f * c[i] * c[j] * T(J[i * 6 + j])
                             : T(0.5) * f * c[i] * c[j] * (T(J[i * 6 + j]) + T(J[j * 6 + i])));
  return true;
}

// Stress from a general Voigt tangent D (tensor stress, engineering shear strain) and sym(H).
// (rare path inside the operator: rows are read one at a time so that this branch does
// not raise the register budget of the whole kernel)
template <typename T> __device__ __forceinline__ void general_apply(const T H[3][3], const float* D, T S[3][3]) {
  const T e[6] = {H[0][0], H[1][1], H[2][2], H[1][2] + H[2][1], H[0][2] + H[2][0], H[0][1] + H[1][0]};
  T s[6];
#pragma unroll 1
  for (int i = 0; i < 6; ++i) {
    T acc = 0;
#pragma unroll
    for (int j = 0; j < 6; ++j) acc += T(D[i * 6 + j]) * e[j];
    s[i] = acc;
  }
  S[0][0] = s[0];
  S[1][1] = s[1];
  S[2][2] = s[2];
  S[1][2] = S[2][1] = s[3];
  S[0][2] = S[2][0] = s[4];
  S[0][1] = S[1][0] = s[5];
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
// Per-(element, Gauss point) tangent data used by the diagonal and CSR kernels.

struct TanArgs {
  int n;
  double h;
  int64_t n_el;
  const uint8_t* phase;
  const void* scale;
  const void* tangent;
  const uint8_t* mask;
  Phases mat;
  const int* sur_map;   // surrogate points: slot of their general Voigt tangent in sur_D
  const void* sur_D;
};

template <typename T> struct QpTangent {
  int kind;  // 0: small strain D = lp 1x1 + 2 mp I_sym - beta N x N; 1: Neo-Hookean at F; 2: general Voigt D
  T lp, mp, beta, N[6];
  T mu, lam, lnJ, FiT[3][3];
  const float* D;  // kind 2: the surrogate's Voigt tangent (stored in FP32, as the network computes it)
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
    if (tn[0] < T(-1.5)) {
      t.kind = 2;
      t.D = static_cast<const float*>(a.sur_D) + (int64_t)a.sur_map[(int64_t)qp * ne + e] * 36;
    } else {
      j2_tangent_coeffs(tn, T(pc.K) * sc, T(pc.G) * sc, T(pc.H), t.lp, t.mp, t.beta, t.N);
    }
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
  if (t.kind == 2) {
    // B_a^T D B_b with the 6x3 strain-displacement blocks of the two nodes
    const T Ba[6][3] = {{ga[0], 0, 0}, {0, ga[1], 0}, {0, 0, ga[2]},
                        {0, ga[2], ga[1]}, {ga[2], 0, ga[0]}, {ga[1], ga[0], 0}};
    const T Bb[6][3] = {{gb[0], 0, 0}, {0, gb[1], 0}, {0, 0, gb[2]},
                        {0, gb[2], gb[1]}, {gb[2], 0, gb[0]}, {gb[1], gb[0], 0}};
    T DB[6][3];
#pragma unroll
    for (int p = 0; p < 6; ++p)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        T s = 0;
#pragma unroll
        for (int q = 0; q < 6; ++q) s += T(t.D[p * 6 + q]) * Bb[q][k];
        DB[p][k] = s;
      }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        T s = 0;
#pragma unroll
        for (int p = 0; p < 6; ++p) s += Ba[p][i] * DB[p][k];
        B[i][k] += w * s;
      }
  } else if (t.kind == 0) {
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

}  // namespace fe
