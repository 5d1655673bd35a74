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
//   4. nodal forces are summed into LDS in FP64 by workgroup-scope LDS atomic adds;
//      nodes owned by the brick alone are stored, nodes on the brick's faces are
//      added with hardware FP atomics.
// Bricks are numbered so that consecutive bricks land on one XCD (workgroups
// are dealt round-robin over the 8 XCDs), keeping shared face nodes in one L2.
#include "fe_internal.hpp"
#include "fe_device.hpp"

namespace fe {

LaunchEvents& launch_events() {
  static thread_local LaunchEvents ev;
  return ev;
}

constexpr int TX = 16, TY = 4, TZ = 4;
constexpr int NX = TX + 1, NY = TY + 1, NZ = TZ + 1, NN = NX * NY * NZ;
constexpr int EBLOCK = TX * TY * TZ;
static_assert(EBLOCK == 256, "one element per lane");

// CG direction step of iteration k (see the CG section below); false when the
// iteration stops (block 0 records the status).
__device__ __forceinline__ bool cg_direction_step(CgCtrl* ctrl, const double* pu, long k, double* sh, double* bc,
                                                  double& beta) {
  const double rr = sum_partials_all(pu, CG_UGRID, sh, bc);
  const double rz = sum_partials_all(pu + CG_UGRID, CG_UGRID, sh, bc + 1);
  const double tol2 = k == 0 ? ctrl->rtol2 * rr : ctrl->tol2;
  int st = CG_RUNNING;
  if (!finite(rr) || !finite(rz))
    st = FE_ERR_NONFINITE;
  else if (k == 0 ? rr == 0.0 : rr <= tol2)
    st = CG_CONVERGED;
  else if (k >= ctrl->max_it)
    st = FE_ERR_NOT_CONVERGED;
  beta = k == 0 ? 0.0 : rz / ctrl->rz[(k - 1) & 1];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (k == 0) {
      ctrl->bb = rr;
      ctrl->tol2 = tol2;
    }
    ctrl->rr = rr;
    ctrl->iters = (int)k;
    ctrl->beta = beta;
    ctrl->rz[k & 1] = rz;
    if (st != CG_RUNNING) ctrl->status = st;
  }
  return st == CG_RUNNING;
}

// (M^-1 r)[dof]: point Jacobi (M holds 1/diag, [n_dof]) or node-block Jacobi (M holds the
// symmetric 3x3 inverse blocks [n_nodes][6], order xx yy zz yz xz xy).  Every caller forms
// the same expression, so a node's value does not depend on who computes it.
template <typename T>
__device__ __forceinline__ T pc_apply(const T* M, const T* R, int64_t dof, int block) {
  if (!block) return M[dof] * R[dof];
  const int64_t nd = dof / 3;
  const int c = (int)(dof - 3 * nd);
  const T* m = M + 6 * nd;
  const T* r = R + 3 * nd;
  const T m0 = c == 0 ? m[0] : (c == 1 ? m[5] : m[4]);
  const T m1 = c == 0 ? m[5] : (c == 1 ? m[1] : m[3]);
  const T m2 = c == 0 ? m[4] : (c == 1 ? m[3] : m[2]);
  return m0 * r[0] + m1 * r[1] + m2 * r[2];
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
// Single-reduction CG, staging of a brick's nodes for launch j (see ElemArgs): every lane
// requests the previous launch's slot sums, then the loads of all its dofs (vector loads return
// in order, so the scalar step below waits for the slot sums alone), forms alpha, beta, and then
//   s_{j-1} = w_{j-1} + beta s_{j-2},  r_j = r_{j-1} - alpha s_{j-1},  u_j = M^-1 r_j
// (launch 0: r_0 = b, u_0 = M^-1 b).  Every brick that touches a node forms the same u_j; the
// owner also stores s_{j-1}, r_j, p_{j-1} = u_{j-1} + beta p_{j-2}, x_j = x_{j-1} + alpha p_{j-1},
// zeroes the w buffer of launch j+1 and adds its shares of (r_j, u_j) and ||r_j||^2.
// u_j goes to s_x (0 on constrained dofs, whose value goes to s_b), s_y is cleared.
constexpr int STAGE_IT = (NN * 3 + EBLOCK - 1) / EBLOCK;

template <typename T>
__device__ __forceinline__ bool cg_scalars(const ElemArgs& a, const double v_in[3], double (*sh)[EBLOCK / 64],
                                           T& alpha_out, T& beta_out);

template <typename T, bool NEED_L, bool BLK, typename Acc, typename Early>
__device__ __forceinline__ bool cg_stage_brick(const ElemArgs& a, int n, int a0, int b0, int c0,
                                               double (*sh)[EBLOCK / 64], T* s_x, Acc* s_y, T* s_b, T* s_l,
                                               unsigned char* s_fx, double& g, double& rr, Early&& early) {
  static_assert(CGS_SLOTS == EBLOCK, "one reduction slot per lane");
  // the previous launch's slot sums are requested before the staging loads (loads return in
  // order), so the scalar reduction overlaps the staging traffic
  double acc_v[3] = {0, 0, 0};
  const bool prev = a.cg_j > 0;
  if (prev) {
#pragma unroll
    for (int k = 0; k < 3; ++k) acc_v[k] = a.cg_acc_in[k * CGS_SLOTS + threadIdx.x];
  }
  T alpha = 0, beta = 0;
  const T* __restrict__ RO = static_cast<const T*>(a.cg_rold);
  const T* __restrict__ WO = static_cast<const T*>(a.cg_wold);
  const T* __restrict__ SO = static_cast<const T*>(a.cg_sold);
  const T* __restrict__ M = static_cast<const T*>(a.cg_dinv);
  const T* __restrict__ XL = static_cast<const T*>(a.xlin);
  T* __restrict__ RN = static_cast<T*>(a.cg_rnew);
  T* __restrict__ SN = static_cast<T*>(a.cg_snew);
  T* __restrict__ P = static_cast<T*>(a.cg_pvec);
  T* __restrict__ X = static_cast<T*>(a.cg_x);
  T* __restrict__ WZ = static_cast<T*>(a.cg_wzero);
  const unsigned char* __restrict__ mask = a.mask;
  constexpr bool blk = BLK;
  const bool first = a.cg_j == 0;
  const int64_t np1 = n + 1;
  // loads in batches of SB rounds (all loads of a batch, then its updates and stores):
  // FP64 takes all rounds at once, FP32 two batches, which measured faster there
  constexpr int SB = sizeof(T) == 8 ? STAGE_IT : (STAGE_IT + 1) / 2;
#pragma unroll
  for (int t0 = 0; t0 < STAGE_IT; t0 += SB) {
    int64_t dofs[SB];
    int cs[SB];
    bool in[SB], own[SB];
    unsigned char mk[SB];
    T ro[SB][3], wo[SB][3], so[SB][3], m[SB][3], po[SB], xo[SB], lv[SB];
#pragma unroll
    for (int t = 0; t < SB; ++t) {
      const int i = threadIdx.x + (t0 + t) * EBLOCK;
      const int c = i % 3, nd = i / 3;
      const int li = nd % NX, lj = (nd / NX) % NY, lk = nd / (NX * NY);
      const int gi = a0 + li, gj = b0 + lj, gk = c0 + lk;
      in[t] = i < NN * 3 && gi <= n && gj <= n && gk <= n;
      own[t] = in[t] && (min(gi, n - 1) - a0 < TX) && (min(gj, n - 1) - b0 < TY) && (min(gk, n - 1) - c0 < TZ);
      cs[t] = c;
      const int64_t dof = in[t] ? 3 * (gi + np1 * (gj + np1 * gk)) + c : 0;
      dofs[t] = dof;
      const int64_t b3 = dof - c;
      if (blk) {  // the node's three components (slot k = component k)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          ro[t][k] = in[t] ? RO[b3 + k] : T(0);
          wo[t][k] = in[t] && !first ? WO[b3 + k] : T(0);
          so[t][k] = in[t] && !first ? SO[b3 + k] : T(0);
        }
      } else {  // the lane's own component only (slot 0): one coalesced load per vector
        ro[t][0] = in[t] ? RO[dof] : T(0);
        wo[t][0] = in[t] && !first ? WO[dof] : T(0);
        so[t][0] = in[t] && !first ? SO[dof] : T(0);
        ro[t][1] = ro[t][2] = wo[t][1] = wo[t][2] = so[t][1] = so[t][2] = T(0);
      }
      if (blk) {
        const T* mb = M + 2 * b3;  // 6 entries per node: xx, yy, zz, yz, xz, xy
        const int i0 = c == 0 ? 0 : (c == 1 ? 5 : 4), i1 = c == 0 ? 5 : (c == 1 ? 1 : 3),
                  i2 = c == 0 ? 4 : (c == 1 ? 3 : 2);
        m[t][0] = in[t] ? mb[i0] : T(0);
        m[t][1] = in[t] ? mb[i1] : T(0);
        m[t][2] = in[t] ? mb[i2] : T(0);
      } else {  // (one word: a copy of a register with a load in flight would wait for it)
        m[t][0] = in[t] ? M[dof] : T(0);
        m[t][1] = m[t][2] = T(0);
      }
      mk[t] = mask ? mask[dof] : (unsigned char)0;  // dof is 0 outside the mesh
      po[t] = own[t] && !first ? P[dof] : T(0);
      xo[t] = own[t] && !first ? X[dof] : T(0);
      lv[t] = NEED_L && in[t] ? XL[dof] : T(0);
    }
    if (t0 == 0) {
      early();
      if (prev && !cg_scalars<T>(a, acc_v, sh, alpha, beta)) return false;
    }
#pragma unroll
    for (int t = 0; t < SB; ++t) {
      const int i = threadIdx.x + (t0 + t) * EBLOCK;
      if (i >= NN * 3) break;
      const int c = cs[t];
      int mkv = mk[t];
      asm volatile("" : "+v"(mkv));  // keeps the flag test here, after every load of the batch was issued
      const bool fixed = in[t] && mkv != 0;
      T rn[3], sn[3];
#pragma unroll
      for (int k = 0; k < (blk ? 3 : 1); ++k) {
        sn[k] = wo[t][k] + beta * so[t][k];
        rn[k] = first ? ro[t][k] : ro[t][k] - alpha * sn[k];
      }
      T u, uo;
      int cc = 0;  // slot of the lane's own component
      if (blk) {
        u = m[t][0] * rn[0] + m[t][1] * rn[1] + m[t][2] * rn[2];
        uo = m[t][0] * ro[t][0] + m[t][1] * ro[t][1] + m[t][2] * ro[t][2];
        cc = c;
      } else {
        u = m[t][0] * rn[0];
        uo = m[t][0] * ro[t][0];
      }
      if (own[t]) {
        const int64_t dof = dofs[t];
        WZ[dof] = 0;
        if (!first) {
          const T pn = uo + beta * po[t];
          P[dof] = pn;
          X[dof] = xo[t] + alpha * pn;
          SN[dof] = sn[cc];
          RN[dof] = rn[cc];
        }
        g += (double)rn[cc] * (double)u;
        rr += (double)rn[cc] * (double)rn[cc];
      }
      if (fixed) {
        s_b[i] = u;
        u = 0;
      }
      s_fx[i] = fixed ? 1 : 0;
      s_x[i] = in[t] ? u : T(0);
      s_y[i] = 0;
      if (NEED_L) s_l[i] = lv[t];
    }
  }
  return true;
}

// Start of single-reduction CG launch j >= 1, run redundantly by every workgroup (no
// inter-workgroup synchronisation inside a launch): sum the slots of launch j-1 in fixed
// order into d = (u, A u), g = (r, u), rr = ||r||^2 of iterate j-1 and form
// (Chronopoulos & Gear 1989)
//   beta_{j-1} = g_{j-1} / g_{j-2},  alpha_{j-1} = g_{j-1} / (d_{j-1} - beta g_{j-1} / alpha_{j-2})
// (j = 1: beta_0 = 0, alpha_0 = g_0 / d_0), or a stop: ||r_{j-1}|| <= rtol ||b||,
// j - 1 = max_it, breakdown, non-finite.  Workgroup 0 records the scalars and the status;
// (g, alpha) of iterate j-1 go to history slot (j-1) & 1 while slot j & 1 is read.
// Returns false when the iteration stops (every workgroup reaches the same decision).
template <typename T>
__device__ __forceinline__ bool cg_scalars(const ElemArgs& a, const double v_in[3], double (*sh)[EBLOCK / 64],
                                           T& alpha_out, T& beta_out) {
  const long j = a.cg_j;
  double v[3] = {v_in[0], v_in[1], v_in[2]};
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < 3; ++k) sh[k][threadIdx.x >> 6] = v[k];
  __syncthreads();
  double d = 0, g = 0, rr = 0;
  for (int w = 0; w < EBLOCK / 64; ++w) {
    d += sh[0][w];
    g += sh[1][w];
    rr += sh[2][w];
  }
  __syncthreads();  // sh is reused by the caller
  const CgCtrl* c = a.ctrl;
  const int slot = (int)(j & 1);  // history of iterate j-2
  const double tol2 = j == 1 ? c->rtol2 * rr : c->tol2;
  int st = CG_RUNNING;
  double alpha = 0, beta = 0;
  if (!finite(d) || !finite(g) || !finite(rr)) {
    st = FE_ERR_NONFINITE;
  } else if (j == 1 ? rr == 0.0 : rr <= tol2) {
    st = CG_CONVERGED;
  } else if (j - 1 >= c->max_it) {
    st = FE_ERR_NOT_CONVERGED;
  } else {
    beta = j == 1 ? 0.0 : g / c->ghist[slot];
    const double den = j == 1 ? d : d - beta * g / c->ahist[slot];
    if (!finite(den)) st = FE_ERR_NONFINITE;
    else if (den <= 0.0) st = FE_ERR_BREAKDOWN;
    else alpha = g / den;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    CgCtrl* w = a.ctrl;
    if (j == 1) {
      w->bb = rr;
      w->tol2 = tol2;
    }
    w->rr = rr;
    w->pq = d;
    w->iters = (int)(j - 1);
    w->alpha = alpha;
    w->beta = beta;
    w->ghist[slot ^ 1] = g;
    w->ahist[slot ^ 1] = alpha;
    if (st != CG_RUNNING) w->status = st;
  }
  alpha_out = T(alpha);
  beta_out = T(beta);
  return st == CG_RUNNING;
}

// ---------------------------------------------------------------------------
// element brick kernel

// (at least two waves per SIMD: some FP64 instances sit at the 256-register edge, where
// the allocator would otherwise fall back to one wave per SIMD)
// ACC32 (FP32 problems only): the nodal sums accumulate in FP32 LDS as well; by default they
// are formed in FP64 in both precisions.
template <typename T, int OP, int MS, bool ACC32 = false>
__global__ __launch_bounds__(EBLOCK) __attribute__((amdgpu_waves_per_eu(2))) void elem_kernel(ElemArgs a,
                                                                                              const int* stop) {
  static_assert(!ACC32 || sizeof(T) == 4, "FP32 accumulation is an FP32-problem variant");
  using Acc = typename std::conditional<ACC32, float, double>::type;
  constexpr bool APPLY_LIKE = (OP == OP_APPLY) || (OP == OP_CG_APPLY);
  constexpr bool NEED_L = OP == OP_VJP;
  __shared__ T s_x[NN * 3];
  __shared__ Acc s_y[OP == OP_VJP ? 1 : NN * 3];  // nodal sums
  __shared__ T s_l[NEED_L ? NN * 3 : 1];
  __shared__ T s_b[OP == OP_CG_APPLY ? NN * 3 : 1];  // CG: u on constrained dofs (A u = u there)
  __shared__ double s_red[6][EBLOCK / 64];
  __shared__ unsigned char s_fx[NN * 3];  // constrained dof flags of the brick (apply_bc)

  if (stop && *stop) return;
  const int n = a.n;
  const int ntx = (n + TX - 1) / TX, nty = (n + TY - 1) / TY, ntz = (n + TZ - 1) / TZ;
  const int nb = ntx * nty * ntz;
  const int per = (nb + 7) >> 3;
  const int tile = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (tile >= nb) {  // padding block of the XCD-aware numbering
    if constexpr (OP == OP_RESID)  // (deterministic mode sums every workgroup's stress slot)
      if (a.stress_part && a.stress_sum && threadIdx.x < 6) a.stress_part[(int64_t)blockIdx.x * 6 + threadIdx.x] = 0.0;
    return;
  }
  const int a0 = (tile % ntx) * TX, b0 = ((tile / ntx) % nty) * TY, c0 = (tile / (ntx * nty)) * TZ;
  const int tid = threadIdx.x;
  const T* X = static_cast<const T*>(a.x);
  const T* XL = static_cast<const T*>(a.xlin);
  const int ex = tid % TX, ey = (tid / TX) % TY, ez = tid / (TX * TY);
  const int ga = a0 + ex, gb = b0 + ey, gc = c0 + ez;
  const bool valid = ga < n && gb < n && gc < n;
  const int64_t e = valid ? (ga + (int64_t)n * (gb + (int64_t)n * gc)) : 0;
  const int64_t ne = a.n_el;
  const T h = T(a.h), inv_h = T(1.0 / a.h);
  // the element's phase is requested before the staging loads; the operator's first stored-
  // tangent word of every Gauss point right after them (both arrive before they are used)
  const int ph = valid ? (int)a.phase[e] : 0;
  const T* tang_c = static_cast<const T*>(a.tangent);
  T tq0[8];
  T nw[2][10];  // Neo-Hookean operator: F^-T and ln J of two Gauss points (see below)
  // (FP32 requests the first point's words with the staging, measured faster there; FP64 after
  // the gradients, measured faster there)
  constexpr bool NH_EARLY = sizeof(T) == 4;
  auto early = [&]() {
    if (APPLY_LIKE && MS == MS_J2) {
      const bool j2 = valid && a.mat.ph[ph].model == FE_J2;
#pragma unroll
      for (int qq = 0; qq < 8; ++qq) tq0[qq] = j2 ? tang_c[(int64_t)qq * ne + e] : T(-1);
    }
    if (APPLY_LIKE && MS == MS_NH && NH_EARLY) {
      const bool nh = valid && a.mat.ph[ph].model == FE_NEOHOOKE;
#pragma unroll
      for (int k = 0; k < 10; ++k) nw[0][k] = nh ? tang_c[(int64_t)(k * 8) * ne + e] : T(0);
    }
  };

  double cg_g = 0, cg_rr = 0;  // owners' shares of (r_j, u_j) and ||r_j||^2
  const int64_t np1 = n + 1;

  if (OP == OP_CG_APPLY) {
    if (blockIdx.x == 0)
      for (int i = tid; i < 3 * CGS_SLOTS; i += EBLOCK) a.cg_acc_zero[i] = 0.0;  // slots of launch j+1
    // (one instance per preconditioner form, so each staging path is branch-free)
    const bool go =
        a.cg_block
            ? cg_stage_brick<T, NEED_L, true>(a, n, a0, b0, c0, s_red, s_x, s_y, s_b, s_l, s_fx, cg_g, cg_rr, early)
            : cg_stage_brick<T, NEED_L, false>(a, n, a0, b0, c0, s_red, s_x, s_y, s_b, s_l, s_fx, cg_g, cg_rr, early);
    if (!go) return;
  } else {  // all loads of the lane first, then the LDS stores
    T v[STAGE_IT], vl[STAGE_IT];
    unsigned char mk[STAGE_IT];
    bool in[STAGE_IT];
    const bool bc = a.apply_bc && a.mask;
#pragma unroll
    for (int t = 0; t < STAGE_IT; ++t) {
      const int i = tid + t * EBLOCK;
      const int c = i % 3, nd = i / 3;
      const int li = nd % NX, lj = (nd / NX) % NY, lk = nd / (NX * NY);
      const int gi = a0 + li, gj = b0 + lj, gk = c0 + lk;
      in[t] = i < NN * 3 && gi <= n && gj <= n && gk <= n;
      const int64_t dof = in[t] ? 3 * (gi + np1 * (gj + np1 * gk)) + c : 0;
      v[t] = in[t] ? X[dof] : T(0);
      vl[t] = NEED_L && in[t] ? XL[dof] : T(0);
      mk[t] = bc ? a.mask[dof] : (unsigned char)0;
    }
    early();
#pragma unroll
    for (int t = 0; t < STAGE_IT; ++t) {
      const int i = tid + t * EBLOCK;
      if (i >= NN * 3) break;
      int mkv = mk[t];
      asm volatile("" : "+v"(mkv));  // (the flag test stays here, see cg_stage_brick)
      const bool fx = in[t] && mkv != 0;
      s_fx[i] = fx ? 1 : 0;
      s_x[i] = (APPLY_LIKE && fx) ? T(0) : v[t];
      if (OP != OP_VJP) s_y[i] = 0;
      if (NEED_L) s_l[i] = vl[t];
    }
  }
  __syncthreads();

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

    // Neo-Hookean operator: F^-T and ln J of the linearisation, stored by the residual per
    // Gauss point ([10][8][n_el]), requested one point ahead of their use
    const bool nh_el = MS == MS_NH && pc.model == FE_NEOHOOKE;
    auto load_nh = [&](int qp, T* w) {
#pragma unroll
      for (int k = 0; k < 10; ++k) w[k] = nh_el ? tang_c[(int64_t)(k * 8 + qp) * ne + e] : T(0);
    };
    if (APPLY_LIKE && MS == MS_NH && !NH_EARLY) load_nh(0, nw[0]);

    T Px[2][2][3], Py[2][2][3], Pz[2][2][3];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int c = 0; c < 3; ++c) Px[x][y][c] = Py[x][y][c] = Pz[x][y][c] = 0;

    // J2 operator: the first stored-tangent word of every Gauss point arrived with the staging
    // (tq0); the five plastic-point words are requested PF Gauss points ahead of their use (a
    // ring of PF + 1 register sets: 2 measured best, 3 costs more registers than it hides)
    constexpr int PF = 2;
    T pw[PF + 1][5];
    auto load_pw = [&](int qp, T* w) {
#pragma unroll
      for (int k = 1; k < 6; ++k) w[k - 1] = tq0[qp] >= 0 ? tang_c[(int64_t)(k * 8 + qp) * ne + e] : T(0);
    };
    if (APPLY_LIKE && MS == MS_J2)
#pragma unroll
      for (int q0 = 0; q0 < PF; ++q0) load_pw(q0, pw[q0]);
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
          if (APPLY_LIKE && MS == MS_J2 && qp + PF < 8) load_pw(qp + PF, pw[(qp + PF) % (PF + 1)]);
          if (APPLY_LIKE && MS == MS_NH && qp < 7) load_nh(qp + 1, nw[(qp + 1) & 1]);
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
              if (a.sur_mode != SUR_OFF) {
                const int64_t pidx = (int64_t)qp * ne + e;
                const bool ptrial = tn[0] >= 0;  // elastic trial is plastic: the surrogate's domain
                if (a.sur_mode == SUR_CAPTURE) {
                  const bool keep = ptrial && (((unsigned)pidx * 2654435761u + a.sur_salt) % a.sur_stride == 0);
                  const unsigned slot = wave_append(a.sur_count, keep);
                  if (keep && slot < a.sur_cap) {
                    sur_inputs(H, epn, an, a.sur_sin, a.sur_x + (int64_t)slot * 13);
                    const T rt2 = T(1.41421356237309504880), is = T(1) / T(a.sur_sout);
                    float* yo = a.sur_y + (int64_t)slot * 6;
                    yo[0] = float(S[0][0] * is);
                    yo[1] = float(S[1][1] * is);
                    yo[2] = float(S[2][2] * is);
                    yo[3] = float(S[1][2] * rt2 * is);
                    yo[4] = float(S[0][2] * rt2 * is);
                    yo[5] = float(S[0][1] * rt2 * is);
                  }
                } else if (a.sur_mode == SUR_CLASSIFY) {
                  const unsigned slot = wave_append(a.sur_count, ptrial);
                  const bool listed = ptrial && slot < a.sur_cap;
                  a.sur_map[pidx] = listed ? (int)slot : -1;
                  if (listed) sur_inputs(H, epn, an, a.sur_sin, a.sur_x + (int64_t)slot * 13);
                } else {  // SUR_CONSUME
                  const int slot = a.sur_map[pidx];
                  bool accepted = false, fallback = false;
                  if (ptrial && slot >= 0) {
                    T Ss[3][3], eps2[6], al2;
                    float* Dsym = static_cast<float*>(a.sur_D) + (int64_t)slot * 36;
                    accepted = sur_consume(H, epn, an, Kb, Gs, sy, Hh, a.sur_y + (int64_t)slot * 6,
                                           a.sur_jac + (int64_t)slot * 36, a.sur_sin, a.sur_sout, a.sur_tol, tn,
                                           Ss, eps2, al2, Dsym, a.sur_full);
                    fallback = !accepted;
                    if (accepted) {
#pragma unroll
                      for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int j = 0; j < 3; ++j) S[i][j] = Ss[i][j];
#pragma unroll
                      for (int k = 0; k < 6; ++k) ep[k] = eps2[k];
                      al = al2;
                      tn[0] = T(SUR_FLAG);
                    }
                  }
                  wave_count(a.sur_stats, accepted);
                  wave_count(a.sur_stats + 1, fallback);
                }
              }
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
              tn[0] = tq0[qp];
              if (tn[0] < T(-1.5)) {  // surrogate tangent of this point
                const int slot = a.sur_map[(int64_t)qp * ne + e];
                general_apply(H, static_cast<const float*>(a.sur_D) + (int64_t)slot * 36, S);
              } else {
#pragma unroll
                for (int k = 1; k < 6; ++k) tn[k] = pw[qp % (PF + 1)][k - 1];
                j2_tangent_coeffs(tn, Kb, Gs, Hh, lp, mp, beta, N);
                j2_apply(H, lp, mp, beta, N, S);
              }
              done = true;
            }
          }
          if (MS == MS_NH && pc.model == FE_NEOHOOKE) {
            if (APPLY_LIKE) {
              T FiT[3][3];
#pragma unroll
              for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) FiT[i][j] = nw[qp & 1][3 * i + j];
              nh_apply(H, FiT, nw[qp & 1][9], lam, mu, S);
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

  // deterministic mode: the element's nodal forces to the per-element buffer (summed later in
  // fixed order by det_gather), the stress integral to this workgroup's partial slot
  if constexpr (OP == OP_RESID || OP == OP_APPLY) {
    if (a.elf) {
      if (valid) {
        T* F = static_cast<T*>(a.elf);
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
          for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
              for (int c = 0; c < 3; ++c) F[(int64_t)(3 * (i + 2 * j + 4 * k) + c) * ne + e] = Fo[k][j][i][c];
      }
      if (OP == OP_RESID && a.stress_sum) {
        __syncthreads();
        if (tid < 6) {
          double v = 0;
          for (int w = 0; w < EBLOCK / 64; ++w) v += s_red[tid][w];
          a.stress_part[(int64_t)blockIdx.x * 6 + tid] = v;
        }
      }
      return;
    }
  }

  if (OP == OP_VJP) {
    if (valid) {
      // the element's nodal forces sum to zero, so lambda may be taken relative to its
      // element mean: exact, and it removes the cancellation of a large rigid part
      double lm[3] = {0, 0, 0};
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int c = 0; c < 3; ++c) lm[c] += (double)s_l[3 * ((ex + i) + NX * ((ey + j) + NY * (ez + k))) + c];
      double d = 0;
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int c = 0; c < 3; ++c)
              d += (double)Fo[k][j][i][c] *
                   ((double)s_l[3 * ((ex + i) + NX * ((ey + j) + NY * (ez + k))) + c] - 0.125 * lm[c]);
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

  // nodal sums in LDS: workgroup-scope FP64 atomic adds by all lanes at once (one corner per
  // instruction, so the lanes of a wave address distinct nodes); measured 12 % faster per
  // FP64 CG iteration than 8 colour passes with a barrier each (FP32 float LDS atomics were
  // twice as slow as the passes, hence FP64 sums for FP32 problems as well)
  if (valid) {
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int c = 0; c < 3; ++c)
            __hip_atomic_fetch_add(&s_y[3 * ((ex + i) + NX * ((ey + j) + NY * (ez + k))) + c],
                                   (Acc)Fo[k][j][i][c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  __syncthreads();

  if (OP == OP_RESID && a.stress_sum && tid < 6) {
    double v = 0;
    for (int w = 0; w < EBLOCK / 64; ++w) v += s_red[tid][w];
    atomic_add(a.stress_sum + tid, v);
  }

  T* Y = static_cast<T*>(a.y);
  if (!Y) return;
#pragma unroll 1  // (unrolled, the instance spills)
  for (int t = 0; t < STAGE_IT; ++t) {
    const int i = tid + t * EBLOCK;
    if (i >= NN * 3) break;
    const int c = i % 3, nd = i / 3;
    const int li = nd % NX, lj = (nd / NX) % NY, lk = nd / (NX * NY);
    const int gi = a0 + li, gj = b0 + lj, gk = c0 + lk;
    if (gi > n || gj > n || gk > n) continue;
    const int64_t dof = 3 * (gi + np1 * (gj + np1 * gk)) + c;
    const bool own = (min(gi, n - 1) - a0 < TX) && (min(gj, n - 1) - b0 < TY) && (min(gk, n - 1) - c0 < TZ);
    const bool priv = (gi == 0 || li >= 1) && (gi == n || li < TX) && (gj == 0 || lj >= 1) && (gj == n || lj < TY) &&
                      (gk == 0 || lk >= 1) && (gk == n || lk < TZ);
    if (s_fx[i]) {
      if (own) {
        if (OP == OP_CG_APPLY) {  // A u = u on constrained dofs; their (u, A u) share is u^2
          const T v = s_b[i];
          Y[dof] = v;
          pq += (double)v * (double)v;
        } else {
          Y[dof] = (OP == OP_APPLY) ? X[dof] : T(0);
        }
      }
      continue;
    }
    if (priv)
      Y[dof] = T(s_y[i]);
    else
      atomic_add(Y + dof, T(s_y[i]));
  }
  if (OP == OP_CG_APPLY) {  // partials of (u_j, A u_j), (r_j, u_j), ||r_j||^2
    double q3[3] = {pq, cg_g, cg_rr};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) q3[k] += __shfl_down(q3[k], off, 64);
    }
    if ((tid & 63) == 0)
#pragma unroll
      for (int k = 0; k < 3; ++k) s_red[3 + k][tid >> 6] = q3[k];
    __syncthreads();
    if (threadIdx.x == 0) {  // workgroups share CGS_SLOTS slots per quantity
      double t0 = 0, t1 = 0, t2 = 0;
      for (int w = 0; w < EBLOCK / 64; ++w) {
        t0 += s_red[3][w];
        t1 += s_red[4][w];
        t2 += s_red[5][w];
      }
      const int sl = (int)(blockIdx.x % CGS_SLOTS);
      atomic_add(a.cg_acc_out + sl, t0);
      atomic_add(a.cg_acc_out + CGS_SLOTS + sl, t1);
      atomic_add(a.cg_acc_out + 2 * CGS_SLOTS + sl, t2);
    }
  }
}

static int elem_grid(int n) {
  const int nb = ((n + TX - 1) / TX) * ((n + TY - 1) / TY) * ((n + TZ - 1) / TZ);
  return 8 * ((nb + 7) / 8);
}

template <typename T, int OP>
static hipError_t launch_elem_t(const fe_problem* p, const ElemArgs& a, const int* stop, hipStream_t s) {
  const dim3 grid(elem_grid(p->n)), block(EBLOCK);
  if constexpr (sizeof(T) == 4 && OP != OP_VJP) {
    if (p->acc32) {
      switch (p->model_set) {
        case MS_J2: timed_launch((elem_kernel<T, OP, MS_J2, true>), grid, block, 0, s, a, stop); break;
        case MS_NH: timed_launch((elem_kernel<T, OP, MS_NH, true>), grid, block, 0, s, a, stop); break;
        default: timed_launch((elem_kernel<T, OP, MS_LINEAR, true>), grid, block, 0, s, a, stop);
      }
      return hipGetLastError();
    }
  }
  switch (p->model_set) {
    case MS_J2:
      timed_launch((elem_kernel<T, OP, MS_J2>), grid, block, 0, s, a, stop);
      break;
    case MS_NH:
      timed_launch((elem_kernel<T, OP, MS_NH>), grid, block, 0, s, a, stop);
      break;
    default:
      timed_launch((elem_kernel<T, OP, MS_LINEAR>), grid, block, 0, s, a, stop);
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_elem_op(const fe_problem* p, int op, const ElemArgs& a, const int* stop, hipStream_t s) {
  if (p->deterministic && (op == OP_RESID || op == OP_APPLY)) {
    // element forces to the buffer, then the fixed-order node gather (no atomics)
    ElemArgs d = a;
    d.elf = p->w_elf;
    d.stress_part = p->stress_part;
    hipError_t e = op == OP_RESID ? launch_elem_t<T, OP_RESID>(p, d, stop, s) : launch_elem_t<T, OP_APPLY>(p, d, stop, s);
    if (e != hipSuccess) return e;
    if (op == OP_RESID && a.stress_sum && (e = det_stress_reduce(p, s)) != hipSuccess) return e;
    if (!a.y) return hipSuccess;
    return det_gather(p, p->w_elf, op == OP_RESID ? 0 : 1, a.apply_bc, a.x, a.y, stop, nullptr, s);
  }
  if (op == OP_RESID) return launch_elem_t<T, OP_RESID>(p, a, stop, s);
  if (op == OP_APPLY) return launch_elem_t<T, OP_APPLY>(p, a, stop, s);
  return launch_elem_t<T, OP_VJP>(p, a, stop, s);
}

hipError_t launch_elem_stop(const fe_problem* p, int op, const ElemArgs& a, const int* stop, hipStream_t s) {
  if (p->general) return gen_launch_elem(p, op, a, stop, s);
  return p->prec == FE_F64 ? launch_elem_op<double>(p, op, a, stop, s) : launch_elem_op<float>(p, op, a, stop, s);
}

hipError_t launch_elem(const fe_problem* p, int op, const ElemArgs& a, hipStream_t s) {
  if (p->general) return gen_launch_elem(p, op, a, nullptr, s);
  return p->prec == FE_F64 ? launch_elem_op<double>(p, op, a, nullptr, s) : launch_elem_op<float>(p, op, a, nullptr, s);
}

// ---------------------------------------------------------------------------
// Gradient of the basis function of brick-local node (i,j,k) at Gauss point (p,q,r).
template <typename T>
__device__ __forceinline__ void basis_grad(int i, int j, int k, int p, int q, int r, T inv_h, T g[3]) {
  const T mi = (i == p) ? T(GA) : T(GB), mj = (j == q) ? T(GA) : T(GB), mk = (k == r) ? T(GA) : T(GB);
  const T si = i ? inv_h : -inv_h, sj = j ? inv_h : -inv_h, sk = k ? inv_h : -inv_h;
  g[0] = si * mj * mk;
  g[1] = mi * sj * mk;
  g[2] = mi * mj * sk;
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
  a.sur_map = p->sur_map;
  a.sur_D = p->sur_D;
  return a;
}

// Diagonal of K: one lane per element, 24 entries added atomically (d zeroed before).
template <typename T, int MS>
__global__ __launch_bounds__(256) void diag_kernel(TanArgs a, T* d, T* elf) {
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
        for (int c = 0; c < 3; ++c) {
          if (elf)  // deterministic mode: summed later in fixed element order
            elf[(int64_t)(3 * (i + 2 * j + 4 * k) + c) * a.n_el + e] = acc[k][j][i][c];
          else
            atomic_add(d + 3 * ((ea + i) + np1 * ((eb + j) + np1 * (ec + k))) + c, acc[k][j][i][c]);
        }
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
  T* elf = p->deterministic ? static_cast<T*>(p->w_elf) : nullptr;
  if (!elf) hipLaunchKernelGGL(fill_kernel<T>, dim3(vgrid(p->n_dof)), dim3(VBLOCK), 0, s, d, p->n_dof, T(0));
  const TanArgs a = tan_args(p);
  const dim3 grid((unsigned)((p->n_el + 255) / 256));
  switch (p->model_set) {
    case MS_J2: hipLaunchKernelGGL((diag_kernel<T, MS_J2>), grid, dim3(256), 0, s, a, d, elf); break;
    case MS_NH: hipLaunchKernelGGL((diag_kernel<T, MS_NH>), grid, dim3(256), 0, s, a, d, elf); break;
    default: hipLaunchKernelGGL((diag_kernel<T, MS_LINEAR>), grid, dim3(256), 0, s, a, d, elf);
  }
  if (elf) return det_gather(p, elf, 2, apply_bc, nullptr, d, nullptr, nullptr, s);
  if (apply_bc && p->mask)
    hipLaunchKernelGGL(mask_set_kernel<T>, dim3(vgrid(p->n_dof)), dim3(VBLOCK), 0, s, d, p->mask, p->n_dof, T(1));
  return hipGetLastError();
}

hipError_t launch_diag(const fe_problem* p, void* d, int apply_bc, hipStream_t s) {
  if (p->general) return gen_diag(p, d, 3, apply_bc, tan_args(p), s);
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
  if (p->general) return gen_csr_pattern(p, row_ptr, col_idx, s);
  hipLaunchKernelGGL(csr_pattern_kernel, dim3((unsigned)((p->n_nodes + 255) / 256)), dim3(256), 0, s, p->n, row_ptr,
                     col_idx);
  return hipGetLastError();
}

// CSR values (linear, J2 with the surrogate's Voigt tangents, Neo-Hookean): a workgroup takes
// TR_NODES consecutive nodes of one x-row of nodes, whose CSR rows are one contiguous segment.
// Phase 1 forms the Gauss-point coefficients of the elements around the tile once into LDS
// ((lp, mp, beta, N) of the small-strain laws; lam, mu, F^-T, ln J at Neo-Hookean points).  Phase 2: lane (node, task), one wave per node; the 64 tasks
// of a node are the (neighbour, shared element) pairs: per axis the neighbour offset d and the
// element offset o (element = node + o) take (d, o) = (-1, -1), (0, -1), (0, 0) or (1, 0), so
// 4^3 tasks cover the 27 neighbours with their 1, 2, 4 or 8 shared elements; each lane sums
// its element's 3x3 block over the 8 Gauss points.  Phase 3 writes the tile's rows in order,
// each entry the fixed-order sum of its neighbour's tasks (deterministic, no atomics).
constexpr int TR_NODES = 4;
constexpr int TR_SETS = (TR_NODES + 1) * 2 * 2 * 8;  // (element, Gauss point) coefficient sets

template <typename T, int MS>
__global__ __launch_bounds__(256) void tangent_rows_kernel(TanArgs a, T* vals, int apply_bc) {
  // per set, component-major: small-strain laws lp, mp, beta, N (xx yy zz yz xz xy); Neo-Hookean
  // problems lam, mu, a flag (1: Neo-Hookean point, 0: linear phase), F^-T (row-major), ln J
  constexpr int NCO = MS == MS_NH ? 13 : 9;
  __shared__ T s_co[NCO][TR_SETS];
  __shared__ int s_sur[TR_SETS];  // surrogate points: slot of their Voigt tangent, else -1
  __shared__ T s_part[9][256];    // each task's 3x3 block, component-major (conflict-free)
  __shared__ uint8_t s_mk[3][3][TR_NODES + 2][3];  // constrained flags of the tile's nodes and neighbours
  __shared__ uint8_t s_uni[TR_SETS / 8];           // element with one isotropic (lp, mp) at all 8 points
  const int n = a.n;
  const int64_t np1 = n + 1, ne = a.n_el;
  const int tiles_x = (n + TR_NODES) / TR_NODES;  // ceil((n + 1) / TR_NODES)
  const int64_t nrow = (int64_t)blockIdx.x / tiles_x;
  const int i0 = (int)(blockIdx.x % tiles_x) * TR_NODES;
  const int j = (int)(nrow % np1), k = (int)(nrow / np1);
  const int tid = threadIdx.x;
  const T inv_h = T(1.0 / a.h), w = T(0.125 * a.h * a.h * a.h);

  // phase 1: elements (i0 - 1 .. i0 + TR_NODES - 1) x (j - 1, j) x (k - 1, k), all 8 points.
  // Every load of the phase is issued before any of them is used: the constrained-dof flags of
  // the tile's nodes, and per set the phase id, modulus scale and the stored-tangent words (six
  // for J2, ten for Neo-Hookean problems; read for every element: the words exist for all of
  // them and are used at points of that law only)
  static_assert(TR_SETS <= 256, "one coefficient set per lane");
  uint8_t mk_v = 0;
  const bool mk_lane = tid < 27 * (TR_NODES + 2);
  int mk_c = 0, mk_x = 0, mk_y = 0, mk_z = 0;
  if (mk_lane) {  // nodes (i0 - 1 .. i0 + TR_NODES) x (j - 1 .. j + 1) x (k - 1 .. k + 1)
    mk_c = tid % 3;
    mk_x = (tid / 3) % (TR_NODES + 2);
    mk_y = (tid / (3 * (TR_NODES + 2))) % 3;
    mk_z = tid / (9 * (TR_NODES + 2));
    const int gx = i0 - 1 + mk_x, gy = j - 1 + mk_y, gz = k - 1 + mk_z;
    const bool in = apply_bc && a.mask && gx >= 0 && gx <= n && gy >= 0 && gy <= n && gz >= 0 && gz <= n;
    mk_v = in ? a.mask[3 * (gx + np1 * (gy + np1 * (int64_t)gz)) + mk_c] : (uint8_t)0;
  }
  {
    const int si = tid;
    const int qp = si & 7, el = si >> 3;
    const int xl = el % (TR_NODES + 1), yl = (el / (TR_NODES + 1)) & 1, zl = el / (2 * (TR_NODES + 1));
    const int ea = i0 - 1 + xl, eb = j - 1 + yl, ec = k - 1 + zl;
    T co[NCO];
#pragma unroll
    for (int q = 0; q < NCO; ++q) co[q] = 0;
    int sur = -1;
    if (si < TR_SETS && ea >= 0 && ea < n && eb >= 0 && eb < n && ec >= 0 && ec < n) {
      const int64_t e = ea + (int64_t)n * (eb + (int64_t)n * ec);
      const int ph = a.phase[e];
      const T sc = a.scale ? static_cast<const T*>(a.scale)[e] : T(1);
      constexpr int NW = MS == MS_NH ? 10 : 6;
      T tn[NW];
      if (MS != MS_LINEAR) {
        const T* tg = static_cast<const T*>(a.tangent);
#pragma unroll
        for (int q = 0; q < NW; ++q) tn[q] = tg[(int64_t)(q * 8 + qp) * ne + e];
      }
      const PhaseConst pc = a.mat.ph[ph];
      co[0] = T(pc.lam) * sc;
      co[1] = T(pc.mu) * sc;
      if (MS == MS_NH && pc.model == FE_NEOHOOKE) {
        co[2] = 1;
#pragma unroll
        for (int q = 0; q < 10; ++q) co[3 + q] = tn[q];
      }
      if (MS == MS_J2 && pc.model == FE_J2) {
        T N[6];
        if (tn[0] < T(-1.5)) {
          sur = a.sur_map[(int64_t)qp * ne + e];
        } else {
          j2_tangent_coeffs(tn, T(pc.K) * sc, T(pc.G) * sc, T(pc.H), co[0], co[1], co[2], N);
#pragma unroll
          for (int q = 0; q < 6; ++q) co[3 + q] = N[q];
        }
      }
    }
    // an element whose 8 points share lp, mp and have no plastic or surrogate term is summed in
    // closed form in phase 2 (the 8 lanes of an element are one aligned group of a wave)
    const T lp0 = __shfl(co[0], tid & ~7, 64), mp0 = __shfl(co[1], tid & ~7, 64);
    const bool iso = si < TR_SETS && co[2] == T(0) && sur < 0 && co[0] == lp0 && co[1] == mp0;
    const unsigned long long bal = __ballot(iso);
    if (si < TR_SETS) {
#pragma unroll
      for (int q = 0; q < NCO; ++q) s_co[q][si] = co[q];
      s_sur[si] = sur;
      if ((si & 7) == 0) s_uni[si >> 3] = ((bal >> (tid & 63 & ~7)) & 0xffull) == 0xffull ? 1 : 0;
    }
  }
  if (mk_lane) s_mk[mk_z][mk_y][mk_x][mk_c] = mk_v;
  __syncthreads();

  // phase 2: one task per lane
  const int nl = tid >> 6, task = tid & 63;
  const int i = i0 + nl;
  const int tx = task & 3, ty = (task >> 2) & 3, tz = task >> 4;
  const int dx = tx == 0 ? -1 : (tx == 3 ? 1 : 0), dy = ty == 0 ? -1 : (ty == 3 ? 1 : 0),
            dz = tz == 0 ? -1 : (tz == 3 ? 1 : 0);
  const int ox = tx <= 1 ? -1 : 0, oy = ty <= 1 ? -1 : 0, oz = tz <= 1 ? -1 : 0;
  const int ea = i + ox, eb = j + oy, ec = k + oz;
  T B[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  const int sb = (((oz + 1) * 2 + (oy + 1)) * (TR_NODES + 1) + (nl + ox + 1)) * 8;
  const bool task_ok = i <= n && ea >= 0 && ea < n && eb >= 0 && eb < n && ec >= 0 && ec < n;
  if (task_ok && s_uni[sb >> 3]) {
    // sum over the 8 points in closed form: with A = sum_q w ga gb^T (geometry only),
    // B = lp A + mp (tr(A) I + A^T); per axis the Gauss sums of the two corners' 1-D factors are
    // S = sum_p phi_a(g_p) phi_b(g_p) (GA^2 + GB^2 on equal corners, 2 GA GB otherwise) and
    // sum_p phi(g_p) = 1, the derivative factors are +-1/h
    const T lp = s_co[0][sb], mp = s_co[1][sb];
    const int ca[3] = {-ox, -oy, -oz}, cb[3] = {dx - ox, dy - oy, dz - oz};
    T sg[3], S[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      sg[c] = (ca[c] == cb[c] ? inv_h : -inv_h) * inv_h;  // s_a s_b
      S[c] = ca[c] == cb[c] ? T(GA * GA + GB * GB) : T(2 * GA * GB);
    }
    const T sa[3] = {ca[0] ? inv_h : -inv_h, ca[1] ? inv_h : -inv_h, ca[2] ? inv_h : -inv_h};
    const T sbv[3] = {cb[0] ? inv_h : -inv_h, cb[1] ? inv_h : -inv_h, cb[2] ? inv_h : -inv_h};
    T A[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int d = 0; d < 3; ++d)
        A[c][d] = c == d ? w * 2 * sg[c] * S[(c + 1) % 3] * S[(c + 2) % 3] : w * sa[c] * sbv[d] * S[3 - c - d];
    const T tr = mp * (A[0][0] + A[1][1] + A[2][2]);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int d = 0; d < 3; ++d) B[c][d] = lp * A[c][d] + mp * A[d][c] + (c == d ? tr : T(0));
  } else if (task_ok) {
#pragma unroll
    for (int qp = 0; qp < 8; ++qp) {
      const int p = qp & 1, q = (qp >> 1) & 1, r = qp >> 2;
      T ga[3], gb[3];
      basis_grad(-ox, -oy, -oz, p, q, r, inv_h, ga);               // the row node's corner
      basis_grad(dx - ox, dy - oy, dz - oz, p, q, r, inv_h, gb);   // the neighbour's corner
      T co[NCO];
#pragma unroll
      for (int q = 0; q < NCO; ++q) co[q] = s_co[q][sb + qp];
      const int sur = MS == MS_J2 ? s_sur[sb + qp] : -1;
      if (MS == MS_NH && co[2] != T(0)) {
        // w (mu (ga.gb) I + (mu - lam ln J) (F^-T gb)(F^-T ga)^T + lam (F^-T ga)(F^-T gb)^T)
        T va[3], vb[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          va[c] = co[3 + 3 * c] * ga[0] + co[4 + 3 * c] * ga[1] + co[5 + 3 * c] * ga[2];
          vb[c] = co[3 + 3 * c] * gb[0] + co[4 + 3 * c] * gb[1] + co[5 + 3 * c] * gb[2];
        }
        const T wm = w * co[1], wc = w * (co[1] - co[0] * co[12]), wl = w * co[0];
        const T t = wm * (ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2]);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          B[c][c] += t;
#pragma unroll
          for (int d = 0; d < 3; ++d) B[c][d] += wc * vb[c] * va[d] + wl * va[c] * vb[d];
        }
      } else if (sur >= 0) {
        QpTangent<T> t;
        t.kind = 2;
        t.D = static_cast<const float*>(a.sur_D) + (int64_t)sur * 36;
        block_add(t, ga, gb, w, B);
      } else {
        // w (lp ga gb^T + mp (ga.gb I + gb ga^T) - beta (N ga)(N gb)^T), three FMAs an entry
        const T wl = w * co[0], wm = w * co[1];
        const T u[3] = {wl * ga[0], wl * ga[1], wl * ga[2]}, v[3] = {wm * ga[0], wm * ga[1], wm * ga[2]};
        const T t = v[0] * gb[0] + v[1] * gb[1] + v[2] * gb[2];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          B[c][c] += t;
#pragma unroll
          for (int d = 0; d < 3; ++d) B[c][d] += u[c] * gb[d] + v[d] * gb[c];
        }
        if (MS == MS_J2 && co[2] != T(0)) {  // (a wave skips it when its elements are elastic there)
          const T wb = w * co[2];
          const T na[3] = {wb * (co[3] * ga[0] + co[8] * ga[1] + co[7] * ga[2]),
                           wb * (co[8] * ga[0] + co[4] * ga[1] + co[6] * ga[2]),
                           wb * (co[7] * ga[0] + co[6] * ga[1] + co[5] * ga[2])};
          const T nb[3] = {co[3] * gb[0] + co[8] * gb[1] + co[7] * gb[2], co[8] * gb[0] + co[4] * gb[1] + co[6] * gb[2],
                           co[7] * gb[0] + co[6] * gb[1] + co[5] * gb[2]};
#pragma unroll
          for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int d = 0; d < 3; ++d) B[c][d] -= na[c] * nb[d];
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int d = 0; d < 3; ++d) s_part[3 * c + d][tid] = B[c][d];
  __syncthreads();

  // phase 3: one lane per (node, neighbour) block: the fixed-order sum of the neighbour's tasks,
  // written as three column triplets into the node's three rows (the tile's rows are one
  // contiguous segment of the CSR values, neighbours in rank order inside each row)
  const int cy = axis_cnt(j, n), cz = axis_cnt(k, n);
  if (tid < 27 * TR_NODES) {
    const int m = tid / 27, nb = tid - 27 * m;
    const int ii = i0 + m;
    const int ddx = nb % 3 - 1, ddy = (nb / 3) % 3 - 1, ddz = nb / 9 - 1;
    const int cx = ii <= n ? axis_cnt(ii, n) : 0;
    if (ii <= n && ii + ddx >= 0 && ii + ddx <= n && j + ddy >= 0 && j + ddy <= n && k + ddz >= 0 &&
        k + ddz <= n) {
      const int len = 3 * cx * cy * cz;
      const int rank = (axis_rank(k, ddz) * cy + axis_rank(j, ddy)) * cx + axis_rank(ii, ddx);
      // the neighbour's tasks per axis: d = -1 -> task 0, d = 0 -> tasks 1, 2, d = 1 -> task 3
      const int ax0 = ddx < 0 ? 0 : (ddx == 0 ? 1 : 3), ax1 = ddx == 0 ? 2 : ax0;
      const int ay0 = ddy < 0 ? 0 : (ddy == 0 ? 1 : 3), ay1 = ddy == 0 ? 2 : ay0;
      const int az0 = ddz < 0 ? 0 : (ddz == 0 ? 1 : 3), az1 = ddz == 0 ? 2 : az0;
      T v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
      for (int zz = az0; zz <= az1; ++zz)
        for (int yy = ay0; yy <= ay1; ++yy)
          for (int xx = ax0; xx <= ax1; ++xx) {
            const int tk = m * 64 + xx + 4 * yy + 16 * zz;
#pragma unroll
            for (int q = 0; q < 9; ++q) v[q] += s_part[q][tk];
          }
      const bool self = ddx == 0 && ddy == 0 && ddz == 0;
      T* out = vals + node_row_start(ii, j, k, n) + 3 * rank;
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          T x = v[3 * c + d];
          if (s_mk[1][1][m + 1][c] || s_mk[1 + ddz][1 + ddy][m + 1 + ddx][d]) x = (self && c == d) ? T(1) : T(0);
          out[(int64_t)c * len + d] = x;
        }
    }
  }
}

hipError_t launch_tangent_csr(const fe_problem* p, void* vals, int apply_bc, hipStream_t s) {
  if (p->general) return gen_tangent(p, vals, apply_bc, tan_args(p), s);
  const TanArgs a = tan_args(p);
  const int64_t np1 = p->n + 1;
  const dim3 grid((unsigned)(np1 * np1 * ((np1 + TR_NODES - 1) / TR_NODES))), block(256);
  if (p->prec == FE_F64) {
    double* v = (double*)vals;
    switch (p->model_set) {
      case MS_J2: timed_launch((tangent_rows_kernel<double, MS_J2>), grid, block, 0, s, a, v, apply_bc); break;
      case MS_NH: timed_launch((tangent_rows_kernel<double, MS_NH>), grid, block, 0, s, a, v, apply_bc); break;
      default: timed_launch((tangent_rows_kernel<double, MS_LINEAR>), grid, block, 0, s, a, v, apply_bc);
    }
  } else {
    float* v = (float*)vals;
    switch (p->model_set) {
      case MS_J2: timed_launch((tangent_rows_kernel<float, MS_J2>), grid, block, 0, s, a, v, apply_bc); break;
      case MS_NH: timed_launch((tangent_rows_kernel<float, MS_NH>), grid, block, 0, s, a, v, apply_bc); break;
      default: timed_launch((tangent_rows_kernel<float, MS_LINEAR>), grid, block, 0, s, a, v, apply_bc);
    }
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// CSR sparse mat-vec: LPR lanes per row, contiguous row segments (coalesced),
// butterfly reduction inside the lane group.

// One lane's share of a CSR row dot product: entries b + lane, b + lane + LPR, ... < e, two
// column steps per batch with both index loads, gathers and values issued before the
// multiply-adds (the gather depends on its index load; one step at a time serialises the two),
// summed in entry order.
template <typename T, int LPR>
__device__ __forceinline__ T csr_row_dot(const int32_t* __restrict__ ci, const T* __restrict__ v,
                                         const T* __restrict__ x, int b, int e, int lane) {
  T acc = 0;
  int k = b + lane;
  for (; k + LPR < e; k += 2 * LPR) {
    const int c0 = ci[k], c1 = ci[k + LPR];
    const T v0 = v[k], v1 = v[k + LPR];
    const T x0 = x[c0], x1 = x[c1];
    acc += v0 * x0;
    acc += v1 * x1;
  }
  if (k < e) acc += v[k] * x[ci[k]];
  return acc;
}

template <typename T, int LPR>
__global__ __launch_bounds__(256) void spmv_kernel(int64_t n_rows, const int32_t* __restrict__ rp,
                                                   const int32_t* __restrict__ ci, const T* __restrict__ v,
                                                   const T* __restrict__ x, T* __restrict__ y, const int* stop) {
  if (stop && *stop) return;
  const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / LPR;
  const int lane = threadIdx.x % LPR;
  T acc = 0;
  if (row < n_rows) acc = csr_row_dot<T, LPR>(ci, v, x, rp[row], rp[row + 1], lane);
#pragma unroll
  for (int off = LPR / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, LPR);
  if (row < n_rows && lane == 0) y[row] = acc;
}

constexpr int SPMV_LPR = 16;

// Node-structured CSR (the pattern of the structured mesh): rows 3a, 3a+1, 3a+2 share one
// column list, so the column indices and the gathered x of the first row serve all three.
// LPN lanes per node; y = A x.
// Partial sums of the three rows b0, b1, b2 (one column list) against x for the columns
// k = lane, lane + LPN, ...: two column steps per batch, all their index loads, gathers and
// values issued before the multiply-adds (measured at 64^3 / 128^3: 0.44 -> 0.52-0.58 of 8 TB/s
// in FP32, 0.57 -> 0.63-0.65 in FP64, against one step at a time).
template <typename T, int LPN>
__device__ __forceinline__ void nodal_row_dot(const int32_t* __restrict__ ci, const T* __restrict__ v,
                                              const T* __restrict__ x, int b0, int b1, int b2, int len, int lane,
                                              T& a0, T& a1, T& a2) {
  int k = lane;
  for (; k + LPN < len; k += 2 * LPN) {
    const int c0 = ci[b0 + k], c1 = ci[b0 + k + LPN];
    const T v00 = v[b0 + k], v10 = v[b1 + k], v20 = v[b2 + k];
    const T v01 = v[b0 + k + LPN], v11 = v[b1 + k + LPN], v21 = v[b2 + k + LPN];
    const T x0 = x[c0], x1 = x[c1];
    a0 += v00 * x0 + v01 * x1;
    a1 += v10 * x0 + v11 * x1;
    a2 += v20 * x0 + v21 * x1;
  }
  if (k < len) {
    const T xv = x[ci[b0 + k]];
    a0 += v[b0 + k] * xv;
    a1 += v[b1 + k] * xv;
    a2 += v[b2 + k] * xv;
  }
}

template <typename T, int LPN>
__global__ __launch_bounds__(256) void spmv_nodal_kernel(int64_t n_nodes, const int32_t* __restrict__ rp,
                                                         const int32_t* __restrict__ ci, const T* __restrict__ v,
                                                         const T* __restrict__ x, T* __restrict__ y,
                                                         const int* stop) {
  if (stop && *stop) return;
  const int64_t nd = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / LPN;
  const int lane = threadIdx.x % LPN;
  T a0 = 0, a1 = 0, a2 = 0;
  if (nd < n_nodes) {
    const int b0 = rp[3 * nd], b1 = rp[3 * nd + 1], b2 = rp[3 * nd + 2];
    const int len = b1 - b0;
    nodal_row_dot<T, LPN>(ci, v, x, b0, b1, b2, len, lane, a0, a1, a2);
  }
#pragma unroll
  for (int off = LPN / 2; off > 0; off >>= 1) {
    a0 += __shfl_xor(a0, off, LPN);
    a1 += __shfl_xor(a1, off, LPN);
    a2 += __shfl_xor(a2, off, LPN);
  }
  if (nd < n_nodes && lane < 3) y[3 * nd + lane] = lane == 0 ? a0 : (lane == 1 ? a1 : a2);
}

constexpr int SPMV_LPN = 32;

template <typename T>
static hipError_t launch_spmv_nodal_t(const fe_problem* p, const int32_t* rp, const int32_t* ci, const T* v,
                                      const T* x, T* y, const int* stop, hipStream_t s) {
  const int64_t threads = p->n_nodes * SPMV_LPN;
  timed_launch((spmv_nodal_kernel<T, SPMV_LPN>), dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s,
               p->n_nodes, rp, ci, v, x, y, stop);
  return hipGetLastError();
}

hipError_t launch_spmv_nodal(const fe_problem* p, const int32_t* rp, const int32_t* ci, const void* v, const void* x,
                             void* y, hipStream_t s) {
  return p->prec == FE_F64
             ? launch_spmv_nodal_t(p, rp, ci, (const double*)v, (const double*)x, (double*)y, nullptr, s)
             : launch_spmv_nodal_t(p, rp, ci, (const float*)v, (const float*)x, (float*)y, nullptr, s);
}

template <typename T>
static hipError_t launch_spmv_t(const fe_problem* p, const int32_t* rp, const int32_t* ci, const T* v, const T* x,
                                T* y, const int* stop, hipStream_t s) {
  const int64_t threads = p->n_dof * SPMV_LPR;
  timed_launch((spmv_kernel<T, SPMV_LPR>), dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, p->n_dof,
                     rp, ci, v, x, y, stop);
  return hipGetLastError();
}

hipError_t launch_spmv(const fe_problem* p, const int32_t* rp, const int32_t* ci, const void* v, const void* x,
                       void* y, hipStream_t s) {
  return p->prec == FE_F64 ? launch_spmv_t(p, rp, ci, (const double*)v, (const double*)x, (double*)y, nullptr, s)
                           : launch_spmv_t(p, rp, ci, (const float*)v, (const float*)x, (float*)y, nullptr, s);
}

hipError_t launch_spmv_stop(const fe_problem* p, const int32_t* rp, const int32_t* ci, const void* v,
                            const void* x, void* y, const int* stop, hipStream_t s) {
  if (p->csr_nodal)
    return p->prec == FE_F64
               ? launch_spmv_nodal_t(p, rp, ci, (const double*)v, (const double*)x, (double*)y, stop, s)
               : launch_spmv_nodal_t(p, rp, ci, (const float*)v, (const float*)x, (float*)y, stop, s);
  return p->prec == FE_F64 ? launch_spmv_t(p, rp, ci, (const double*)v, (const double*)x, (double*)y, stop, s)
                           : launch_spmv_t(p, rp, ci, (const float*)v, (const float*)x, (float*)y, stop, s);
}

// One wave per node: rows 3a, 3a+1, 3a+2 must have one length and one column list.
__global__ __launch_bounds__(256) void csr_nodal_check_kernel(int64_t n_nodes, const int32_t* rp,
                                                              const int32_t* ci, int* flag) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t nd = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64; nd < n_nodes; nd += waves) {
    const int b0 = rp[3 * nd], b1 = rp[3 * nd + 1], b2 = rp[3 * nd + 2], e = rp[3 * nd + 3];
    bool bad = (b1 - b0 != b2 - b1) || (e - b2 != b1 - b0);
    if (!bad)
      for (int k = lane; k < b1 - b0; k += 64) bad = bad || ci[b0 + k] != ci[b1 + k] || ci[b0 + k] != ci[b2 + k];
    if (bad) *flag = 1;
  }
}

hipError_t launch_csr_nodal_check(const fe_problem* p, const int32_t* rp, const int32_t* ci, int* flag,
                                  hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((p->n_nodes + 3) / 4, 4096);
  hipLaunchKernelGGL(csr_nodal_check_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p->n_nodes, rp, ci, flag);
  return hipGetLastError();
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
// Node-block Jacobi: the 3x3 blocks of A on the diagonal, one per node, stored
// as 6 symmetric entries [n_nodes][6] in the order xx yy zz yz xz xy.

// Blocks of the matrix-free operator: one lane per element, 8 x 6 entries added atomically (blk zeroed before).
template <typename T, int MS>
__global__ __launch_bounds__(256) void block_diag_kernel(TanArgs a, T* blk) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= a.n_el) return;
  const int n = a.n;
  const int ea = (int)(e % n), eb = (int)((e / n) % n), ec = (int)(e / ((int64_t)n * n));
  const T inv_h = T(1.0 / a.h), w = T(0.125 * a.h * a.h * a.h);
  T acc[8][6] = {};
  for (int qp = 0; qp < 8; ++qp) {
    const int p = qp & 1, q = (qp >> 1) & 1, r = qp >> 2;
    QpTangent<T> t;
    load_qp_tangent<T, MS>(a, e, qp, t);
#pragma unroll
    for (int l = 0; l < 8; ++l) {
      T g[3], B[3][3] = {};
      basis_grad(l & 1, (l >> 1) & 1, l >> 2, p, q, r, inv_h, g);
      block_add(t, g, g, w, B);
      acc[l][0] += B[0][0];
      acc[l][1] += B[1][1];
      acc[l][2] += B[2][2];
      acc[l][3] += B[1][2];
      acc[l][4] += B[0][2];
      acc[l][5] += B[0][1];
    }
  }
  const int64_t np1 = n + 1;
#pragma unroll
  for (int l = 0; l < 8; ++l) {
    const int64_t node = (ea + (l & 1)) + np1 * ((eb + ((l >> 1) & 1)) + np1 * (ec + (l >> 2)));
#pragma unroll
    for (int k = 0; k < 6; ++k) atomic_add(blk + 6 * node + k, acc[l][k]);
  }
}

// Blocks of a CSR matrix with sorted columns: row 3a+c holds columns 3a..3a+2 next to each other.
template <typename T>
__global__ void csr_block_kernel(int64_t n_dof, const int32_t* rp, const int32_t* ci, const T* v, T* blk) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n_dof; r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t node = r / 3;
    const int c = (int)(r - 3 * node);
    T row[3] = {0, 0, 0};
    int lo = rp[r], hi = rp[r + 1] - 1;
    while (lo <= hi) {  // first stored column >= 3 node
      const int mid = (lo + hi) >> 1;
      if (ci[mid] < 3 * node)
        lo = mid + 1;
      else
        hi = mid - 1;
    }
    for (int k = lo; k < rp[r + 1] && ci[k] < 3 * node + 3; ++k) row[ci[k] - 3 * node] = v[k];
    T* b = blk + 6 * node;
    if (c == 0) {
      b[0] = row[0];
      b[5] = row[1];
      b[4] = row[2];
    } else if (c == 1) {
      b[1] = row[1];
      b[3] = row[2];
    } else {
      b[2] = row[2];
    }
  }
}

// In place: eliminate constrained components (zero row and column, 1 on the diagonal), then invert.
// The inverse is formed in double precision from the adjugate.
template <typename T>
__global__ void block_inv_kernel(int64_t n_nodes, const uint8_t* mask, T* blk, int* flags) {
  for (int64_t nd = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; nd < n_nodes;
       nd += (int64_t)gridDim.x * blockDim.x) {
    T* b = blk + 6 * nd;
    double m00 = b[0], m11 = b[1], m22 = b[2], m12 = b[3], m02 = b[4], m01 = b[5];
    if (mask) {
      const bool c0 = mask[3 * nd], c1 = mask[3 * nd + 1], c2 = mask[3 * nd + 2];
      if (c0) m00 = 1, m01 = 0, m02 = 0;
      if (c1) m11 = 1, m01 = 0, m12 = 0;
      if (c2) m22 = 1, m02 = 0, m12 = 0;
    }
    const double a00 = m11 * m22 - m12 * m12, a01 = m02 * m12 - m01 * m22, a02 = m01 * m12 - m02 * m11;
    const double a11 = m00 * m22 - m02 * m02, a12 = m01 * m02 - m00 * m12, a22 = m00 * m11 - m01 * m01;
    const double det = m00 * a00 + m01 * a01 + m02 * a02;
    if (!(det > 0.0) && flags) atomicOr(flags, 2);
    const double id = 1.0 / det;
    b[0] = T(a00 * id);
    b[1] = T(a11 * id);
    b[2] = T(a22 * id);
    b[3] = T(a12 * id);
    b[4] = T(a02 * id);
    b[5] = T(a01 * id);
  }
}

template <typename T> static hipError_t launch_block_t(const fe_problem* p, const int32_t* rp, const int32_t* ci,
                                                       const T* v, T* blk, hipStream_t s) {
  if (rp) {
    hipLaunchKernelGGL(csr_block_kernel<T>, dim3(vgrid(p->n_dof)), dim3(VBLOCK), 0, s, p->n_dof, rp, ci, v, blk);
  } else if (p->general) {
    const hipError_t e = gen_diag(p, blk, 6, 0, tan_args(p), s);
    if (e != hipSuccess) return e;
  } else {
    hipLaunchKernelGGL(fill_kernel<T>, dim3(vgrid(6 * p->n_nodes)), dim3(VBLOCK), 0, s, blk, 6 * p->n_nodes, T(0));
    const TanArgs a = tan_args(p);
    const dim3 grid((unsigned)((p->n_el + 255) / 256));
    switch (p->model_set) {
      case MS_J2: hipLaunchKernelGGL((block_diag_kernel<T, MS_J2>), grid, dim3(256), 0, s, a, blk); break;
      case MS_NH: hipLaunchKernelGGL((block_diag_kernel<T, MS_NH>), grid, dim3(256), 0, s, a, blk); break;
      default: hipLaunchKernelGGL((block_diag_kernel<T, MS_LINEAR>), grid, dim3(256), 0, s, a, blk);
    }
  }
  hipLaunchKernelGGL(block_inv_kernel<T>, dim3(vgrid(p->n_nodes)), dim3(VBLOCK), 0, s, p->n_nodes, p->mask, blk,
                     p->flags);
  return hipGetLastError();
}

hipError_t launch_block_jacobi(const fe_problem* p, const int32_t* rp, const int32_t* ci, const void* v, void* blk,
                               hipStream_t s) {
  return p->prec == FE_F64 ? launch_block_t(p, rp, ci, (const double*)v, (double*)blk, s)
                           : launch_block_t(p, rp, ci, (const float*)v, (float*)blk, s);
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
  if (p->general) return gen_lift(p, E, u, zero_free, s);
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
    hipLaunchKernelGGL(dot_kernel<double>, dim3(std::min(vgrid(n), 64)), dim3(VBLOCK), 0, s, (const double*)a, (const double*)b, n,
                       p->partials, p->counter, out);
  else
    hipLaunchKernelGGL(dot_kernel<float>, dim3(std::min(vgrid(n), 64)), dim3(VBLOCK), 0, s, (const float*)a, (const float*)b, n,
                       p->partials, p->counter, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Jacobi-preconditioned CG on the CSR operator, with device-resident scalars and no
// grid-wide fences (the matrix-free solve runs the single-reduction form further down).
// Every kernel of an iteration writes per-block partial sums; the next kernel
// re-reduces them in every block in the same order (identical results in all
// blocks; the kernel boundary makes the partials visible), and block 0 records
// the scalars for the host.  Kernels return at once when ctrl->status is set, so
// the host can enqueue several iterations between convergence checks.
//   direction step k: rr, rz from the update partials -> stop tests, beta = rz / rz_old,
//                     p = M^-1 r + beta p
//   operator k:       q = A p, partials of p.q
//   update k:         alpha = rz / p.q, x += alpha p, r -= alpha q, q = 0, partials of r.r, r.M^-1 r

// x = 0, r = b, q = 0, p = 0, d <- 1/d; partials of b.b and b.M^-1 b (CG_UGRID blocks)
// (block: M already holds the inverse blocks and is left unchanged)
template <typename T> __global__ __launch_bounds__(VBLOCK) void cg_init_kernel(
    int64_t n, const T* b, T* x, T* r, T* p, T* q, T* dinv, int block, CgCtrl* ctrl, double rtol, int max_it,
    double* pu) {
  __shared__ double sh[VBLOCK / 64];
  double rz = 0, bb = 0;
  for (int64_t i = (int64_t)blockIdx.x * VBLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * VBLOCK) {
    const T bi = b[i];
    T zi;
    if (block) {
      zi = pc_apply(dinv, b, i, 1);
    } else {
      const T di = T(1) / dinv[i];
      dinv[i] = di;
      zi = di * bi;
    }
    x[i] = 0;
    r[i] = bi;
    q[i] = 0;
    p[i] = 0;
    rz += (double)bi * (double)zi;
    bb += (double)bi * (double)bi;
  }
  rz = block_sum(rz, sh);
  bb = block_sum(bb, sh);
  if (threadIdx.x == 0) {
    pu[blockIdx.x] = bb;
    pu[CG_UGRID + blockIdx.x] = rz;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctrl->rz[0] = ctrl->rz[1] = 0;
    ctrl->rtol2 = rtol * rtol;
    ctrl->iters = 0;
    ctrl->max_it = max_it;
    ctrl->alpha = ctrl->beta = ctrl->pq = 0;
    ctrl->status = CG_RUNNING;
  }
}

// Direction step as a kernel of its own (the mat-vec needs the whole p first)
template <typename T> __global__ __launch_bounds__(VBLOCK) void cg_direction_kernel(int64_t n, const T* r,
                                                                                     const T* dinv, int block, T* p,
                                                                                     CgCtrl* ctrl, const double* pu,
                                                                                     long k) {
  __shared__ double sh[VBLOCK / 64], bc[2];
  if (ctrl->status) return;
  double beta;
  if (!cg_direction_step(ctrl, pu, k, sh, bc, beta)) return;
  const T tb = T(beta);
  for (int64_t i = (int64_t)blockIdx.x * VBLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * VBLOCK)
    p[i] = pc_apply(dinv, r, i, block) + tb * p[i];
}

// alpha = rz / p.q (from the operator's partials); x += alpha p; r -= alpha q; q = 0.
// One thread per node (so r.M^-1 r uses the node's three new residual entries), UPB nodes
// per thread whose loads are all issued before the partial sums are reduced.
constexpr int UPB = 2;
template <typename T> struct UpdBatch {
  T x[UPB][3], r[UPB][3], p[UPB][3], q[UPB][3], m[UPB][6];
};

template <typename T>
__device__ __forceinline__ void upd_load(UpdBatch<T>& b, int64_t nd0, int64_t stride, int64_t n_nodes,
                                         const T* __restrict__ x, const T* __restrict__ r, const T* __restrict__ p,
                                         const T* __restrict__ q, const T* __restrict__ dinv, int block) {
#pragma unroll
  for (int u = 0; u < UPB; ++u) {
    const int64_t nd = nd0 + u * stride;
    const bool ok = nd < n_nodes;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t i = ok ? 3 * nd + c : 0;
      b.x[u][c] = ok ? x[i] : T(0);
      b.r[u][c] = ok ? r[i] : T(0);
      b.p[u][c] = ok ? p[i] : T(0);
      b.q[u][c] = ok ? q[i] : T(0);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) b.m[u][c] = (ok && (block || c < 3)) ? dinv[(block ? 6 : 3) * nd + c] : T(0);
  }
}

template <typename T>
__device__ __forceinline__ void upd_store(const UpdBatch<T>& b, T ta, int64_t nd0, int64_t stride, int64_t n_nodes,
                                          T* __restrict__ x, T* __restrict__ r, T* __restrict__ q, int block,
                                          double& rr, double& rzn) {
#pragma unroll
  for (int u = 0; u < UPB; ++u) {
    const int64_t nd = nd0 + u * stride;
    if (nd >= n_nodes) continue;
    T rn[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t i = 3 * nd + c;
      x[i] = b.x[u][c] + ta * b.p[u][c];
      rn[c] = b.r[u][c] - ta * b.q[u][c];
      r[i] = rn[c];
      q[i] = 0;
      rr += (double)rn[c] * (double)rn[c];
    }
    const T* m = b.m[u];
    if (block) {
      const T z0 = m[0] * rn[0] + m[5] * rn[1] + m[4] * rn[2];
      const T z1 = m[5] * rn[0] + m[1] * rn[1] + m[3] * rn[2];
      const T z2 = m[4] * rn[0] + m[3] * rn[1] + m[2] * rn[2];
      rzn += (double)rn[0] * (double)z0 + (double)rn[1] * (double)z1 + (double)rn[2] * (double)z2;
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) rzn += (double)rn[c] * (double)(m[c] * rn[c]);
    }
  }
}

template <typename T> __global__ __launch_bounds__(VBLOCK) void cg_update_kernel(
    int64_t n, T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p, T* __restrict__ q,
    const T* __restrict__ dinv, int block, CgCtrl* ctrl, const double* pa, int nba, double* pu, long k) {
  __shared__ double sh[VBLOCK / 64], bc[1];
  if (ctrl->status) return;
  const int64_t n_nodes = n / 3;
  const int64_t stride = (int64_t)gridDim.x * VBLOCK;
  int64_t nd0 = (int64_t)blockIdx.x * VBLOCK + threadIdx.x;
  UpdBatch<T> b;
  upd_load(b, nd0, stride, n_nodes, x, r, p, q, dinv, block);  // in flight while the partials are reduced
  const double pq = sum_partials_all(pa, nba, sh, bc);
  const double rz = ctrl->rz[k & 1];
  const int st = !finite(pq) ? FE_ERR_NONFINITE : (pq <= 0.0 ? FE_ERR_BREAKDOWN : CG_RUNNING);
  const double alpha = rz / pq;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctrl->pq = pq;
    ctrl->alpha = alpha;
    if (st != CG_RUNNING) ctrl->status = st;
  }
  if (st != CG_RUNNING) return;
  const T ta = T(alpha);
  double rr = 0, rzn = 0;
  upd_store(b, ta, nd0, stride, n_nodes, x, r, q, block, rr, rzn);
  for (nd0 += UPB * stride; nd0 < n_nodes; nd0 += UPB * stride) {
    upd_load(b, nd0, stride, n_nodes, x, r, p, q, dinv, block);
    upd_store(b, ta, nd0, stride, n_nodes, x, r, q, block, rr, rzn);
  }
  rr = block_sum(rr, sh);
  rzn = block_sum(rzn, sh);
  if (threadIdx.x == 0) {
    pu[blockIdx.x] = rr;
    pu[CG_UGRID + blockIdx.x] = rzn;
  }
}

template <typename T>
static hipError_t cg_init_t(const fe_problem* p, const T* b, T* x, double rtol, int max_it, hipStream_t s) {
  const int64_t n = p->n_dof;
  hipLaunchKernelGGL(cg_init_kernel<T>, dim3(CG_UGRID), dim3(VBLOCK), 0, s, n, b, x, (T*)p->w_r, (T*)p->w_p,
                     (T*)p->w_q, (T*)pc_buffer(p), p->precond, p->ctrl, rtol, max_it, p->partials + cg_pa_size(p));
  return hipGetLastError();
}

hipError_t cg_init(const fe_problem* p, const void* b, void* x, double rtol, int max_it, hipStream_t s) {
  return p->prec == FE_F64 ? cg_init_t(p, (const double*)b, (double*)x, rtol, max_it, s)
                           : cg_init_t(p, (const float*)b, (float*)x, rtol, max_it, s);
}

int elem_grid_size(int n) { return elem_grid(n); }

// CG mat-vec: q = A p with LPR lanes per row (grid-stride over rows) and per-workgroup partials of p.q.
template <typename T, int LPR>
__global__ __launch_bounds__(256) void cg_spmv_kernel(int64_t n_rows, const int32_t* __restrict__ rp,
                                                      const int32_t* __restrict__ ci, const T* __restrict__ v,
                                                      const T* __restrict__ p, T* __restrict__ q, const int* stop,
                                                      double* pa) {
  __shared__ double sh[VBLOCK / 64];
  if (*stop) return;
  constexpr int RPB = 256 / LPR;
  const int lane = threadIdx.x % LPR;
  double pq = 0;
  for (int64_t row0 = (int64_t)blockIdx.x * RPB; row0 < n_rows; row0 += (int64_t)gridDim.x * RPB) {
    const int64_t row = row0 + threadIdx.x / LPR;
    T acc = 0;
    if (row < n_rows) acc = csr_row_dot<T, LPR>(ci, v, p, rp[row], rp[row + 1], lane);
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, LPR);
    if (row < n_rows && lane == 0) {
      q[row] = acc;
      pq += (double)p[row] * (double)acc;
    }
  }
  pq = block_sum(pq, sh);
  if (threadIdx.x == 0) pa[blockIdx.x] = pq;
}

// Node-structured form of the same (rows 3a..3a+2 share their column list): LPN lanes per
// node, grid-stride over node groups.
template <typename T, int LPN>
__global__ __launch_bounds__(256) void cg_spmv_nodal_kernel(int64_t n_nodes, const int32_t* __restrict__ rp,
                                                            const int32_t* __restrict__ ci, const T* __restrict__ v,
                                                            const T* __restrict__ p, T* __restrict__ q,
                                                            const int* stop, double* pa) {
  __shared__ double sh[VBLOCK / 64];
  if (*stop) return;
  constexpr int NPB = 256 / LPN;
  const int lane = threadIdx.x % LPN;
  double pq = 0;
  for (int64_t n0 = (int64_t)blockIdx.x * NPB; n0 < n_nodes; n0 += (int64_t)gridDim.x * NPB) {
    const int64_t nd = n0 + threadIdx.x / LPN;
    T a0 = 0, a1 = 0, a2 = 0;
    if (nd < n_nodes) {
      const int b0 = rp[3 * nd], b1 = rp[3 * nd + 1], b2 = rp[3 * nd + 2];
      const int len = b1 - b0;
      nodal_row_dot<T, LPN>(ci, v, p, b0, b1, b2, len, lane, a0, a1, a2);
    }
#pragma unroll
    for (int off = LPN / 2; off > 0; off >>= 1) {
      a0 += __shfl_xor(a0, off, LPN);
      a1 += __shfl_xor(a1, off, LPN);
      a2 += __shfl_xor(a2, off, LPN);
    }
    if (nd < n_nodes && lane < 3) {
      const T a = lane == 0 ? a0 : (lane == 1 ? a1 : a2);
      q[3 * nd + lane] = a;
      pq += (double)p[3 * nd + lane] * (double)a;
    }
  }
  pq = block_sum(pq, sh);
  if (threadIdx.x == 0) pa[blockIdx.x] = pq;
}

static int cg_spmv_grid(const fe_problem* p) {
  const int64_t blocks = p->csr_nodal ? (p->n_nodes + (256 / SPMV_LPN) - 1) / (256 / SPMV_LPN)
                                      : (p->n_dof + (256 / SPMV_LPR) - 1) / (256 / SPMV_LPR);
  return (int)std::min<int64_t>(blocks, SPMV_MAXGRID);
}

static int cg_operator_grid(const fe_problem* p, int op) {
  if (op != FE_OP_CSR && (p->general || p->deterministic)) return GEN_CG_GRID;
  return op == FE_OP_CSR ? cg_spmv_grid(p) : elem_grid(p->n);
}

template <typename T>
static hipError_t cg_operator_t(const fe_problem* p, int op, const int32_t* rp, const int32_t* ci, const T* vals,
                                long k, hipStream_t s) {
  const int* stop = &p->ctrl->status;
  T* Q = (T*)p->w_q;
  double* pa = p->partials;
  if (op == FE_OP_CSR) {
    if (p->csr_nodal)
      timed_launch((cg_spmv_nodal_kernel<T, SPMV_LPN>), dim3(cg_spmv_grid(p)), dim3(256), 0, s, p->n_nodes, rp, ci,
                   vals, (const T*)p->w_p, Q, stop, pa);
    else
      timed_launch((cg_spmv_kernel<T, SPMV_LPR>), dim3(cg_spmv_grid(p)), dim3(256), 0, s, p->n_dof, rp, ci, vals,
                   (const T*)p->w_p, Q, stop, pa);
    return hipGetLastError();
  }
  if (p->general) return gen_cg_operator(p, s);
  if (p->deterministic) {  // q = A p element by element, fixed-order gather with the p.q partials
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
    a.x = p->w_p;
    a.y = p->w_q;
    a.apply_bc = 1;
    a.elf = p->w_elf;
    const hipError_t e = launch_elem_t<T, OP_APPLY>(p, a, stop, s);
    if (e != hipSuccess) return e;
    return det_gather(p, p->w_elf, 1, 1, p->w_p, p->w_q, stop, p->partials, s);
  }
  return hipErrorInvalidValue;  // the structured matrix-free operator runs through cgs_operator
}

// ---------------------------------------------------------------------------
// Matrix-free CG with one operator launch per iteration (single-reduction form of
// Chronopoulos & Gear 1989; exact-arithmetic equivalent of the CG recursion):
//   launch j forms u_j = M^-1 r_j, w_j = A u_j and the partials of (u_j, w_j),
//   (r_j, u_j), ||r_j||^2; its staging applies update j-1 (see cg_stage) and its last
//   workgroup reduces the partials into alpha_j, beta_j or a stop (see cg_finish).
// Vectors: x (caller), p (in place, owners only), r in two buffers, s in two, w in three
// (launch j writes w into the buffer that launch j-1 zeroed).

template <typename T> __global__ __launch_bounds__(VBLOCK) void cgs_init_kernel(
    int64_t n, const T* b, T* x, T* r0, T* p, T* s1, T* w0, T* dinv, int block, CgCtrl* ctrl, double rtol,
    int max_it, double* acc0) {
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < 3 * CGS_SLOTS; i += VBLOCK) acc0[i] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * VBLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * VBLOCK) {
    x[i] = 0;
    r0[i] = b[i];
    p[i] = 0;
    s1[i] = 0;
    w0[i] = 0;
    if (!block) dinv[i] = T(1) / dinv[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctrl->rtol2 = rtol * rtol;
    ctrl->iters = 0;
    ctrl->max_it = max_it;
    ctrl->alpha = ctrl->beta = ctrl->pq = 0;
    ctrl->ghist[0] = ctrl->ghist[1] = ctrl->ahist[0] = ctrl->ahist[1] = 0;
    ctrl->status = CG_RUNNING;
  }
}

template <typename T> static T* cgs_vec(const fe_problem* p, int k) {  // 0 r_1, 1 s_0, 2 s_1, 3 w_0, 4 w_1, 5 w_2
  return static_cast<T*>(p->w_cg) + (int64_t)k * p->n_dof;
}

template <typename T> static T* cgs_r(const fe_problem* p, long j) { return (j & 1) ? cgs_vec<T>(p, 0) : (T*)p->w_r; }
template <typename T> static T* cgs_s(const fe_problem* p, long j) { return cgs_vec<T>(p, 1 + (int)(j & 1)); }
template <typename T> static T* cgs_w(const fe_problem* p, long j) { return cgs_vec<T>(p, 3 + (int)(j % 3)); }

template <typename T>
static hipError_t cgs_init_t(const fe_problem* p, const T* b, T* x, double rtol, int max_it, hipStream_t s) {
  hipLaunchKernelGGL(cgs_init_kernel<T>, dim3(CG_UGRID), dim3(VBLOCK), 0, s, p->n_dof, b, x, (T*)p->w_r,
                     (T*)p->w_p, cgs_s<T>(p, 1), cgs_w<T>(p, 0), (T*)pc_buffer(p), p->precond, p->ctrl, rtol,
                     max_it, p->partials);
  return hipGetLastError();
}

hipError_t cgs_init(const fe_problem* p, const void* b, void* x, double rtol, int max_it, hipStream_t s) {
  return p->prec == FE_F64 ? cgs_init_t(p, (const double*)b, (double*)x, rtol, max_it, s)
                           : cgs_init_t(p, (const float*)b, (float*)x, rtol, max_it, s);
}

template <typename T> static hipError_t cgs_operator_t(const fe_problem* p, T* x, long j, hipStream_t s) {
  ElemArgs a{};
  a.n = p->n;
  a.h = p->h;
  a.n_el = p->n_el;
  a.phase = p->phase;
  a.scale = p->scale;
  a.mask = p->mask;
  a.tangent = p->tangent;
  a.apply_bc = 1;
  a.mat = p->mat;
  a.sur_map = p->sur_map;
  a.sur_D = p->sur_D;
  a.cg_dinv = pc_buffer(p);
  a.cg_block = p->precond;
  a.ctrl = p->ctrl;
  a.cg_j = j;
  // launch j: reads r_{j-1} (r_0 = b at j = 0), w_{j-1}, s_{j-2}; writes r_j, s_{j-1}, w_j
  a.cg_rold = j == 0 ? (const void*)p->w_r : cgs_r<T>(p, j - 1);
  a.cg_rnew = cgs_r<T>(p, j);
  a.cg_wold = j == 0 ? nullptr : cgs_w<T>(p, j - 1);
  a.cg_sold = j == 0 ? nullptr : cgs_s<T>(p, j);  // s_{j-2} lives in the slot of parity j
  a.cg_snew = j == 0 ? nullptr : cgs_s<T>(p, j - 1);
  a.cg_wzero = cgs_w<T>(p, j + 1);
  a.y = cgs_w<T>(p, j);
  a.cg_pvec = p->w_p;
  a.cg_x = x;
  double* acc = p->partials;  // three sets of 3 * CGS_SLOTS, cycled over launches
  a.cg_acc_in = j == 0 ? nullptr : acc + ((j + 2) % 3) * 3 * CGS_SLOTS;
  a.cg_acc_out = acc + (j % 3) * 3 * CGS_SLOTS;
  a.cg_acc_zero = acc + ((j + 1) % 3) * 3 * CGS_SLOTS;
  return launch_elem_t<T, OP_CG_APPLY>(p, a, &p->ctrl->status, s);
}

hipError_t cgs_operator(const fe_problem* p, void* x, long j, hipStream_t s) {
  return p->prec == FE_F64 ? cgs_operator_t(p, (double*)x, j, s) : cgs_operator_t(p, (float*)x, j, s);
}

hipError_t cg_operator(const fe_problem* p, int op, const int32_t* rp, const int32_t* ci, const void* vals, long k,
                       hipStream_t s) {
  return p->prec == FE_F64 ? cg_operator_t(p, op, rp, ci, (const double*)vals, k, s)
                           : cg_operator_t(p, op, rp, ci, (const float*)vals, k, s);
}

// CSR iterations form the direction in a kernel of their own before the mat-vec.
template <typename T> static hipError_t cg_pre_t(const fe_problem* p, int op, long k, hipStream_t s) {
  if (op != FE_OP_CSR && !p->general && !p->deterministic) return hipSuccess;
  hipLaunchKernelGGL(cg_direction_kernel<T>, dim3(CG_UGRID), dim3(VBLOCK), 0, s, p->n_dof, (const T*)p->w_r,
                     (const T*)pc_buffer(p), p->precond, (T*)p->w_p, p->ctrl,
                     (const double*)(p->partials + cg_pa_size(p)), k);
  return hipGetLastError();
}

hipError_t cg_pre(const fe_problem* p, int op, long k, hipStream_t s) {
  return p->prec == FE_F64 ? cg_pre_t<double>(p, op, k, s) : cg_pre_t<float>(p, op, k, s);
}

template <typename T> static hipError_t cg_vectors_t(const fe_problem* p, int op, T* x, long k, hipStream_t s) {
  const int64_t n = p->n_dof;
  T* P = (T*)p->w_p;
  hipLaunchKernelGGL(cg_update_kernel<T>, dim3(CG_UGRID), dim3(VBLOCK), 0, s, n, x, (T*)p->w_r, (const T*)P,
                     (T*)p->w_q, (const T*)pc_buffer(p), p->precond, p->ctrl, (const double*)p->partials,
                     cg_operator_grid(p, op), p->partials + cg_pa_size(p), k);
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
  const bool j2 = e < ne && mat.ph[phase[e]].model == FE_J2;
  unsigned long long cnt = 0, pl = 0;
  if (j2) {
    cnt = 8;
    for (int q = 0; q < 8; ++q) pl += tangent[(int64_t)q * ne + e] >= T(0) ? 1 : 0;
  }
  // wave sums, one atomic per wave
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    cnt += __shfl_down(cnt, off, 64);
    pl += __shfl_down(pl, off, 64);
  }
  if (__lane_id() == 0) {
    atomicAdd(out, cnt);
    atomicAdd(out + 1, pl);
  }
}

// ---------------------------------------------------------------------------
// Preconditioned BiCGStab (nonsymmetric operators) with device-resident scalars.
// Vector kernels write per-workgroup partial sums; the next vector kernel reduces
// them redundantly in every workgroup (same order, same result) and workgroup 0
// records the scalars.  Per iteration:
//   DIR:    rho = (r_hat, r); stop test on ||r||; p = r + beta (p - omega v); p_hat = M^-1 p; v = 0
//   (operator) v = A p_hat
//   HALF:   alpha = rho / (r_hat, v); s = r - alpha v; s_hat = M^-1 s; partial ||s||^2
//   (operator) t = A s_hat
//   DOTS:   partials of (t, s), (t, t)
//   UPDATE: ||s|| small: x += alpha p_hat, stop; else omega = (t,s)/(t,t),
//           x += alpha p_hat + omega s_hat, r = s - omega t, t = 0; partials (r_hat, r), ||r||^2
// Partial slots: 0 (r_hat, r), 1 ||r||^2, 2 (r_hat, v), 3 ||s||^2, 4 (t, s), 5 (t, t).

enum { BICG_DIR = 0, BICG_HALF = 1, BICG_DOTS = 2, BICG_UPDATE = 3 };

template <typename T> struct BicgVec {
  T *x, *r, *rh, *p, *v, *sv, *t, *ph, *sh;
  const T* M;
  int block;
};

// dst[node] = M^-1 v for one node (point Jacobi: inverse diagonal; node blocks: symmetric 3x3
// inverse; ILU(0), block = 2: a copy, which the host then sweeps in place)
template <typename T>
__device__ __forceinline__ void bicg_precond(const BicgVec<T>& w, int64_t nd, const T v[3], T* dst) {
  if (w.block == 2) {
#pragma unroll
    for (int c = 0; c < 3; ++c) dst[3 * nd + c] = v[c];
  } else if (w.block) {
    const T* m = w.M + 6 * nd;
    dst[3 * nd] = m[0] * v[0] + m[5] * v[1] + m[4] * v[2];
    dst[3 * nd + 1] = m[5] * v[0] + m[1] * v[1] + m[3] * v[2];
    dst[3 * nd + 2] = m[4] * v[0] + m[3] * v[1] + m[2] * v[2];
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) dst[3 * nd + c] = w.M[3 * nd + c] * v[c];
  }
}

__device__ __forceinline__ double bicg_sum(const double* part, int slot, double* sh, double* bc) {
  return sum_partials_all(part + (int64_t)slot * BICG_GRID, BICG_GRID, sh, bc);
}

template <typename T>
__global__ __launch_bounds__(VBLOCK) void bicg_kernel(int stage, int64_t n, BicgVec<T> w, BicgCtrl* ctrl,
                                                      double* part) {
  __shared__ double sh[VBLOCK / 64], bc[2];
  if (ctrl->status) return;
  const int64_t stride = (int64_t)gridDim.x * VBLOCK;
  const int64_t i0 = (int64_t)blockIdx.x * VBLOCK + threadIdx.x;
  double a0 = 0, a1 = 0;
  if (stage == BICG_DIR) {
    if (ctrl->finish) {  // the last update met the tolerance (its workgroups all completed x)
      if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->status = CG_CONVERGED;
      return;
    }
    const double rho = bicg_sum(part, 0, sh, bc);
    const double rr = bicg_sum(part, 1, sh, bc + 1);
    const bool first = ctrl->iters == 0 && ctrl->rho_old == 0.0;
    const double tol2 = first ? ctrl->rtol2 * rr : ctrl->tol2;
    int st = CG_RUNNING;
    if (!finite(rho) || !finite(rr)) st = FE_ERR_NONFINITE;
    else if (first ? rr == 0.0 : rr <= tol2) st = CG_CONVERGED;
    else if (ctrl->iters >= ctrl->max_it) st = FE_ERR_NOT_CONVERGED;
    else if (rho == 0.0 || (!first && ctrl->omega == 0.0)) st = FE_ERR_BREAKDOWN;
    const double beta = first ? 0.0 : (rho / ctrl->rho_old) * (ctrl->alpha / ctrl->omega);
    const double omega = first ? 0.0 : ctrl->omega;
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      if (first) {
        ctrl->bb = rr;
        ctrl->tol2 = tol2;
      }
      ctrl->rr = rr;
      ctrl->rho = rho;
      ctrl->beta = beta;
      if (st != CG_RUNNING) ctrl->status = st;
    }
    if (st != CG_RUNNING) return;
    const T tb = T(beta), to = T(omega);
    for (int64_t nd = i0; nd < n / 3; nd += stride) {  // one node per thread: M^-1 may couple its dofs
      T pv[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int64_t i = 3 * nd + c;
        pv[c] = w.r[i] + tb * (w.p[i] - to * w.v[i]);
        w.p[i] = pv[c];
        w.v[i] = 0;
      }
      bicg_precond(w, nd, pv, w.ph);
    }
  } else if (stage == BICG_HALF) {
    const double rv = bicg_sum(part, 2, sh, bc);
    const double rho = ctrl->rho;
    const int st = !finite(rv) ? FE_ERR_NONFINITE : (rv == 0.0 ? FE_ERR_BREAKDOWN : CG_RUNNING);
    const double alpha = rho / rv;
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ctrl->alpha = alpha;
      if (st != CG_RUNNING) ctrl->status = st;
    }
    if (st != CG_RUNNING) return;
    const T ta = T(alpha);
    for (int64_t nd = i0; nd < n / 3; nd += stride) {
      T sv[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int64_t i = 3 * nd + c;
        sv[c] = w.r[i] - ta * w.v[i];
        w.sv[i] = sv[c];
        a0 += (double)sv[c] * (double)sv[c];
      }
      bicg_precond(w, nd, sv, w.sh);
    }
  } else if (stage == BICG_DOTS) {
    for (int64_t i = i0; i < n; i += stride) {
      a0 += (double)w.t[i] * (double)w.sv[i];
      a1 += (double)w.t[i] * (double)w.t[i];
    }
  } else {  // BICG_UPDATE
    const double ss = bicg_sum(part, 3, sh, bc);
    const double ts = bicg_sum(part, 4, sh, bc + 1);
    const double tt = bicg_sum(part, 5, sh, bc);
    const double alpha = ctrl->alpha;
    const bool done = ss <= ctrl->tol2;
    const double omega = done ? 0.0 : (tt > 0.0 ? ts / tt : 0.0);
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ctrl->omega = omega;
      ctrl->rho_old = ctrl->rho;
      ctrl->iters += 1;
      if (done) {  // not the status word: the other workgroups of this launch still update x
        ctrl->rr = ss;
        ctrl->finish = 1;
      }
    }
    const T ta = T(alpha), to = T(omega);
    for (int64_t i = i0; i < n; i += stride) {
      if (done) {
        w.x[i] += ta * w.ph[i];
        continue;
      }
      w.x[i] += ta * w.ph[i] + to * w.sh[i];
      const T ri = w.sv[i] - to * w.t[i];
      w.r[i] = ri;
      w.t[i] = 0;
      a0 += (double)w.rh[i] * (double)ri;
      a1 += (double)ri * (double)ri;
    }
  }
  const int s0 = stage == BICG_HALF ? 3 : (stage == BICG_DOTS ? 4 : 0);
  if (stage != BICG_DIR) {
    a0 = block_sum(a0, sh);
    a1 = block_sum(a1, sh);
    if (threadIdx.x == 0) {
      part[(int64_t)s0 * BICG_GRID + blockIdx.x] = a0;
      if (stage != BICG_HALF) part[(int64_t)(s0 + 1) * BICG_GRID + blockIdx.x] = a1;
    }
  }
}

// (r_hat, v) partials after the operator
template <typename T>
__global__ __launch_bounds__(VBLOCK) void bicg_rv_kernel(int64_t n, const T* rh, const T* v, BicgCtrl* ctrl,
                                                         double* part) {
  __shared__ double sh[VBLOCK / 64];
  if (ctrl->status) return;
  double a = 0;
  for (int64_t i = (int64_t)blockIdx.x * VBLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * VBLOCK)
    a += (double)rh[i] * (double)v[i];
  a = block_sum(a, sh);
  if (threadIdx.x == 0) part[2 * BICG_GRID + blockIdx.x] = a;
}

// x = 0, r = r_hat = b, p = v = t = 0; partials (r_hat, r) = ||b||^2 and ||r||^2
template <typename T>
__global__ __launch_bounds__(VBLOCK) void bicg_init_kernel(int64_t n, const T* b, BicgVec<T> w, BicgCtrl* ctrl,
                                                           double* part, double rtol, int max_it, int invert) {
  __shared__ double sh[VBLOCK / 64];
  double bb = 0;
  for (int64_t i = (int64_t)blockIdx.x * VBLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * VBLOCK) {
    const T bi = b[i];
    w.x[i] = 0;
    w.r[i] = bi;
    w.rh[i] = bi;
    w.p[i] = 0;
    w.v[i] = 0;
    w.t[i] = 0;
    if (invert) const_cast<T*>(w.M)[i] = T(1) / w.M[i];
    bb += (double)bi * (double)bi;
  }
  bb = block_sum(bb, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = bb;
    part[BICG_GRID + blockIdx.x] = bb;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctrl->rho = ctrl->rho_old = ctrl->alpha = ctrl->omega = ctrl->beta = 0;
    ctrl->rtol2 = rtol * rtol;
    ctrl->iters = 0;
    ctrl->max_it = max_it;
    ctrl->status = CG_RUNNING;
    ctrl->finish = 0;
  }
}

template <typename T> static BicgVec<T> bicg_vec(const fe_problem* p, void* x) {
  BicgVec<T> w;
  T* base = static_cast<T*>(p->w_bicg);
  const int64_t n = p->n_dof;
  w.x = static_cast<T*>(x);
  w.r = base;
  w.rh = base + n;
  w.p = base + 2 * n;
  w.v = base + 3 * n;
  w.sv = base + 4 * n;
  w.t = base + 5 * n;
  w.ph = base + 6 * n;
  w.sh = base + 7 * n;
  w.M = static_cast<const T*>(pc_buffer(p));
  w.block = p->precond == FE_PC_BLOCK_JACOBI ? 1 : (p->precond == FE_PC_ILU0 ? 2 : 0);
  return w;
}

template <typename T>
static hipError_t bicg_init_t(const fe_problem* p, const T* b, void* x, double rtol, int max_it, hipStream_t s) {
  hipLaunchKernelGGL(bicg_init_kernel<T>, dim3(BICG_GRID), dim3(VBLOCK), 0, s, p->n_dof, b, bicg_vec<T>(p, x),
                     p->bicg_ctrl, p->bicg_part, rtol, max_it, p->precond == FE_PC_JACOBI ? 1 : 0);
  return hipGetLastError();
}

hipError_t bicg_init(const fe_problem* p, const void* b, void* x, double rtol, int max_it, hipStream_t s) {
  return p->prec == FE_F64 ? bicg_init_t(p, (const double*)b, x, rtol, max_it, s)
                           : bicg_init_t(p, (const float*)b, x, rtol, max_it, s);
}

template <typename T> static hipError_t bicg_step_t(const fe_problem* p, int stage, void* x, hipStream_t s) {
  const BicgVec<T> w = bicg_vec<T>(p, x);
  if (stage == 4) {  // (r_hat, v) after the first operator
    hipLaunchKernelGGL(bicg_rv_kernel<T>, dim3(BICG_GRID), dim3(VBLOCK), 0, s, p->n_dof, (const T*)w.rh,
                       (const T*)w.v, p->bicg_ctrl, p->bicg_part);
  } else {
    hipLaunchKernelGGL(bicg_kernel<T>, dim3(BICG_GRID), dim3(VBLOCK), 0, s, stage, p->n_dof, w, p->bicg_ctrl,
                       p->bicg_part);
  }
  return hipGetLastError();
}

hipError_t bicg_step(const fe_problem* p, int stage, void* x, hipStream_t s) {
  return p->prec == FE_F64 ? bicg_step_t<double>(p, stage, x, s) : bicg_step_t<float>(p, stage, x, s);
}

// ---------------------------------------------------------------------------
// Path adjoint through the return map (FP64).  Forward-mode dual numbers give the
// Jacobian of one Gauss point's update (eps, eps_p_n, alpha_n, s) -> (sigma, eps_p,
// alpha) column by column, from the same j2_update the residual uses; the
// cotangents are contracted with it.

struct Dual {
  double v, d;
  __device__ Dual(double x = 0.0, double y = 0.0) : v(x), d(y) {}
  __device__ Dual& operator+=(Dual b) { v += b.v; d += b.d; return *this; }
  __device__ Dual& operator-=(Dual b) { v -= b.v; d -= b.d; return *this; }
};
__device__ inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
__device__ inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
__device__ inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
__device__ inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
__device__ inline Dual operator/(Dual a, Dual b) { return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)); }
__device__ inline Dual sqrt(Dual a) {
  const double r = ::sqrt(a.v);
  return Dual(r, r > 0.0 ? a.d / (2.0 * r) : 0.0);
}
__device__ inline bool operator>(Dual a, Dual b) { return a.v > b.v; }
__device__ inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
__device__ inline bool operator>=(Dual a, Dual b) { return a.v >= b.v; }

struct PathArgs {
  int n;
  double h;
  int64_t n_el;
  const uint8_t* phase;
  const double* scale;   // [n_el] or null (1)
  Phases mat;
  const double* u;       // linearisation displacement [n_dof]
  const double* hist;    // state at the start of the step [7][8][n_el]
  const double* c;       // cotangent of the residual [n_dof] or null
  const double* mu_in;   // cotangent of the step's trial state [7][8][n_el] or null
  double* mu_out;        // cotangent of the starting state [7][8][n_el] (written)
  double* u_bar;         // += history part of the displacement cotangent [n_dof] or null
  double* s_bar;         // += cotangent of the modulus scale [n_el] or null
};

__global__ __launch_bounds__(256) void path_vjp_kernel(PathArgs a) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= a.n_el) return;
  const int n = a.n;
  const int64_t ne = a.n_el, np1 = n + 1;
  const int ea = (int)(e % n), eb = (int)((e / n) % n), ec = (int)(e / ((int64_t)n * n));
  const double inv_h = 1.0 / a.h, w = 0.125 * a.h * a.h * a.h;
  const PhaseConst pc = a.mat.ph[a.phase[e]];
  const double sc = a.scale ? a.scale[e] : 1.0;
  const bool j2 = pc.model == FE_J2;
  double U[8][3], C[8][3], UB[8][3];
  int64_t node[8];
#pragma unroll
  for (int l = 0; l < 8; ++l) {
    node[l] = (ea + (l & 1)) + np1 * ((eb + ((l >> 1) & 1)) + np1 * (ec + (l >> 2)));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      U[l][c] = a.u[3 * node[l] + c];
      C[l][c] = a.c ? a.c[3 * node[l] + c] : 0.0;
      UB[l][c] = 0.0;
    }
  }
  double sbar = 0.0;
  for (int qp = 0; qp < 8; ++qp) {
    const int p = qp & 1, q = (qp >> 1) & 1, r = qp >> 2;
    double g[8][3];
#pragma unroll
    for (int l = 0; l < 8; ++l) basis_grad(l & 1, (l >> 1) & 1, l >> 2, p, q, r, inv_h, g[l]);
    double H[3][3] = {}, Hc[3][3] = {};
#pragma unroll
    for (int l = 0; l < 8; ++l)
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int J = 0; J < 3; ++J) {
          H[c][J] += U[l][c] * g[l][J];
          Hc[c][J] += C[l][c] * g[l][J];
        }
    // stress cotangent: c . R = sum_q w (B_q c_e) . sigma_q (engineering-shear pairing)
    const double sb[6] = {w * Hc[0][0], w * Hc[1][1], w * Hc[2][2], w * (Hc[1][2] + Hc[2][1]),
                          w * (Hc[0][2] + Hc[2][0]), w * (Hc[0][1] + Hc[1][0])};
    double mu[7], ebar[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 7; ++k) mu[k] = a.mu_in ? a.mu_in[(int64_t)(k * 8 + qp) * ne + e] : 0.0;
    if (j2) {
      double hn[7];
#pragma unroll
      for (int k = 0; k < 7; ++k) hn[k] = a.hist ? a.hist[(int64_t)(k * 8 + qp) * ne + e] : 0.0;
      for (int col = 0; col < 14; ++col) {
        Dual Hd[3][3], epd[6], ad, Kd(pc.K * sc), Gd(pc.G * sc);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) Hd[i][j] = Dual(H[i][j]);
#pragma unroll
        for (int k = 0; k < 6; ++k) epd[k] = Dual(hn[k]);
        ad = Dual(hn[6]);
        if (col < 3) {
          Hd[col][col].d = 1.0;
        } else if (col < 6) {  // engineering shear strain: half to each off-diagonal entry
          const int i = col == 3 ? 1 : 0, j = col == 5 ? 1 : 2;
          Hd[i][j].d = 0.5;
          Hd[j][i].d = 0.5;
        } else if (col < 12) {
          epd[col - 6].d = 1.0;
        } else if (col == 12) {
          ad.d = 1.0;
        } else {
          Kd.d = pc.K;
          Gd.d = pc.G;
        }
        Dual S[3][3], ep[6], al, tn[6];
        j2_update(Hd, epd, ad, Kd, Gd, Dual(pc.sy), Dual(pc.H), S, ep, al, tn);
        const double hon = mu[0] * ep[0].d + mu[1] * ep[1].d + mu[2] * ep[2].d + mu[3] * ep[3].d +
                           mu[4] * ep[4].d + mu[5] * ep[5].d + mu[6] * al.d;
        const double tot = hon + sb[0] * S[0][0].d + sb[1] * S[1][1].d + sb[2] * S[2][2].d + sb[3] * S[1][2].d +
                           sb[4] * S[0][2].d + sb[5] * S[0][1].d;
        if (col < 6)
          ebar[col] = hon;
        else if (col < 13)
          a.mu_out[(int64_t)((col - 6) * 8 + qp) * ne + e] = tot;
        else
          sbar += tot;
      }
    } else {  // history-free phase: the state passes through; sigma = s D_hat eps
      double S[3][3];
      hooke(H, pc.lam, pc.mu, S);
      sbar += sb[0] * S[0][0] + sb[1] * S[1][1] + sb[2] * S[2][2] + sb[3] * S[1][2] + sb[4] * S[0][2] +
              sb[5] * S[0][1];
#pragma unroll
      for (int k = 0; k < 7; ++k) a.mu_out[(int64_t)(k * 8 + qp) * ne + e] = mu[k];
    }
    if (a.u_bar && j2) {  // d/dH of the engineering strain: symmetric split of the shear entries
      const double Hb[3][3] = {{ebar[0], ebar[5], ebar[4]}, {ebar[5], ebar[1], ebar[3]}, {ebar[4], ebar[3], ebar[2]}};
#pragma unroll
      for (int l = 0; l < 8; ++l)
#pragma unroll
        for (int c = 0; c < 3; ++c) UB[l][c] += Hb[c][0] * g[l][0] + Hb[c][1] * g[l][1] + Hb[c][2] * g[l][2];
    }
  }
  if (a.s_bar) a.s_bar[e] += sbar;
  if (a.u_bar)
#pragma unroll
    for (int l = 0; l < 8; ++l)
#pragma unroll
      for (int c = 0; c < 3; ++c) atomic_add(a.u_bar + 3 * node[l] + c, UB[l][c]);
}

hipError_t launch_path_vjp(const fe_problem* p, const void* u, const void* hist, const void* c, const void* mu_in,
                           void* mu_out, void* u_bar, void* s_bar, hipStream_t s) {
  PathArgs a;
  a.n = p->n;
  a.h = p->h;
  a.n_el = p->n_el;
  a.phase = p->phase;
  a.scale = static_cast<const double*>(p->scale);
  a.mat = p->mat;
  a.u = static_cast<const double*>(u);
  a.hist = static_cast<const double*>(hist);
  a.c = static_cast<const double*>(c);
  a.mu_in = static_cast<const double*>(mu_in);
  a.mu_out = static_cast<double*>(mu_out);
  a.u_bar = static_cast<double*>(u_bar);
  a.s_bar = static_cast<double*>(s_bar);
  hipLaunchKernelGGL(path_vjp_kernel, dim3((unsigned)((p->n_el + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_lin_stats(const fe_problem* p, unsigned long long* out, hipStream_t s) {
  const dim3 g((unsigned)((p->n_el + 255) / 256)), b(256);
  if (p->prec == FE_F64)
    hipLaunchKernelGGL(lin_stats_kernel<double>, g, b, 0, s, p->n_el, p->phase, p->mat, (const double*)p->tangent, out);
  else
    hipLaunchKernelGGL(lin_stats_kernel<float>, g, b, 0, s, p->n_el, p->phase, p->mat, (const float*)p->tangent, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// deterministic mode: fixed-order sums of per-element nodal values

// One thread per dof: the (up to 8) elements around its node in the order (c, b, a) ascending,
// each element's value of this node's corner.
template <typename T>
__global__ __launch_bounds__(VBLOCK) void det_gather_kernel(int n, int64_t n_el, const T* __restrict__ elf, const uint8_t* mask,
                                                            int mode, int apply_bc, const T* __restrict__ x, T* __restrict__ y,
                                                            const int* stop, double* pa) {
  __shared__ double sh[VBLOCK / 64];
  if (stop && *stop) return;
  const int64_t np1 = n + 1, n_dof = 3 * np1 * np1 * np1;
  double v = 0;
  for (int64_t d = (int64_t)blockIdx.x * VBLOCK + threadIdx.x; d < n_dof; d += (int64_t)gridDim.x * VBLOCK) {
    const int64_t P = d / 3;
    const int c = (int)(d - 3 * P);
    const int gi = (int)(P % np1), gj = (int)((P / np1) % np1), gk = (int)(P / (np1 * np1));
    T sum = 0;
#pragma unroll
    for (int dk = 1; dk >= 0; --dk)
#pragma unroll
      for (int dj = 1; dj >= 0; --dj)
#pragma unroll
        for (int di = 1; di >= 0; --di) {
          const int ea = gi - di, eb = gj - dj, ec = gk - dk;  // element whose corner (di, dj, dk) is this node
          if (ea < 0 || eb < 0 || ec < 0 || ea >= n || eb >= n || ec >= n) continue;
          const int64_t e = ea + (int64_t)n * (eb + (int64_t)n * ec);
          sum += elf[(int64_t)(3 * (di + 2 * dj + 4 * dk) + c) * n_el + e];
        }
    if (apply_bc && mask && mask[d]) sum = mode == 0 ? T(0) : (mode == 1 ? x[d] : T(1));
    y[d] = sum;
    if (pa) v += (double)x[d] * (double)sum;
  }
  if (pa) {
    v = block_sum(v, sh);
    if (threadIdx.x == 0) pa[blockIdx.x] = v;
  }
}

template <typename T>
static hipError_t det_gather_t(const fe_problem* p, const T* elf, int mode, int apply_bc, const T* x, T* y, const int* stop,
                               double* pa, hipStream_t s) {
  const unsigned grid = pa ? (unsigned)GEN_CG_GRID : (unsigned)vgrid(p->n_dof);
  hipLaunchKernelGGL(det_gather_kernel<T>, dim3(grid), dim3(VBLOCK), 0, s, p->n, p->n_el, elf, p->mask, mode, apply_bc, x,
                     y, stop, pa);
  return hipGetLastError();
}

hipError_t det_gather(const fe_problem* p, const void* elf, int mode, int apply_bc, const void* x, void* y,
                      const int* stop, double* pa, hipStream_t s) {
  return p->prec == FE_F64 ? det_gather_t(p, (const double*)elf, mode, apply_bc, (const double*)x, (double*)y, stop, pa, s)
                           : det_gather_t(p, (const float*)elf, mode, apply_bc, (const float*)x, (float*)y, stop, pa, s);
}

// stress_sum[k] = sum of the workgroup partials in workgroup order (one thread per component)
__global__ void det_stress_kernel(const double* part, int nb, double* out) {
  const int k = threadIdx.x;
  if (k >= 6) return;
  double v = 0;
  for (int b = 0; b < nb; ++b) v += part[(int64_t)b * 6 + k];
  out[k] = v;
}

hipError_t det_stress_reduce(const fe_problem* p, hipStream_t s) {
  hipLaunchKernelGGL(det_stress_kernel, dim3(1), dim3(64), 0, s, p->stress_part, elem_grid(p->n), p->stress_sum);
  return hipGetLastError();
}

}  // namespace fe

