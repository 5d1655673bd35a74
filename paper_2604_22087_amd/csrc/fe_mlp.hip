// Learned constitutive surrogate: MLP 13 -> 128 -> 128 -> 128 -> 6 (SiLU) on gfx950.
//
// Inference (forward + 6 forward-mode tangent columns) is a chain of dense
// products, so it runs on the FP32 matrix cores (v_mfma_f32_16x16x4f32): a
// workgroup stages 64 rows in LDS -- per sample the value row, the six tangent
// rows (input e_j) and one pad row -- and each wave multiplies one 16-row tile
// by the layer's weights (read input-major, so 16 consecutive lanes load 16
// consecutive floats).  The epilogue applies SiLU to value rows and scales the
// tangent rows by SiLU'(z) of their sample's value row, fetched with a lane shuffle.
// Training (backward pass, Adam) is lighter and runs on the vector units.
#include "fe_internal.hpp"

namespace fe {

constexpr int HID = FE_MLP_HIDDEN, NIN = FE_MLP_IN, NOUT = FE_MLP_OUT;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NIN * HID;
constexpr int OFF_W2 = OFF_B1 + HID, OFF_B2 = OFF_W2 + HID * HID;
constexpr int OFF_W3 = OFF_B2 + HID, OFF_B3 = OFF_W3 + HID * HID;
constexpr int OFF_W4 = OFF_B3 + HID, OFF_B4 = OFF_W4 + HID * NOUT;
static_assert(OFF_B4 + NOUT == FE_MLP_PARAMS, "parameter layout");

constexpr int MROWS = 64;       // rows staged per workgroup (4 tiles of 16, one per wave)
constexpr int LDA = HID + 4;    // LDS row stride in floats

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float sigm(float z) { return 1.0f / (1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_f(float z) { return z * sigm(z); }
__device__ __forceinline__ float silu_d(float z) {
  const float s = sigm(z);
  return s * (1.0f + z * (1.0f - s));
}

// One hidden layer: Dst = act(A Wt + b) for MROWS rows.  RPS rows per sample
// (1: values only; 8: value, six tangents, pad).  Lane layout of the 16x16x4
// FP32 MFMA: A[l%16][l/16], B[l/16][l%16], D[4(l/16)+r][l%16].
template <int RPS, int KPAD>
__device__ __forceinline__ void hidden_layer(const float* A, float* Dst, const float* __restrict__ Wt,
                                             const float* __restrict__ b, int K, float* cache, int64_t s0,
                                             int64_t n, int layer) {
  const int lane = threadIdx.x & 63, rt = threadIdx.x >> 6;
  v4f acc[HID / 16];
#pragma unroll
  for (int ct = 0; ct < HID / 16; ++ct) acc[ct] = v4f{0.f, 0.f, 0.f, 0.f};
  const float* arow = A + (rt * 16 + (lane & 15)) * LDA;
  for (int k0 = 0; k0 < KPAD; k0 += 4) {
    const int k = k0 + (lane >> 4);
    const float a = arow[k];
    const bool kin = k < K;
#pragma unroll
    for (int ct = 0; ct < HID / 16; ++ct) {
      const float bv = kin ? Wt[k * HID + ct * 16 + (lane & 15)] : 0.0f;
      acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv, acc[ct], 0, 0, 0);
    }
  }
  // value row of this lane's sample (RPS = 8): row 0 of the 8-row group -> lane base + column
  const int src = ((lane >> 5) << 5) + (lane & 15);
#pragma unroll
  for (int ct = 0; ct < HID / 16; ++ct) {
    const int col = ct * 16 + (lane & 15);
    const float bias = b[col];
    const float zv = __shfl(acc[ct][0], src, 64) + bias;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = rt * 16 + 4 * (lane >> 4) + r;
      float out;
      if (RPS == 1) {
        const float z = acc[ct][r] + bias;
        out = silu_f(z);
        const int64_t gs = s0 + row;
        if (cache && gs < n) cache[gs * (3 * HID) + layer * HID + col] = z;
      } else {
        const int path = row % RPS;
        if (path == 0) {
          out = silu_f(zv);
          const int64_t gs = s0 + row / RPS;
          if (cache && gs < n) cache[gs * (3 * HID) + layer * HID + col] = zv;
        } else if (path <= NOUT) {
          out = silu_d(zv) * acc[ct][r];
        } else {
          out = 0.0f;
        }
      }
      Dst[row * LDA + col] = out;
    }
  }
}

template <int RPS>
__global__ __launch_bounds__(256) void mlp_fwd_kernel(const float* __restrict__ W, const float* __restrict__ x,
                                                      float* __restrict__ y, float* __restrict__ jac,
                                                      float* __restrict__ cache, int64_t n) {
  constexpr int SPB = MROWS / RPS;
  __shared__ float act[2][MROWS * LDA];
  const int64_t s0 = (int64_t)blockIdx.x * SPB;
  for (int i = threadIdx.x; i < MROWS * 16; i += 256) {
    const int row = i / 16, k = i % 16;
    const int path = row % RPS;
    const int64_t gs = s0 + row / RPS;
    float v = 0.0f;
    if (gs < n) {
      if (path == 0)
        v = (k < NIN) ? x[gs * NIN + k] : 0.0f;
      else if (path <= NOUT)
        v = (k == path - 1) ? 1.0f : 0.0f;
    }
    act[0][row * LDA + k] = v;
  }
  __syncthreads();
  hidden_layer<RPS, 16>(act[0], act[1], W + OFF_W1, W + OFF_B1, NIN, cache, s0, n, 0);
  __syncthreads();
  hidden_layer<RPS, HID>(act[1], act[0], W + OFF_W2, W + OFF_B2, HID, cache, s0, n, 1);
  __syncthreads();
  hidden_layer<RPS, HID>(act[0], act[1], W + OFF_W3, W + OFF_B3, HID, cache, s0, n, 2);
  __syncthreads();
  // output layer: 6 columns padded to one 16-wide tile, no activation
  const int lane = threadIdx.x & 63, rt = threadIdx.x >> 6;
  const int col = lane & 15;
  v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
  const float* arow = act[1] + (rt * 16 + (lane & 15)) * LDA;
  const float* W4 = W + OFF_W4;
  for (int k0 = 0; k0 < HID; k0 += 4) {
    const int k = k0 + (lane >> 4);
    const float bv = col < NOUT ? W4[k * NOUT + col] : 0.0f;
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(arow[k], bv, acc, 0, 0, 0);
  }
  if (col < NOUT) {
    const float bias = W[OFF_B4 + col];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = rt * 16 + 4 * (lane >> 4) + r;
      const int path = row % RPS;
      const int64_t gs = s0 + row / RPS;
      if (gs >= n) continue;
      if (path == 0)
        y[gs * NOUT + col] = acc[r] + bias;
      else if (path <= NOUT && jac)
        jac[gs * (NOUT * NOUT) + col * NOUT + (path - 1)] = acc[r];
    }
  }
}

// ---------------------------------------------------------------------------
// backward pass of the mean squared error, SB samples per workgroup; weight
// gradients are summed over workgroups with FP32 atomics (dW zeroed first).

constexpr int SB = 32;
constexpr int LDB = HID + 1;

__device__ __forceinline__ double block_sum_d(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < 4; ++i) r += sh[i];
  return r;
}

// Given delta (dL/dz_l, [SB][nout]) and the layer input h ([SB][nin]):
// dWt[i][o] += sum_s h[s][i] delta[s][o], db[o] += sum_s delta[s][o].
__device__ __forceinline__ void weight_grad(const float* h, const float* delta, int nin, int nout, int ns,
                                            float* dWt, float* db) {
  for (int idx = threadIdx.x; idx < nin * nout; idx += 256) {
    const int i = idx / nout, o = idx % nout;
    float acc = 0.0f;
    for (int s = 0; s < ns; ++s) acc += h[s * LDB + i] * delta[s * LDB + o];
    unsafeAtomicAdd(dWt + idx, acc);
  }
  for (int o = threadIdx.x; o < nout; o += 256) {
    float acc = 0.0f;
    for (int s = 0; s < ns; ++s) acc += delta[s * LDB + o];
    unsafeAtomicAdd(db + o, acc);
  }
}

// delta_prev[s][i] = silu'(z_prev[s][i]) * sum_o Wt[i][o] delta[s][o]
__device__ __forceinline__ void back_delta(const float* delta, const float* Wt, const float* zprev, int nin, int nout,
                                           int ns, float* out) {
  for (int idx = threadIdx.x; idx < ns * nin; idx += 256) {
    const int s = idx / nin, i = idx % nin;
    float acc = 0.0f;
    for (int o = 0; o < nout; ++o) acc += Wt[i * nout + o] * delta[s * LDB + o];
    out[s * LDB + i] = silu_d(zprev[s * LDB + i]) * acc;
  }
}

__global__ __launch_bounds__(256) void mlp_bwd_kernel(const float* __restrict__ W, const float* __restrict__ x,
                                                      const float* __restrict__ cache, const float* __restrict__ y,
                                                      const float* __restrict__ t, float* dW, double* loss,
                                                      int64_t n) {
  __shared__ float z[3][SB * LDB];   // pre-activations of the three hidden layers
  __shared__ float hbuf[SB * LDB];   // layer input (activation or x)
  __shared__ float d0[SB * LDB], d1[SB * LDB];
  __shared__ double sh[4];
  const int64_t s0 = (int64_t)blockIdx.x * SB;
  const int ns = (int)min<int64_t>(SB, n - s0);
  for (int idx = threadIdx.x; idx < SB * 3 * HID; idx += 256) {
    const int s = idx / (3 * HID), rem = idx % (3 * HID), l = rem / HID, c = rem % HID;
    z[l][s * LDB + c] = s < ns ? cache[(s0 + s) * 3 * HID + rem] : 0.0f;
  }
  const float scale = 2.0f / (float)n;
  double lsum = 0;
  for (int idx = threadIdx.x; idx < SB * NOUT; idx += 256) {
    const int s = idx / NOUT, o = idx % NOUT;
    float d = 0.0f;
    if (s < ns) {
      const float e = y[(s0 + s) * NOUT + o] - t[(s0 + s) * NOUT + o];
      lsum += (double)e * (double)e;
      d = scale * e;
    }
    d0[s * LDB + o] = d;
  }
  lsum = block_sum_d(lsum, sh);
  if (threadIdx.x == 0) unsafeAtomicAdd(loss, lsum / (double)n);
  // layer 4 (input h3 = silu(z3))
  for (int idx = threadIdx.x; idx < SB * HID; idx += 256) {
    const int s = idx / HID, c = idx % HID;
    hbuf[s * LDB + c] = silu_f(z[2][s * LDB + c]);
  }
  __syncthreads();
  weight_grad(hbuf, d0, HID, NOUT, ns, dW + OFF_W4, dW + OFF_B4);
  back_delta(d0, W + OFF_W4, z[2], HID, NOUT, ns, d1);
  __syncthreads();
  // layer 3 (input h2)
  for (int idx = threadIdx.x; idx < SB * HID; idx += 256) {
    const int s = idx / HID, c = idx % HID;
    hbuf[s * LDB + c] = silu_f(z[1][s * LDB + c]);
  }
  __syncthreads();
  weight_grad(hbuf, d1, HID, HID, ns, dW + OFF_W3, dW + OFF_B3);
  back_delta(d1, W + OFF_W3, z[1], HID, HID, ns, d0);
  __syncthreads();
  // layer 2 (input h1)
  for (int idx = threadIdx.x; idx < SB * HID; idx += 256) {
    const int s = idx / HID, c = idx % HID;
    hbuf[s * LDB + c] = silu_f(z[0][s * LDB + c]);
  }
  __syncthreads();
  weight_grad(hbuf, d0, HID, HID, ns, dW + OFF_W2, dW + OFF_B2);
  back_delta(d0, W + OFF_W2, z[0], HID, HID, ns, d1);
  __syncthreads();
  // layer 1 (input x)
  for (int idx = threadIdx.x; idx < SB * NIN; idx += 256) {
    const int s = idx / NIN, c = idx % NIN;
    hbuf[s * LDB + c] = s < ns ? x[(s0 + s) * NIN + c] : 0.0f;
  }
  __syncthreads();
  weight_grad(hbuf, d1, NIN, HID, ns, dW + OFF_W1, dW + OFF_B1);
}

__global__ void adam_kernel(float* W, const float* dW, float* m, float* v, int64_t np, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x) {
    const float g = dW[i];
    const float mi = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    W[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  }
}

__global__ void zero_kernel(float* a, int64_t n, double* d) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) a[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0 && d) *d = 0;
}

}  // namespace fe

using namespace fe;

#define HIPCHK(x)                                  \
  do {                                             \
    hipError_t _e = (x);                           \
    if (_e != hipSuccess) return hip_fail(_e, #x); \
  } while (0)

extern "C" int fe_mlp_forward(const float* W, const float* x, float* y, float* jac, float* cache, int64_t n,
                              void* stream) {
  if (!W || !x || !y || n < 0) {
    set_error("fe_mlp_forward: W, x and y are required, n >= 0");
    return FE_ERR_ARG;
  }
  if (n == 0) return FE_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (jac) {
    const int64_t blocks = (n + MROWS / 8 - 1) / (MROWS / 8);
    hipLaunchKernelGGL(mlp_fwd_kernel<8>, dim3((unsigned)blocks), dim3(256), 0, s, W, x, y, jac, cache, n);
  } else {
    const int64_t blocks = (n + MROWS - 1) / MROWS;
    hipLaunchKernelGGL(mlp_fwd_kernel<1>, dim3((unsigned)blocks), dim3(256), 0, s, W, x, y, jac, cache, n);
  }
  HIPCHK(hipGetLastError());
  return FE_OK;
}

extern "C" int fe_mlp_backward(const float* W, const float* x, const float* cache, const float* y, const float* target,
                               float* dW, double* loss, int64_t n, void* stream) {
  if (!W || !x || !cache || !y || !target || !dW || !loss || n <= 0) {
    set_error("fe_mlp_backward: all arrays are required, n > 0");
    return FE_ERR_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(zero_kernel, dim3(64), dim3(256), 0, s, dW, (int64_t)FE_MLP_PARAMS, loss);
  hipLaunchKernelGGL(mlp_bwd_kernel, dim3((unsigned)((n + SB - 1) / SB)), dim3(256), 0, s, W, x, cache, y, target,
                     dW, loss, n);
  HIPCHK(hipGetLastError());
  return FE_OK;
}

extern "C" int fe_adam_step(float* W, const float* dW, float* m, float* v, int64_t np, double lr, double beta1,
                            double beta2, double eps, int t, void* stream) {
  if (!W || !dW || !m || !v || np <= 0 || t < 1) {
    set_error("fe_adam_step: arrays required, n_param > 0, t >= 1");
    return FE_ERR_ARG;
  }
  const double c1 = 1.0 / (1.0 - std::pow(beta1, t)), c2 = 1.0 / (1.0 - std::pow(beta2, t));
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)std::min<int64_t>((np + 255) / 256, 1024)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), W, dW, m, v, np, (float)lr, (float)beta1, (float)beta2,
                     (float)eps, (float)c1, (float)c2);
  HIPCHK(hipGetLastError());
  return FE_OK;
}
