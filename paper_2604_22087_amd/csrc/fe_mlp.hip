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
#include <mutex>

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
// backward pass of the mean squared error.  (1) per sample, the pre-activation
// gradients delta_l = dL/dz_l of all layers go to a workspace [n][3*128+6];
// (2) the weight gradients dWt_l[i][o] = sum_s h_{l-1}[s][i] delta_l[s][o] are
// batch-reduced GEMMs: 32x32 tiles, the batch split into chunks of WG_K samples
// whose partial tiles are added with FP32 atomics (dW zeroed first).

constexpr int SB = 32;
constexpr int LDB = HID + 1;
constexpr int WSTRIDE = 3 * HID + NOUT;  // workspace row: delta1, delta2, delta3, delta4
constexpr int WG_K = 1024;

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

// out[s][i] = silu'(zprev[s][i]) * sum_o Wt[i][o] delta[s][o]
__device__ __forceinline__ void back_delta(const float* delta, const float* Wt, const float* zprev, int nin, int nout,
                                           float* out) {
  for (int idx = threadIdx.x; idx < SB * nin; idx += 256) {
    const int s = idx / nin, i = idx % nin;
    float acc = 0.0f;
    for (int o = 0; o < nout; ++o) acc += Wt[i * nout + o] * delta[s * LDB + o];
    out[s * LDB + i] = silu_d(zprev[s * LDB + i]) * acc;
  }
}

__global__ __launch_bounds__(256) void mlp_delta_kernel(const float* __restrict__ W, const float* __restrict__ cache,
                                                        const float* __restrict__ y, const float* __restrict__ t,
                                                        float* __restrict__ work, double* loss, int64_t n) {
  __shared__ float z[3][SB * LDB];
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
      work[(s0 + s) * WSTRIDE + 3 * HID + o] = d;
    }
    d0[s * LDB + o] = d;
  }
  lsum = block_sum_d(lsum, sh);  // (synchronises the block)
  if (threadIdx.x == 0) unsafeAtomicAdd(loss, lsum / (double)n);
  back_delta(d0, W + OFF_W4, z[2], HID, NOUT, d1);  // delta3
  __syncthreads();
  back_delta(d1, W + OFF_W3, z[1], HID, HID, d0);   // delta2
  __syncthreads();
  for (int idx = threadIdx.x; idx < ns * HID; idx += 256) {
    const int s = idx / HID, c = idx % HID;
    work[(s0 + s) * WSTRIDE + 2 * HID + c] = d1[s * LDB + c];
    work[(s0 + s) * WSTRIDE + HID + c] = d0[s * LDB + c];
  }
  back_delta(d0, W + OFF_W2, z[0], HID, HID, d1);   // delta1
  __syncthreads();
  for (int idx = threadIdx.x; idx < ns * HID; idx += 256) {
    const int s = idx / HID, c = idx % HID;
    work[(s0 + s) * WSTRIDE + c] = d1[s * LDB + c];
  }
}

// Weight-gradient tiles: blockIdx.y enumerates (layer, input tile, output tile), 40 in all;
// blockIdx.x the batch chunk.
__global__ __launch_bounds__(256) void mlp_wgrad_kernel(const float* __restrict__ x, const float* __restrict__ cache,
                                                        const float* __restrict__ work, float* dW, int64_t n) {
  __shared__ float hs[32][33], ds[32][33];
  const int tile = blockIdx.y;
  int layer, it, ot;
  if (tile < 4) {
    layer = 0; it = 0; ot = tile;
  } else if (tile < 20) {
    layer = 1; it = (tile - 4) / 4; ot = (tile - 4) % 4;
  } else if (tile < 36) {
    layer = 2; it = (tile - 20) / 4; ot = (tile - 20) % 4;
  } else {
    layer = 3; it = tile - 36; ot = 0;
  }
  const int nin = layer == 0 ? NIN : HID, nout = layer == 3 ? NOUT : HID;
  const int woff = layer == 0 ? OFF_W1 : (layer == 1 ? OFF_W2 : (layer == 2 ? OFF_W3 : OFF_W4));
  const int boff = layer == 0 ? OFF_B1 : (layer == 1 ? OFF_B2 : (layer == 2 ? OFF_B3 : OFF_B4));
  const int doff = layer * HID;  // delta_{layer+1} column offset in the workspace
  const int64_t k0 = (int64_t)blockIdx.x * WG_K, k1 = min<int64_t>(n, k0 + WG_K);
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads, 4 outputs each
  float acc[4] = {0.f, 0.f, 0.f, 0.f}, bacc = 0.f;
  for (int64_t sb = k0; sb < k1; sb += 32) {
    for (int idx = threadIdx.x; idx < 32 * 32; idx += 256) {
      const int s = idx / 32, c = idx % 32;
      const int64_t gs = sb + s;
      const int i = it * 32 + c, o = ot * 32 + c;
      float hv = 0.f, dv = 0.f;
      if (gs < k1) {
        if (i < nin) hv = layer == 0 ? x[gs * NIN + i] : silu_f(cache[gs * 3 * HID + (layer - 1) * HID + i]);
        if (o < nout) dv = work[gs * WSTRIDE + doff + o];
      }
      hs[s][c] = hv;
      ds[s][c] = dv;
    }
    __syncthreads();
#pragma unroll 8
    for (int s = 0; s < 32; ++s) {
      const float dv = ds[s][tx];
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] += hs[s][ty * 4 + r] * dv;
      if (it == 0 && ty == 0) bacc += dv;
    }
    __syncthreads();
  }
  const int o = ot * 32 + tx;
  if (o < nout) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = it * 32 + ty * 4 + r;
      if (i < nin) unsafeAtomicAdd(dW + woff + i * nout + o, acc[r]);
    }
    if (it == 0 && ty == 0) unsafeAtomicAdd(dW + boff + o, bacc);
  }
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
                               float* dW, double* loss, float* work, int64_t n, void* stream) {
  if (!W || !x || !cache || !y || !target || !dW || !loss || !work || n <= 0) {
    set_error("fe_mlp_backward: all arrays are required, n > 0");
    return FE_ERR_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(zero_kernel, dim3(64), dim3(256), 0, s, dW, (int64_t)FE_MLP_PARAMS, loss);
  hipLaunchKernelGGL(mlp_delta_kernel, dim3((unsigned)((n + SB - 1) / SB)), dim3(256), 0, s, W, cache, y, target,
                     work, loss, n);
  hipLaunchKernelGGL(mlp_wgrad_kernel, dim3((unsigned)((n + WG_K - 1) / WG_K), 40), dim3(256), 0, s, x, cache, work,
                     dW, n);
  HIPCHK(hipGetLastError());
  return FE_OK;
}

// Workspace of fe_mlp_backward_static: the per-sample pre-activation gradients of at most
// FE_MLP_STATIC_MAX samples, in a file-scope device array (each GPU the library runs on holds its
// own copy, 12.8 MB, until the process ends).  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol): the device address is looked up
// once per device with hipGetSymbolAddress and kept in g_scratch_dev.
static __device__ __align__(256) float scratch[(size_t)FE_MLP_STATIC_MAX * WSTRIDE];

constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static float* g_scratch_dev[SCRATCH_MAX_DEVICES];

// Device address of `scratch` on the current device, or null (error recorded) on failure.
static float* scratch_on_current_device() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    hip_fail(e, "hipGetDevice");
    return nullptr;
  }
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) {
    set_error("fe_mlp_backward_static: device index beyond the supported range");
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
      return nullptr;
    }
    g_scratch_dev[dev] = static_cast<float*>(ptr);
  }
  return g_scratch_dev[dev];
}

extern "C" int fe_mlp_backward_static(const float* W, const float* x, const float* cache, const float* y,
                                      const float* target, float* dW, double* loss, int64_t n, void* stream) {
  if (!W || !x || !cache || !y || !target || !dW || !loss || n <= 0) {
    set_error("fe_mlp_backward_static: all arrays are required, n > 0");
    return FE_ERR_ARG;
  }
  if (n > FE_MLP_STATIC_MAX) {
    set_error("fe_mlp_backward_static: n exceeds FE_MLP_STATIC_MAX samples (use fe_mlp_backward with a workspace)");
    return FE_ERR_ARG;
  }
  float* work = scratch_on_current_device();
  if (!work) return FE_ERR_HIP;
  // the delta kernel writes every workspace entry the weight-gradient kernel reads
  // (rows 0..n-1), so the array's contents from an earlier call never matter
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(zero_kernel, dim3(64), dim3(256), 0, s, dW, (int64_t)FE_MLP_PARAMS, loss);
  hipLaunchKernelGGL(mlp_delta_kernel, dim3((unsigned)((n + SB - 1) / SB)), dim3(256), 0, s, W, cache, y, target,
                     work, loss, n);
  hipLaunchKernelGGL(mlp_wgrad_kernel, dim3((unsigned)((n + WG_K - 1) / WG_K), 40), dim3(256), 0, s, x, cache, work,
                     dW, n);
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
