// Learned cost model for scheduling: a 4 -> 64 -> 64 -> 1 ReLU MLP that maps
// per-vertex features (log1p of degree, core number, triangles, length-2
// walks) to log(search nodes of the vertex's subproblem).  It only orders the
// work queue; it never changes the cliques.
//
// Parameter block (float, kMlpParams entries), row-major:
//   W1[64][4], b1[64], W2[64][64], b2[64], w3[64], b3[1],
//   mu[4], sigma[4]   (feature standardisation: x' = (x - mu) / sigma)
// One wavefront handles 64 samples at a time (lane = sample); weights are
// read from LDS with wave-uniform addresses (broadcast).  The batch is a few
// hundred thousand vertices, i.e. ~1 GFLOP per forward pass: VALU FP32 is
// ample, so the kernels stay on the vector units.

#include "dev.h"
#include "internal.h"

#include <mutex>

namespace mce {

namespace {

constexpr int H = 64;
constexpr int kW1 = 0, kB1 = kW1 + H * 4, kW2 = kB1 + H, kB2 = kW2 + H * H, kW3 = kB2 + H, kB3 = kW3 + H,
              kMu = kB3 + 1, kSig = kMu + 4, kTotal = kSig + 4;
static_assert(kTotal == 4553, "parameter block layout");

__device__ __forceinline__ float relu(float a) { return a > 0.0f ? a : 0.0f; }

// bfloat16 by round-to-nearest-even on the float's bits (NaN stays NaN).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ float round_bf16(float f) { return bf16_to_f32(f32_to_bf16(f)); }

template <bool BF16>
__global__ void __launch_bounds__(64) k_forward(const float* __restrict__ prm, const uint16_t* __restrict__ prm16,
                                                const float* __restrict__ x, uint64_t n, float* __restrict__ y) {
  __shared__ float P[kTotal];
  __shared__ float H1[H][64];  // [unit][sample]
  const int lane = threadIdx.x;
  for (int i = lane; i < kTotal; i += 64) {
    float v = BF16 ? bf16_to_f32(prm16[i]) : prm[i];
    if (BF16 && i >= kMu) v = prm[i];  // standardisation constants stay FP32
    P[i] = v;
  }
  __syncthreads();
  for (uint64_t base = (uint64_t)blockIdx.x * 64; base < n; base += (uint64_t)gridDim.x * 64) {
    const uint64_t s = base + lane;
    float xin[4];
    for (int k = 0; k < 4; ++k) {
      float v = s < n ? (x[4 * s + k] - P[kMu + k]) / P[kSig + k] : 0.0f;
      xin[k] = BF16 ? round_bf16(v) : v;
    }
    for (int i = 0; i < H; ++i) {
      float a = P[kB1 + i];
      for (int k = 0; k < 4; ++k) a += P[kW1 + i * 4 + k] * xin[k];
      H1[i][lane] = BF16 ? round_bf16(relu(a)) : relu(a);
    }
    float out = P[kB3];
    for (int j = 0; j < H; ++j) {
      float a = P[kB2 + j];
      for (int i = 0; i < H; ++i) a += P[kW2 + j * H + i] * H1[i][lane];
      const float h2 = BF16 ? round_bf16(relu(a)) : relu(a);
      out += P[kW3 + j] * h2;
    }
    if (s < n) y[s] = out;
  }
}

// Gradient of L = (1/n) sum (yhat - t)^2 with respect to the first kMu
// parameters: block b writes its samples' share to row b of `part` (kRow
// floats: the kMu gradient entries, then its share of L); k_grad_reduce adds
// the rows in block order, so the result does not depend on scheduling.
// One wave per block; lanes are samples in the forward/backward sweep and
// hidden units in the weight-gradient sweep.
constexpr int kRow = kMu + 1;

__global__ void __launch_bounds__(64) k_backward(const float* __restrict__ prm, const float* __restrict__ x,
                                                 const float* __restrict__ t, uint64_t n, float* part) {
  __shared__ float P[kTotal];
  __shared__ float H1[H][65];   // [unit][sample]
  __shared__ float H2[H][65];
  __shared__ float DA2[H][65];
  __shared__ float DA1[H][65];
  __shared__ float XS[4][65];
  __shared__ float DY[64];
  const int lane = threadIdx.x;
  for (int i = lane; i < kTotal; i += 64) P[i] = prm[i];
  __syncthreads();
  const float inv_n = 1.0f / (float)n;
  float gW2[H];
  for (int i = 0; i < H; ++i) gW2[i] = 0.0f;
  float gW1[4] = {0, 0, 0, 0};
  float gb1 = 0, gb2 = 0, gw3 = 0, gb3 = 0, l = 0;
  for (uint64_t base = (uint64_t)blockIdx.x * 64; base < n; base += (uint64_t)gridDim.x * 64) {
    const uint64_t s = base + lane;
    const bool valid = s < n;
    // forward, lane = sample
    float xin[4];
    for (int k = 0; k < 4; ++k) {
      xin[k] = valid ? (x[4 * s + k] - P[kMu + k]) / P[kSig + k] : 0.0f;
      XS[k][lane] = xin[k];
    }
    float h1[H];
    for (int i = 0; i < H; ++i) {
      float a = P[kB1 + i];
      for (int k = 0; k < 4; ++k) a += P[kW1 + i * 4 + k] * xin[k];
      h1[i] = relu(a);
      H1[i][lane] = h1[i];
    }
    float out = P[kB3];
    for (int j = 0; j < H; ++j) {
      float a = P[kB2 + j];
      for (int i = 0; i < H; ++i) a += P[kW2 + j * H + i] * h1[i];
      const float h2 = relu(a);
      H2[j][lane] = h2;
      out += P[kW3 + j] * h2;
    }
    const float dy = valid ? 2.0f * (out - t[s]) * inv_n : 0.0f;
    if (valid) l += (out - t[s]) * (out - t[s]) * inv_n;
    DY[lane] = dy;
    for (int j = 0; j < H; ++j) DA2[j][lane] = H2[j][lane] > 0.0f ? dy * P[kW3 + j] : 0.0f;
    __syncthreads();
    // dh1 = W2^T da2, masked by relu'(a1)
    for (int i = 0; i < H; ++i) {
      float a = 0;
      for (int j = 0; j < H; ++j) a += P[kW2 + j * H + i] * DA2[j][lane];
      DA1[i][lane] = h1[i] > 0.0f ? a : 0.0f;
    }
    __syncthreads();
    // weight gradients, lane = hidden unit
    const int u = lane;
    for (int smp = 0; smp < 64; ++smp) {
      const float d2 = DA2[u][smp];
      gb2 += d2;
      gw3 += DY[smp] * H2[u][smp];
      for (int i = 0; i < H; ++i) gW2[i] += d2 * H1[i][smp];
      const float d1 = DA1[u][smp];
      gb1 += d1;
      for (int k = 0; k < 4; ++k) gW1[k] += d1 * XS[k][smp];
    }
    if (lane == 0)
      for (int smp = 0; smp < 64; ++smp) gb3 += DY[smp];
    __syncthreads();
  }
  const int u = lane;
  float* row = part + (uint64_t)blockIdx.x * kRow;
  for (int i = 0; i < H; ++i) row[kW2 + u * H + i] = gW2[i];
  for (int k = 0; k < 4; ++k) row[kW1 + u * 4 + k] = gW1[k];
  row[kB1 + u] = gb1;
  row[kB2 + u] = gb2;
  row[kW3 + u] = gw3;
  if (lane == 0) row[kB3] = gb3;
  for (int o = 32; o >= 1; o >>= 1) l += __shfl_xor(l, o, 64);
  if (lane == 0) row[kMu] = l;
}

// grad[i] = sum over blocks b (in order) of part[b][i] for the trainable
// parameters, 0 for mu/sigma; loss[0] = sum of the blocks' loss shares.
__global__ void k_grad_reduce(const float* __restrict__ part, uint32_t nb, float* grad, float* loss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > kTotal) return;
  const int col = i < kMu ? i : kMu;
  float a = 0.0f;
  if (i < kMu || i == kTotal)
    for (uint32_t b = 0; b < nb; ++b) a += part[(uint64_t)b * kRow + col];
  if (i < kTotal)
    grad[i] = i < kMu ? a : 0.0f;
  else
    loss[0] = a;
}

// per-device rows of the blocks' partial gradients
std::mutex g_part_mu;
DevBuf g_part[64];

// Adam (Kingma & Ba) on the trainable parameters; step >= 1.
__global__ void k_adam(float* prm, float* m, float* v, const float* grad, float lr, float b1, float b2, float eps,
                       uint32_t step) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kMu) return;
  const float g = grad[i];
  const float mi = b1 * m[i] + (1.0f - b1) * g;
  const float vi = b2 * v[i] + (1.0f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / (1.0f - powf(b1, (float)step));
  const float vh = vi / (1.0f - powf(b2, (float)step));
  prm[i] -= lr * mh / (sqrtf(vh) + eps);
}

// Feature standardisation constants (mean and standard deviation per column).
__global__ void __launch_bounds__(256) k_norm(const float* __restrict__ x, uint64_t n, float* prm) {
  __shared__ double acc[8][256];
  double s[4] = {0, 0, 0, 0}, q[4] = {0, 0, 0, 0};
  for (uint64_t i = threadIdx.x; i < n; i += blockDim.x)
    for (int k = 0; k < 4; ++k) {
      double v = x[4 * i + k];
      s[k] += v;
      q[k] += v * v;
    }
  for (int k = 0; k < 4; ++k) {
    acc[k][threadIdx.x] = s[k];
    acc[4 + k][threadIdx.x] = q[k];
  }
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < 8; ++k) acc[k][threadIdx.x] += acc[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) {
    const int k = threadIdx.x;
    const double mean = acc[k][0] / (double)n;
    double var = acc[4 + k][0] / (double)n - mean * mean;
    if (var < 1e-12) var = 1.0;
    prm[kMu + k] = (float)mean;
    prm[kSig + k] = (float)sqrt(var);
  }
}

__global__ void k_to_bf16(const float* prm, uint16_t* out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kTotal) out[i] = f32_to_bf16(prm[i]);
}

__global__ void k_labels(const uint64_t* __restrict__ nodes, uint64_t n, float* y) {
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = logf((float)(nodes[i] > 0 ? nodes[i] : 1));
}

uint32_t grid_for(uint64_t n) {
  uint64_t g = (n + 63) / 64;
  return (uint32_t)(g < 4096 ? (g ? g : 1) : 4096);
}

}  // namespace

// BF16 prediction on stream s without a wait (the static call's schedule).
hipError_t launch_mlp_forward_bf16(const float* prm, const uint16_t* prm16, const float* feat, uint64_t n, float* out,
                                   hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_forward<true>, dim3(grid_for(n)), dim3(64), 0, s, prm, prm16, feat, n, out);
  return hipGetLastError();
}

}  // namespace mce

using namespace mce;

extern "C" {

uint32_t mce_mlp_param_count(void) { return (uint32_t)kTotal; }

int mce_mlp_forward(const float* params, const float* feat, uint64_t n, float* out, void* hip_stream) {
  if (!params || (n && (!feat || !out))) {
    set_error("NULL argument");
    return MCE_EINVAL;
  }
  if (n == 0) return MCE_OK;
  hipStream_t s = (hipStream_t)hip_stream;
  hipLaunchKernelGGL(k_forward<false>, dim3(grid_for(n)), dim3(64), 0, s, params, nullptr, feat, n, out);
  MCE_TRY_HIP(hipGetLastError());
  MCE_TRY_HIP(hipStreamSynchronize(s));
  return MCE_OK;
}

int mce_mlp_forward_bf16(const uint16_t* params_bf16, const float* params, const float* feat, uint64_t n, float* out,
                         void* hip_stream) {
  if (!params_bf16 || !params || (n && (!feat || !out))) {
    set_error("NULL argument");
    return MCE_EINVAL;
  }
  if (n == 0) return MCE_OK;
  hipStream_t s = (hipStream_t)hip_stream;
  hipLaunchKernelGGL(k_forward<true>, dim3(grid_for(n)), dim3(64), 0, s, params, params_bf16, feat, n, out);
  MCE_TRY_HIP(hipGetLastError());
  MCE_TRY_HIP(hipStreamSynchronize(s));
  return MCE_OK;
}

int mce_mlp_grad(const float* params, const float* feat, const float* target, uint64_t n, float* grad, float* loss,
                 void* hip_stream) {
  if (!params || !grad || !loss || (n && (!feat || !target))) {
    set_error("NULL argument");
    return MCE_EINVAL;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  int dev = 0;
  MCE_TRY_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) {
    set_error("device index %d out of range", dev);
    return MCE_ENOTSUP;
  }
  const uint32_t nb = n ? (grid_for(n) < 1024 ? grid_for(n) : 1024) : 0;
  std::lock_guard<std::mutex> lk(g_part_mu);
  DevBuf& part = g_part[dev];
  MCE_TRY(part.ensure((uint64_t)std::max<uint32_t>(nb, 1) * kRow * sizeof(float)));
  if (n) {
    hipLaunchKernelGGL(k_backward, dim3(nb), dim3(64), 0, s, params, feat, target, n, part.as<float>());
    MCE_TRY_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_grad_reduce, dim3((kTotal + 1 + 255) / 256), dim3(256), 0, s, part.as<float>(), nb, grad, loss);
  MCE_TRY_HIP(hipGetLastError());
  MCE_TRY_HIP(hipStreamSynchronize(s));
  return MCE_OK;
}

int mce_mlp_adam(float* params, float* m, float* v, const float* grad, float lr, uint32_t step, void* hip_stream) {
  if (!params || !m || !v || !grad || step == 0) {
    set_error("bad argument");
    return MCE_EINVAL;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  hipLaunchKernelGGL(k_adam, dim3((kMu + 255) / 256), dim3(256), 0, s, params, m, v, grad, lr, 0.9f, 0.999f, 1e-8f,
                     step);
  MCE_TRY_HIP(hipGetLastError());
  return MCE_OK;
}

int mce_mlp_fit_norm(float* params, const float* feat, uint64_t n, void* hip_stream) {
  if (!params || !feat || n == 0) {
    set_error("bad argument");
    return MCE_EINVAL;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  hipLaunchKernelGGL(k_norm, dim3(1), dim3(256), 0, s, feat, n, params);
  MCE_TRY_HIP(hipGetLastError());
  MCE_TRY_HIP(hipStreamSynchronize(s));
  return MCE_OK;
}

int mce_mlp_to_bf16(const float* params, uint16_t* params_bf16, void* hip_stream) {
  if (!params || !params_bf16) {
    set_error("NULL argument");
    return MCE_EINVAL;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  hipLaunchKernelGGL(k_to_bf16, dim3((kTotal + 255) / 256), dim3(256), 0, s, params, params_bf16);
  MCE_TRY_HIP(hipGetLastError());
  MCE_TRY_HIP(hipStreamSynchronize(s));
  return MCE_OK;
}

int mce_mlp_labels(const uint64_t* nodes, uint64_t n, float* target, void* hip_stream) {
  if (n && (!nodes || !target)) {
    set_error("NULL argument");
    return MCE_EINVAL;
  }
  if (n == 0) return MCE_OK;
  hipStream_t s = (hipStream_t)hip_stream;
  hipLaunchKernelGGL(k_labels, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, nodes, n, target);
  MCE_TRY_HIP(hipGetLastError());
  MCE_TRY_HIP(hipStreamSynchronize(s));
  return MCE_OK;
}

}  // extern "C"
