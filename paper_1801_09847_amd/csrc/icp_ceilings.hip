// Measured ceilings of the device, against which the kernels of this library
// are judged: the issue rate of unpacked float32 / float64 vector arithmetic
// (independent dependency chains, one instruction per operation, no packed
// forms) and the streaming bandwidth of device memory (a plain copy and a
// plain read of buffers larger than the last-level cache).
//
// These are measurement hooks, not part of the registration method: the
// figures they return are the denominators of the bench's "alu" and copy
// fractions, taken on the same device in the same process.

#include <hip/hip_runtime.h>

#include <string>

#include "icp_runtime.h"

#pragma clang fp contract(off)

namespace {

constexpr int kChains = 8;  // independent dependency chains per thread

// kind 0: v_mul_f32 then v_add_f32 per chain step; kind 2: the same in
// float64.  Every operation is one instruction; the multiplier keeps values
// bounded and normal.
template <int KIND>
__global__ __launch_bounds__(256) void valu_chain_kernel(float* out, int iters, float a, float b) {
  using F = typename std::conditional<(KIND >= 2), double, float>::type;
  F x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = (F)(threadIdx.x + c) * (F)1e-3;
  const F fa = (F)a, fb = (F)b;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      x[c] = x[c] * fa;
      x[c] = x[c] + fb;
    }
  }
  F s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s = s + x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = (float)s;
}

// kind 1: two v_fma_f32 per chain step; kind 3: two v_fma_f64.
template <int KIND>
__global__ __launch_bounds__(256) void valu_fma_kernel(float* out, int iters, float a, float b) {
  using F = typename std::conditional<(KIND >= 2), double, float>::type;
  F x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = (F)(threadIdx.x + c) * (F)1e-3;
  const F fa = (F)a, fb = (F)b;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      if constexpr (KIND == 1) {
        x[c] = __builtin_fmaf(x[c], fa, fb);
        x[c] = __builtin_fmaf(x[c], fa, fb);
      } else {
        x[c] = __builtin_fma(x[c], fa, fb);
        x[c] = __builtin_fma(x[c], fa, fb);
      }
    }
  }
  F s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s = s + x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = (float)s;
}

// kind 4: the squared-distance pattern of a 36-dimensional feature comparison
// (per dimension one v_sub, one v_mul and one v_add for each of two queries
// against a target held in scalar registers): many independent instructions
// per wave, the shape in which the SIMDs reach their highest unpacked rate.
__global__ __launch_bounds__(256) void valu_distance_kernel(float* out, const float* __restrict__ tg,
                                                            int iters) {
  float q0[36], q1[36];
#pragma unroll
  for (int k = 0; k < 36; ++k) {
    q0[k] = (float)(threadIdx.x + k) * 1e-3f;
    q1[k] = (float)(3 * threadIdx.x + k) * 1e-3f;
  }
  float b0 = 1e30f, b1 = 1e30f;
  for (int it = 0; it < iters; ++it) {
    const float* t = tg + (it & 63) * 36;
    float s0 = 0.f, s1 = 0.f;
#pragma unroll
    for (int k = 0; k < 36; ++k) {
      const float tk = t[k];
      const float d0 = q0[k] - tk, d1 = q1[k] - tk;
      s0 = s0 + d0 * d0;
      s1 = s1 + d1 * d1;
    }
    b0 = fminf(b0, s0);
    b1 = fminf(b1, s1);
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = b0 + b1;
}

__global__ __launch_bounds__(256) void copy_kernel(const float4* __restrict__ src, float4* __restrict__ dst,
                                                   int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

__global__ __launch_bounds__(256) void read_kernel(const float4* __restrict__ src, float* __restrict__ out,
                                                   int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  float s = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float4 v = src[i];
    s = s + ((v.x + v.y) + (v.z + v.w));
  }
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

struct Scoped {
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  void* a = nullptr;
  void* b = nullptr;
  ~Scoped() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (s) (void)hipStreamDestroy(s);
  }
};

}  // namespace

extern "C" int icp_measure_valu(int device, int kind, double* lane_ops_per_s, double* best_ms) {
  if (!lane_ops_per_s || kind < 0 || kind > 4) return icp_rt::fail(ICP_E_INVALID_ARG, "icp_measure_valu: bad argument");
  HIP_TRY(hipSetDevice(device), "hipSetDevice");
  int n_cu = 0;
  HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device), "hipDeviceGetAttribute");
  Scoped z;
  HIP_TRY(hipStreamCreateWithFlags(&z.s, hipStreamNonBlocking), "hipStreamCreate");
  HIP_TRY(hipEventCreate(&z.e0), "hipEventCreate");
  HIP_TRY(hipEventCreate(&z.e1), "hipEventCreate");
  // 8 waves per SIMD (4 SIMDs per CU): enough to cover the dependent-issue
  // latency of each chain several times over
  const int blocks = n_cu * 8;
  const int iters = 2048;
  HIP_TRY(hipMalloc(&z.a, (size_t)blocks * 256 * sizeof(float)), "hipMalloc");
  HIP_TRY(hipMalloc(&z.b, 64 * 36 * sizeof(float)), "hipMalloc");
  HIP_TRY(hipMemsetAsync(z.b, 0, 64 * 36 * sizeof(float), z.s), "hipMemsetAsync");
  float* out = static_cast<float*>(z.a);
  const float* tg = static_cast<const float*>(z.b);
  const float a = 0.999f, b = 1e-3f;
  const int dist_iters = iters / 8;
  auto launch = [&]() {
    switch (kind) {
      case 0: valu_chain_kernel<0><<<blocks, 256, 0, z.s>>>(out, iters, a, b); break;
      case 1: valu_fma_kernel<1><<<blocks, 256, 0, z.s>>>(out, iters, a, b); break;
      case 2: valu_chain_kernel<2><<<blocks, 256, 0, z.s>>>(out, iters, a, b); break;
      case 3: valu_fma_kernel<3><<<blocks, 256, 0, z.s>>>(out, iters, a, b); break;
      default: valu_distance_kernel<<<blocks, 256, 0, z.s>>>(out, tg, dist_iters); break;
    }
  };
  launch();  // warm-up (clocks ramp, code object loads)
  HIP_TRY(hipGetLastError(), "valu kernel launch");
  float best = 1e30f;
  for (int rep = 0; rep < 5; ++rep) {
    HIP_TRY(hipEventRecord(z.e0, z.s), "hipEventRecord");
    launch();
    HIP_TRY(hipEventRecord(z.e1, z.s), "hipEventRecord");
    HIP_TRY(hipEventSynchronize(z.e1), "hipEventSynchronize");
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, z.e0, z.e1), "hipEventElapsedTime");
    if (ms < best) best = ms;
  }
  // lane operations: two per chain per trip; the distance pattern six per
  // dimension per trip
  const double ops = kind == 4 ? (double)blocks * 256.0 * dist_iters * 36.0 * 6.0
                               : (double)blocks * 256.0 * iters * kChains * 2.0;
  *lane_ops_per_s = ops / (best * 1e-3);
  if (best_ms) *best_ms = best;
  return ICP_SUCCESS;
}

extern "C" int icp_measure_copy(int device, int64_t bytes, int kind, double* gb_per_s, double* best_ms) {
  if (!gb_per_s || bytes < (1 << 20) || (kind != 0 && kind != 1))
    return icp_rt::fail(ICP_E_INVALID_ARG, "icp_measure_copy: bad argument");
  HIP_TRY(hipSetDevice(device), "hipSetDevice");
  int n_cu = 0;
  HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device), "hipDeviceGetAttribute");
  Scoped z;
  HIP_TRY(hipStreamCreateWithFlags(&z.s, hipStreamNonBlocking), "hipStreamCreate");
  HIP_TRY(hipEventCreate(&z.e0), "hipEventCreate");
  HIP_TRY(hipEventCreate(&z.e1), "hipEventCreate");
  const int64_t n4 = bytes / 16;
  const int blocks = n_cu * 16;
  HIP_TRY(hipMalloc(&z.a, (size_t)n4 * 16), "hipMalloc");
  if (kind == 0) {
    HIP_TRY(hipMalloc(&z.b, (size_t)n4 * 16), "hipMalloc");
  } else {
    HIP_TRY(hipMalloc(&z.b, (size_t)blocks * 256 * sizeof(float)), "hipMalloc");
  }
  HIP_TRY(hipMemsetAsync(z.a, 0, (size_t)n4 * 16, z.s), "hipMemsetAsync");
  auto launch = [&]() {
    if (kind == 0)
      copy_kernel<<<blocks, 256, 0, z.s>>>(static_cast<const float4*>(z.a), static_cast<float4*>(z.b), n4);
    else
      read_kernel<<<blocks, 256, 0, z.s>>>(static_cast<const float4*>(z.a), static_cast<float*>(z.b), n4);
  };
  launch();
  HIP_TRY(hipGetLastError(), "copy kernel launch");
  float best = 1e30f;
  for (int rep = 0; rep < 5; ++rep) {
    HIP_TRY(hipEventRecord(z.e0, z.s), "hipEventRecord");
    launch();
    HIP_TRY(hipEventRecord(z.e1, z.s), "hipEventRecord");
    HIP_TRY(hipEventSynchronize(z.e1), "hipEventSynchronize");
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, z.e0, z.e1), "hipEventElapsedTime");
    if (ms < best) best = ms;
  }
  const double moved = (double)n4 * 16.0 * (kind == 0 ? 2.0 : 1.0);
  *gb_per_s = moved / (best * 1e-3) / 1e9;
  if (best_ms) *best_ms = best;
  return ICP_SUCCESS;
}
