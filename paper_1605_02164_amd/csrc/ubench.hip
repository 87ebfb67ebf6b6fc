// Peak probes of the device (bf_ubench): the rates the roofline of the fused
// kernel is read against -- FP32 and FP16 matrix products, FP32 FMAs,
// the transcendental unit, LDS reads, and a device copy through HBM.  Each
// probe is one small kernel whose work is counted exactly (instructions x
// lanes x the operation's flops or bytes) and timed with HIP events; the
// best of a few launches is reported.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "bfvec.h"
#include "host.h"

namespace bfvec {
namespace {

typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));

constexpr int kWaves = 8;            // waves per workgroup (two per SIMD)
constexpr int kThreads = 64 * kWaves;

// C independent accumulator chains of 16x16x4 FP32 products per wave.
template <int C>
__global__ __launch_bounds__(kThreads) void ub_mfma_f32(float* out, int iters) {
  f32x4_t acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
  const float a = 1.0f + threadIdx.x * 1e-7f, b = 1e-3f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < C; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

// C chains of 16x16x32 FP16 products per wave.
template <int C>
__global__ __launch_bounds__(kThreads) void ub_mfma_f16(float* out, int iters) {
  f32x4_t acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
  f16x8_t a, b;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    a[k] = (_Float16)(1.0f + k * 1e-3f);
    b[k] = (_Float16)(1e-3f * (threadIdx.x & 7));
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < C; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

// C chains of FP32 FMAs per lane (the build disables packed FP32 issue).
template <int C>
__global__ __launch_bounds__(kThreads) void ub_valu_f32(float* out, int iters) {
  float x[C];
#pragma unroll
  for (int c = 0; c < C; ++c) x[c] = 1.0f + (threadIdx.x + c) * 1e-7f;
  const float m = 0.999999f, k = 1e-7f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < C; ++c) x[c] = fmaf(x[c], m, k);
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < C; ++c) s += x[c];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

// 8 chains of v_sin_f32 (argument in turns) per lane.
__global__ __launch_bounds__(kThreads) void ub_sin_f32(float* out, int iters) {
  float x[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) x[c] = 0.1f + (threadIdx.x + c) * 1e-6f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = __builtin_amdgcn_sinf(x[c]);
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < 8; ++c) s += x[c];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

// 128-bit LDS reads: lane l of each wave reads 16 bytes at 16 l (+ a
// wave-uniform step), so a wave's 64 reads cover 1 KB without conflicts.
__global__ __launch_bounds__(kThreads) void ub_lds_read(float* out, int iters) {
  __shared__ float4 buf[2048];   // 32 KB
  for (int i = threadIdx.x; i < 2048; i += kThreads) buf[i] = make_float4(i, i + 1, i + 2, i + 3);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  for (int i = 0; i < iters; ++i) {
    const float4 v = buf[((i & 31) << 6) + lane];
    acc.x += v.x;
    acc.y += v.y;
    acc.z += v.z;
    acc.w += v.w;
  }
  out[blockIdx.x * kThreads + threadIdx.x] = acc.x + acc.y + acc.z + acc.w;
}

// Matrix and vector work side by side: waves 0-3 (one per SIMD) run two
// chains of FP32 (F16 = false) or FP16 matrix products when WHAT & 1, waves
// 4-7 eight chains of FP32 FMAs when WHAT & 2.
template <bool F16, int WHAT>
__global__ __launch_bounds__(kThreads) void ub_mix(float* out, int iters, int fma_iters) {
  const int w = threadIdx.x >> 6;
  float s = 0.0f;
  if (w < 4 && (WHAT & 1)) {
    f32x4_t acc0 = {0.0f, 0.0f, 0.0f, 0.0f}, acc1 = acc0;
    if constexpr (F16) {
      f16x8_t a, b;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        a[k] = (_Float16)(1.0f + k * 1e-3f);
        b[k] = (_Float16)(1e-3f * (threadIdx.x & 7));
      }
      for (int i = 0; i < iters; ++i) {
        acc0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc1, 0, 0, 0);
      }
    } else {
      const float a = 1.0f + threadIdx.x * 1e-7f, b = 1e-3f;
      for (int i = 0; i < iters; ++i) {
        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc1, 0, 0, 0);
      }
    }
    s = acc0[0] + acc1[3];
  } else if (w >= 4 && (WHAT & 2)) {
    float x[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = 1.0f + (threadIdx.x + c) * 1e-7f;
    for (int i = 0; i < fma_iters; ++i) {
#pragma unroll
      for (int c = 0; c < 8; ++c) x[c] = fmaf(x[c], 0.999999f, 1e-7f);
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) s += x[c];
  }
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

// Grid-stride copy of n float4.
__global__ __launch_bounds__(256) void ub_copy(const float4* __restrict__ src,
                                               float4* __restrict__ dst, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    dst[i] = src[i];
}

int cu_count() {
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return ncu;
}

// Best of 3 timed launches (after one untimed), in ms.
template <class F>
int best_ms(F launch, float* best) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) {
    launch();
    e = hipGetLastError();
  }
  *best = 1e30f;
  for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
    e = hipEventRecord(e0, nullptr);
    if (e != hipSuccess) break;
    launch();
    if ((e = hipGetLastError()) != hipSuccess) break;
    if ((e = hipEventRecord(e1, nullptr)) != hipSuccess) break;
    if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
    float ms = 0.0f;
    if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
    *best = std::min(*best, ms);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return e == hipSuccess ? BF_OK : fail(BF_EDEVICE, std::string("bf_ubench: ") + hipGetErrorString(e));
}

}  // namespace
}  // namespace bfvec

using namespace bfvec;

extern "C" int bf_ubench(int probe, int param, double* rate) {
  clear_error();
  if (!rate) return fail(BF_EINVAL, "bf_ubench: rate must be non-null");
  *rate = 0.0;
  const bool chains = probe == BF_UB_MFMA_F32 || probe == BF_UB_MFMA_F16 ||
                      probe == BF_UB_VALU_F32 || probe == BF_UB_MFMA_F32_SOLO;
  const bool overlap = probe == BF_UB_OVERLAP_F32 || probe == BF_UB_OVERLAP_F16;
  if (chains && param != 1 && param != 2 && param != 4 && param != 8)
    return fail(BF_EINVAL, "bf_ubench: chains must be 1, 2, 4 or 8");
  if (probe == BF_UB_HBM_COPY && (param < 1 || param > 16384))
    return fail(BF_EINVAL, "bf_ubench: copy size must be 1..16384 MiB");
  if (overlap && param != 0) return fail(BF_EINVAL, "bf_ubench: overlap probes take param 0");
  if (probe < BF_UB_MFMA_F32 || probe > BF_UB_OVERLAP_F16)
    return fail(BF_EINVAL, "bf_ubench: unknown probe");
  const int ncu = cu_count();
  if (ncu <= 0) return fail(BF_EDEVICE, "bf_ubench: no device");
  float ms = 0.0f;
  int rc = BF_OK;
  if (probe == BF_UB_HBM_COPY) {
    const size_t bytes = (size_t)param << 20, n = bytes / sizeof(float4);
    float4 *src = nullptr, *dst = nullptr;
    hipError_t e = hipMalloc(&src, bytes);
    if (e == hipSuccess) e = hipMalloc(&dst, bytes);
    if (e == hipSuccess) e = hipMemset(src, 0, bytes);
    if (e == hipSuccess) {
      const int blocks = ncu * 8;
      rc = best_ms([&] { ub_copy<<<blocks, 256>>>(src, dst, n); }, &ms);
      if (rc == BF_OK) *rate = 2.0 * (double)bytes / (ms * 1e-3) / 1e12;   // read + write
    } else {
      rc = fail(BF_EDEVICE, std::string("bf_ubench: ") + hipGetErrorString(e));
    }
    if (src) (void)hipFree(src);
    if (dst) (void)hipFree(dst);
    return rc;
  }
  float* out = nullptr;
  hipError_t e = hipMalloc(&out, (size_t)ncu * kThreads * sizeof(float));
  if (e != hipSuccess) return fail(BF_EDEVICE, std::string("bf_ubench: ") + hipGetErrorString(e));
  const int iters = 2000;
  double work = 0.0;   // flops or bytes per launch
  const double waves = (double)ncu * kWaves;
  // (solo: one wave per SIMD, so a wave's dependent chain is not hidden
  // behind another wave's)
  const int nthr = probe == BF_UB_MFMA_F32_SOLO ? kThreads / 2 : kThreads;
  auto mfma32 = [&](auto C) {
    constexpr int c = decltype(C)::value;
    rc = best_ms([&] { ub_mfma_f32<c><<<ncu, nthr>>>(out, iters); }, &ms);
    work = (double)ncu * (nthr / 64) * iters * c * (2.0 * 16 * 16 * 4);
  };
  auto mfma16 = [&](auto C) {
    constexpr int c = decltype(C)::value;
    rc = best_ms([&] { ub_mfma_f16<c><<<ncu, kThreads>>>(out, iters); }, &ms);
    work = waves * iters * c * (2.0 * 16 * 16 * 32);
  };
  auto valu = [&](auto C) {
    constexpr int c = decltype(C)::value;
    rc = best_ms([&] { ub_valu_f32<c><<<ncu, kThreads>>>(out, iters * 8); }, &ms);
    work = waves * 64.0 * iters * 8 * c * 2.0;
  };
  if (overlap) {
    // durations chosen so that each side alone takes about the same time
    // (one wave per SIMD: ~36 cycles per FP32 product pair member, ~9 per
    // FMA instruction; FP16 products are 4x shorter)
    const bool f16 = probe == BF_UB_OVERLAP_F16;
    const int mi = f16 ? 16000 : 4000, fi = 4000;
    float tm = 0.0f, tf = 0.0f, tb = 0.0f;
    if (f16) {
      rc = best_ms([&] { ub_mix<true, 1><<<ncu, kThreads>>>(out, mi, fi); }, &tm);
      if (rc == BF_OK) rc = best_ms([&] { ub_mix<true, 2><<<ncu, kThreads>>>(out, mi, fi); }, &tf);
      if (rc == BF_OK) rc = best_ms([&] { ub_mix<true, 3><<<ncu, kThreads>>>(out, mi, fi); }, &tb);
    } else {
      rc = best_ms([&] { ub_mix<false, 1><<<ncu, kThreads>>>(out, mi, fi); }, &tm);
      if (rc == BF_OK) rc = best_ms([&] { ub_mix<false, 2><<<ncu, kThreads>>>(out, mi, fi); }, &tf);
      if (rc == BF_OK) rc = best_ms([&] { ub_mix<false, 3><<<ncu, kThreads>>>(out, mi, fi); }, &tb);
    }
    (void)hipFree(out);
    if (rc == BF_OK) *rate = (tm + tf - tb) / std::min(tm, tf);
    return rc;
  }
  switch (probe) {
    case BF_UB_MFMA_F32:
    case BF_UB_MFMA_F32_SOLO:
      if (param == 1) mfma32(std::integral_constant<int, 1>{});
      else if (param == 2) mfma32(std::integral_constant<int, 2>{});
      else if (param == 4) mfma32(std::integral_constant<int, 4>{});
      else mfma32(std::integral_constant<int, 8>{});
      break;
    case BF_UB_MFMA_F16:
      if (param == 1) mfma16(std::integral_constant<int, 1>{});
      else if (param == 2) mfma16(std::integral_constant<int, 2>{});
      else if (param == 4) mfma16(std::integral_constant<int, 4>{});
      else mfma16(std::integral_constant<int, 8>{});
      break;
    case BF_UB_VALU_F32:
      if (param == 1) valu(std::integral_constant<int, 1>{});
      else if (param == 2) valu(std::integral_constant<int, 2>{});
      else if (param == 4) valu(std::integral_constant<int, 4>{});
      else valu(std::integral_constant<int, 8>{});
      break;
    case BF_UB_TRANS_F32:
      rc = best_ms([&] { ub_sin_f32<<<ncu, kThreads>>>(out, iters); }, &ms);
      work = waves * 64.0 * iters * 8;   // operations, not flops
      break;
    case BF_UB_LDS_READ:
      rc = best_ms([&] { ub_lds_read<<<ncu, kThreads>>>(out, iters * 4); }, &ms);
      work = waves * 64.0 * iters * 4 * 16.0;   // bytes
      break;
  }
  (void)hipFree(out);
  if (rc == BF_OK) *rate = work / (ms * 1e-3) / 1e12;
  return rc;
}
