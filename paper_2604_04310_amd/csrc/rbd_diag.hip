// Diagnostics: the FP32 fused-multiply-add issue rate of the device at a given
// launch shape, and the streaming HBM bandwidth (write-only and copy), the
// measured ceilings beside the published FP32 and HBM peaks.
#include <hip/hip_runtime.h>

#include "rbd_internal.hpp"

namespace rbd {
namespace {

// ILP independent chains of 16 * iters FMAs per lane (no memory traffic in the
// loop); one store per lane keeps the work alive.
template <int ILP>
__global__ __launch_bounds__(256) void k_fma_rate(float* __restrict__ out, int iters, float a, float b) {
  float x[ILP];
#pragma unroll
  for (int k = 0; k < ILP; ++k) x[k] = threadIdx.x * 1e-3f + k;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int r = 0; r < 16; ++r)
#pragma unroll
      for (int k = 0; k < ILP; ++k) x[k] = __builtin_fmaf(x[k], a, b);
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < ILP; ++k) s += x[k];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <int ILP>
rbd_status time_rate(float* buf, int blocks, int fma_per_lane, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                     float* ms) {
  const int iters = fma_per_lane / (16 * ILP);
  for (int w = 0; w < 3; ++w)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fma_rate<ILP>), dim3(blocks), dim3(256), 0, s, buf, iters, 0.999f, 0.001f);
  const int n = 10;
  if (hipEventRecord(e0, s) != hipSuccess) return fail(RBD_E_LAUNCH, "event record failed");
  for (int w = 0; w < n; ++w)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fma_rate<ILP>), dim3(blocks), dim3(256), 0, s, buf, iters, 0.999f, 0.001f);
  if (hipGetLastError() != hipSuccess) return fail(RBD_E_LAUNCH, "launch failed");
  if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
    return fail(RBD_E_LAUNCH, "event failed");
  if (hipEventElapsedTime(ms, e0, e1) != hipSuccess) return fail(RBD_E_LAUNCH, "event timing failed");
  *ms /= n;
  return RBD_OK;
}

// Streaming HBM kernels over n float4 elements, consecutive lanes on
// consecutive 16-byte elements. COPY reads src and writes dst, else a value
// is written; NT selects non-temporal stores (as the pose, mass-matrix and
// Jacobian outputs are written). With grid-stride = false each thread handles
// kUnroll elements a block's width apart (one 64 KiB tile per block, no
// loop); with grid-stride = true the grid strides over the whole array.
constexpr int kUnroll = 16;
typedef float f4 __attribute__((ext_vector_type(4)));
template <bool COPY, bool NT, bool STRIDE>
__global__ __launch_bounds__(256) void k_hbm_stream(const f4* __restrict__ src, f4* __restrict__ dst, int64_t n,
                                                    float v) {
  auto put = [&](int64_t i) __attribute__((always_inline)) {
    f4 x;
    if constexpr (COPY) x = src[i];
    else x = f4{v, v, v, v};
    if constexpr (NT) __builtin_nontemporal_store(x, &dst[i]);
    else dst[i] = x;
  };
  if constexpr (STRIDE) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) put(i);
  } else {
    const int64_t base = (int64_t)blockIdx.x * kUnroll * blockDim.x + threadIdx.x;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = base + (int64_t)u * blockDim.x;
      if (i < n) put(i);
    }
  }
}

}  // namespace
}  // namespace rbd

// Best of 10 timed launches (after 3 warm-up launches) of the streaming kernel
// over `bytes` bytes (rounded down to 16), 256-thread blocks; GB/s counts the
// bytes moved to and from HBM (copy: read + write).
extern "C" rbd_status rbd_diag_hbm_rate(int device, int64_t bytes, int mode, int blocks, double* gbs) {
  using namespace rbd;
  if (!gbs) return fail(RBD_E_INVAL, "gbs is NULL");
  if (mode < 0 || mode > 2) return fail(RBD_E_INVAL, "mode = %d, expected 0 (write), 1 (copy) or 2 (plain write)", mode);
  if (bytes < (1 << 20) || bytes > (int64_t(16) << 30))
    return fail(RBD_E_INVAL, "bytes = %lld, expected 1 MiB .. 16 GiB", (long long)bytes);
  if (blocks < 0 || blocks > (1 << 20)) return fail(RBD_E_INVAL, "blocks = %d, expected 0..2^20", blocks);
  if (device < 0 || device >= rbd_device_count()) return fail(RBD_E_NODEVICE, "device %d is not available", device);
  if (hipSetDevice(device) != hipSuccess) return fail(RBD_E_NODEVICE, "cannot select device %d", device);
  const int64_t n = bytes / 16;
  f4 *src = nullptr, *dst = nullptr;
  if (hipMalloc(&dst, n * 16) != hipSuccess) return fail(RBD_E_NOMEM, "allocation failed");
  if (mode == 1 && hipMalloc(&src, n * 16) != hipSuccess) {
    (void)hipFree(dst);
    return fail(RBD_E_NOMEM, "allocation failed");
  }
  if (src) (void)hipMemset(src, 0, n * 16);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const unsigned tiles = (unsigned)((n + (int64_t)kUnroll * 256 - 1) / ((int64_t)kUnroll * 256));
  const dim3 grid(blocks > 0 ? (unsigned)blocks : tiles), block(256);
  auto launch = [&]() {
    if (blocks > 0) {
      if (mode == 1) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_hbm_stream<true, true, true>), grid, block, 0, nullptr, src, dst, n, 0.0f);
      else if (mode == 0) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_hbm_stream<false, true, true>), grid, block, 0, nullptr, src, dst, n, 1.0f);
      else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_hbm_stream<false, false, true>), grid, block, 0, nullptr, src, dst, n, 1.0f);
    } else {
      if (mode == 1) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_hbm_stream<true, true, false>), grid, block, 0, nullptr, src, dst, n, 0.0f);
      else if (mode == 0) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_hbm_stream<false, true, false>), grid, block, 0, nullptr, src, dst, n, 1.0f);
      else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_hbm_stream<false, false, false>), grid, block, 0, nullptr, src, dst, n, 1.0f);
    }
  };
  rbd_status st = RBD_OK;
  float best = 0.0f;
  for (int w = 0; w < 3; ++w) launch();
  for (int r = 0; r < 10 && st == RBD_OK; ++r) {
    float ms = 0.0f;
    if (hipEventRecord(e0, nullptr) != hipSuccess) st = fail(RBD_E_LAUNCH, "event record failed");
    launch();
    if (st == RBD_OK && hipGetLastError() != hipSuccess) st = fail(RBD_E_LAUNCH, "launch failed");
    if (st == RBD_OK && (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      st = fail(RBD_E_LAUNCH, "event timing failed");
    if (st == RBD_OK && (best == 0.0f || ms < best)) best = ms;
  }
  (void)hipDeviceSynchronize();
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(dst);
  if (src) (void)hipFree(src);
  if (st != RBD_OK) return st;
  *gbs = (mode == 1 ? 2.0 : 1.0) * (double)(n * 16) / (best * 1e-3) / 1e9;
  return RBD_OK;
}

extern "C" rbd_status rbd_diag_fma_rate(int device, int blocks, int ilp, double* tflops) {
  using namespace rbd;
  if (!tflops) return fail(RBD_E_INVAL, "tflops is NULL");
  if (blocks < 1 || blocks > 65536) return fail(RBD_E_INVAL, "blocks = %d, expected 1..65536", blocks);
  if (ilp != 1 && ilp != 4 && ilp != 16) return fail(RBD_E_INVAL, "ilp = %d, expected 1, 4 or 16", ilp);
  if (device < 0 || device >= rbd_device_count()) return fail(RBD_E_NODEVICE, "device %d is not available", device);
  if (hipSetDevice(device) != hipSuccess) return fail(RBD_E_NODEVICE, "cannot select device %d", device);
  float* buf = nullptr;
  if (hipMalloc(&buf, (size_t)blocks * 256 * sizeof(float)) != hipSuccess) return fail(RBD_E_NOMEM, "allocation failed");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const int fma_per_lane = 16384;
  float ms = 0.0f;
  rbd_status st = ilp == 1 ? time_rate<1>(buf, blocks, fma_per_lane, nullptr, e0, e1, &ms)
                : ilp == 4 ? time_rate<4>(buf, blocks, fma_per_lane, nullptr, e0, e1, &ms)
                           : time_rate<16>(buf, blocks, fma_per_lane, nullptr, e0, e1, &ms);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(buf);
  if (st != RBD_OK) return st;
  *tflops = 2.0 * fma_per_lane * (double)blocks * 256 / (ms * 1e-3) / 1e12;
  return RBD_OK;
}
