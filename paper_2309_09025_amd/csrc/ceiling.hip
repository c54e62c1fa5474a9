// Measured ceilings of the two resources the bootstrapping kernels can be
// bound by: binary64 VALU issue (the exact modular arithmetic of the
// transforms) and HBM streaming.  The VALU probe runs the blind rotation's
// own instruction forms (the modular product of ntt_fp64.h inside a
// butterfly or a multiply-accumulate, or a bare FMA) on registers only, at
// a chosen number of waves per SIMD, so the fraction of peak a kernel
// reaches can be set against what this chip issues at that occupancy.
#include <hip/hip_runtime.h>

#include <string>

#include "fs_internal.h"
#include "kernels.h"

namespace fs {
namespace {

constexpr int kProbeThreads = 256;  // four waves: one per SIMD of a CU

// One butterfly stage over the register pairs (r, r + 2^B): 8 butterflies
// (x, y) -> (x + w y, x - w y) with the modular product, 8 instructions each.
template <int B>
__device__ __forceinline__ void probe_stage(double x[16], double w) {
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    if (r & (1 << B)) continue;
    const int r2 = r | (1 << B);
    const double m = mulmod(x[r2], w);
    const double a = x[r] + m, d = x[r] - m;
    x[r] = a;
    x[r2] = d;
  }
}

// kind 0: four butterfly stages per iteration (32 butterflies, 256
// instructions), the data flow of a transform round.  kind 1: acc_r +=
// w (acc_{r^1} + x_r) (modular product and sum, 7 instructions, plus the
// add that keeps the operand loop-carried), 16 per iteration.
// kind 2: x_r = fma(x_r, a, c), 16 per iteration.  The multipliers come
// from the kernel arguments, so nothing folds; every value stays finite
// (w < 2^10 keeps the growth additive).
template <int KIND>
__global__ void __launch_bounds__(kProbeThreads)
valu_probe_kernel(double w0, double w1, uint32_t iters, double* __restrict__ out) {
  double x[16], acc[16];
  const double t = (double)(threadIdx.x + 1);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    x[r] = t * (r + 3);
    acc[r] = 0.0;
  }
  for (uint32_t it = 0; it < iters; ++it) {
    if constexpr (KIND == 0) {
      probe_stage<0>(x, w0);
      probe_stage<1>(x, w1);
      probe_stage<2>(x, w0);
      probe_stage<3>(x, w1);
    } else if constexpr (KIND == 1) {
#pragma unroll
      for (int r = 0; r < 16; r += 2) {  // each product reads the other sum of its pair
        const double m0 = mulmod(acc[r + 1] + x[r], w0), m1 = mulmod(acc[r] + x[r + 1], w1);
        acc[r] += m0;
        acc[r + 1] += m1;
      }
    } else {
#pragma unroll
      for (int r = 0; r < 16; ++r) x[r] = __builtin_fma(x[r], w0, w1);
    }
  }
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < 16; ++r) s += x[r] + acc[r];
  out[(size_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256)
hbm_copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * 256;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// Makes `device` current for the probe and restores the caller's device.
struct ProbeDevice {
  int prev = -1;
  hipError_t err;
  explicit ProbeDevice(int device) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    err = hipSetDevice(device);
  }
  ~ProbeDevice() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

}  // namespace
}  // namespace fs

using namespace fs;

extern "C" {

int fs_probe_valu(int device, uint32_t waves_per_simd, uint32_t kind, double* lane_instr_per_s,
                  double* ms) {
  if (!lane_instr_per_s || kind > 2 || waves_per_simd == 0 || waves_per_simd > 8)
    return fail(FS_EINVAL, "fs_probe_valu: kind 0..2, 1..8 waves per SIMD, non-null output");
  ProbeDevice g(device);
  if (g.err != hipSuccess) return fail(FS_EDEVICE, "fs_probe_valu: no such device");
  int cus = 0;
  size_t lds = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    return fail(FS_EDEVICE, "fs_probe_valu: device attributes");
  int lds_cu = 0;
  if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device) !=
      hipSuccess)
    return fail(FS_EDEVICE, "fs_probe_valu: device attributes");
  // LDS per workgroup so that at most waves_per_simd workgroups (of one
  // wave per SIMD) fit a CU; the grid is exactly that many per CU
  lds = (size_t)lds_cu / waves_per_simd - 1024;
  const uint32_t blocks = (uint32_t)cus * waves_per_simd;
  const double per_iter[3] = {256.0, 128.0, 16.0};  // VALU instructions per thread
  // about 2e12 lane-instructions per launch, whatever the occupancy
  const uint32_t iters =
      (uint32_t)(2.0e12 / ((double)blocks * kProbeThreads * per_iter[kind]));
  double* out = nullptr;
  if (hipMalloc(&out, (size_t)blocks * kProbeThreads * sizeof(double)) != hipSuccess)
    return fail(FS_ENOMEM, "fs_probe_valu: allocation");
  auto launch = [&](uint32_t n) {
    const double w0 = 977.0, w1 = 613.0;
    switch (kind) {
      case 0: valu_probe_kernel<0><<<blocks, kProbeThreads, lds>>>(w0, w1, n, out); break;
      case 1: valu_probe_kernel<1><<<blocks, kProbeThreads, lds>>>(w0, w1, n, out); break;
      default:
        valu_probe_kernel<2><<<blocks, kProbeThreads, lds>>>(1.0 - 0x1p-40, 0x1p-30, n, out);
    }
  };
  (void)hipFuncSetAttribute((const void*)valu_probe_kernel<0>,
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  (void)hipFuncSetAttribute((const void*)valu_probe_kernel<1>,
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  (void)hipFuncSetAttribute((const void*)valu_probe_kernel<2>,
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  launch(iters / 16);  // warm-up
  (void)hipEventRecord(e0, nullptr);
  launch(iters);
  (void)hipEventRecord(e1, nullptr);
  const hipError_t e = hipEventSynchronize(e1);
  float t = 0.f;
  (void)hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(out);
  const hipError_t le = hipGetLastError();
  if (e != hipSuccess || le != hipSuccess || t <= 0.f)
    return fail(FS_EDEVICE, std::string("fs_probe_valu: ") +
                                hipGetErrorString(e != hipSuccess ? e : le));
  *lane_instr_per_s = (double)blocks * kProbeThreads * iters * per_iter[kind] / (t * 1e-3);
  if (ms) *ms = t;
  return FS_OK;
}

int fs_probe_hbm(int device, size_t bytes, double* bytes_per_s, double* ms) {
  if (!bytes_per_s || bytes < (1u << 20))
    return fail(FS_EINVAL, "fs_probe_hbm: at least 1 MiB, non-null output");
  ProbeDevice g(device);
  if (g.err != hipSuccess) return fail(FS_EDEVICE, "fs_probe_hbm: no such device");
  const size_t n = bytes / 2 / sizeof(uint4);  // half read, half written
  uint4 *src = nullptr, *dst = nullptr;
  if (hipMalloc(&src, n * sizeof(uint4)) != hipSuccess)
    return fail(FS_ENOMEM, "fs_probe_hbm: allocation");
  if (hipMalloc(&dst, n * sizeof(uint4)) != hipSuccess) {
    (void)hipFree(src);
    return fail(FS_ENOMEM, "fs_probe_hbm: allocation");
  }
  (void)hipMemset(src, 1, n * sizeof(uint4));
  int cus = 0;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  const uint32_t blocks = (uint32_t)cus * 8;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  hbm_copy_kernel<<<blocks, 256>>>(src, dst, n);  // warm-up
  (void)hipEventRecord(e0, nullptr);
  const int reps = 5;
  for (int k = 0; k < reps; ++k) hbm_copy_kernel<<<blocks, 256>>>(src, dst, n);
  (void)hipEventRecord(e1, nullptr);
  const hipError_t e = hipEventSynchronize(e1);
  float t = 0.f;
  (void)hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(src);
  (void)hipFree(dst);
  const hipError_t le = hipGetLastError();
  if (e != hipSuccess || le != hipSuccess || t <= 0.f)
    return fail(FS_EDEVICE, std::string("fs_probe_hbm: ") +
                                hipGetErrorString(e != hipSuccess ? e : le));
  *bytes_per_s = 2.0 * n * sizeof(uint4) * reps / (t * 1e-3);
  if (ms) *ms = t / reps;
  return FS_OK;
}

}  // extern "C"
