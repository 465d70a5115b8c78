// Measured peaks of the matrix units the chain kernels use (ctr_probe_peaks
// in include/ctrace.h): register-only loops of independent MFMA
// instructions on every SIMD, timed with HIP events.  The roofline figures
// of the benchmark are the published ones; these say what the device at hand
// delivers at its clock.
#include <hip/hip_runtime.h>

#include "ctrace_internal.h"

namespace ctr {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kProbeIter = 4096;
constexpr int kProbeThreads = 256;

// The sink write is never taken for these inputs; it keeps the loops alive.
__global__ __launch_bounds__(kProbeThreads) void k_probe_f64_16(double* sink, double s) {
  const double a = s + threadIdx.x, b = s - threadIdx.x;
  d4 c0 = {0, 0, 0, 0}, c1 = c0, c2 = c0, c3 = c0;
  for (int i = 0; i < kProbeIter; ++i) {
    c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c3, 0, 0, 0);
  }
  const d4 r = c0 + c1 + c2 + c3;
  if (r[0] == 12345.0) sink[threadIdx.x] = r[1] + r[2] + r[3];
}

__global__ __launch_bounds__(kProbeThreads) void k_probe_f64_4(double* sink, double s) {
  const double a = s + threadIdx.x, b = s - threadIdx.x;
  double c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = 0; i < kProbeIter; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) c[j] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c[j], 0, 0, 0);
  }
  double r = 0.0;
  for (int j = 0; j < 8; ++j) r += c[j];
  if (r == 12345.0) sink[threadIdx.x] = r;
}

__global__ __launch_bounds__(kProbeThreads) void k_probe_f32_16(double* sink, double s) {
  const float a = (float)(s + threadIdx.x), b = (float)(s - threadIdx.x);
  f4 c0 = {0, 0, 0, 0}, c1 = c0, c2 = c0, c3 = c0;
  for (int i = 0; i < kProbeIter; ++i) {
    c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c3, 0, 0, 0);
  }
  const f4 r = c0 + c1 + c2 + c3;
  if (r[0] == 12345.0f) sink[threadIdx.x] = r[1] + r[2] + r[3];
}

}  // namespace

// flops per wavefront and loop trip: 16x16x4 -> 2048 per instruction, x4 instructions;
// 4x4x4 (four 4x4 blocks) -> 512 per instruction, x8 instructions.
hipError_t probe_peaks(int device, hipStream_t stream, double* sink, double* out) {
  int cus = 0, clock_khz = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeClockRate, device)) != hipSuccess) return e;
  const int blocks = cus * 8;  // 8 workgroups of 4 wavefronts per CU: 8 wavefronts per SIMD
  const double waves = (double)blocks * (kProbeThreads / 64);
  struct K {
    const void* fn;
    double flop_per_wave_iter;
  } ks[3] = {{reinterpret_cast<const void*>(&k_probe_f64_16), 4 * 2048.0},
             {reinterpret_cast<const void*>(&k_probe_f64_4), 8 * 512.0},
             {reinterpret_cast<const void*>(&k_probe_f32_16), 4 * 2048.0}};
  hipEvent_t t0, t1;
  if ((e = hipEventCreate(&t0)) != hipSuccess) return e;
  if ((e = hipEventCreate(&t1)) != hipSuccess) {
    (void)hipEventDestroy(t0);
    return e;
  }
  for (int k = 0; k < 3 && e == hipSuccess; ++k) {
    double s = 0.5;
    void* args[] = {&sink, &s};
    // one warm-up launch, then the timed one
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
      if (rep == 1) e = hipEventRecord(t0, stream);
      if (e == hipSuccess) e = hipLaunchKernel(ks[k].fn, dim3(blocks), dim3(kProbeThreads), args, 0, stream);
      if (e == hipSuccess && rep == 1) e = hipEventRecord(t1, stream);
    }
    if (e == hipSuccess) e = hipEventSynchronize(t1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
    if (e == hipSuccess) out[k] = waves * kProbeIter * ks[k].flop_per_wave_iter / (ms * 1e-3) / 1e12;
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  out[3] = clock_khz / 1000.0;
  out[4] = cus;
  return e;
}

}  // namespace ctr
