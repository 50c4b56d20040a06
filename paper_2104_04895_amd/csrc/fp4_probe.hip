// fp4_probe.hip -- measured throughput of the matrix cores against the vector units on the
// current device, the evidence for where the branch-block contraction of Eq. V4 runs.
//
// Six timed kernels (every loop bounded, one output store per lane):
//   0 FP64 MFMA 16x16x4 (four independent accumulators per wavefront)
//   1 FP64 VALU FMA (sixteen independent chains per lane)
//   2 half of the wavefronts of every work-group as in 0, the other half as in 1
//   3 BF16 MFMA 16x16x32 with FP32 accumulation (four accumulators)
//   4 FP32 VALU FMA (sixteen chains; the build disables packed FP32)
//   5 half as in 3, half as in 4
// Reported as TFLOP/s of the work each kernel performs (2 M N K per MFMA, 2 per FMA).  If the
// matrix core ran beside the vector unit, the mixed kernels would finish in about the time of
// the slower half; if they share the issue or the arithmetic, in about the mean.
#include "fp4_internal.h"

#include <hip/hip_runtime.h>

namespace fp4 {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kProbeIter = 2048;
constexpr int kProbeBlocks = 2048;

__device__ double probe_mfma64(double a, double b) {
  v4d c0 = {0, 0, 0, 0}, c1 = c0, c2 = c0, c3 = c0;
  for (int i = 0; i < kProbeIter; ++i) {
    c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(b, a, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, a, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f64_16x16x4f64(b, b, c3, 0, 0, 0);
  }
  return c0[0] + c1[1] + c2[2] + c3[3];
}

__device__ double probe_valu64(double a, double b) {
  double x[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) x[j] = a + j;
  for (int i = 0; i < kProbeIter * 4; ++i)
#pragma unroll
    for (int j = 0; j < 16; ++j) x[j] = __builtin_fma(x[j], b, a);
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < 16; ++j) s += x[j];
  return s;
}

__device__ double probe_mfma_bf16(float a, float b) {
  bf16x8 A, B;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    A[i] = (__bf16)(a + 0.125f * i);
    B[i] = (__bf16)(b - 0.125f * i);
  }
  v4f c0 = {0, 0, 0, 0}, c1 = c0, c2 = c0, c3 = c0;
  for (int i = 0; i < kProbeIter; ++i) {
    c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(B, A, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, A, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(B, B, c3, 0, 0, 0);
  }
  return (double)(c0[0] + c1[1] + c2[2] + c3[3]);
}

__device__ double probe_valu32(float a, float b) {
  float x[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) x[j] = a + j;
  for (int i = 0; i < kProbeIter * 4; ++i)
#pragma unroll
    for (int j = 0; j < 16; ++j) x[j] = __builtin_fmaf(x[j], b, a);
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < 16; ++j) s += x[j];
  return (double)s;
}

__global__ __launch_bounds__(256) void k_probe(int mode, double a, double b, double *out) {
  const int w = threadIdx.x >> 6;
  const bool first = (w & 1) == 0;
  double r;
  switch (mode) {
    case 0: r = probe_mfma64(a, b); break;
    case 1: r = probe_valu64(a, b); break;
    case 2: r = first ? probe_mfma64(a, b) : probe_valu64(a, b); break;
    case 3: r = probe_mfma_bf16((float)a, (float)b); break;
    case 4: r = probe_valu32((float)a, (float)b); break;
    default: r = first ? probe_mfma_bf16((float)a, (float)b) : probe_valu32((float)a, (float)b); break;
  }
  out[(size_t)blockIdx.x * 256 + threadIdx.x] = r;
}

}  // namespace

size_t probe_out_doubles() { return (size_t)kProbeBlocks * 256; }

// Times each of the six kernels (one warm-up launch, then one timed) on stream s into
// tflops[6]; `out` holds probe_out_doubles() doubles of device memory.
hipError_t run_probe(double *out, double *tflops, hipStream_t s) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const double waves = kProbeBlocks * 4.0;
  const double f_mfma64 = kProbeIter * 4.0 * (2.0 * 16 * 16 * 4);
  const double f_valu = kProbeIter * 4.0 * 16.0 * 2.0 * 64.0;
  const double f_bf16 = kProbeIter * 4.0 * (2.0 * 16 * 16 * 32);
  const double flops[6] = {waves * f_mfma64, waves * f_valu, waves / 2 * (f_mfma64 + f_valu),
                           waves * f_bf16, waves * f_valu, waves / 2 * (f_bf16 + f_valu)};
  for (int mode = 0; mode < 6 && e == hipSuccess; ++mode) {
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
      e = hipEventRecord(e0, s);
      if (e != hipSuccess) break;
      hipLaunchKernelGGL(k_probe, dim3(kProbeBlocks), dim3(256), 0, s, mode, 1.0000001, 0.9999999, out);
      e = hipGetLastError();
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess && rep == 1) tflops[mode] = flops[mode] / ((double)ms * 1e9);
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return e;
}

}  // namespace fp4
