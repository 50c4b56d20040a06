// fp4_device.h -- small device helpers shared by the kernels of the library: complex
// arithmetic, exact roots of unity, and the fixed-order FP64 energy-window predicate.
#pragma once
#include <hip/hip_runtime.h>

namespace fp4 {
namespace {

// ------------------------------------------------------------------ complex helpers

template <typename R> struct CT;
template <> struct CT<double> { using T = double2; };
template <> struct CT<float> { using T = float2; };

__device__ __forceinline__ double fmaR(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaR(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <typename V> __device__ __forceinline__ V czero() { V z; z.x = 0; z.y = 0; return z; }
template <typename V> __device__ __forceinline__ V cconj(V a) { a.y = -a.y; return a; }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  V r;
  r.x = fmaR(a.x, b.x, -a.y * b.y);
  r.y = fmaR(a.x, b.y, a.y * b.x);
  return r;
}
// acc += a * b
template <typename V> __device__ __forceinline__ void cmac(V &acc, V a, V b) {
  acc.x = fmaR(a.x, b.x, acc.x);
  acc.x = fmaR(-a.y, b.y, acc.x);
  acc.y = fmaR(a.x, b.y, acc.y);
  acc.y = fmaR(a.y, b.x, acc.y);
}
// acc += a * conj(b)
template <typename V> __device__ __forceinline__ void cmac_cb(V &acc, V a, V b) {
  acc.x = fmaR(a.x, b.x, acc.x);
  acc.x = fmaR(a.y, b.y, acc.x);
  acc.y = fmaR(-a.x, b.y, acc.y);
  acc.y = fmaR(a.y, b.x, acc.y);
}
template <typename V> __device__ __forceinline__ V cadd(V a, V b) { a.x += b.x; a.y += b.y; return a; }

__device__ __forceinline__ float2 to32(double2 a) { return make_float2((float)a.x, (float)a.y); }
template <typename V> __device__ __forceinline__ V fromd(double2 a);
template <> __device__ __forceinline__ double2 fromd<double2>(double2 a) { return a; }
template <> __device__ __forceinline__ float2 fromd<float2>(double2 a) { return to32(a); }

// exp(2 pi i k / N) with exact conjugate symmetry between k and N - k
__device__ __forceinline__ double2 root_of_unity(long long k, int N) {
  const bool upper = 2 * k > N;
  const long long kk = upper ? N - k : k;
  double s, co;
  sincospi(2.0 * (double)kk / (double)N, &s, &co);
  return make_double2(co, upper ? -s : s);
}

__device__ __forceinline__ int wrap(int x, int g) {
  x = x >= g ? x - g : x;
  x = x >= g ? x - g : x;
  x = x < 0 ? x + g : x;
  x = x < 0 ? x + g : x;
  return x;
}

// Energy-window predicate in a fixed FP64 order without contraction:
//   dw = bw - w3 (bw = (w s' w') s'' w'' formed by the caller, left to right)
//   s2 = (dx*dx + dy*dy) + dz*dz, d = v'' - v'''
//   keep <=> dw*dw <= c_win * s2
__device__ __forceinline__ bool window_keep(double bw, double w3, double4 v2, double4 v3,
                                            double c_win, double &dw, double &s2) {
#pragma clang fp contract(off)
  dw = bw - w3;
  const double dx = v2.x - v3.x, dy = v2.y - v3.y, dz = v2.z - v3.z;
  s2 = (dx * dx + dy * dy) + dz * dz;
  return dw * dw <= c_win * s2;
}

__device__ __forceinline__ double add_signed(double a, double b, int s) {
#pragma clang fp contract(off)
  return s > 0 ? a + b : a - b;
}

}  // namespace
}  // namespace fp4
