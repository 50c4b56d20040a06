// fp4_kappa.hip -- RTA lattice thermal conductivity from the three- and four-phonon rates.
//
// kappa^{ab}(T) = 1/(N Omega) sum_lambda C_lambda v^a v^b tau_lambda with
// C_lambda = k_B x^2 n0 (n0 + 1), x = hbar w / (k_B T), and 1/tau = 1/tau3 + 1/tau4 (the
// relaxation time of Eq. tao0 without the isotope term; F = tau v, Eq. BTE under the
// relaxation-time approximation).  The paper states that its conductivity follows ShengBTE
// and does not print the expression; this is the standard kinetic form.  Modes with w <= 0
// or with a zero total rate take no part.
#include "fp4_internal.h"

#include <hip/hip_runtime.h>

namespace fp4 {
namespace {

constexpr int kKappaThreads = 256;

// a + b with the rounding error carried in c (Neumaier)
__device__ __forceinline__ void neumaier_add(double &s, double &c, double x) {
  const double t = s + x;
  c += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
  s = t;
}

// One work-group per temperature.  Thread i sums modes i, i + 256, ... in order with
// compensation; the 256 partial sums are then added in a fixed pairwise tree.  Output
// kappa [nT][9] in W/(m K); skipped [nT] active modes with a zero total rate.
__global__ __launch_bounds__(kKappaThreads) void k_kappa(const double *omega, const double4 *vel,
                                                         int nmodes, const double *T, double hk,
                                                         const double *occ, const double *r3,
                                                         const double *r4, double scale,
                                                         double kb, double *kappa,
                                                         long long *skipped) {
  __shared__ double red[9][kKappaThreads];
  __shared__ unsigned long long nsk[kKappaThreads];
  const int t = blockIdx.x, tid = threadIdx.x;
  double s[9], c[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    s[e] = 0.0;
    c[e] = 0.0;
  }
  unsigned long long sk = 0;
  const double Tt = T[t];
  for (int mu = tid; mu < nmodes; mu += kKappaThreads) {
    const double w = omega[mu];
    const double rate = r3[(size_t)t * nmodes + mu] + r4[(size_t)t * nmodes + mu];
    if (!(w > 0.0)) continue;
    if (!(rate > 0.0)) {
      ++sk;
      continue;
    }
    const double x = hk * w / Tt;
    const double n0 = occ[(size_t)t * nmodes + mu];
    const double cap = kb * x * x * n0 * (n0 + 1.0);   // J/K
    const double tau = 1e-12 / rate;                    // s
    const double4 v = vel[mu];
    const double vm[3] = {v.x * 100.0, v.y * 100.0, v.z * 100.0};   // m/s
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) neumaier_add(s[3 * a + b], c[3 * a + b], cap * vm[a] * vm[b] * tau);
  }
#pragma unroll
  for (int e = 0; e < 9; ++e) red[e][tid] = s[e] + c[e];
  nsk[tid] = sk;
  __syncthreads();
  for (int h = kKappaThreads / 2; h > 0; h >>= 1) {
    if (tid < h) {
#pragma unroll
      for (int e = 0; e < 9; ++e) red[e][tid] += red[e][tid + h];
      nsk[tid] += nsk[tid + h];
    }
    __syncthreads();
  }
  if (tid < 9) kappa[(size_t)t * 9 + tid] = red[tid][0] * scale;
  if (tid == 0 && skipped) skipped[t] = (long long)nsk[0];
}

}  // namespace

hipError_t launch_kappa(const Crystal &c, const double *T, int nT, double hk, const double *occ,
                        const double *r3, const double *r4, double scale, double kb,
                        double *kappa, long long *skipped, hipStream_t s) {
  hipLaunchKernelGGL(k_kappa, dim3(nT), dim3(kKappaThreads), 0, s, c.omega, c.vel, c.N * c.nb, T,
                     hk, occ, r3, r4, scale, kb, kappa, skipped);
  return hipGetLastError();
}

}  // namespace fp4
