// fp4_features.hip -- per-mode input features of the learned surrogate (FourPhonon paper,
// Eq. 4phgamma inputs: frequency, group velocity, branch, equilibrium occupation; the
// three-phonon rate of Eq. 3phgamma; and the mode's fourth-order coupling strength).
//
//   k_fc4_strength  g4(lambda) = sum over combos c and components of |U_c|^2, with U the
//                   slot-1 precontraction of the four-phonon path (the fourth-order force
//                   constants seen through the mode's own eigenvector and phase)
//   k_features      one row of FP4_NFEAT floats per (temperature, target), optionally
//                   standardised: x = (f - shift) * scale
#include "fp4.h"
#include "fp4_internal.h"
#include "fp4_device.h"

#include <hip/hip_runtime.h>

namespace fp4 {
namespace {

constexpr int FT_THREADS = 256;

__global__ void __launch_bounds__(FT_THREADS)
k_fc4_strength(Crystal c, const int *targets, double *g4) {
  __shared__ double red[FT_THREADS];
  const int t = blockIdx.x;
  const int mu = targets[t];
  const int iq = mu / c.nb, j = mu % c.nb;
  const double2 *e1 = c.E64 + ((size_t)iq * c.nb + j) * c.nb;
  double sum = 0.0;
  const int total = c.nc * 27;
  for (int id = threadIdx.x; id < total; id += FT_THREADS) {
    const int e = id % 27, ci = id / 27;
    double2 acc = make_double2(0.0, 0.0);
    for (int n = c.cq_start[ci]; n < c.cq_start[ci + 1]; ++n) {
      const int i = c.q_i[n];
      const double2 ph = c.PHB64[(size_t)iq * c.nbv + c.q_b[n]];
      const double *phi = c.q_phi + 81 * (size_t)n + e;
      for (int al = 0; al < 3; ++al) {
        const double2 x = cmul(e1[3 * i + al], ph);
        const double f = phi[27 * al];
        acc.x = fma(f, x.x, acc.x);
        acc.y = fma(f, x.y, acc.y);
      }
    }
    sum += acc.x * acc.x + acc.y * acc.y;
  }
  red[threadIdx.x] = sum;
  __syncthreads();
  for (int h = FT_THREADS / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) g4[t] = red[0];
}

__global__ void k_features(Crystal c, const int *targets, int nt, const double *T, int nT,
                           const double *occ, const double *r3, const double *g4,
                           const float *shift, const float *scale, float *X) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long long)nT * nt) return;
  const int t = (int)(id / nt), i = (int)(id % nt);
  const int mu = targets[i];
  const int j = mu % c.nb;
  const size_t nmodes = (size_t)c.N * c.nb;
  const double w = c.omega[mu];
  const double4 v = c.vel[mu];
  double f[FP4_NFEAT];
  f[0] = w > 0.0 ? log(w) : 0.0;
  f[1] = log(sqrt(v.x * v.x + v.y * v.y + v.z * v.z) + 1e-2);
  for (int k = 0; k < 12; ++k) f[2 + k] = k == j ? 1.0 : 0.0;
  const double n0 = occ[(size_t)t * nmodes + mu];
  f[14] = n0 > 0.0 ? log(n0) : 0.0;
  f[15] = log(r3[(size_t)t * nt + i] + 1e-8);
  f[16] = log(T[t] / 300.0);
  f[17] = log(g4[i] + 1e-30);
  float *x = X + (size_t)id * FP4_NFEAT;
  for (int k = 0; k < FP4_NFEAT; ++k) {
    float val = (float)f[k];
    if (shift) val = (val - shift[k]) * scale[k];
    x[k] = val;
  }
}

}  // namespace

hipError_t launch_fc4_strength(const Crystal &c, const int *targets, int nt, double *g4,
                               hipStream_t s) {
  if (nt <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fc4_strength, dim3((unsigned)nt), dim3(FT_THREADS), 0, s, c, targets, g4);
  return hipGetLastError();
}

hipError_t launch_features(const Crystal &c, const int *targets, int nt, const double *T, int nT,
                           const double *occ, const double *r3, const double *g4,
                           const float *shift, const float *scale, float *X, hipStream_t s) {
  const long long n = (long long)nT * nt;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_features, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, c, targets,
                     nt, T, nT, occ, r3, g4, shift, scale, X);
  return hipGetLastError();
}

}  // namespace fp4
