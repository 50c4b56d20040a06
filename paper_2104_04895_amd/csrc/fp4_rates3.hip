// fp4_rates3.hip -- three-phonon RTA rate (FourPhonon paper, Eq. tao0 three-phonon bracket,
// Eq. 3phgamma, Eq. V3), an input feature of the learned surrogate.
//
// Factorisation.  For triplet t with atoms (i, j, k) and cells (0, Rj, Rk) the phase of
// Eq. V3 of a momentum-conserving process q'' = q + s' q' is
//   exp(i s' q'.Rj) exp(-i q''.Rk) = exp(-i q.Rk) exp(i s' q'.d),  d = Rj - Rk,
// so with the slot-1 factor and exp(-i q.Rk) folded into a per-target precontraction
//   U_t[b][c] = exp(-i q.Rk) sum_a Phi_t^{abc} e^lambda_a(i)/sqrt(M_i)
// the matrix element of a branch pair is
//   V(j', j'') = sum_{B=(k,c)} conj(E''_B(j'')) Y_B(j'),
//   Y_{(k,c)}(j') = sum_{t: atom k} exp(i s' q'.d_t) sum_b U_t[b][c] X'_{(j_t,b)}(j'),
// with X' = E' (s' = +1) or conj(E') (s' = -1) and E = e/sqrt(M).
//
//   k_tables3       exp(i q.d) for every q and distinct d, stored [d][q]
//   k_precontract3  U for a batch of targets
//   k_rates3<NAT>   one work-group per target mode, one lane per q' (strided); per channel:
//                   FP64 window predicate of each branch row j' (all j''), Y for the rows
//                   with a kept process, then V, the Gaussian and the occupation factors of
//                   every kept (j', j''); per-lane sums in LDS and an ordered tree reduction,
//                   one store per target and temperature
#include "fp4_internal.h"
#include "fp4_device.h"

#include <hip/hip_runtime.h>

namespace fp4 {
namespace {

constexpr int R3_THREADS = 256;

__global__ void k_tables3(int g0, int g1, int g2, int N, const int *dvec, int nd,
                          double2 *PH3) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long long)nd * N) return;
  const int d = (int)(id / N), iq = (int)(id % N);
  const int n1 = iq % g0, n2 = (iq / g0) % g1, n3 = iq / (g0 * g1);
  const int *R = dvec + 3 * d;
  const long long k = (long long)((((long long)n1 * R[0]) % g0 + g0) % g0) * (N / g0) +
                      (long long)((((long long)n2 * R[1]) % g1 + g1) % g1) * (N / g1) +
                      (long long)((((long long)n3 * R[2]) % g2 + g2) % g2) * (N / g2);
  PH3[id] = root_of_unity(k % N, N);
}

// U[t][n][b*3 + c] for targets[t], triplet n
__global__ void k_precontract3(Crystal c, Fc3Dev f, const int *targets, int nt, double2 *U) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = (long long)nt * f.n3 * 9;
  if (id >= total) return;
  const int bc = (int)(id % 9);
  const long long tn = id / 9;
  const int n = (int)(tn % f.n3);
  const int t = (int)(tn / f.n3);
  const int mu = targets[t];
  const int iq = mu / c.nb, j = mu % c.nb;
  const double2 *e1 = c.E64 + ((size_t)iq * c.nb + j) * c.nb + 3 * f.t_i[n];
  const double *ph = f.t_phi + (size_t)27 * n;
  double2 acc = make_double2(0.0, 0.0);
  for (int a = 0; a < 3; ++a) {
    const double p = ph[a * 9 + bc];
    acc.x = fma(p, e1[a].x, acc.x);
    acc.y = fma(p, e1[a].y, acc.y);
  }
  // exp(-i q.Rk) from the grid triple of q and the integer cell Rk
  const int4 qn = c.qn[iq];
  const int *R = f.rk_vec + 3 * f.t_rk[n];
  const long long k = (long long)((((long long)qn.x * R[0]) % c.g0 + c.g0) % c.g0) * (c.N / c.g0) +
                      (long long)((((long long)qn.y * R[1]) % c.g1 + c.g1) % c.g1) * (c.N / c.g1) +
                      (long long)((((long long)qn.z * R[2]) % c.g2 + c.g2) % c.g2) * (c.N / c.g2);
  const double2 e = cconj(root_of_unity(k % c.N, c.N));
  U[id] = cmul(acc, e);
}

template <int NAT>
__global__ void __launch_bounds__(R3_THREADS)
k_rates3(Crystal c, Fc3Dev f, Rate3Args a, const double2 *__restrict__ U) {
  constexpr int NB = 3 * NAT;
  extern __shared__ double lds3[];
  double *acc = lds3;                                              // [nT][256]
  unsigned long long *cnt = (unsigned long long *)(lds3 + a.nT * R3_THREADS);  // [2][256]
  const int tid = threadIdx.x;
  const int it = a.t0 + (int)blockIdx.x;   // index of the target in the output
  const int mu = a.targets[it];
  const int iq = mu / NB;
  const double w = c.omega[mu];
  for (int t = 0; t < a.nT; ++t) acc[t * R3_THREADS + tid] = 0.0;
  unsigned long long n_plus = 0ull, n_minus = 0ull;
  const double2 *Ut = U + (size_t)blockIdx.x * f.n3 * 9;
  if (w > 0.0) {
    const int4 qn = c.qn[iq];
    const double iw = c.inv_omega[mu];
    for (int iq1 = tid; iq1 < c.N; iq1 += R3_THREADS) {
      const int4 qn1 = c.qn[iq1];
#pragma unroll 1
      for (int ch = 0; ch < 2; ++ch) {
        const int s = ch == 0 ? 1 : -1;
        const int iq2 = wrap(qn.x + s * qn1.x, c.g0) +
                        c.g0 * (wrap(qn.y + s * qn1.y, c.g1) + c.g1 * wrap(qn.z + s * qn1.z, c.g2));
#pragma unroll 1
        for (int j1 = 0; j1 < NB; ++j1) {
          const int mu1 = iq1 * NB + j1;
          const double4 m1 = c.mode4[mu1];
          if (!(m1.w > 0.0)) continue;
          const double bw = add_signed(w, m1.w, s);
          unsigned row = 0u;
          for (int j2 = 0; j2 < NB; ++j2) {
            const double4 m2 = c.mode4[iq2 * NB + j2];
            double dw, s2;
            if (m2.w > 0.0 && window_keep(bw, m2.w, m1, m2, a.c_win, dw, s2)) row |= 1u << j2;
          }
          if (!row) continue;
          // slot-2 factor of row j'
          double2 X[NB];
          const double2 *e2 = c.E64 + (size_t)mu1 * NB;
#pragma unroll
          for (int A = 0; A < NB; ++A) X[A] = s > 0 ? e2[A] : cconj(e2[A]);
          double2 Y[NB];
#pragma unroll
          for (int B = 0; B < NB; ++B) Y[B] = make_double2(0.0, 0.0);
#pragma unroll
          for (int ja = 0; ja < NAT; ++ja)
#pragma unroll
            for (int ka = 0; ka < NAT; ++ka) {
              const int t0 = f.jk_start[ja * NAT + ka], t1 = f.jk_start[ja * NAT + ka + 1];
#pragma unroll 1
              for (int t = t0; t < t1; ++t) {
                double2 ph = f.PH3[(size_t)f.t_d[t] * c.N + iq1];
                if (s < 0) ph = cconj(ph);
                const double2 *u = Ut + (size_t)t * 9;
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) {
                  double2 z = make_double2(0.0, 0.0);
#pragma unroll
                  for (int b = 0; b < 3; ++b) cmac(z, u[b * 3 + cc], X[ja * 3 + b]);
                  cmac(Y[ka * 3 + cc], ph, z);
                }
              }
            }
          const double iw1 = c.inv_omega[mu1];
          while (row) {
            const int j2 = __builtin_ctz(row);
            row &= row - 1u;
            const int mu2 = iq2 * NB + j2;
            const double4 m2 = c.mode4[mu2];
            double dw, s2;
            window_keep(bw, m2.w, m1, m2, a.c_win, dw, s2);
            const double2 *e3 = c.E64 + (size_t)mu2 * NB;
            double2 V = make_double2(0.0, 0.0);
#pragma unroll
            for (int B = 0; B < NB; ++B) cmac_cb(V, Y[B], e3[B]);
            const double v2 = V.x * V.x + V.y * V.y;
            const double sig2 = a.c_sig * s2;
            double delta = 1.0;
            if (!(sig2 < a.c_min)) {
              const double is2 = 1.0 / sig2;
              delta = exp(-(dw * dw) * is2) * (0.5641895835477563 * sqrt(is2));
            }
            const double base = a.kpref * iw * iw1 * c.inv_omega[mu2] * v2 * delta;
            n_plus += ch == 0;
            n_minus += ch != 0;
            for (int t = 0; t < a.nT; ++t) {
              const double *n0 = a.occ + (size_t)t * c.N * NB;
              const double fo = ch == 0 ? n0[mu1] - n0[mu2] : 0.5 * (n0[mu1] + n0[mu2] + 1.0);
              acc[t * R3_THREADS + tid] += base * fo;
            }
          }
        }
      }
    }
  }
  cnt[tid] = n_plus;
  cnt[R3_THREADS + tid] = n_minus;
  __syncthreads();
  for (int h = R3_THREADS / 2; h > 0; h >>= 1) {
    if (tid < h) {
      for (int t = 0; t < a.nT; ++t) acc[t * R3_THREADS + tid] += acc[t * R3_THREADS + tid + h];
      cnt[tid] += cnt[tid + h];
      cnt[R3_THREADS + tid] += cnt[R3_THREADS + tid + h];
    }
    __syncthreads();
  }
  if (tid < a.nT) a.rates[(size_t)tid * a.nt_total + it] = acc[tid * R3_THREADS];
  if (tid < 2 && a.counts) a.counts[2 * (size_t)it + tid] = (long long)cnt[tid * R3_THREADS];
}

}  // namespace

hipError_t launch_tables3(const Crystal &c, const int *dvec, int nd, double2 *PH3, hipStream_t s) {
  const long long n = (long long)nd * c.N;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tables3, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, c.g0, c.g1,
                     c.g2, c.N, dvec, nd, PH3);
  return hipGetLastError();
}

hipError_t launch_precontract3(const Crystal &c, const Fc3Dev &f, const int *targets, int nt,
                               double2 *U, hipStream_t s) {
  const long long n = (long long)nt * f.n3 * 9;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_precontract3, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, c, f,
                     targets, nt, U);
  return hipGetLastError();
}

size_t rates3_lds_bytes(int nT) { return (size_t)R3_THREADS * (nT * sizeof(double) + 2 * sizeof(unsigned long long)); }

hipError_t launch_rates3(const Crystal &c, const Fc3Dev &f, const Rate3Args &a,
                         const double2 *U, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  const size_t lds = rates3_lds_bytes(a.nT);
  const dim3 grid((unsigned)nblocks), block(R3_THREADS);
  switch (c.nat) {
    case 1: hipLaunchKernelGGL(k_rates3<1>, grid, block, lds, s, c, f, a, U); break;
    case 2: hipLaunchKernelGGL(k_rates3<2>, grid, block, lds, s, c, f, a, U); break;
    case 3: hipLaunchKernelGGL(k_rates3<3>, grid, block, lds, s, c, f, a, U); break;
    case 4: hipLaunchKernelGGL(k_rates3<4>, grid, block, lds, s, c, f, a, U); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace fp4
