// fp4_kernels.hip -- CDNA4 (gfx950) kernels of the four-phonon RTA rate.
//
// Hot path (FourPhonon paper, Eq. tao0, Eq. 4phgamma, Eq. V4, Sec. 2.4):
//   k_tables       per-q tables: E = e/sqrt(M), grid triples, lattice phase tables
//   k_occupations  n0 and 1/n0 for every mode and temperature
//   k_precontract  per target mode lambda: U_c = sum over the quartets of combo c of
//                  Phi contracted with the slot-1 factor e^lambda(i) exp(i q.b)
//   k_rates        per (lambda, block of q'): W'' for each lambda' (slot-2 contraction,
//                  grouped by slot-3/slot-4 atoms and relative cell), then for every q'' and
//                  channel: FP64 energy-window prefilter of the nb x nb branch block, and for
//                  blocks with a surviving process the branch-block contraction
//                  V = E3 F E4^T with F = sum_d exp(i s'' q''.d) W''_d, followed by the
//                  Gaussian, occupation factors and per-lane FP64 accumulation
//   k_reduce       ordered sum of the per-work-group partial rates
#include <type_traits>

#include "fp4_internal.h"
#include "fp4_device.h"

#include <hip/hip_runtime.h>

#include <mutex>

namespace fp4 {
namespace {

template <typename R> __device__ __forceinline__ const typename CT<R>::T *Etab(const Crystal &c);
template <> __device__ __forceinline__ const double2 *Etab<double>(const Crystal &c) { return c.E64; }
template <> __device__ __forceinline__ const float2 *Etab<float>(const Crystal &c) { return c.E32; }
template <typename R> __device__ __forceinline__ const typename CT<R>::T *PHDtab(const Crystal &c);
template <> __device__ __forceinline__ const double2 *PHDtab<double>(const Crystal &c) { return c.PHD64; }
template <> __device__ __forceinline__ const float2 *PHDtab<float>(const Crystal &c) { return c.PHD32; }

// Keep a complex value in registers at this point of the instruction stream: the arithmetic
// that produces it cannot sink below, and (with the memory clobber) later loads cannot be
// hoisted above.  Used to bound the number of LDS rows in flight in the branch-block products.
__device__ __forceinline__ void pin(double2 &v) { __asm__ volatile("" : "+v"(v.x), "+v"(v.y)::"memory"); }
__device__ __forceinline__ void pin(float2 &v) { __asm__ volatile("" : "+v"(v.x), "+v"(v.y)::"memory"); }

// q = x / g, r = x % g for 0 <= x < 2^24 and 1 <= g: a single-precision estimate of the
// quotient (off by at most one since x is exact in FP32) corrected by one integer step.
__device__ __forceinline__ void divmod_small(int x, int g, float inv_g, int &q, int &r) {
  q = (int)((float)x * inv_g);
  r = x - q * g;
  if (r < 0) {
    q -= 1;
    r += g;
  } else if (r >= g) {
    q += 1;
    r -= g;
  }
}

// A value that is the same in every lane (work-group constants such as the frequencies of
// lambda and lambda'), moved to scalar registers so it takes no vector register
__device__ __forceinline__ double uniform_d(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Elements per group tile: an NB x NB block of V, H, F or E4 rows, or the NB column records
// (4 doubles each) of the window test, whichever is larger.  FP64 tiles are padded by one
// element, which spreads the tiles of a wavefront's lane groups over more LDS banks
// (measured 0.7% faster; with FP32 tiles the same padding measured 11% slower).
__host__ __device__ constexpr int xtile(int nb, int cbytes) {
  return (nb * nb * cbytes >= 32 * nb ? nb * nb : (32 * nb) / cbytes) + (cbytes == 16 ? 1 : 0);
}

// LDS stride of a group of W'' (nine entries, padded to ten): the lanes of the two atom rows
// of a lane group read different groups at once, and the padding moves their reads onto
// different banks (measured 0.4% faster in FP64, 1.2% in FP32).
constexpr int WSTR = 10;

// ------------------------------------------------------------------ table kernels

__global__ void k_tables(Crystal c, double4 *qbound, double4 *mode4, double *speed, double *inv_omega, double2 *E64, float2 *E32,
                         const double *evec, const double *mass, int4 *qn, double2 *PHA64, double2 *PHB64,
                         double2 *PHD64, float2 *PHD32, const int *avec, const int *bvec,
                         const int *dvec) {
  const int iq = blockIdx.x * blockDim.x + threadIdx.x;
  if (iq >= c.N) return;
  const int n1 = iq % c.g0, n2 = (iq / c.g0) % c.g1, n3 = iq / (c.g0 * c.g1);
  qn[iq] = make_int4(n1, n2, n3, 0);
  const int nb = c.nb;
  for (int j = 0; j < nb; ++j) {
    const double w = c.omega[(size_t)iq * nb + j];
    inv_omega[(size_t)iq * nb + j] = w > 0.0 ? 1.0 / w : 0.0;
    const double4 v = c.vel[(size_t)iq * nb + j];
    mode4[(size_t)iq * nb + j] = make_double4(v.x, v.y, v.z, w);
    speed[(size_t)iq * nb + j] = sqrt(v.x * v.x + v.y * v.y + v.z * v.z);
  }
  // frequency range and largest speed of the active branches at this q (an empty range,
  // w_min > w_max, when no branch is active)
  {
    double wmin = 1e300, wmax = -1e300, vmax = 0.0;
    for (int j = 0; j < nb; ++j) {
      const double w = c.omega[(size_t)iq * nb + j];
      if (!(w > 0.0)) continue;
      const double4 v = c.vel[(size_t)iq * nb + j];
      wmin = fmin(wmin, w);
      wmax = fmax(wmax, w);
      vmax = fmax(vmax, sqrt(v.x * v.x + v.y * v.y + v.z * v.z));
    }
    qbound[iq] = make_double4(wmin, wmax, vmax, 0.0);
  }
  for (int j = 0; j < nb; ++j)
    for (int col = 0; col < nb; ++col) {
      const size_t o = ((size_t)iq * nb + j) * nb + col;
      const double sm = 1.0 / sqrt(mass[col / 3]);
      const double2 e = make_double2(evec[2 * o] * sm, evec[2 * o + 1] * sm);
      E64[o] = e;
      E32[o] = to32(e);
    }
  auto phase = [&](const int *R) {
    const long long k = (long long)(((long long)n1 * R[0]) % c.g0 + c.g0) % c.g0 * (c.N / c.g0) +
                        (long long)(((long long)n2 * R[1]) % c.g1 + c.g1) % c.g1 * (c.N / c.g1) +
                        (long long)(((long long)n3 * R[2]) % c.g2 + c.g2) % c.g2 * (c.N / c.g2);
    return root_of_unity(k % c.N, c.N);
  };
  for (int i = 0; i < c.na; ++i) PHA64[(size_t)iq * c.na + i] = phase(avec + 3 * i);
  for (int i = 0; i < c.nbv; ++i) PHB64[(size_t)iq * c.nbv + i] = phase(bvec + 3 * i);
  for (int i = 0; i < c.nd; ++i) {
    const double2 p = phase(dvec + 3 * i);
    PHD64[(size_t)iq * c.nd + i] = p;
    PHD32[(size_t)iq * c.nd + i] = to32(p);
  }
}

// temperatures passed by value
struct TempList {
  double T[8];
};

// n0 = 1/expm1(hbar w / k T) (after Eq. 4phgamma); 1/n0 = expm1(.)  (0 for inactive modes)
__global__ void k_occupations_v(const double *omega, int nmodes, TempList T, int nT, double hk,
                                double *occ, double *inv_occ) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nmodes * nT) return;
  const int t = i / nmodes, m = i % nmodes;
  const double w = omega[m];
  double Tt = T.T[0];
#pragma unroll
  for (int k = 1; k < 8; ++k)
    if (k == t) Tt = T.T[k];
  if (w > 0.0) {
    const double em = expm1(hk * w / Tt);
    occ[i] = 1.0 / em;
    inv_occ[i] = em;
  } else {
    occ[i] = 0.0;
    inv_occ[i] = 0.0;
  }
}

__global__ void k_occupations(const double *omega, int nmodes, const double *T, int nT,
                              double hk, double *occ, double *inv_occ) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nmodes * nT) return;
  const int t = i / nmodes, m = i % nmodes;
  const double w = omega[m];
  if (w > 0.0) {
    const double em = expm1(hk * w / T[t]);
    occ[i] = 1.0 / em;
    inv_occ[i] = em;
  } else {
    occ[i] = 0.0;
    inv_occ[i] = 0.0;
  }
}

// U[t][c][beta*9 + gamma*3 + theta] = sum_{n in combo c} sum_alpha Phi_n^{abgt}
//                                     e^{lambda_t}_alpha(i_n)/sqrt(M) exp(i q.b_n)
template <typename CR>
__global__ void k_precontract(Crystal c, const int *targets, int tbase, int nt, CR *U) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = (long long)nt * c.nc * 27;
  if (id >= total) return;
  const int e = (int)(id % 27);
  const long long tc = id / 27;
  const int ci = (int)(tc % c.nc);
  const int t = (int)(tc / c.nc);
  const int mu = targets ? targets[t] : tbase + t;
  const int iq = mu / c.nb, j = mu % c.nb;
  const double2 *e1 = c.E64 + ((size_t)iq * c.nb + j) * c.nb;
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
  U[id] = fromd<CR>(acc);
}

// ------------------------------------------------------------------ W'' build

// W[s][g][gamma*3 + theta] (WSTR elements per g), s = 0 for s' = + and 1 for s' = -:
//   sum over combos c of g, beta: U_c[beta][gt] (E[q'][j'][3 j_c + beta] exp(i q'.a_c))^(s')
// The slot-2 factors p[c][beta] = E[q'][j'][3 j_c + beta] exp(i q'.a_c), shared by the nine
// entries of a group, are formed once into `stage` (LDS, free while W is built) when it holds
// them, so the entry loop reads only U from memory.
template <typename R>
__device__ void build_W(const Crystal &c, const typename CT<R>::T *Ut, int iq1, int j1,
                        typename CT<R>::T *W, typename CT<R>::T *stage, int stage_cap, int tid,
                        int nthr) {
  using CR = typename CT<R>::T;
  const CR *e2 = Etab<R>(c) + ((size_t)iq1 * c.nb + j1) * c.nb;
  const int tot = c.ng * 9;
  if (3 * c.nc <= stage_cap) {
    for (int i = tid; i < 3 * c.nc; i += nthr) {
      const int ci = i / 3, be = i - 3 * ci;
      const CR ph = fromd<CR>(c.PHA64[(size_t)iq1 * c.na + c.c_a[ci]]);
      stage[i] = cmul(e2[3 * c.c_jat[ci] + be], ph);
    }
    __syncthreads();
    for (int idx = tid; idx < tot; idx += nthr) {
      const int g = idx / 9, gt = idx - 9 * g;
      CR ap = czero<CR>(), am = czero<CR>();
      for (int ci = c.c_start[g]; ci < c.c_start[g + 1]; ++ci) {
        const CR *u = Ut + (size_t)ci * 27 + gt;
#pragma unroll
        for (int be = 0; be < 3; ++be) {
          const CR p = stage[3 * ci + be];
          const CR uu = u[9 * be];
          cmac(ap, uu, p);
          cmac_cb(am, uu, p);
        }
      }
      W[g * WSTR + gt] = ap;
      W[c.ng * WSTR + g * WSTR + gt] = am;
    }
    return;
  }
  for (int idx = tid; idx < tot; idx += nthr) {
    const int g = idx / 9, gt = idx - 9 * g;
    CR ap = czero<CR>(), am = czero<CR>();
    for (int ci = c.c_start[g]; ci < c.c_start[g + 1]; ++ci) {
      const int jat = c.c_jat[ci];
      const CR ph = fromd<CR>(c.PHA64[(size_t)iq1 * c.na + c.c_a[ci]]);
      const CR *u = Ut + (size_t)ci * 27 + gt;
#pragma unroll
      for (int be = 0; be < 3; ++be) {
        const CR p = cmul(e2[3 * jat + be], ph);
        const CR uu = u[9 * be];
        cmac(ap, uu, p);
        cmac_cb(am, uu, p);
      }
    }
    W[g * WSTR + gt] = ap;
    W[c.ng * WSTR + g * WSTR + gt] = am;
  }
}

// ------------------------------------------------------------------ branch block

// With the FP64 contraction the rate kernel leaves H = E3 F in the group tile and forms
// V[r][cc] = H[r][:] . conj(E4[cc][:]) only for the kept entries, in the Gamma list (a
// third of the 36 per block); with the FP32 contraction the dense V = H E4^T measured
// faster.
template <typename R> constexpr bool VLIST = sizeof(R) == 8;

// Row r (= j'') of V[j''][j'''] for the block (lambda, lambda', q'', channel with sign S2):
//   F[(k,gamma)][(l,theta)] = sum_{d of (k,l)} exp(i s'' q''.d) W[(k,l,d)][gamma theta]
//   V = E3 F E4^T,  E3[j''][(k,gamma)] = (E[q''][j''][3k+gamma])^(s''),
//                   E4[j'''][(l,theta)] = conj(E[q'''][j'''][3l+theta])
// The nb lanes of a group hold one row each and exchange F rows and E4 rows through the
// group's LDS tile Xg[nb][nb] (all lanes of a group belong to one wavefront).
template <typename R, int NB, bool HONLY = false>
__device__ __forceinline__ void block_row(const Crystal &c, const typename CT<R>::T *Ws, int S2,
                                          int iq2, int iq3, int r,
                                          typename CT<R>::T *Xg, typename CT<R>::T *Pg,
                                          const int *sg_d, const int *skl,
                                          typename CT<R>::T (&V)[NB]) {
  using CR = typename CT<R>::T;
  constexpr int NAT = NB / 3;
  const int k = r / 3, gam = r - 3 * k;
  // the row of E3 is fetched first, so that its latency overlaps the phase staging and F
  const CR *e3 = Etab<R>(c) + ((size_t)iq2 * NB + r) * NB;
  CR e3v[NB];
#pragma unroll
  for (int kg = 0; kg < NB; ++kg) e3v[kg] = e3[kg];
  // stage exp(i s'' q''.d) of every distinct d in the group's phase tile
  {
    const CR *phd = PHDtab<R>(c) + (size_t)iq2 * c.nd;
    for (int i = r; i < c.nd; i += NB) {
      CR ph = phd[i];
      if (S2 < 0) ph = cconj(ph);
      Pg[i] = ph;
    }
  }
  wave_sync();
  // F row r, accumulated in the atom order l = k, k+1, ... (mod NAT) so that the
  // register index is static
  CR Frel[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) Frel[i] = czero<CR>();
#pragma unroll
  for (int rl = 0; rl < NAT; ++rl) {
    const int l = (k + rl) % NAT;
    const int gb = skl[k * NAT + l], ge = skl[k * NAT + l + 1];
#pragma unroll 2
    for (int g = gb; g < ge; ++g) {
      const CR ph = Pg[sg_d[g]];
      const CR *wg = Ws + g * WSTR + gam * 3;
#pragma unroll
      for (int th = 0; th < 3; ++th) cmac(Frel[rl * 3 + th], ph, wg[th]);
    }
  }
#pragma unroll
  for (int l = 0; l < NAT; ++l) {
    const int rl = (l - k + NAT) % NAT;
#pragma unroll
    for (int th = 0; th < 3; ++th) {
      CR f = Frel[th];
#pragma unroll
      for (int rr = 1; rr < NAT; ++rr)
        if (rr == rl) f = Frel[rr * 3 + th];
      Xg[r * NB + l * 3 + th] = f;
    }
  }
  wave_sync();
  // the row of E4 (lane r: conj(E[q'''][r][:])) is fetched before H = E3[r][:] F when the
  // registers allow it (FP32)
  const CR *e4 = Etab<R>(c) + ((size_t)iq3 * NB + r) * NB;
  constexpr bool PRE4 = sizeof(R) == 4 && !HONLY;
  CR e4v[NB];
  if (PRE4) {
#pragma unroll
    for (int col = 0; col < NB; ++col) e4v[col] = e4[col];
  }
  CR H[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) H[i] = czero<CR>();
#pragma unroll
  for (int kg = 0; kg < NB; ++kg) {
    CR e = e3v[kg];
    if (S2 < 0) e = cconj(e);
#pragma unroll
    for (int col = 0; col < NB; ++col) cmac(H[col], e, Xg[kg * NB + col]);
#pragma unroll
    for (int col = 0; col < NB; ++col) pin(H[col]);
  }
  wave_sync();
  if constexpr (HONLY) {
    // the rate kernel forms V[r][cc] = H[r][:] . conj(E4[cc][:]) only for the kept
    // entries, in the Gamma list: lane r leaves its row of H in the tile
#pragma unroll
    for (int col = 0; col < NB; ++col) Xg[r * NB + col] = H[col];
    return;
  }
#pragma unroll
  for (int col = 0; col < NB; ++col) Xg[r * NB + col] = cconj(PRE4 ? e4v[col] : e4[col]);
  wave_sync();
#pragma unroll
  for (int cc = 0; cc < NB; ++cc) {
    CR v = czero<CR>();
#pragma unroll
    for (int col = 0; col < NB; ++col) cmac(v, H[col], Xg[cc * NB + col]);
    pin(v);
    V[cc] = v;
  }
  wave_sync();
}

// ------------------------------------------------------------------ rate kernel

template <int NT>
struct Acc {
  double r[3][NT];
  unsigned cnt[3];
  unsigned blocks;
};

// Window-prefilter bits of one row of a branch block.  Lane r owns row mode mu_r = (q'', r)
// with record vr; column cc is (q''', cc), whose (v, w) records the lanes of the group share
// through LDS (cs: record cc as the double2 pair cs[2cc], cs[2cc+1]).  b0 tests the processes
// (lambda'' = row, lambda''' = column), b1 (mirror rows of the redistribution channel only)
// the mirrored ones (lambda'' = column, lambda''' = row).  Each candidate is evaluated in the
// same FP64 order as a stand-alone process.
//
// A row is skipped without testing its candidates when no candidate can pass: dw of the row
// lies in x - [w_min, w_max] of q''' (qb = (w_min, w_max, v_max, 0) over its active
// branches) and a kept process needs |dw| <= sqrt(c_win) |v'' - v'''| <= sqrt(c_win)
// (|v_row| + v_max(q''')); the bound is applied with a relative margin of 1e-6, far above
// FP64 rounding, so it never drops a process the exact test would keep.
//
// The two orientations of a mirror row share s2: d = v'' - v''' of one is the negative of the
// other's, so their squares and s2 = (dx*dx + dy*dy) + dz*dz are bitwise equal, and only dw
// is formed twice, each in its own stand-alone order.
template <int NB>
__device__ __forceinline__ void row_bits_cols(const RateArgs &a, double aw, int S2, const double4 vr,
                                              double speed, const double4 qb, const double2 *cs,
                                              bool mirror_row, unsigned &b0, unsigned &b1) {
#pragma clang fp contract(off)
  b0 = 0u;
  b1 = 0u;
  if (!(vr.w > 0.0)) return;
  const double lim = a.sqrt_c_win * (speed + qb.z) * (1.0 + 1e-6) + 1e-12;
  auto dist = [&](double x) {
    const double lo = x - qb.y, hi = x - qb.x;
    return lo > 0.0 ? lo : (hi < 0.0 ? -hi : 0.0);
  };
  const bool t0 = !(dist(add_signed(aw, vr.w, S2)) > lim);
  const bool t1 = mirror_row && !(dist(aw - vr.w) > lim);
  if (!t0 && !t1) return;
  const double bw = add_signed(aw, vr.w, S2);
#pragma unroll
  for (int cc = 0; cc < NB; ++cc) {
    const double2 p0 = cs[2 * cc], p1 = cs[2 * cc + 1];
    const double4 vc = make_double4(p0.x, p0.y, p1.x, p1.y);
    if (vc.w > 0.0) {
      const double dx = vr.x - vc.x, dy = vr.y - vc.y, dz = vr.z - vc.z;
      const double lim2 = a.c_win * ((dx * dx + dy * dy) + dz * dz);
      if (t0) {
        const double dw = bw - vc.w;
        if (dw * dw <= lim2) b0 |= 1u << cc;
      }
      if (t1) {
        const double dw = add_signed(aw, vc.w, S2) - vr.w;
        if (dw * dw <= lim2) b1 |= 1u << cc;
      }
    }
  }
}

// What Gamma needs of a mode besides V: (v, w), 1/w and n0 at each temperature.
template <int NT>
struct ModeRec {
  double4 m;
  double iw;
  double n[NT];
};

template <int NB, int NT>
__device__ __forceinline__ ModeRec<NT> load_rec(const Crystal &c, const RateArgs &a, int mu) {
  ModeRec<NT> r;
  r.m = c.mode4[mu];
  r.iw = c.inv_omega[mu];
#pragma unroll
  for (int t = 0; t < NT; ++t) r.n[t] = (t < a.nT) ? a.occ[(size_t)t * c.N * NB + mu] : 0.0;
  return r;
}

// Gamma (Eq. 4phgamma) of a compacted list of kept processes of the wavefront's blocks,
// accumulated into the lane's FP64 partial rates.  Entry i of L is (s << 6) | b for source
// lane s = (group g, row r) and code b: b < NB is the process (lambda'' = (q''_g, r),
// lambda''' = (q'''_g, b)), NB <= b < 2 NB the mirrored one (lambda'' = (q'''_g, b - NB),
// lambda''' = (q''_g, r)), b >= 2 NB both of column b - 2 NB (redistribution or splitting
// channel, both kept).  The two members of a mirror pair share |V| (V transposed), |v'' - v'''| and so
// sigma, 1/(w'' w''') and the occupation factor; one evaluation serves both, each with its
// own dw formed in its stand-alone order and its own Gaussian.  V comes from the group's
// tile (dense V, or H and a row of E4, see VLIST), (q''_g, q'''_g) from Gq (bit 30 of
// q'''_g: the block's processes are Umklapp ones).  Consecutive lanes take consecutive
// entries, so every lane has work while the list lasts.
// With a.qclass == 3 the sums go by class instead of by channel: normal processes to
// acc.r[0], Umklapp ones to acc.r[1].
// exp(-x) for x >= 0 (in the Gaussian x <= window_w^2, a few units): x = k ln2 - t with
// k = rint(x / ln2) and |t| <= ln2 / 2, reduced in two steps after Cody and Waite with ln2
// split into a 40-bit head (k ln2_hi exact for |k| < 2^13) and the rest; exp(t) by its
// Taylor series to t^12 (truncation below 2e-16 relative for |t| <= ln2 / 2, Horner in
// FP64), scaled by 2^-k.  x is capped at 800, where exp(-x) is 0 in FP64 already.
__device__ __forceinline__ double exp_neg(double x) {
  x = fmin(x, 800.0);
  const double k = rint(x * 1.4426950408889634);
  double t = fma(k, 0.6931471805592082, -x);
  t = fma(k, 7.371002565167799e-13, t);
  double p = 2.08767569878681e-09;           // 1/12!
  p = fma(p, t, 2.505210838544172e-08);      // 1/11!
  p = fma(p, t, 2.755731922398589e-07);      // 1/10!
  p = fma(p, t, 2.7557319223985893e-06);     // 1/9!
  p = fma(p, t, 2.48015873015873e-05);       // 1/8!
  p = fma(p, t, 0.0001984126984126984);      // 1/7!
  p = fma(p, t, 0.001388888888888889);       // 1/6!
  p = fma(p, t, 0.008333333333333333);       // 1/5!
  p = fma(p, t, 0.041666666666666664);       // 1/4!
  p = fma(p, t, 0.16666666666666666);        // 1/3!
  p = fma(p, t, 0.5);
  p = fma(p, t, 1.0);
  p = fma(p, t, 1.0);
  return ldexp(p, -(int)k);
}

// The pair (lambda, lambda'): grid digits of q and q', the two modes and their frequencies.
struct PairIn {
  int4 nq, nq1;
  int mu, mu1;
  double w, w1;
};

// Per-pair constants of the channels, index 0 for s' = + (++ and +-), 1 for s' = - (--):
// aw = w s' w', and kw = the channel weight of Eq. tao0 (1/2 for ++ and +-, 1/6 for --)
// times the prefactor C4/N^2 and 1/(w w') of Eq. 4phgamma (the phase space P4 keeps only the
// channel weight and 1/N^2).
struct ChanK {
  double aw[2];
  double kw[2];
  __device__ __forceinline__ ChanK(const Crystal &c, const RateArgs &a, const PairIn &pi) {
    aw[0] = add_signed(pi.w, pi.w1, 1);
    aw[1] = add_signed(pi.w, pi.w1, -1);
    if (a.harmonic == 2) {
      kw[0] = 0.5 * a.kpref;
      kw[1] = (1.0 / 6.0) * a.kpref;
    } else {
      kw[0] = 0.5 * a.kpref * c.inv_omega[pi.mu] * c.inv_omega[pi.mu1];
      kw[1] = (1.0 / 6.0) * a.kpref * c.inv_omega[pi.mu] * c.inv_omega[pi.mu1];
    }
  }
};

// Gamma (Eq. 4phgamma) of a compacted list of kept processes of the wavefront's blocks,
// accumulated into the lane's FP64 partial rates.  Entry i of L is (s << 6) | b for source
// lane s = (group g, row r) and code b: b < NB is the process (lambda'' = (q''_g, r),
// lambda''' = (q'''_g, b)), NB <= b < 2 NB the mirrored one (lambda'' = (q'''_g, b - NB),
// lambda''' = (q''_g, r)), b >= 2 NB both of column b - 2 NB (redistribution or splitting
// channel, both kept).  The two members of a mirror pair share |V| (V transposed), |v'' - v'''| and so
// sigma, 1/(w'' w''') and the occupation factor; one evaluation serves both, each with its
// own dw formed in its stand-alone order and its own Gaussian.  V comes from the group's
// tile (dense V, or H and a row of E4, see VLIST), (q''_g, q'''_g) from Gq (bit 30 of
// q'''_g: the block's processes are Umklapp ones; with CH = 3, bit 29: the block is a --
// one, else a ++ one).  CH = 1 is the redistribution channel; CH = 3 a list whose blocks
// belong to ++ or to --.  Consecutive lanes take consecutive entries, so every lane has work
// while the list lasts.  With a.qclass == 3 the sums go by class instead of by channel:
// normal processes to acc.r[0], Umklapp ones to acc.r[1].
template <typename R, int NB, int NT, int CH>
__device__ __forceinline__ void gamma_list(const Crystal &c, const RateArgs &a,
                                           const unsigned short *L, int cnt, int lane,
                                           const typename CT<R>::T *Xw, const int2 *Gq,
                                           const ChanK &ck, const double (&invn)[NT],
                                           const double (&n1)[NT], Acc<NT> &acc) {
  using CR = typename CT<R>::T;
  static_assert(CH == 1 || CH == 3, "redistribution, or a list of ++ and -- blocks");
  auto decode = [&](int i, int &mu2, int &mu3, int &vi, int &cc, int &m4, bool &pair, bool &umk,
                    bool &neg) {
    const unsigned d = L[i];
    const int s = (int)(d >> 6), b = (int)(d & 63u);
    const int g = s / NB, r = s - g * NB;
    const int2 q = Gq[g];
    umk = ((q.y >> 30) & 1) != 0;
    neg = CH == 3 && ((q.y >> 29) & 1) != 0;
    const bool mir = b >= NB && b < 2 * NB;
    pair = b >= 2 * NB;
    cc = pair ? b - 2 * NB : (mir ? b - NB : b);
    const int mr = q.x * NB + r, mc = (q.y & 0x1fffffff) * NB + cc;
    mu2 = mir ? mc : mr;
    mu3 = mir ? mr : mc;
    vi = g * xtile(NB, sizeof(CR)) + r * NB;
    m4 = mc;
  };
#pragma unroll 1
  for (int i = lane; i < cnt; i += 64) {
    int mu2, mu3, vi, cc, m4;
    bool pair, umk, neg;
    decode(i, mu2, mu3, vi, cc, m4, pair, umk, neg);
    // s'' = - for +- and --, + for ++; the channel index of the sums
    const int S2 = (CH == 1 || neg) ? -1 : 1;
    const int chi = CH == 1 ? 1 : (neg ? 2 : 0);
    const double aw = neg ? ck.aw[1] : ck.aw[0];
    const double kw = neg ? ck.kw[1] : ck.kw[0];
    const bool split = a.qclass == 3;
    const ModeRec<NT> p2 = load_rec<NB, NT>(c, a, mu2), p3 = load_rec<NB, NT>(c, a, mu3);
    double dw, s2, dwm = 0.0;
    window_keep(add_signed(aw, p2.m.w, S2), p3.m.w, p2.m, p3.m, a.c_win, dw, s2);
    if (pair) {
      // the mirrored member (lambda'' and lambda''' exchanged); its s2 equals s2 exactly
      double s2m;
      window_keep(add_signed(aw, p3.m.w, S2), p2.m.w, p3.m, p2.m, a.c_win, dwm, s2m);
    }
    double v2abs = 1.0;
    if (a.harmonic == 0) {
      CR vv;
      if constexpr (VLIST<R>) {
        // V[r][cc] = H[r][:] . conj(E4[cc][:]) (the same products in the same order as the
        // dense V = H E4^T), H from the group's tile, the row of E4 (q''', cc) from the table
        const CR *e4 = Etab<R>(c) + (size_t)m4 * NB;
        vv = czero<CR>();
#pragma unroll
        for (int col = 0; col < NB; ++col) cmac(vv, Xw[vi + col], cconj(e4[col]));
      } else {
        vv = Xw[vi + cc];
      }
      v2abs = (double)vv.x * (double)vv.x + (double)vv.y * (double)vv.y;
    }
    const double sig2 = a.c_sig * s2;
    double delta = pair ? 2.0 : 1.0;
    if (!(sig2 < a.c_min)) {
      // adaptive Gaussian exp(-dw^2/sigma^2) / (sqrt(pi) sigma), 1/sqrt(pi) =
      // 0.5641895835477563; y = 1/sigma from the hardware reciprocal square root refined
      // by two Newton steps (relative error at the FP64 rounding level)
      double y = __builtin_amdgcn_rsq(sig2);
      y = fma(0.5 * y, fma(-sig2 * y, y, 1.0), y);
      y = fma(0.5 * y, fma(-sig2 * y, y, 1.0), y);
      const double y2 = y * y, x0 = (dw * dw) * y2;
      const double e0 = exp_neg(x0);
      delta = e0 * (0.5641895835477563 * y);
      if (pair) {
        // the mirrored member's exponent differs from x0 only by the rounding of its dw
        // (|x0 - x1| <= 1e-8 for any sigma above the floor), so exp(-x1) =
        // e0 exp(d) = e0 (1 + d + d^2/2) to far below the FP64 rounding, d = x0 - x1
        const double d = x0 - (dwm * dwm) * y2;
        delta += fma(e0, fma(0.5 * d, d, d), e0) * (0.5641895835477563 * y);
      }
    }
    // P4 (harmonic 2): channel weight / N^2 times delta only
    const bool p4 = a.harmonic == 2;
    const double base = p4 ? kw * delta : kw * p2.iw * p3.iw * v2abs * delta;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (t < a.nT) {
        // occupation factor: (1 + n')(1 + n'') n''' (++), (1 + n') n'' n''' (+-),
        // n' n'' n''' (--)
        const double n2 = p2.n[t];
        const double n3 = p3.n[t];
        double f;
        if (CH == 1) f = (1.0 + n1[t]) * n2 * n3;
        else f = (neg ? n1[t] : 1.0 + n1[t]) * (neg ? n2 : 1.0 + n2) * n3;
        const double x = p4 ? base : base * f * invn[t];
        if (split) {
          if (umk) acc.r[1][t] += x;
          else acc.r[0][t] += x;
        } else if (CH == 1) {
          acc.r[1][t] += x;
        } else if (neg) {
          acc.r[2][t] += x;
        } else {
          acc.r[0][t] += x;
        }
      }
    }
    const unsigned inc = pair ? 2u : 1u;
    if (chi == 1) acc.cnt[1] += inc;
    else if (chi == 2) acc.cnt[2] += inc;
    else acc.cnt[0] += inc;
  }
}

// Per wavefront, a.qseg blocks are queued at a time and a.lseg kept processes evaluated per
// pass (both set by the host; the autotuner picks them with the q'-chunk).

// Where q''' = fold(q + s' q' + s'' q'') lies, for one (s', s''): with b = q + s' q' folded
// into the grid once, each digit of b + s'' q'' lies in (-g, 2g) and needs at most one
// correction by g; on the linear index the three corrections add to idx(b) + s'' idx(q'')
// (iq2 = idx(q''), n2 its digits).
struct Fold {
  int4 bw;
  int Bw;
  // b = q + s' q'
  __device__ __forceinline__ Fold(const Crystal &c, const PairIn &pi, int s1) {
    bw = make_int4(wrap(pi.nq.x + s1 * pi.nq1.x, c.g0), wrap(pi.nq.y + s1 * pi.nq1.y, c.g1),
                   wrap(pi.nq.z + s1 * pi.nq1.z, c.g2), 0);
    Bw = bw.x + c.g0 * (bw.y + c.g1 * bw.z);
  }
  __device__ __forceinline__ int operator()(const Crystal &c, int s2, int iq2, int4 n2) const {
    const int G01 = c.g0 * c.g1;
    if (s2 < 0)
      return Bw - iq2 + (bw.x < n2.x ? c.g0 : 0) + (bw.y < n2.y ? G01 : 0) + (bw.z < n2.z ? c.N : 0);
    return Bw + iq2 - (bw.x + n2.x >= c.g0 ? c.g0 : 0) - (bw.y + n2.y >= c.g1 ? G01 : 0) -
           (bw.z + n2.z >= c.g2 ? c.N : 0);
  }
};

// The contraction phase: the wavefront's lane groups take the queued blocks GPW at a time
// (lane r of a group owns branch row j'' = r), test their rows (the exact window predicate
// per candidate), contract the blocks with a kept process, and evaluate the kept processes
// of the blocks in flight as one compacted list.  CH = 1: redistribution blocks; CH = 3: ++
// and -- blocks (bit 30 of the queue entry: --), whose signs s' = s'' are taken per group.
// Queue entries hold q'' and q''' packed (15 bits each) on grids of up to 2^15 points (no
// fold here), q'' alone on larger ones.
template <typename R, int NB, int NT, int CH>
__device__ __forceinline__ void contract_queue(const Crystal &c, const RateArgs &a,
                                               const typename CT<R>::T *W, int lane, int gw,
                                               int r, bool glane, typename CT<R>::T *Xg,
                                               typename CT<R>::T *Pg, const int *sg_d,
                                               const int *skl, const int *Qw, int cnt,
                                               const typename CT<R>::T *Xw, int2 *Gq,
                                               unsigned short *Lw, const PairIn &pi,
                                               const double (&invn)[NT],
                                               const double (&n1)[NT], Acc<NT> &acc) {
  using CR = typename CT<R>::T;
  constexpr int GPW = 64 / NB;
  constexpr unsigned long long GMASK = (1ull << NB) - 1ull;
  const unsigned long long lt = (1ull << lane) - 1ull;
  const int LSEG = a.lseg;
  const ChanK ck(c, a, pi);
  const int mu = pi.mu, mu1 = pi.mu1;
  const bool pack = c.N <= 32768;
  const float inv_g0 = 1.0f / (float)c.g0, inv_g1 = 1.0f / (float)c.g1;
  for (int e0 = 0; e0 < cnt; e0 += GPW) {
    const int e = e0 + gw;
    const bool act = glane && e < cnt;
    int iq2 = 0, iq3 = 0;
    bool neg = false;
    unsigned bA = 0u, bB = 0u;
    if (act) {
      const int qv = Qw[e];
      neg = CH == 3 && ((qv >> 30) & 1) != 0;
      if (pack) {
        iq2 = qv & 0x7fff;
        iq3 = (qv >> 15) & 0x7fff;
      } else {
        // grid digits of q'' by division (no index-table load on the critical path)
        iq2 = qv & 0x3fffffff;
        int4 n2;
        int t;
        divmod_small(iq2, c.g0, inv_g0, t, n2.x);
        divmod_small(t, c.g1, inv_g1, n2.z, n2.y);
        iq3 = Fold(c, pi, neg ? -1 : 1)(c, (CH == 1 || neg) ? -1 : 1, iq2, n2);
      }
      // lane r reads column record r; the group shares the six through its tile
      const double4 vc = c.mode4[iq3 * NB + r];
      double2 *cs = reinterpret_cast<double2 *>(Xg);
      cs[2 * r] = make_double2(vc.x, vc.y);
      cs[2 * r + 1] = make_double2(vc.z, vc.w);
    }
    // redistribution: s' = +, s'' = -; ++: both +; --: both -
    const int S1 = neg ? -1 : 1;
    const int S2 = (CH == 1 || neg) ? -1 : 1;
    const double aw = neg ? ck.aw[1] : ck.aw[0];
    // in the redistribution and splitting channels slots 3 and 4 are both conjugated, so
    // for a slot-3/slot-4 symmetric quartet list the blocks q'' and q''' are transposes:
    // one contraction serves the mirror pair (its other orientation tested alongside)
    const bool mir = (CH == 1 || neg) && a.mirror != 0;
    wave_sync();
    if (act)
      row_bits_cols<NB>(a, aw, S2, c.mode4[iq2 * NB + r], c.speed[iq2 * NB + r], c.qbound[iq3],
                        reinterpret_cast<const double2 *>(Xg), mir && iq2 != iq3, bA, bB);
    bool umk = false;
    if (a.qclass != 0 && act) {
      // normal / Umklapp class of the block (the same for every branch and, for a mirror
      // pair, both orientations): Q = k(q''') - (k(q) + s' k(q') + s'' k(q'')) on the
      // first-zone image numerators of the four points
      const int4 k0 = c.qimg[mu / NB], k1 = c.qimg[mu1 / NB], k2 = c.qimg[iq2], k3 = c.qimg[iq3];
      umk = (k0.x + S1 * k1.x + S2 * k2.x != k3.x) || (k0.y + S1 * k1.y + S2 * k2.y != k3.y) ||
            (k0.z + S1 * k1.z + S2 * k2.z != k3.z);
      if (a.qclass != 3 && umk != (a.qclass == 2)) {
        bA = 0u;
        bB = 0u;
      }
    }
    const unsigned long long bal = __ballot((bA | bB) != 0u);
    const bool blk = act && ((bal >> (gw * NB)) & GMASK) != 0ull;
    if (blk && r == 0) acc.blocks += 1;
    if (blk && a.harmonic == 0) {   // the phase spaces take |V|^2 := 1
      CR V[NB];
      block_row<R, NB, VLIST<R>>(c, W + (S1 > 0 ? 0 : c.ng * WSTR), S2, iq2, iq3, r, Xg, Pg,
                                 sg_d, skl, V);
      if constexpr (!VLIST<R>) {
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) Xg[r * NB + cc] = V[cc];
      }
    }
    if (act && r == 0) Gq[gw] = make_int2(iq2, iq3 | (neg ? (1 << 29) : 0) | (umk ? (1 << 30) : 0));
    // the lane's list entries: single orientations, then mirror pairs with both kept
    // (codes as in gamma_list, one per column, so at most NB < 32 per lane); their place in
    // the wavefront's list is a prefix sum of the per-lane counts (the codes fit 32 bits up
    // to NB = 10; a list that fits one pass needs no bound check)
    using MT = std::conditional_t<(3 * NB <= 32), unsigned, unsigned long long>;
    const unsigned pr = bA & bB;
    const MT m = blk ? ((MT)(bA & ~pr) | ((MT)(bB & ~pr) << NB) | ((MT)pr << (2 * NB))) : (MT)0;
    const int n = sizeof(MT) == 4 ? __popc((unsigned)m) : __popcll((unsigned long long)m);
    int pre = 0, tot = 0;
    if constexpr (sizeof(R) == 8) {
      // FP64 kernel (measured 0.7% faster; the FP32 one keeps the ballots): an inclusive
      // scan over the wavefront, all 64 lanes active here, by DPP row shifts by 1, 2, 4, 8
      // within rows of 16 lanes, then row broadcasts of lane 15 into the odd rows and of
      // lane 31 into rows 2 and 3
      int x = n;
      x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);
      x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);
      x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);
      x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);
      x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);
      x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);
      pre = x - n;
      tot = __builtin_amdgcn_readlane(x, 63);
    } else {
#pragma unroll
      for (int bsl = 0; bsl < 5; ++bsl) {
        const unsigned long long bb = __ballot((n >> bsl) & 1);
        pre += __popcll(bb & lt) << bsl;
        tot += __popcll(bb) << bsl;
      }
    }
    auto ctz = [](MT x) {
      return sizeof(MT) == 4 ? __builtin_ctz((unsigned)x) : __builtin_ctzll((unsigned long long)x);
    };
    for (int base = 0; base < tot; base += LSEG) {
      MT mm = m;
      int idx = pre - base;
      if (tot <= LSEG) {
        while (mm) {
          const int b = ctz(mm);
          mm &= mm - (MT)1;
          Lw[idx++] = (unsigned short)((lane << 6) | b);
        }
      } else {
        while (mm) {
          const int b = ctz(mm);
          mm &= mm - (MT)1;
          if ((unsigned)idx < (unsigned)LSEG) Lw[idx] = (unsigned short)((lane << 6) | b);
          ++idx;
        }
      }
      wave_sync();
      gamma_list<R, NB, NT, CH>(c, a, Lw, min(LSEG, tot - base), lane, Xw, Gq, ck, invn, n1, acc);
      wave_sync();
    }
  }
  wave_sync();
}

// Redistribution (+-) blocks of one pair (lambda, lambda'): every q'' in grid order, one
// block of each mirror pair {q'', q'''} (V of the pair members are transposes of each other
// when the quartet list is symmetric under the slot-3/slot-4 exchange, a.mirror; otherwise
// every q'' block is queued and contracted on its own).  q'' is dealt out in rounds of 256
// consecutive points, every fourth to a wavefront and one to each of its lanes, so that
// every wavefront samples the whole grid evenly (mirror leaders, the lower-index member of
// each pair, gather at low indices: contiguous shares would load the wavefronts unevenly);
// each wavefront queues a segment of rounds in a fixed order (ballot + prefix count), then
// contracts the queue.
template <typename R, int NB, int NT>
__device__ __forceinline__ void redistribution_blocks(
    const Crystal &c, const RateArgs &a, const typename CT<R>::T *W, int wave, int lane, int gw,
    int r, bool glane, typename CT<R>::T *Xg, typename CT<R>::T *Pg, const int *sg_d,
    const int *skl, int *Qw, const typename CT<R>::T *Xw, int2 *Gq, unsigned short *Lw,
    const PairIn &pi, const double (&invn)[NT], const double (&n1)[NT], Acc<NT> &acc) {
  const unsigned long long lt = (1ull << lane) - 1ull;
  const bool pack = c.N <= 32768;
  const bool mir = a.mirror != 0;
  const Fold fp(c, pi, 1);
  const int nk = (c.N + 255) / 256;
  const int KSEG = a.qseg / 64;
  // grid digits of the per-round step 256 of q'' (one carry per digit at most: each step
  // digit is below its grid dimension)
  const int4 DK = make_int4(256 % c.g0, (256 / c.g0) % c.g1, 256 / (c.g0 * c.g1), 0);
  for (int k0 = 0; k0 < nk; k0 += KSEG) {
    const int k1 = min(nk, k0 + KSEG);
    int cnt = 0;
    // the grid digits of q'' advance arithmetically by DK per round (no index-table load);
    // past the grid (q'' >= N, never queued) they run on unchecked
    int iq2 = (k0 * 64 + lane) * 4 + wave;
    int4 d2 = c.qn[min(iq2, c.N - 1)];
    for (int k = k0; k < k1; ++k) {
      const int iq2c = iq2, iq3c = fp(c, -1, iq2, d2);
      iq2 += 256;
      d2.x += DK.x;
      const int cx = d2.x >= c.g0;
      d2.x -= cx ? c.g0 : 0;
      d2.y += DK.y + cx;
      const int cy = d2.y >= c.g1;
      d2.y -= cy ? c.g1 : 0;
      d2.z += DK.z + cy;
      const bool lead = iq2c < c.N && (!mir || iq2c <= iq3c);
      const unsigned long long lb = __ballot(lead);
      if (lead) Qw[cnt + __popcll(lb & lt)] = pack ? (iq2c | (iq3c << 15)) : iq2c;
      cnt += __popcll(lb);
    }
    wave_sync();
    contract_queue<R, NB, NT, 1>(c, a, W, lane, gw, r, glane, Xg, Pg, sg_d, skl, Qw, cnt, Xw, Gq,
                                 Lw, pi, invn, n1, acc);
  }
}

// The threshold of the scan of ++ (CH = 0) or -- (CH = 2) and its length: the sorted entries
// <= thr, counted in whole 64ths of the list first, then in the boundary one.
template <int CH>
__device__ __forceinline__ double sorted_thr(const Crystal &c, const RateArgs &a,
                                             const PairIn &pi) {
  constexpr int S2 = (CH == 0) ? 1 : -1;
  const double aw = add_signed(pi.w, pi.w1, S2);
  const double win = 2.0 * a.sqrt_c_win * c.v_hi * (1.0 + 1e-6) + 1e-9 * (fabs(aw) + c.w_hi) + 1e-12;
  return (S2 > 0 ? c.w_hi - aw : aw - c.w_lo) + win;
}

template <int CH>
__device__ __forceinline__ int sorted_scan(const Crystal &c, const RateArgs &a, int lane,
                                           const PairIn &pi) {
  const double thr = sorted_thr<CH>(c, a, pi);
  const int seg = (c.N + 63) >> 6;
  const bool le = lane * seg < c.N && c.qord_w[min(c.N, (lane + 1) * seg) - 1] <= thr;
  const int full = __popcll(__ballot(le));
  int nscan = full * seg;
  for (int i0 = 0; i0 < seg; i0 += 64) {
    const int i = i0 + lane, p = full * seg + i;
    const bool b = i < seg && p < c.N && c.qord_w[p] <= thr;
    nscan += __popcll(__ballot(b));
  }
  return nscan;
}

// One segment, rounds [k0, k1), of the scan of ++ (CH = 0) or -- (CH = 2): the blocks with
// a kept process are appended to the queue (tagged with bit 30 for --).  The sorted list is
// dealt out in rounds of 4 GPW consecutive points, every fourth point to a wavefront, so
// that the four wavefronts sample the list (and its blocks with kept processes, which
// gather at low frequencies) evenly.
template <int NB, int CH>
__device__ __forceinline__ void sorted_segment(const Crystal &c, const RateArgs &a, int wave,
                                               int lane, int gw, int r, bool glane,
                                               double2 *cs, int *Qw, int &cnt,
                                               const PairIn &pi, int nscan, int k0, int k1) {
  constexpr int GPW = 64 / NB;
  constexpr int S2 = (CH == 0) ? 1 : -1;
  constexpr unsigned long long GMASK = (1ull << NB) - 1ull;
  const unsigned long long lt = (1ull << lane) - 1ull;
  const bool pack = c.N <= 32768;
  const unsigned tag = CH == 2 ? (1u << 30) : 0u;
  // splitting with mirror pairs: the pair {q'', q'''} is taken from its lower index, with
  // both orientations tested
  const bool mir = CH == 2 && a.mirror != 0;
  const Fold fold(c, pi, S2);
  const double aw = add_signed(pi.w, pi.w1, S2);
  // (formed again here rather than carried across the contraction: fewer live registers)
  const double thr = sorted_thr<CH>(c, a, pi);
  const float inv_g0 = 1.0f / (float)c.g0, inv_g1 = 1.0f / (float)c.g1;
  const int npt = (k1 - k0) * GPW;
  auto staged = [&](int v, int &iq2, int &iq3) {
    if (pack) {
      iq2 = v & 0x7fff;
      iq3 = v >> 15;
    } else {
      iq2 = v;
      int4 n2;
      int t;
      divmod_small(iq2, c.g0, inv_g0, t, n2.x);
      divmod_small(t, c.g1, inv_g1, n2.z, n2.y);
      iq3 = fold(c, S2, iq2, n2);
    }
  };
  const int c0 = cnt;
  // stage A: every lane tests one point of the segment's part of the sorted list against
  // a bound on its whole block: dw of any process of (q'', q''') lies in
  // [aw + w''_min - w'''_max, aw + w''_max - w'''_min] (++) or
  // [aw - w''_max - w'''_max, aw - w''_min - w'''_min] (--), and a kept one has
  // |dw| <= sqrt(c_win) (v''_max + v'''_max); the interval is widened by 1e-9 of the
  // frequencies entering it (far above its FP64 rounding) and the bound by 1e-6, so no
  // block with a kept process is dropped.  In the splitting channel the interval is the
  // same for both orientations of a mirror pair.  The survivors are staged at Qw[c0...].
  const double bmar = 1e-9 * (fabs(aw) + 2.0 * c.w_hi) + 1e-12;
  int ns = 0;
  for (int i0 = 0; i0 < npt; i0 += 64) {
    const int i = i0 + lane;
    const int p = ((k0 * GPW + i) << 2) + wave;
    bool sv = false;
    int iq2 = 0, iq3 = 0;
    if (i < npt && p < nscan) {
      const int4 s = c.qord[p];
      iq2 = s.x;
      iq3 = fold(c, S2, iq2, make_int4(s.y, s.z, s.w, 0));
      const double4 b2 = c.qbound[iq2], b3 = c.qbound[iq3];
      const double lo = S2 > 0 ? (aw + b2.x) - b3.y : (aw - b2.y) - b3.y;
      const double hi = S2 > 0 ? (aw + b2.y) - b3.x : (aw - b2.x) - b3.x;
      const double lim = a.sqrt_c_win * (b2.z + b3.z) * (1.0 + 1e-6) + bmar;
      sv = !(lo > lim) && !(hi < -lim);
      // a mirror pair is taken from its lower index; a q''' outside the scanned part
      // holds no kept process
      if (mir) sv = sv && iq2 <= iq3 && b3.x <= thr;
    }
    const unsigned long long bal = __ballot(sv);
    if (sv) Qw[c0 + ns + __popcll(bal & lt)] = pack ? (iq2 | (iq3 << 15)) : iq2;
    ns += __popcll(bal);
  }
  wave_sync();
  // stage B: the lane groups take the surviving points GPW at a time and test their rows
  // against the six columns (the next round's records are fetched while the current one
  // is tested); the blocks with a kept process are queued in place, below the entries
  // still to be read
  int e = gw;
  bool live = glane && e < ns;
  int iq2 = 0, iq3 = 0;
  if (live) staged(Qw[c0 + e], iq2, iq3);
  const double4 z4 = make_double4(0.0, 0.0, 0.0, 0.0);
  double4 vr = live ? c.mode4[iq2 * NB + r] : z4;
  double sp = live ? c.speed[iq2 * NB + r] : 0.0;
  double4 qb = live ? c.qbound[iq3] : z4;
  double4 vc = live ? c.mode4[iq3 * NB + r] : z4;
  for (int j0 = 0; j0 < ns; j0 += GPW) {
    const bool livec = live;
    const int iq2c = iq2, iq3c = iq3;
    const double4 vrc = vr, qbc = qb;
    const double spc = sp;
    // lane r holds column record r of the round; the group shares the six through its tile
    if (livec) {
      cs[2 * r] = make_double2(vc.x, vc.y);
      cs[2 * r + 1] = make_double2(vc.z, vc.w);
    }
    e += GPW;
    live = glane && e < ns;
    if (live) {
      staged(Qw[c0 + e], iq2, iq3);
      vr = c.mode4[iq2 * NB + r];
      sp = c.speed[iq2 * NB + r];
      qb = c.qbound[iq3];
      vc = c.mode4[iq3 * NB + r];
    }
    wave_sync();
    bool keep = false;
    if (livec) {
      unsigned b0, b1;
      row_bits_cols<NB>(a, aw, S2, vrc, spc, qbc, cs, mir && iq2c != iq3c, b0, b1);
      const unsigned long long bal = __ballot((b0 | b1) != 0u);
      keep = ((bal >> (gw * NB)) & GMASK) != 0ull;
    }
    wave_sync();
    const bool lead = keep && r == 0;
    const unsigned long long lb = __ballot(lead);
    if (lead) Qw[cnt + __popcll(lb & lt)] = (int)((pack ? (unsigned)(iq2c | (iq3c << 15)) : (unsigned)iq2c) | tag);
    cnt += __popcll(lb);
  }
  wave_sync();
}

// Recombination (++) and splitting (--) blocks of one pair: q'' is scanned in ascending order
// of its lowest active frequency, and only as far as a row can pass the window.  A kept
// process has |dw| <= sqrt(c_win) |v'' - v'''| <= 2 sqrt(c_win) v_hi, with
// dw = aw + w'' - w''' (++) or aw - w'' - w''' (--), so its row frequency w'' is at most
// thr = w_hi - aw + win (++) or aw - w_lo + win (--).  The margins are far above the FP64
// rounding of the exact test, so no kept process is skipped.  In the splitting channel the
// same bound holds for w''' (the two slots enter dw alike), so a block whose q''' has its
// lowest frequency above thr holds no kept process, and a mirror pair has both members in
// the scanned part of the list or no kept process.  The blocks with a kept process of both
// channels go to one queue, contracted when the next segment would not fit and at the end,
// so the few blocks of the two channels fill common rounds (one call site of the
// contraction).
template <typename R, int NB, int NT>
__device__ __forceinline__ void sorted_blocks(
    const Crystal &c, const RateArgs &a, const typename CT<R>::T *W, int wave, int lane, int gw,
    int r, bool glane, typename CT<R>::T *Xg, typename CT<R>::T *Pg, const int *sg_d,
    const int *skl, int *Qw, const typename CT<R>::T *Xw, int2 *Gq, unsigned short *Lw,
    const PairIn &pi, const double (&invn)[NT], const double (&n1)[NT], Acc<NT> &acc) {
  constexpr int GPW = 64 / NB;
  const int KSEG = a.qseg / GPW;
  const int ns0 = (a.mask & 1u) ? sorted_scan<0>(c, a, lane, pi) : 0;
  const int ns2 = (a.mask & 4u) ? sorted_scan<2>(c, a, lane, pi) : 0;
  const int nk0 = (ns0 + 4 * GPW - 1) / (4 * GPW), nk2 = (ns2 + 4 * GPW - 1) / (4 * GPW);
  const int sg0 = (nk0 + KSEG - 1) / KSEG, sg2 = (nk2 + KSEG - 1) / KSEG;
  double2 *cs = reinterpret_cast<double2 *>(Xg);
  int cnt = 0;
  for (int sgi = 0; sgi <= sg0 + sg2; ++sgi) {
    const bool last = sgi == sg0 + sg2;
    const bool m2 = sgi >= sg0;
    const int k0 = (m2 ? sgi - sg0 : sgi) * KSEG;
    const int k1 = min(m2 ? nk2 : nk0, k0 + KSEG);
    const int npt = last ? 0 : (k1 - k0) * GPW;
    if (last || cnt + npt > a.qseg) {
      contract_queue<R, NB, NT, 3>(c, a, W, lane, gw, r, glane, Xg, Pg, sg_d, skl, Qw, cnt, Xw,
                                   Gq, Lw, pi, invn, n1, acc);
      cnt = 0;
    }
    if (last) break;
    if (m2) sorted_segment<NB, 2>(c, a, wave, lane, gw, r, glane, cs, Qw, cnt, pi, ns2, k0, k1);
    else sorted_segment<NB, 0>(c, a, wave, lane, gw, r, glane, cs, Qw, cnt, pi, ns0, k0, k1);
  }
}

// The work of one (target t of the batch, q'-chunk) item: every lambda' of the chunk, all
// channels, partial rates and counts written to the item's slot.  Called by the whole
// work-group (it synchronises internally).
template <typename R, int NB, int NT>
__device__ __forceinline__ void rate_body(const Crystal &c, const RateArgs &a, int t, int chunk,
                                          unsigned char *smem) {
  using CR = typename CT<R>::T;
  constexpr int GPW = 64 / NB;
  constexpr int NGRP = 4 * GPW;
  CR *W = reinterpret_cast<CR *>(smem);                 // [2][ng][WSTR]
  constexpr int XT = xtile(NB, sizeof(CR));
  CR *X = W + 2 * c.ng * WSTR;                             // [NGRP][XT]
  CR *P = X + NGRP * XT;                                // [NGRP][nd]
  int2 *Gq = reinterpret_cast<int2 *>(P + NGRP * c.nd); // [NGRP] current block of each group
  int *sg_d = reinterpret_cast<int *>(Gq + NGRP);       // [ng]
  int *skl = sg_d + c.ng;                               // [nat*nat + 1]
  int *Q = skl + c.nat * c.nat + 1;                     // [4][qseg] block queues
  unsigned short *L = reinterpret_cast<unsigned short *>(Q + 4 * a.qseg);  // [4][lseg]

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int gw = lane / NB, r = lane - gw * NB;
  const bool glane = gw < GPW;
  const int G = wave * GPW + gw;
  CR *Xg = X + (size_t)(glane ? G : 0) * XT;
  CR *Pg = P + (size_t)(glane ? G : 0) * c.nd;
  int *Qw = Q + wave * a.qseg;
  const CR *Xw = X + (size_t)wave * GPW * XT;
  int2 *Gqw = Gq + wave * GPW;
  unsigned short *Lw = L + wave * a.lseg;
  for (int i = tid; i < c.ng; i += 256) sg_d[i] = c.g_d[i];
  for (int i = tid; i <= c.nat * c.nat; i += 256) skl[i] = c.kl_start[i];

  const int mu = a.targets ? a.targets[t] : a.tbase + t;
  const int iq = mu / NB;
  Acc<NT> acc;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) acc.r[ch][tt] = 0.0;
    acc.cnt[ch] = 0;
  }
  acc.blocks = 0;
  const double w = uniform_d(c.omega[mu]);
  __syncthreads();
  if (w > 0.0) {
    const int4 nq = c.qn[iq];
    const CR *Ut = reinterpret_cast<const CR *>(a.U) + (size_t)t * c.nc * 27;
    double invn[NT];
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) invn[tt] = (tt < a.nT) ? uniform_d(a.inv_occ[(size_t)tt * c.N * NB + mu]) : 0.0;
    const int q1b = chunk * a.qchunk;
    const int q1e = min(c.N, q1b + a.qchunk);
    for (int iq1 = q1b; iq1 < q1e; ++iq1) {
      const int4 nq1 = c.qn[iq1];
      for (int j1 = 0; j1 < NB; ++j1) {
        const int mu1 = iq1 * NB + j1;
        const double w1 = uniform_d(c.omega[mu1]);
        if (!(w1 > 0.0)) continue;
        __syncthreads();
        build_W<R>(c, Ut, iq1, j1, W, X, NGRP * (XT + c.nd), tid, 256);
        __syncthreads();
        double n1[NT];
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) n1[tt] = (tt < a.nT) ? uniform_d(a.occ[(size_t)tt * c.N * NB + mu1]) : 0.0;
        const PairIn pi{nq, nq1, mu, mu1, w, w1};
        if (a.mask & 5u)
          sorted_blocks<R, NB, NT>(c, a, W, wave, lane, gw, r, glane, Xg, Pg, sg_d, skl, Qw, Xw, Gqw, Lw, pi, invn, n1, acc);
        if (a.mask & 2u)
          redistribution_blocks<R, NB, NT>(c, a, W, wave, lane, gw, r, glane, Xg, Pg, sg_d, skl, Qw, Xw, Gqw, Lw, pi, invn, n1, acc);
      }
    }
  }
  // work-group reduction in a fixed order: wave shuffles, then the four waves in order
  __syncthreads();
  double *red = reinterpret_cast<double *>(smem);
  constexpr int NV = 3 * NT;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch)
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) {
      double v = acc.r[ch][tt];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      if (lane == 0) red[wave * NV + ch * NT + tt] = v;
    }
  unsigned long long cv[4] = {acc.cnt[0], acc.cnt[1], acc.cnt[2], acc.blocks};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    unsigned long long v = cv[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    cv[i] = v;
  }
  unsigned long long *redc = reinterpret_cast<unsigned long long *>(red + 4 * NV);
  if (lane == 0)
    for (int i = 0; i < 4; ++i) redc[wave * 4 + i] = cv[i];
  __syncthreads();
  const size_t pbase = ((size_t)(a.t0 + t) * a.nchunk + chunk);
  if (tid < NV) {
    const int ch = tid / NT, tt = tid - ch * NT;
    if (tt < a.nT) {
      const double v = ((red[tid] + red[NV + tid]) + red[2 * NV + tid]) + red[3 * NV + tid];
      a.partial[pbase * 3 * a.nT + ch * a.nT + tt] = v;
    }
  }
  if (tid < 3) a.pcount[pbase * 3 + tid] = redc[tid] + redc[4 + tid] + redc[8 + tid] + redc[12 + tid];
  if (tid == 0) {
    const unsigned long long b = redc[3] + redc[7] + redc[11] + redc[15];
    if (b) atomicAdd(a.blocks, b);
  }
}

template <typename R, int NB, int NT>
// 3 work-groups (12 wavefronts) per CU, or 4 for the FP32 contraction of up to 6 branches,
// whose registers and LDS fit a fourth at a small spill (measured faster)
__global__ __launch_bounds__(256, (sizeof(R) == 4 && NB <= 6) ? 4 : 3) void k_rates(Crystal c, RateArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  // Work-groups reach the XCDs round-robin by blockIdx.  Remap so that XCD x walks the
  // contiguous range x*q + min(x, rem) ... of the target-major item list: the work-groups
  // resident on one XCD then share a few targets, whose precontraction U (re-read for every
  // lambda') stays in that XCD's L2.
  const unsigned nx = (unsigned)a.nxcd, b = blockIdx.x;
  const unsigned q = gridDim.x / nx, rem = gridDim.x - q * nx;
  const unsigned x = b % nx;
  const unsigned item = x * q + min(x, rem) + b / nx;
  const int t = (int)(item / (unsigned)a.nchunk), chunk = (int)(item - (unsigned)t * a.nchunk);
  rate_body<R, NB, NT>(c, a, t, chunk, smem);
}

// Persistent form over several crystals with the same branch count (uneven grids, quartet
// lists and mode counts): every work-group takes (instance, target, q'-chunk) items from
// atomic work queues (below) until all are exhausted; items are numbered instance by
// instance (the host orders the instances by cost per item, most expensive first).  Crystals
// of different branch counts run as separate persistent kernels of the same graph.
template <typename R, int NB, int NT>
__global__ __launch_bounds__(256, (sizeof(R) == 4 && NB <= 6) ? 4 : 3) void k_rates_batch(const BatchInst *__restrict__ insts, int ninst,
                                                        long long total,
                                                        unsigned long long *counter) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ long long item_s;
  // Work-groups reach the XCDs round-robin by blockIdx, and the item list is target-major.
  // The list is cut into one contiguous range per XCD with its own counter: a work-group
  // takes items of its XCD's range first (the work-groups resident on an XCD then share
  // targets, whose precontraction U stays in that XCD's L2), then those of the following
  // ranges in turn.  Every item is handed out once; a work-group stops after finding all
  // ranges exhausted.
  const int home = (int)(blockIdx.x % kBatchQueues);
  const long long q = total / kBatchQueues, rem = total % kBatchQueues;
  int visited = 0;   // ranges found exhausted (thread 0)
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) {
      long long it = total;
      while (visited < kBatchQueues) {
        const int x = (home + visited) % kBatchQueues;
        const long long lo = x * q + (x < rem ? x : rem), n = q + (x < rem ? 1 : 0);
        const long long k = (long long)atomicAdd(counter + (size_t)x * kQueueStride, 1ull);
        if (k < n) {
          it = lo + k;
          break;
        }
        ++visited;
      }
      item_s = it;
    }
    __syncthreads();
    // the item and the instance index are wave-uniform: keep them (and so the instance
    // descriptor loads) in scalar registers
    const long long iv = item_s;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(iv & 0xffffffffll));
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)iv >> 32));
    const long long item = (long long)(((unsigned long long)hi << 32) | lo);
    if (item >= total) break;
    int i = 0;
    while (i + 1 < ninst && item >= insts[i + 1].item0) ++i;
    i = __builtin_amdgcn_readfirstlane(i);
    const long long local = item - insts[i].item0;
    const int nchunk = insts[i].a.nchunk;
    const int t = (int)(local / nchunk), chunk = (int)(local - (long long)t * nchunk);
    rate_body<R, NB, NT>(insts[i].c, insts[i].a, t, chunk, smem);
  }
}

// ordered reduction over q'-chunks of targets 0 .. nt-1 of the partial buffers:
// rates[T][off + t] (row stride `stride`), per channel, counts
__global__ void k_reduce(const double *partial, const unsigned long long *pcount, int nt,
                         int nchunk, int nT, int stride, int off, double *rates,
                         double *rates_ch, long long *counts) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  const size_t o = (size_t)off + t;
  for (int tt = 0; tt < nT; ++tt) {
    double tot = 0.0;
    for (int ch = 0; ch < 3; ++ch) {
      double s = 0.0;
      for (int k = 0; k < nchunk; ++k) s += partial[(((size_t)t * nchunk + k) * 3 + ch) * nT + tt];
      if (rates_ch) rates_ch[((size_t)tt * 3 + ch) * stride + o] = s;
      tot += s;
    }
    rates[(size_t)tt * stride + o] = tot;
  }
  if (counts)
    for (int ch = 0; ch < 3; ++ch) {
      unsigned long long s = 0;
      for (int k = 0; k < nchunk; ++k) s += pcount[((size_t)t * nchunk + k) * 3 + ch];
      counts[o * 3 + ch] = (long long)s;
    }
}

// Scratch area of the allocation-free entry point (kScratchBytes per GPU, held while the
// process lives).  Host code never uses this name as an address: the device address comes
// from hipGetSymbolAddress (scratch_init) and is kept per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// V for explicit processes through the same W'' build and branch-block contraction.
// One wavefront per process; lanes 0..NB-1 form the group.
template <typename R, int NB>
__global__ __launch_bounds__(64) void k_debug_v(Crystal c, const int *quads, const int *tslot,
                                                const typename CT<R>::T *U, double2 *Vout) {
  using CR = typename CT<R>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  CR *W = reinterpret_cast<CR *>(smem);
  CR *Xg = W + 2 * c.ng * WSTR;
  CR *Pg = Xg + NB * NB;
  int *sg_d = reinterpret_cast<int *>(Pg + c.nd);
  int *skl = sg_d + c.ng;
  const int p = blockIdx.x, tid = threadIdx.x;
  for (int i = tid; i < c.ng; i += 64) sg_d[i] = c.g_d[i];
  for (int i = tid; i <= c.nat * c.nat; i += 64) skl[i] = c.kl_start[i];
  const int *qd = quads + 8 * p;
  const int iq = qd[0], iq1 = qd[2], j1 = qd[3], iq2 = qd[4], j2 = qd[5], j3 = qd[6], ch = qd[7];
  const CR *Ut = U + (size_t)tslot[p] * c.nc * 27;
  build_W<R>(c, Ut, iq1, j1, W, nullptr, 0, tid, 64);
  __syncthreads();
  if (tid >= NB) return;
  const int s1 = ch == 2 ? -1 : 1, s2 = ch == 0 ? 1 : -1;
  const int4 nq = c.qn[iq], nq1 = c.qn[iq1], nq2 = c.qn[iq2];
  const int x = wrap(nq.x + s1 * nq1.x + s2 * nq2.x, c.g0);
  const int y = wrap(nq.y + s1 * nq1.y + s2 * nq2.y, c.g1);
  const int z = wrap(nq.z + s1 * nq1.z + s2 * nq2.z, c.g2);
  const int iq3 = x + c.g0 * (y + c.g1 * z);
  CR V[NB];
  const CR *Ws = W + (s1 > 0 ? 0 : c.ng * WSTR);
  block_row<R, NB>(c, Ws, s2, iq2, iq3, tid, Xg, Pg, sg_d, skl, V);
  if (tid == j2) {
#pragma unroll
    for (int cc = 0; cc < NB; ++cc)
      if (cc == j3) Vout[p] = make_double2((double)V[cc].x, (double)V[cc].y);
  }
}

__global__ void k_zero(unsigned long long *p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

size_t rate_lds_bytes(const Crystal &c, int fp32, int NT, int qseg, int lseg) {
  const size_t cb = fp32 ? sizeof(float2) : sizeof(double2);
  const int NB = c.nb, GPW = 64 / NB;
  const size_t lds = cb * ((size_t)2 * c.ng * WSTR + (size_t)4 * GPW * xtile(NB, (int)cb) + (size_t)4 * GPW * c.nd) +
                     sizeof(int2) * (size_t)4 * GPW +
                     sizeof(int) * ((size_t)c.ng + c.nat * c.nat + 1 + (size_t)4 * qseg) +
                     sizeof(unsigned short) * (size_t)4 * lseg;
  const size_t lds_red = sizeof(double) * 4 * 3 * NT + sizeof(unsigned long long) * 16;
  return lds > lds_red ? lds : lds_red;
}

template <typename R, int NB, int NT>
hipError_t launch_rates_t(const Crystal &c, const RateArgs &a, hipStream_t s) {
  const size_t bytes = rate_lds_bytes(c, sizeof(R) == 4, NT, a.qseg, a.lseg);
  if (bytes > 160 * 1024) return hipErrorInvalidValue;
  const unsigned grid = (unsigned)((size_t)a.nt * a.nchunk);
  hipLaunchKernelGGL((k_rates<R, NB, NT>), dim3(grid), dim3(256), bytes, s, c, a);
  return hipGetLastError();
}

template <typename R, int NB>
hipError_t launch_rates_nb(const Crystal &c, const RateArgs &a, hipStream_t s) {
  if (a.nT <= 1) return launch_rates_t<R, NB, 1>(c, a, s);
  if (a.nT <= 2) return launch_rates_t<R, NB, 2>(c, a, s);
  if (a.nT <= 4) return launch_rates_t<R, NB, 4>(c, a, s);
  return launch_rates_t<R, NB, 8>(c, a, s);
}

template <typename R>
hipError_t launch_rates_r(const Crystal &c, const RateArgs &a, hipStream_t s) {
  switch (c.nb) {
    case 3: return launch_rates_nb<R, 3>(c, a, s);
    case 6: return launch_rates_nb<R, 6>(c, a, s);
    case 9: return launch_rates_nb<R, 9>(c, a, s);
    case 12: return launch_rates_nb<R, 12>(c, a, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename R, int NB>
hipError_t launch_debug_nb(const Crystal &c, const int *quads, int n, const int *tslot,
                           const void *U, double2 *V, hipStream_t s) {
  using CR = typename CT<R>::T;
  const size_t lds = sizeof(CR) * ((size_t)2 * c.ng * WSTR + (size_t)NB * NB + c.nd) +
                     sizeof(int) * ((size_t)c.ng + c.nat * c.nat + 1);
  hipLaunchKernelGGL((k_debug_v<R, NB>), dim3(n), dim3(64), lds, s, c, quads, tslot,
                     reinterpret_cast<const CR *>(U), V);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_debug_r(const Crystal &c, const int *quads, int n, const int *tslot,
                          const void *U, double2 *V, hipStream_t s) {
  switch (c.nb) {
    case 3: return launch_debug_nb<R, 3>(c, quads, n, tslot, U, V, s);
    case 6: return launch_debug_nb<R, 6>(c, quads, n, tslot, U, V, s);
    case 9: return launch_debug_nb<R, 9>(c, quads, n, tslot, U, V, s);
    case 12: return launch_debug_nb<R, 12>(c, quads, n, tslot, U, V, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_tables(const Crystal &c, double4 *qbound, double4 *mode4, double *speed, double *inv_omega, double2 *E64, float2 *E32,
                         const double *evec, const double *mass, int4 *qn, double2 *PHA64, double2 *PHB64,
                         double2 *PHD64, float2 *PHD32, const int *avec, const int *bvec,
                         const int *dvec, hipStream_t s) {
  const int nthr = 128;
  hipLaunchKernelGGL(k_tables, dim3((c.N + nthr - 1) / nthr), dim3(nthr), 0, s, c, qbound, mode4, speed, inv_omega, E64, E32,
                     evec, mass, qn, PHA64, PHB64, PHD64, PHD32, avec, bvec, dvec);
  return hipGetLastError();
}

hipError_t launch_occupations(const Crystal &c, const double *T, int nT, double hk,
                              double *occ, double *inv_occ, hipStream_t s) {
  const int n = c.N * c.nb * nT, nthr = 256;
  hipLaunchKernelGGL(k_occupations, dim3((n + nthr - 1) / nthr), dim3(nthr), 0, s, c.omega,
                     c.N * c.nb, T, nT, hk, occ, inv_occ);
  return hipGetLastError();
}

hipError_t launch_precontract(const Crystal &c, const int *targets, int nt, int fp32, void *U,
                              hipStream_t s, int tbase) {
  const long long total = (long long)nt * c.nc * 27;
  const int nthr = 256;
  const unsigned grid = (unsigned)((total + nthr - 1) / nthr);
  if (fp32)
    hipLaunchKernelGGL(k_precontract<float2>, dim3(grid), dim3(nthr), 0, s, c, targets, tbase, nt,
                       reinterpret_cast<float2 *>(U));
  else
    hipLaunchKernelGGL(k_precontract<double2>, dim3(grid), dim3(nthr), 0, s, c, targets, tbase, nt,
                       reinterpret_cast<double2 *>(U));
  return hipGetLastError();
}

hipError_t launch_occupations_v(const Crystal &c, const double *T, int nT, double hk,
                                double *occ, double *inv_occ, hipStream_t s) {
  if (nT < 1 || nT > 8) return hipErrorInvalidValue;
  TempList tl{};
  for (int i = 0; i < nT; ++i) tl.T[i] = T[i];
  const int n = c.N * c.nb * nT, nthr = 256;
  hipLaunchKernelGGL(k_occupations_v, dim3((n + nthr - 1) / nthr), dim3(nthr), 0, s, c.omega,
                     c.N * c.nb, tl, nT, hk, occ, inv_occ);
  return hipGetLastError();
}

size_t rate_lds_bytes_for(const Crystal &c, int fp32, int nT, int qseg, int lseg) {
  return rate_lds_bytes(c, fp32, nT <= 1 ? 1 : nT <= 2 ? 2 : nT <= 4 ? 4 : 8, qseg, lseg);
}

namespace {
void *g_scratch[64];
bool g_scratch_done[64];
std::mutex g_scratch_mu;
}  // namespace

hipError_t scratch_init(int dev, void **out) {
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_done[dev]) {
    void *p = nullptr;
    // the caller has made `dev` the current device
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = p;
    g_scratch_done[dev] = true;
  }
  if (out) *out = g_scratch[dev];
  return hipSuccess;
}

void *scratch_ptr(int dev) {
  if (dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch[dev];
}

hipError_t launch_rates(const Crystal &c, const RateArgs &a, int fp32, hipStream_t s) {
  return fp32 ? launch_rates_r<float>(c, a, s) : launch_rates_r<double>(c, a, s);
}

size_t batch_lds_bytes(const Crystal &c, int fp32, int nT, int qseg, int lseg) {
  return rate_lds_bytes(c, fp32, nT <= 1 ? 1 : nT <= 2 ? 2 : 4, qseg, lseg) + 64;
}

template <typename R, int NB, int NT>
hipError_t launch_batch_t(const BatchInst *insts, int ninst, long long total,
                          unsigned long long *counter, size_t lds, int *grid_out, hipStream_t s) {
  if (lds > 160 * 1024 - 64) return hipErrorInvalidValue;
  int dev = 0, ncu = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rates_batch<R, NB, NT>, 256, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  long long grid = (long long)ncu * per_cu;
  if (grid > total) grid = total;
  if (grid < 1) grid = 1;
  if (grid_out) *grid_out = (int)grid;
  hipLaunchKernelGGL((k_rates_batch<R, NB, NT>), dim3((unsigned)grid), dim3(256), lds, s, insts,
                     ninst, total, counter);
  return hipGetLastError();
}

template <typename R, int NB>
hipError_t launch_batch_nb(const BatchInst *insts, int ninst, long long total,
                           unsigned long long *counter, size_t lds, int nT, int *grid_out,
                           hipStream_t s) {
  if (nT <= 1) return launch_batch_t<R, NB, 1>(insts, ninst, total, counter, lds, grid_out, s);
  if (nT <= 2) return launch_batch_t<R, NB, 2>(insts, ninst, total, counter, lds, grid_out, s);
  return launch_batch_t<R, NB, 4>(insts, ninst, total, counter, lds, grid_out, s);
}

template <typename R>
hipError_t launch_batch_r(const BatchInst *insts, int ninst, long long total,
                          unsigned long long *counter, size_t lds, int nb, int nT,
                          int *grid_out, hipStream_t s) {
  switch (nb) {
    case 3: return launch_batch_nb<R, 3>(insts, ninst, total, counter, lds, nT, grid_out, s);
    case 6: return launch_batch_nb<R, 6>(insts, ninst, total, counter, lds, nT, grid_out, s);
    case 9: return launch_batch_nb<R, 9>(insts, ninst, total, counter, lds, nT, grid_out, s);
    case 12: return launch_batch_nb<R, 12>(insts, ninst, total, counter, lds, nT, grid_out, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_batch(const BatchInst *insts, int ninst, long long total,
                        unsigned long long *counter, size_t lds, int fp32, int nb, int nT,
                        int *grid_out, hipStream_t s) {
  return fp32 ? launch_batch_r<float>(insts, ninst, total, counter, lds, nb, nT, grid_out, s)
              : launch_batch_r<double>(insts, ninst, total, counter, lds, nb, nT, grid_out, s);
}
hipError_t launch_reduce(const RateArgs &a, int nt_total, double *rates, double *rates_ch,
                         long long *counts, hipStream_t s) {
  return launch_reduce_strided(a, nt_total, nt_total, 0, rates, rates_ch, counts, s);
}

hipError_t launch_reduce_strided(const RateArgs &a, int nt, int stride, int off, double *rates,
                                 double *rates_ch, long long *counts, hipStream_t s) {
  const int nthr = 128;
  hipLaunchKernelGGL(k_reduce, dim3((nt + nthr - 1) / nthr), dim3(nthr), 0, s, a.partial,
                     a.pcount, nt, a.nchunk, a.nT, stride, off, rates, rates_ch, counts);
  return hipGetLastError();
}

hipError_t launch_debug_v(const Crystal &c, const int *quads, int n, const int *tslot,
                          const void *U, int fp32, double2 *V, hipStream_t s) {
  return fp32 ? launch_debug_r<float>(c, quads, n, tslot, U, V, s)
              : launch_debug_r<double>(c, quads, n, tslot, U, V, s);
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t s) {
  const size_t n = bytes / 8;
  if (n == 0) return hipSuccess;
  const int nthr = 256;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + nthr - 1) / nthr)), dim3(nthr), 0, s,
                     reinterpret_cast<unsigned long long *>(p), n);
  return hipGetLastError();
}

}  // namespace fp4
