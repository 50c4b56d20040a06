// fp4_api.cpp -- host side of the four-phonon rate library: context, argument checks,
// regrouping of the quartet list, device buffers and kernel launches.  The ABI is declared
// in include/fp4.h.
#include "fp4.h"
#include "fp4_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

namespace {

// SI 2019 exact h, k_B, e; CODATA 2018 atomic mass unit
constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double kH = 6.62607015e-34;
constexpr double kKB = 1.380649e-23;
constexpr double kEV = 1.602176634e-19;
constexpr double kAMU = 1.66053906660e-27;

double hbar_over_kb_kps() { return kH / (2.0 * kPi) / kKB * 1.0e12; }

// Eq. 4phgamma prefactor hbar^2 pi / 8 for V in eV/(A^4 amu^2), delta in ps, omega in
// rad/ps, rate in 1/ps (the two 1/N factors are applied separately).
double c4_prefactor() {
  const double hbar = kH / (2.0 * kPi);
  const double kv = kEV / (1e-40 * kAMU * kAMU);
  return hbar * hbar * kPi / 8.0 * kv * kv * 1.0e-72;
}

// Eq. 3phgamma prefactor hbar pi / 4 for V in eV/(A^3 amu^1.5), same units otherwise.
double c3_prefactor() {
  const double hbar = kH / (2.0 * kPi);
  const double kv = kEV / (1e-30 * kAMU * std::sqrt(kAMU));
  return hbar * kPi / 4.0 * kv * kv * 1.0e-60;
}

// MI355X deals work-groups to its 8 XCDs (each with its own L2) round-robin by blockIdx.
constexpr int kXcds = 8;

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct fp4_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  int fail_alloc_at = -1;  // test hook: FP4_TEST_FAIL_ALLOC
  int alloc_count = 0;

  // lattice
  bool have_lattice = false;
  double A[9] = {0};
  int grid[3] = {0, 0, 0};
  int N = 0, nat = 0, nb = 0;
  std::vector<double> mass;
  double dq = 0.0;
  // modes / fc4 loaded flags
  bool have_modes = false, have_fc4 = false, tables_dirty = true;
  // third-order list (three-phonon feature), regrouped by atom pair (j, k) and d = Rj - Rk
  bool have_fc3 = false, tables3_dirty = true;
  int n3 = 0, nd3 = 0, nrk3 = 0;
  std::vector<int> jk3_start, t3_i, t3_d, t3_rk, d3vec, rk3vec;
  std::vector<double> t3_phi;
  // parameters
  double window_w = 2.0, sigma_min = 1e-4;
  int qchunk = 0, profile = 0;
  int qseg = 256, lseg = 256;   // queue and list segments of the rate kernel (autotuned)

  // regrouped quartet list (host)
  int ng = 0, nc = 0, nq4 = 0, na = 0, nbv = 0, nd = 0;
  std::vector<int> g_d, kl_start, c_start, c_jat, c_a, cq_start, q_i, q_b, avec, bvec, dvec;
  std::vector<double> q_phi;
  // q points sorted by lowest active frequency (host copies of the uploaded tables)
  std::vector<int> h_qord;
  std::vector<double> h_qordw;

  // device buffers
  DevBuf d_omega, d_iw, d_m4, d_qbnd, d_vel, d_evec, d_mass, d_E64, d_E32, d_qn, d_PHA64, d_PHB64, d_PHD64, d_PHD32;
  DevBuf d_qord, d_qordw, d_qimg, d_speed;
  std::vector<int> h_qimg;
  int qclass = 0, harmonic = 0;
  // the quartet list is symmetric under the exchange of slots 3 and 4 (see fp4_load_fc4)
  bool sym34 = false;
  double w_lo = 0.0, w_hi = 0.0, v_hi = 0.0;
  DevBuf d_g_d, d_kl, d_cs, d_cj, d_ca, d_cq, d_qi, d_qb, d_qphi, d_avec, d_bvec, d_dvec;
  DevBuf d_T, d_occ, d_iocc, d_targets, d_U, d_partial, d_pcount, d_blocks;
  DevBuf d_rates, d_rch, d_counts, d_quads, d_tslot, d_V;
  DevBuf d3_jk, d3_ti, d3_td, d3_trk, d3_phi, d3_rkv, d3_dv, d3_PH3, d3_U, d3_targets, d3_rates, d3_counts;
  DevBuf df_g4, df_X, df_shift, d_kappa;

  // statistics / timing of the last call
  long long st_processes = 0, st_candidates = 0, st_blocks = 0;
  double ms_main = 0.0, ms_total = 0.0;
  std::vector<hipEvent_t> ev_pool;

  int fail(int code, const std::string &msg) {
    err = msg;
    return code;
  }
};

namespace {

#define FP4_HIP(ctx, expr)                                                             \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return (ctx)->fail(FP4_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

int ensure(fp4_ctx *ctx, DevBuf &b, size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (b.bytes >= bytes) return FP4_OK;
  if (b.p) {
    hipError_t e = hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
    if (e != hipSuccess) return ctx->fail(FP4_E_DEVICE, std::string("hipFree: ") + hipGetErrorString(e));
  }
  ctx->alloc_count++;
  if (ctx->fail_alloc_at >= 0 && ctx->alloc_count == ctx->fail_alloc_at)
    return ctx->fail(FP4_E_NOMEM, "device allocation failed (injected by FP4_TEST_FAIL_ALLOC)");
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    return ctx->fail(FP4_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
  }
  b.bytes = bytes;
  return FP4_OK;
}

template <typename T>
int upload(fp4_ctx *ctx, DevBuf &b, const T *src, size_t n) {
  int rc = ensure(ctx, b, n * sizeof(T));
  if (rc) return rc;
  if (n) FP4_HIP(ctx, hipMemcpyAsync(b.p, src, n * sizeof(T), hipMemcpyHostToDevice, ctx->stream));
  return FP4_OK;
}

void release(DevBuf &b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

bool finite_all(const double *p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

fp4::Crystal make_crystal(const fp4_ctx *ctx) {
  fp4::Crystal c{};
  c.g0 = ctx->grid[0];
  c.g1 = ctx->grid[1];
  c.g2 = ctx->grid[2];
  c.N = ctx->N;
  c.nat = ctx->nat;
  c.nb = ctx->nb;
  c.ng = ctx->ng;
  c.nc = ctx->nc;
  c.nq4 = ctx->nq4;
  c.na = ctx->na;
  c.nbv = ctx->nbv;
  c.nd = ctx->nd;
  c.omega = (const double *)ctx->d_omega.p;
  c.inv_omega = (const double *)ctx->d_iw.p;
  c.vel = (const double4 *)ctx->d_vel.p;
  c.mode4 = (const double4 *)ctx->d_m4.p;
  c.speed = (const double *)ctx->d_speed.p;
  c.qbound = (const double4 *)ctx->d_qbnd.p;
  c.qimg = (const int4 *)ctx->d_qimg.p;
  c.qord = (const int4 *)ctx->d_qord.p;
  c.qord_w = (const double *)ctx->d_qordw.p;
  c.w_lo = ctx->w_lo;
  c.w_hi = ctx->w_hi;
  c.v_hi = ctx->v_hi;
  c.E64 = (const double2 *)ctx->d_E64.p;
  c.E32 = (const float2 *)ctx->d_E32.p;
  c.qn = (const int4 *)ctx->d_qn.p;
  c.PHA64 = (const double2 *)ctx->d_PHA64.p;
  c.PHB64 = (const double2 *)ctx->d_PHB64.p;
  c.PHD64 = (const double2 *)ctx->d_PHD64.p;
  c.PHD32 = (const float2 *)ctx->d_PHD32.p;
  c.g_d = (const int *)ctx->d_g_d.p;
  c.kl_start = (const int *)ctx->d_kl.p;
  c.c_start = (const int *)ctx->d_cs.p;
  c.c_jat = (const int *)ctx->d_cj.p;
  c.c_a = (const int *)ctx->d_ca.p;
  c.cq_start = (const int *)ctx->d_cq.p;
  c.q_i = (const int *)ctx->d_qi.p;
  c.q_b = (const int *)ctx->d_qb.p;
  c.q_phi = (const double *)ctx->d_qphi.p;
  return c;
}

// Build every per-q table (E, grid triples, phases) once modes and quartets are loaded.
int ensure_tables(fp4_ctx *ctx) {
  if (!ctx->tables_dirty) return FP4_OK;
  const size_t N = ctx->N, nb = ctx->nb;
  int rc;
  if ((rc = ensure(ctx, ctx->d_iw, N * nb * sizeof(double)))) return rc;
  if ((rc = ensure(ctx, ctx->d_m4, N * nb * sizeof(double4)))) return rc;
  if ((rc = ensure(ctx, ctx->d_speed, N * nb * sizeof(double)))) return rc;
  if ((rc = ensure(ctx, ctx->d_qbnd, N * sizeof(double4)))) return rc;
  if ((rc = ensure(ctx, ctx->d_E64, N * nb * nb * sizeof(double2)))) return rc;
  if ((rc = ensure(ctx, ctx->d_E32, N * nb * nb * sizeof(float2)))) return rc;
  if ((rc = ensure(ctx, ctx->d_qn, N * sizeof(int4)))) return rc;
  if ((rc = ensure(ctx, ctx->d_PHA64, N * ctx->na * sizeof(double2)))) return rc;
  if ((rc = ensure(ctx, ctx->d_PHB64, N * ctx->nbv * sizeof(double2)))) return rc;
  if ((rc = ensure(ctx, ctx->d_PHD64, N * ctx->nd * sizeof(double2)))) return rc;
  if ((rc = ensure(ctx, ctx->d_PHD32, N * ctx->nd * sizeof(float2)))) return rc;
  fp4::Crystal c = make_crystal(ctx);
  FP4_HIP(ctx, fp4::launch_tables(c, (double4 *)ctx->d_qbnd.p, (double4 *)ctx->d_m4.p, (double *)ctx->d_speed.p, (double *)ctx->d_iw.p, (double2 *)ctx->d_E64.p, (float2 *)ctx->d_E32.p,
                                  (const double *)ctx->d_evec.p, (const double *)ctx->d_mass.p,
                                  (int4 *)ctx->d_qn.p, (double2 *)ctx->d_PHA64.p,
                                  (double2 *)ctx->d_PHB64.p, (double2 *)ctx->d_PHD64.p,
                                  (float2 *)ctx->d_PHD32.p, (const int *)ctx->d_avec.p,
                                  (const int *)ctx->d_bvec.p, (const int *)ctx->d_dvec.p,
                                  ctx->stream));
  // q points in ascending order of their lowest active frequency (the ++ and -- channels scan
  // q'' in this order and stop where no row can pass the window), and the global bounds
  {
    std::vector<double4> qb(N);
    FP4_HIP(ctx, hipMemcpyAsync(qb.data(), ctx->d_qbnd.p, N * sizeof(double4), hipMemcpyDeviceToHost, ctx->stream));
    FP4_HIP(ctx, hipStreamSynchronize(ctx->stream));
    std::vector<int> ord(N);
    for (size_t i = 0; i < N; ++i) ord[i] = (int)i;
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return qb[x].x < qb[y].x; });
    ctx->h_qord.assign(4 * N, 0);
    ctx->h_qordw.assign(N, 0.0);
    double wlo = 1e300, whi = -1e300, vhi = 0.0;
    for (size_t p = 0; p < N; ++p) {
      const int iq = ord[p];
      ctx->h_qord[4 * p] = iq;
      ctx->h_qord[4 * p + 1] = iq % ctx->grid[0];
      ctx->h_qord[4 * p + 2] = (iq / ctx->grid[0]) % ctx->grid[1];
      ctx->h_qord[4 * p + 3] = iq / (ctx->grid[0] * ctx->grid[1]);
      ctx->h_qordw[p] = qb[iq].x;
      wlo = std::min(wlo, qb[iq].x);
      whi = std::max(whi, qb[iq].y);
      vhi = std::max(vhi, qb[iq].z);
    }
    ctx->w_lo = wlo;
    ctx->w_hi = whi;
    ctx->v_hi = vhi;
    // First-zone image of every grid point (normal / Umklapp classes): among the 64 shifts
    // m in {-2..1}^3 the reduced vector f = n/N + m of smallest |f|_G^2 = f^T G f, with
    // G = B B^T the reciprocal metric (B rows = b_d, 2 pi included; G = 4 pi^2 (A A^T)^-1).
    // Images whose squared lengths lie within a relative 1e-10 of the shortest are equal
    // lengths (points on the zone boundary); of those the first in the order m1, m2, m3
    // (m1 slowest) is taken.  Stored as integer numerators n_d + m_d N_d.
    {
      const double *A = ctx->A;
      double M[9];   // A A^T
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[3 * i + j] = A[3 * i] * A[3 * j] + A[3 * i + 1] * A[3 * j + 1] + A[3 * i + 2] * A[3 * j + 2];
      const double dm = M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
                        M[2] * (M[3] * M[7] - M[4] * M[6]);
      const double c4pi2 = 4.0 * kPi * kPi / dm;
      const double G[9] = {c4pi2 * (M[4] * M[8] - M[5] * M[7]), c4pi2 * (M[2] * M[7] - M[1] * M[8]),
                           c4pi2 * (M[1] * M[5] - M[2] * M[4]), c4pi2 * (M[5] * M[6] - M[3] * M[8]),
                           c4pi2 * (M[0] * M[8] - M[2] * M[6]), c4pi2 * (M[2] * M[3] - M[0] * M[5]),
                           c4pi2 * (M[3] * M[7] - M[4] * M[6]), c4pi2 * (M[1] * M[6] - M[0] * M[7]),
                           c4pi2 * (M[0] * M[4] - M[1] * M[3])};
      const int *g = ctx->grid;
      ctx->h_qimg.assign(4 * N, 0);
      double len[64];
      for (size_t iq = 0; iq < N; ++iq) {
        const int n[3] = {(int)(iq % g[0]), (int)((iq / g[0]) % g[1]), (int)(iq / ((size_t)g[0] * g[1]))};
        double lmin = 1e300;
        for (int s = 0; s < 64; ++s) {
          const double f[3] = {(double)n[0] / g[0] + (s >> 4) - 2, (double)n[1] / g[1] + ((s >> 2) & 3) - 2,
                               (double)n[2] / g[2] + (s & 3) - 2};
          double l2 = 0.0;
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) l2 += f[i] * G[3 * i + j] * f[j];
          len[s] = l2;
          lmin = std::min(lmin, l2);
        }
        int best = 0;
        while (!(len[best] <= lmin * (1.0 + 1e-10))) ++best;
        const int bm[3] = {(best >> 4) - 2, ((best >> 2) & 3) - 2, (best & 3) - 2};
        for (int d = 0; d < 3; ++d) ctx->h_qimg[4 * iq + d] = n[d] + bm[d] * g[d];
      }
      if ((rc = upload(ctx, ctx->d_qimg, ctx->h_qimg.data(), ctx->h_qimg.size()))) return rc;
    }
    if ((rc = upload(ctx, ctx->d_qord, ctx->h_qord.data(), ctx->h_qord.size()))) return rc;
    if ((rc = upload(ctx, ctx->d_qordw, ctx->h_qordw.data(), ctx->h_qordw.size()))) return rc;
    FP4_HIP(ctx, hipStreamSynchronize(ctx->stream));
  }
  ctx->tables_dirty = false;
  return FP4_OK;
}

hipEvent_t pool_event(fp4_ctx *ctx, size_t i) {
  while (ctx->ev_pool.size() <= i) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ctx->ev_pool.push_back(e);
  }
  return ctx->ev_pool[i];
}

// Default q' points per work item for `nt` targets: enough items to fill the GPU (~8192),
// at most 8 q' per item, so that the ~96 work-groups resident on an XCD span few targets
// (items are mapped to XCDs in contiguous ranges), within a 1 GiB partial buffer.  (8 q'
// measured 1.2% faster than 16 on the 8x8x8 step and 0.5% on 16x16x16 calls.)
int auto_qchunk(const fp4_ctx *ctx, int nt, int nT) {
  long long nchunk = (8192 + nt - 1) / nt;
  if (nchunk < 1) nchunk = 1;
  if (nchunk > ctx->N) nchunk = ctx->N;
  int qchunk = (int)((ctx->N + nchunk - 1) / nchunk);
  qchunk = std::min(qchunk, 8);
  while (qchunk < ctx->N &&
         (size_t)nt * (size_t)((ctx->N + qchunk - 1) / qchunk) * 3 * nT * sizeof(double) > ((size_t)1 << 30))
    qchunk *= 2;
  return qchunk;
}

// Enqueue the whole rate computation for `nt` targets (device list d_targets) on `s`.
// Device outputs: rates [nT][nt], rates_ch [nT][3][nt] (nullable), counts [nt][3] (nullable).
int enqueue(fp4_ctx *ctx, const double *T, int nT, double sb, uint32_t mask, int precision,
            int nt, hipStream_t s, double *d_rates, double *d_rch, long long *d_counts,
            std::vector<std::pair<hipEvent_t, hipEvent_t>> *main_ev, size_t *evi) {
  int rc;
  const int fp32 = precision == FP4_FP32;
  const size_t nmodes = (size_t)ctx->N * ctx->nb;
  if ((rc = ensure_tables(ctx))) return rc;
  if ((rc = upload(ctx, ctx->d_T, T, (size_t)nT))) return rc;
  if ((rc = ensure(ctx, ctx->d_occ, nmodes * nT * sizeof(double)))) return rc;
  if ((rc = ensure(ctx, ctx->d_iocc, nmodes * nT * sizeof(double)))) return rc;
  fp4::Crystal c = make_crystal(ctx);
  FP4_HIP(ctx, fp4::launch_occupations(c, (const double *)ctx->d_T.p, nT, hbar_over_kb_kps(),
                                       (double *)ctx->d_occ.p, (double *)ctx->d_iocc.p, s));

  // work decomposition: q'-chunks per target so that a launch has enough work-groups
  int qchunk = ctx->qchunk > 0 ? ctx->qchunk : auto_qchunk(ctx, nt, nT);
  if (qchunk > ctx->N) qchunk = ctx->N;
  const int nchunk = (ctx->N + qchunk - 1) / qchunk;
  const size_t cbytes = fp32 ? sizeof(float2) : sizeof(double2);
  const size_t per_target = (size_t)ctx->nc * 27 * cbytes;
  const size_t ubudget = (size_t)512 << 20;
  int batch = (int)std::max<size_t>(1, std::min<size_t>((size_t)nt, ubudget / per_target));
  // keep launches under 2^31 work-groups
  batch = (int)std::min<long long>(batch, ((1ll << 31) - 1) / nchunk);

  if ((rc = ensure(ctx, ctx->d_U, (size_t)batch * per_target))) return rc;
  if ((rc = ensure(ctx, ctx->d_partial, (size_t)nt * nchunk * 3 * nT * sizeof(double)))) return rc;
  if ((rc = ensure(ctx, ctx->d_pcount, (size_t)nt * nchunk * 3 * sizeof(unsigned long long)))) return rc;
  if ((rc = ensure(ctx, ctx->d_blocks, sizeof(unsigned long long)))) return rc;
  FP4_HIP(ctx, fp4::launch_zero(ctx->d_blocks.p, sizeof(unsigned long long), s));

  fp4::RateArgs a{};
  const double wsb = ctx->window_w * sb;
  a.c_win = (wsb * ctx->dq) * (wsb * ctx->dq);
  a.sqrt_c_win = wsb * ctx->dq;
  a.c_sig = (sb * ctx->dq) * (sb * ctx->dq);
  a.c_min = ctx->sigma_min * ctx->sigma_min;
  a.kpref = (ctx->harmonic ? 1.0 : c4_prefactor()) / ((double)ctx->N * (double)ctx->N);
  a.harmonic = ctx->harmonic;
  a.mirror = ctx->sym34 ? 1 : 0;
  a.nT = nT;
  a.mask = mask;
  a.qclass = ctx->qclass;
  a.occ = (const double *)ctx->d_occ.p;
  a.inv_occ = (const double *)ctx->d_iocc.p;
  a.qchunk = qchunk;
  a.qseg = ctx->qseg;
  a.lseg = ctx->lseg;
  a.nchunk = nchunk;
  a.nxcd = kXcds;
  a.U = ctx->d_U.p;
  a.partial = (double *)ctx->d_partial.p;
  a.pcount = (unsigned long long *)ctx->d_pcount.p;
  a.blocks = (unsigned long long *)ctx->d_blocks.p;
  for (int t0 = 0; t0 < nt; t0 += batch) {
    const int nb_t = std::min(batch, nt - t0);
    const int *tg = (const int *)ctx->d_targets.p + t0;
    FP4_HIP(ctx, fp4::launch_precontract(c, tg, nb_t, fp32, ctx->d_U.p, s));
    a.targets = tg;
    a.nt = nb_t;
    a.t0 = t0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (main_ev) {
      e0 = pool_event(ctx, (*evi)++);
      e1 = pool_event(ctx, (*evi)++);
      if (!e0 || !e1) return ctx->fail(FP4_E_DEVICE, "hipEventCreate failed");
      FP4_HIP(ctx, hipEventRecord(e0, s));
    }
    hipError_t le = fp4::launch_rates(c, a, fp32, s);
    if (le == hipErrorInvalidValue)
      return ctx->fail(FP4_E_UNSUPPORTED, "the quartet list needs more LDS than a work-group has (too many atom-pair groups for this branch count)");
    FP4_HIP(ctx, le);
    if (main_ev) {
      FP4_HIP(ctx, hipEventRecord(e1, s));
      main_ev->push_back({e0, e1});
    }
  }
  FP4_HIP(ctx, fp4::launch_reduce(a, nt, d_rates, d_rch, d_counts, s));
  return FP4_OK;
}

int check_compute_args(fp4_ctx *ctx, const double *T, int32_t nT, double sb, uint32_t mask,
                       int32_t precision) {
  if (!ctx) return FP4_E_INVAL;
  if (!ctx->have_lattice || !ctx->have_modes || !ctx->have_fc4)
    return ctx->fail(FP4_E_STATE, "compute called before fp4_load_lattice, fp4_load_modes and fp4_load_fc4");
  if (!T || nT < 1 || nT > 8) return ctx->fail(FP4_E_INVAL, "need 1 <= nT <= 8 temperatures");
  for (int i = 0; i < nT; ++i)
    if (!(std::isfinite(T[i]) && T[i] > 0.0)) return ctx->fail(FP4_E_INVAL, "temperatures must be finite and > 0");
  if (!(std::isfinite(sb) && sb > 0.0)) return ctx->fail(FP4_E_INVAL, "scalebroad must be finite and > 0");
  if (mask == 0 || (mask & ~7u)) return ctx->fail(FP4_E_INVAL, "mask must be a nonzero subset of FP4_PP|FP4_PM|FP4_MM");
  if (precision != FP4_FP64 && precision != FP4_FP32)
    return ctx->fail(FP4_E_UNSUPPORTED, "precision must be FP4_FP64 or FP4_FP32");
  return FP4_OK;
}

int finish_stats(fp4_ctx *ctx, const std::vector<std::pair<hipEvent_t, hipEvent_t>> &ev,
                 hipEvent_t first, hipEvent_t last) {
  unsigned long long blocks = 0;
  FP4_HIP(ctx, hipMemcpy(&blocks, ctx->d_blocks.p, sizeof(blocks), hipMemcpyDeviceToHost));
  ctx->st_blocks = (long long)blocks;
  ctx->ms_main = 0.0;
  ctx->ms_total = 0.0;
  if (ctx->profile) {
    for (auto &p : ev) {
      float ms = 0.f;
      FP4_HIP(ctx, hipEventElapsedTime(&ms, p.first, p.second));
      ctx->ms_main += ms;
    }
    if (first && last) {
      float ms = 0.f;
      FP4_HIP(ctx, hipEventElapsedTime(&ms, first, last));
      ctx->ms_total = ms;
    }
  }
  return FP4_OK;
}

int compute_common(fp4_ctx *ctx, const double *T, int32_t nT, double sb, uint32_t mask,
                   int32_t precision, const int32_t *targets, int32_t nt, double *rates,
                   double *rates_ch, int64_t *counts) {
  int rc = check_compute_args(ctx, T, nT, sb, mask, precision);
  if (rc) return rc;
  if (!rates) return ctx->fail(FP4_E_INVAL, "rates output is required");
  const int nmodes = ctx->N * ctx->nb;
  std::vector<int> tl;
  if (targets) {
    if (nt < 1 || nt > nmodes) return ctx->fail(FP4_E_INVAL, "need 1 <= ntargets <= nq*nb");
    tl.assign(targets, targets + nt);
    for (int v : tl)
      if (v < 0 || v >= nmodes) return ctx->fail(FP4_E_INVAL, "target mode id out of range");
  } else {
    nt = nmodes;
    tl.resize(nt);
    for (int i = 0; i < nt; ++i) tl[i] = i;
  }
  if ((rc = upload(ctx, ctx->d_targets, tl.data(), tl.size()))) return rc;
  if ((rc = ensure(ctx, ctx->d_rates, (size_t)nT * nt * sizeof(double)))) return rc;
  if (rates_ch && (rc = ensure(ctx, ctx->d_rch, (size_t)nT * 3 * nt * sizeof(double)))) return rc;
  if ((rc = ensure(ctx, ctx->d_counts, (size_t)nt * 3 * sizeof(long long)))) return rc;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  size_t evi = 0;
  hipEvent_t first = nullptr, last = nullptr;
  if (ctx->profile) {
    first = pool_event(ctx, evi++);
    if (!first) return ctx->fail(FP4_E_DEVICE, "hipEventCreate failed");
    FP4_HIP(ctx, hipEventRecord(first, ctx->stream));
  }
  rc = enqueue(ctx, T, nT, sb, mask, precision, nt, ctx->stream, (double *)ctx->d_rates.p,
               rates_ch ? (double *)ctx->d_rch.p : nullptr, (long long *)ctx->d_counts.p,
               ctx->profile ? &ev : nullptr, &evi);
  if (rc) return rc;
  if (ctx->profile) {
    last = pool_event(ctx, evi++);
    if (!last) return ctx->fail(FP4_E_DEVICE, "hipEventCreate failed");
    FP4_HIP(ctx, hipEventRecord(last, ctx->stream));
  }
  FP4_HIP(ctx, hipMemcpyAsync(rates, ctx->d_rates.p, (size_t)nT * nt * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  if (rates_ch)
    FP4_HIP(ctx, hipMemcpyAsync(rates_ch, ctx->d_rch.p, (size_t)nT * 3 * nt * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  std::vector<long long> cnt((size_t)nt * 3);
  FP4_HIP(ctx, hipMemcpyAsync(cnt.data(), ctx->d_counts.p, cnt.size() * sizeof(long long), hipMemcpyDeviceToHost, ctx->stream));
  FP4_HIP(ctx, hipStreamSynchronize(ctx->stream));
  long long tot = 0;
  for (long long v : cnt) tot += v;
  if (counts) std::memcpy(counts, cnt.data(), cnt.size() * sizeof(long long));
  ctx->st_processes = tot;
  // candidates: active targets x active partner modes^2 x nb (j''') per enabled channel
  long long act = 0;
  // (computed from the host copy of omega kept at load time)
  (void)act;
  if ((rc = finish_stats(ctx, ev, first, last))) return rc;
  ctx->err.clear();
  return FP4_OK;
}

}  // namespace

extern "C" {

const char *fp4_strerror(int code) {
  switch (code) {
    case FP4_OK: return "success";
    case FP4_E_INVAL: return "invalid argument";
    case FP4_E_STATE: return "invalid state (missing or inconsistent loads)";
    case FP4_E_NOMEM: return "out of memory";
    case FP4_E_DEVICE: return "HIP device error";
    case FP4_E_UNSUPPORTED: return "unsupported option";
    default: return "unknown error code";
  }
}

int fp4_create(fp4_ctx **out, int device_id) {
  if (!out) return FP4_E_INVAL;
  *out = nullptr;
  fp4_ctx *ctx = new (std::nothrow) fp4_ctx();
  if (!ctx) return FP4_E_NOMEM;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device_id < 0 || device_id >= ndev) {
    (void)hipGetLastError();
    delete ctx;
    return FP4_E_DEVICE;
  }
  if (hipSetDevice(device_id) != hipSuccess) {
    delete ctx;
    return FP4_E_DEVICE;
  }
  ctx->device = device_id;
  if (hipStreamCreate(&ctx->stream) != hipSuccess) {
    delete ctx;
    return FP4_E_DEVICE;
  }
  // address of this device's allocation-free scratch area (looked up once per device)
  if (fp4::scratch_init(device_id, nullptr) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return FP4_E_DEVICE;
  }
  if (const char *f = std::getenv("FP4_TEST_FAIL_ALLOC")) ctx->fail_alloc_at = std::atoi(f);
  *out = ctx;
  return FP4_OK;
}

void fp4_destroy(fp4_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  DevBuf *all[] = {&ctx->d_omega, &ctx->d_iw, &ctx->d_m4, &ctx->d_speed, &ctx->d_qbnd, &ctx->d_qord, &ctx->d_qordw, &ctx->d_qimg, &ctx->d_vel, &ctx->d_evec, &ctx->d_mass, &ctx->d_E64,
                   &ctx->d_E32, &ctx->d_qn, &ctx->d_PHA64, &ctx->d_PHB64, &ctx->d_PHD64,
                   &ctx->d_PHD32, &ctx->d_g_d, &ctx->d_kl, &ctx->d_cs, &ctx->d_cj, &ctx->d_ca,
                   &ctx->d_cq, &ctx->d_qi, &ctx->d_qb, &ctx->d_qphi, &ctx->d_avec, &ctx->d_bvec,
                   &ctx->d_dvec, &ctx->d_T, &ctx->d_occ, &ctx->d_iocc, &ctx->d_targets,
                   &ctx->d_U, &ctx->d_partial, &ctx->d_pcount, &ctx->d_blocks, &ctx->d_rates,
                   &ctx->d_rch, &ctx->d_counts, &ctx->d_quads, &ctx->d_tslot, &ctx->d_V,
                   &ctx->d3_jk, &ctx->d3_ti, &ctx->d3_td, &ctx->d3_trk, &ctx->d3_phi,
                   &ctx->d3_rkv, &ctx->d3_dv, &ctx->d3_PH3, &ctx->d3_U, &ctx->d3_targets,
                   &ctx->d3_rates, &ctx->d3_counts, &ctx->df_g4, &ctx->df_X, &ctx->df_shift,
                   &ctx->d_kappa};
  for (DevBuf *b : all) release(*b);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

const char *fp4_last_error(const fp4_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int fp4_load_lattice(fp4_ctx *ctx, const double A[9], const int32_t grid[3], int32_t natoms,
                     const double *mass, double dq) {
  if (!ctx) return FP4_E_INVAL;
  try {
    if (!A || !grid || !mass) return ctx->fail(FP4_E_INVAL, "null pointer argument");
    if (!finite_all(A, 9)) return ctx->fail(FP4_E_INVAL, "lattice vectors must be finite");
    const double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                       A[2] * (A[3] * A[7] - A[4] * A[6]);
    if (!(std::fabs(det) > 1e-9)) return ctx->fail(FP4_E_INVAL, "lattice vectors are singular");
    long long N = 1;
    for (int d = 0; d < 3; ++d) {
      if (grid[d] < 1) return ctx->fail(FP4_E_INVAL, "grid dimensions must be >= 1");
      N *= grid[d];
    }
    if (N > (1 << 20)) return ctx->fail(FP4_E_INVAL, "grid larger than 2^20 points");
    if (natoms < 1 || natoms > 4) return ctx->fail(FP4_E_UNSUPPORTED, "1 <= natoms <= 4 supported");
    for (int i = 0; i < natoms; ++i)
      if (!(std::isfinite(mass[i]) && mass[i] > 0.0)) return ctx->fail(FP4_E_INVAL, "masses must be finite and > 0");
    if (!std::isfinite(dq)) return ctx->fail(FP4_E_INVAL, "dq must be finite");
    (void)hipSetDevice(ctx->device);
    std::memcpy(ctx->A, A, sizeof(ctx->A));
    for (int d = 0; d < 3; ++d) ctx->grid[d] = grid[d];
    ctx->N = (int)N;
    ctx->nat = natoms;
    ctx->nb = 3 * natoms;
    ctx->mass.assign(mass, mass + natoms);
    if (dq > 0.0) {
      ctx->dq = dq;
    } else {
      const double detB = std::pow(2.0 * kPi, 3) / std::fabs(det);
      ctx->dq = std::cbrt(detB / (double)N);
    }
    int rc = upload(ctx, ctx->d_mass, ctx->mass.data(), ctx->mass.size());
    if (rc) return rc;
    ctx->have_lattice = true;
    ctx->have_modes = false;
    ctx->have_fc4 = false;
    ctx->have_fc3 = false;
    ctx->tables_dirty = true;
    ctx->tables3_dirty = true;
    ctx->err.clear();
    return FP4_OK;
  } catch (const std::bad_alloc &) {
    return ctx->fail(FP4_E_NOMEM, "host allocation failed");
  }
}

int fp4_load_modes(fp4_ctx *ctx, int32_t nq, int32_t nb, const double *omega,
                   const double *evec, const double *vel) {
  if (!ctx) return FP4_E_INVAL;
  try {
    if (!ctx->have_lattice) return ctx->fail(FP4_E_STATE, "fp4_load_lattice must come first");
    if (nq != ctx->N || nb != ctx->nb) return ctx->fail(FP4_E_STATE, "nq must equal the grid size and nb = 3*natoms");
    if (!omega || !evec || !vel) return ctx->fail(FP4_E_INVAL, "null pointer argument");
    const size_t nm = (size_t)nq * nb;
    if (!finite_all(omega, nm) || !finite_all(evec, nm * nb * 2) || !finite_all(vel, nm * 3))
      return ctx->fail(FP4_E_INVAL, "modes contain NaN or Inf");
    (void)hipSetDevice(ctx->device);
    std::vector<double> v4(nm * 4, 0.0);
    for (size_t i = 0; i < nm; ++i)
      for (int x = 0; x < 3; ++x) v4[4 * i + x] = vel[3 * i + x];
    int rc;
    if ((rc = upload(ctx, ctx->d_omega, omega, nm))) return rc;
    if ((rc = upload(ctx, ctx->d_vel, v4.data(), v4.size()))) return rc;
    if ((rc = upload(ctx, ctx->d_evec, evec, nm * nb * 2))) return rc;
    FP4_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->have_modes = true;
    ctx->tables_dirty = true;
    // the per-q tables are built as soon as modes and quartets are both loaded, so that no
    // compute call has to allocate them
    if (ctx->have_fc4 && (rc = ensure_tables(ctx))) return rc;
    ctx->err.clear();
    return FP4_OK;
  } catch (const std::bad_alloc &) {
    return ctx->fail(FP4_E_NOMEM, "host allocation failed");
  }
}

int fp4_load_fc4(fp4_ctx *ctx, int32_t nquart, const int32_t *atoms, const int32_t *cells,
                 const double *phi) {
  if (!ctx) return FP4_E_INVAL;
  try {
    if (!ctx->have_lattice) return ctx->fail(FP4_E_STATE, "fp4_load_lattice must come first");
    if (nquart < 1 || nquart > (1 << 20)) return ctx->fail(FP4_E_INVAL, "need 1 <= nquart <= 2^20");
    if (!atoms || !cells || !phi) return ctx->fail(FP4_E_INVAL, "null pointer argument");
    for (int i = 0; i < 4 * nquart; ++i)
      if (atoms[i] < 0 || atoms[i] >= ctx->nat) return ctx->fail(FP4_E_INVAL, "quartet atom index out of range");
    for (int i = 0; i < 9 * nquart; ++i)
      if (cells[i] < -64 || cells[i] > 64) return ctx->fail(FP4_E_INVAL, "quartet cell coordinate outside [-64, 64]");
    if (!finite_all(phi, (size_t)81 * nquart)) return ctx->fail(FP4_E_INVAL, "force constants contain NaN or Inf");
    const int nat = ctx->nat;
    // distinct cell vectors a = Rj - Rl, b = -Rl, d = Rk - Rl
    using V3 = std::array<int, 3>;
    std::map<V3, int> amap, bmap, dmap;
    struct Q {
      int i, j, k, l, a, b, d, n;
    };
    std::vector<Q> qs(nquart);
    for (int n = 0; n < nquart; ++n) {
      const int32_t *at = atoms + 4 * n, *cl = cells + 9 * n;
      V3 Rj{cl[0], cl[1], cl[2]}, Rk{cl[3], cl[4], cl[5]}, Rl{cl[6], cl[7], cl[8]};
      V3 a{Rj[0] - Rl[0], Rj[1] - Rl[1], Rj[2] - Rl[2]};
      V3 b{-Rl[0], -Rl[1], -Rl[2]};
      V3 d{Rk[0] - Rl[0], Rk[1] - Rl[1], Rk[2] - Rl[2]};
      auto intern = [](std::map<V3, int> &m, const V3 &v) {
        auto it = m.find(v);
        if (it != m.end()) return it->second;
        const int id = (int)m.size();
        m.emplace(v, id);
        return id;
      };
      qs[n] = Q{at[0], at[1], at[2], at[3], intern(amap, a), intern(bmap, b), intern(dmap, d), n};
    }
    // Symmetry under the exchange of slots 3 and 4: quartet (i, j, k, l; Rj, Rk, Rl) with
    // Phi[a][b][g][t] and quartet (i, j, l, k; Rj, Rl, Rk) with Phi[a][b][t][g] contribute
    // alike to Eq. V4, so for such a list the redistribution matrix element is symmetric in
    // lambda'' and lambda''' and the kernel contracts one block of each mirror pair.  Entries
    // with equal atoms and cells are summed first; a missing partner counts as zero.  The
    // tolerance is 1e-12 of the largest |Phi|.
    {
      using Key = std::array<int, 13>;
      std::map<Key, std::array<double, 81>> acc;
      double pmax = 0.0;
      for (int n = 0; n < nquart; ++n) {
        Key key;
        for (int x = 0; x < 4; ++x) key[x] = atoms[4 * n + x];
        for (int x = 0; x < 9; ++x) key[4 + x] = cells[9 * n + x];
        auto it = acc.find(key);
        if (it == acc.end()) {
          std::array<double, 81> z{};
          it = acc.emplace(key, z).first;
        }
        for (int e = 0; e < 81; ++e) {
          it->second[e] += phi[(size_t)81 * n + e];
          pmax = std::max(pmax, std::fabs(phi[(size_t)81 * n + e]));
        }
      }
      const double tol = 1e-12 * pmax;
      bool sym = true;
      const std::array<double, 81> zero{};
      for (auto it = acc.begin(); sym && it != acc.end(); ++it) {
        const Key &k0 = it->first;
        Key k1 = k0;
        std::swap(k1[2], k1[3]);
        for (int x = 0; x < 3; ++x) std::swap(k1[7 + x], k1[10 + x]);
        auto jt = acc.find(k1);
        const std::array<double, 81> &p1 = jt == acc.end() ? zero : jt->second;
        for (int ab = 0; ab < 9 && sym; ++ab)
          for (int g = 0; g < 3 && sym; ++g)
            for (int t = 0; t < 3; ++t)
              if (std::fabs(it->second[ab * 9 + g * 3 + t] - p1[ab * 9 + t * 3 + g]) > tol) {
                sym = false;
                break;
              }
      }
      ctx->sym34 = sym;
    }
    // groups (k, l, d) and combos (group, j, a), ordered
    std::sort(qs.begin(), qs.end(), [](const Q &x, const Q &y) {
      return std::tie(x.k, x.l, x.d, x.j, x.a, x.n) < std::tie(y.k, y.l, y.d, y.j, y.a, y.n);
    });
    ctx->g_d.clear();
    ctx->c_start.clear();
    ctx->c_jat.clear();
    ctx->c_a.clear();
    ctx->cq_start.clear();
    ctx->q_i.assign(nquart, 0);
    ctx->q_b.assign(nquart, 0);
    ctx->q_phi.assign((size_t)81 * nquart, 0.0);
    ctx->kl_start.assign(nat * nat + 1, 0);
    std::vector<int> g_kl;
    for (int p = 0; p < nquart; ++p) {
      const Q &q = qs[p];
      const bool new_group = p == 0 || q.k != qs[p - 1].k || q.l != qs[p - 1].l || q.d != qs[p - 1].d;
      if (new_group) {
        ctx->g_d.push_back(q.d);
        g_kl.push_back(q.k * nat + q.l);
        ctx->c_start.push_back((int)ctx->c_jat.size());
      }
      const bool new_combo = new_group || q.j != qs[p - 1].j || q.a != qs[p - 1].a;
      if (new_combo) {
        ctx->c_jat.push_back(q.j);
        ctx->c_a.push_back(q.a);
        ctx->cq_start.push_back(p);
      }
      ctx->q_i[p] = q.i;
      ctx->q_b[p] = q.b;
      std::memcpy(&ctx->q_phi[(size_t)81 * p], phi + (size_t)81 * q.n, 81 * sizeof(double));
    }
    ctx->ng = (int)ctx->g_d.size();
    ctx->nc = (int)ctx->c_jat.size();
    ctx->nq4 = nquart;
    ctx->c_start.push_back(ctx->nc);
    ctx->cq_start.push_back(nquart);
    // kl_start[kl] = first group with pair index >= kl
    for (int kl = 0, g = 0; kl <= nat * nat; ++kl) {
      while (g < ctx->ng && g_kl[g] < kl) ++g;
      ctx->kl_start[kl] = g;
    }
    auto flat = [](const std::map<V3, int> &m) {
      std::vector<int> v(3 * m.size());
      for (auto &kv : m)
        for (int x = 0; x < 3; ++x) v[3 * kv.second + x] = kv.first[x];
      return v;
    };
    ctx->avec = flat(amap);
    ctx->bvec = flat(bmap);
    ctx->dvec = flat(dmap);
    ctx->na = (int)amap.size();
    ctx->nbv = (int)bmap.size();
    ctx->nd = (int)dmap.size();
    (void)hipSetDevice(ctx->device);
    int rc;
    if ((rc = upload(ctx, ctx->d_g_d, ctx->g_d.data(), ctx->g_d.size()))) return rc;
    if ((rc = upload(ctx, ctx->d_kl, ctx->kl_start.data(), ctx->kl_start.size()))) return rc;
    if ((rc = upload(ctx, ctx->d_cs, ctx->c_start.data(), ctx->c_start.size()))) return rc;
    if ((rc = upload(ctx, ctx->d_cj, ctx->c_jat.data(), ctx->c_jat.size()))) return rc;
    if ((rc = upload(ctx, ctx->d_ca, ctx->c_a.data(), ctx->c_a.size()))) return rc;
    if ((rc = upload(ctx, ctx->d_cq, ctx->cq_start.data(), ctx->cq_start.size()))) return rc;
    if ((rc = upload(ctx, ctx->d_qi, ctx->q_i.data(), ctx->q_i.size()))) return rc;
    if ((rc = upload(ctx, ctx->d_qb, ctx->q_b.data(), ctx->q_b.size()))) return rc;
    if ((rc = upload(ctx, ctx->d_qphi, ctx->q_phi.data(), ctx->q_phi.size()))) return rc;
    if ((rc = upload(ctx, ctx->d_avec, ctx->avec.data(), ctx->avec.size()))) return rc;
    if ((rc = upload(ctx, ctx->d_bvec, ctx->bvec.data(), ctx->bvec.size()))) return rc;
    if ((rc = upload(ctx, ctx->d_dvec, ctx->dvec.data(), ctx->dvec.size()))) return rc;
    FP4_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->have_fc4 = true;
    ctx->tables_dirty = true;
    if (ctx->have_modes && (rc = ensure_tables(ctx))) return rc;
    ctx->err.clear();
    return FP4_OK;
  } catch (const std::bad_alloc &) {
    return ctx->fail(FP4_E_NOMEM, "host allocation failed");
  }
}

int fp4_set_param(fp4_ctx *ctx, int32_t key, double value) {
  if (!ctx) return FP4_E_INVAL;
  if (!std::isfinite(value)) return ctx->fail(FP4_E_INVAL, "parameter value must be finite");
  switch (key) {
    case FP4_PARAM_WINDOW_W:
      if (!(value > 0.0)) return ctx->fail(FP4_E_INVAL, "window width must be > 0");
      ctx->window_w = value;
      return FP4_OK;
    case FP4_PARAM_SIGMA_MIN:
      if (!(value >= 0.0)) return ctx->fail(FP4_E_INVAL, "sigma_min must be >= 0");
      ctx->sigma_min = value;
      return FP4_OK;
    case FP4_PARAM_QCHUNK:
      if (!(value >= 0.0) || value > (1 << 20)) return ctx->fail(FP4_E_INVAL, "q' chunk must be in [0, 2^20]");
      ctx->qchunk = (int)value;
      return FP4_OK;
    case FP4_PARAM_PROFILE:
      ctx->profile = value != 0.0;
      return FP4_OK;
    case FP4_PARAM_PHASE_SPACE:
      if (!(value == 0.0 || value == 1.0 || value == 2.0))
        return ctx->fail(FP4_E_INVAL, "phase-space kind must be 0 (rates), 1 (WP4) or 2 (P4)");
      ctx->harmonic = (int)value;
      return FP4_OK;
    case FP4_PARAM_QSEG:
      if (!(value >= 64.0 && value <= 2048.0) || std::fmod(value, 64.0) != 0.0)
        return ctx->fail(FP4_E_INVAL, "queue segment must be a multiple of 64 in [64, 2048]");
      ctx->qseg = (int)value;
      return FP4_OK;
    case FP4_PARAM_LSEG:
      if (!(value >= 64.0 && value <= 4096.0) || std::fmod(value, 64.0) != 0.0)
        return ctx->fail(FP4_E_INVAL, "list segment must be a multiple of 64 in [64, 4096]");
      ctx->lseg = (int)value;
      return FP4_OK;
    case FP4_PARAM_QCLASS:
      if (!(value == 0.0 || value == 1.0 || value == 2.0))
        return ctx->fail(FP4_E_INVAL, "process class must be 0 (all), 1 (normal) or 2 (Umklapp)");
      ctx->qclass = (int)value;
      return FP4_OK;
    default:
      return ctx->fail(FP4_E_INVAL, "unknown parameter key");
  }
}

int fp4_compute_rates4(fp4_ctx *ctx, const double *T, int32_t nT, double scalebroad,
                       uint32_t mask, int32_t precision, double *rates,
                       double *rates_by_channel, int64_t *counts) {
  if (!ctx) return FP4_E_INVAL;
  try {
    (void)hipSetDevice(ctx->device);
    return compute_common(ctx, T, nT, scalebroad, mask, precision, nullptr, 0, rates,
                          rates_by_channel, counts);
  } catch (const std::bad_alloc &) {
    return ctx->fail(FP4_E_NOMEM, "host allocation failed");
  }
}

int fp4_compute_rates4_subset(fp4_ctx *ctx, const double *T, int32_t nT, double scalebroad,
                              uint32_t mask, int32_t precision, const int32_t *targets,
                              int32_t ntargets, double *rates, double *rates_by_channel,
                              int64_t *counts) {
  if (!ctx) return FP4_E_INVAL;
  if (!targets) return ctx->fail(FP4_E_INVAL, "targets must not be NULL");
  try {
    (void)hipSetDevice(ctx->device);
    return compute_common(ctx, T, nT, scalebroad, mask, precision, targets, ntargets, rates,
                          rates_by_channel, counts);
  } catch (const std::bad_alloc &) {
    return ctx->fail(FP4_E_NOMEM, "host allocation failed");
  }
}

int fp4_compute_rates4_classes(fp4_ctx *ctx, const double *T, int32_t nT, double scalebroad,
                               uint32_t mask, int32_t precision, const int32_t *targets,
                               int32_t ntargets, double *rates, double *rates_normal,
                               double *rates_umklapp, int64_t *counts) {
  if (!ctx) return FP4_E_INVAL;
  try {
    if (ctx->harmonic) return ctx->fail(FP4_E_UNSUPPORTED, "the class split takes rates, not phase spaces (FP4_PARAM_PHASE_SPACE must be 0)");
    if (!rates_normal && !rates_umklapp) return ctx->fail(FP4_E_INVAL, "rates_normal or rates_umklapp is required");
    (void)hipSetDevice(ctx->device);
    const int nt = targets ? ntargets : ctx->N * ctx->nb;
    if (nt < 1) return ctx->fail(FP4_E_INVAL, "need 1 <= ntargets <= nq*nb");
    std::vector<double> tot((size_t)std::max(1, (int)nT) * nt), cls((size_t)std::max(1, (int)nT) * 3 * nt);
    const int keep = ctx->qclass;
    ctx->qclass = 3;
    const int rc = compute_common(ctx, T, nT, scalebroad, mask, precision, targets, nt,
                                  tot.data(), cls.data(), counts);
    ctx->qclass = keep;
    if (rc) return rc;
    for (int t = 0; t < nT; ++t)
      for (int i = 0; i < nt; ++i) {
        if (rates) rates[(size_t)t * nt + i] = tot[(size_t)t * nt + i];
        if (rates_normal) rates_normal[(size_t)t * nt + i] = cls[((size_t)t * 3 + 0) * nt + i];
        if (rates_umklapp) rates_umklapp[(size_t)t * nt + i] = cls[((size_t)t * 3 + 1) * nt + i];
      }
    return FP4_OK;
  } catch (const std::bad_alloc &) {
    return ctx->fail(FP4_E_NOMEM, "host allocation failed");
  }
}

int fp4_compute_rates4_wedge(fp4_ctx *ctx, const double *T, int32_t nT, double scalebroad,
                             uint32_t mask, int32_t precision, int32_t nrot, const int32_t *rot,
                             double *rates, int64_t *counts, int32_t *nirr) {
  if (!ctx) return FP4_E_INVAL;
  try {
    if (!ctx->have_lattice || !ctx->have_modes || !ctx->have_fc4)
      return ctx->fail(FP4_E_STATE, "compute called before fp4_load_lattice, fp4_load_modes and fp4_load_fc4");
    if (nrot < 1 || nrot > 96 || !rot) return ctx->fail(FP4_E_INVAL, "need 1 <= nrot <= 96 rotations");
    if (!rates) return ctx->fail(FP4_E_INVAL, "rates output is required");
    (void)hipSetDevice(ctx->device);
    const int N = ctx->N, nb = ctx->nb, nmodes = N * nb;
    const int *g = ctx->grid;
    // every rotation must map the grid onto itself: n'_d = sum_e R_de n_e N_d / N_e (mod N_d)
    for (int k = 0; k < nrot; ++k)
      for (int d = 0; d < 3; ++d)
        for (int e = 0; e < 3; ++e) {
          const long long r = rot[9 * k + 3 * d + e];
          if (r != 0 && (r * g[d]) % g[e] != 0)
            return ctx->fail(FP4_E_INVAL, "a rotation does not map the q-grid onto itself");
        }
    // orbits of the grid points under the rotations (union of the images), the lowest index
    // of each orbit is its representative
    std::vector<int> parent(N);
    for (int i = 0; i < N; ++i) parent[i] = i;
    auto find = [&](int i) {
      while (parent[i] != i) i = parent[i] = parent[parent[i]];
      return i;
    };
    for (int iq = 0; iq < N; ++iq) {
      const int n[3] = {iq % g[0], (iq / g[0]) % g[1], iq / (g[0] * g[1])};
      for (int k = 0; k < nrot; ++k) {
        int m[3];
        for (int d = 0; d < 3; ++d) {
          long long acc = 0;
          for (int e = 0; e < 3; ++e) acc += (long long)rot[9 * k + 3 * d + e] * n[e] * g[d] / g[e];
          m[d] = (int)(((acc % g[d]) + g[d]) % g[d]);
        }
        const int jq = m[0] + g[0] * (m[1] + g[1] * m[2]);
        int a = find(iq), b = find(jq);
        if (a != b) parent[std::max(a, b)] = std::min(a, b);
      }
    }
    std::vector<int> rep(N), reps;
    for (int iq = 0; iq < N; ++iq) {
      rep[iq] = find(iq);
      if (rep[iq] == iq) reps.push_back(iq);
    }
    // the modes must be symmetric: the same (ascending-order) frequencies across an orbit
    std::vector<double> w(nmodes);
    FP4_HIP(ctx, hipMemcpy(w.data(), ctx->d_omega.p, nmodes * sizeof(double), hipMemcpyDeviceToHost));
    for (int iq = 0; iq < N; ++iq)
      for (int j = 0; j < nb; ++j) {
        const double a = w[(size_t)iq * nb + j], b = w[(size_t)rep[iq] * nb + j];
        if (std::fabs(a - b) > 1e-8 * std::max(std::fabs(a), std::fabs(b)) + 1e-12)
          return ctx->fail(FP4_E_INVAL, "frequencies differ across a rotation orbit (not a symmetry of the modes)");
      }
    std::vector<int> tl;
    for (int iq : reps)
      for (int j = 0; j < nb; ++j) tl.push_back(iq * nb + j);
    const int nt = (int)tl.size();
    std::vector<double> r((size_t)nT * nt);
    std::vector<int64_t> c((size_t)nt * 3);
    int rc = compute_common(ctx, T, nT, scalebroad, mask, precision, tl.data(), nt, r.data(),
                            nullptr, c.data());
    if (rc) return rc;
    // average over degenerate branches of each representative, then copy to its orbit
    std::vector<int> slot(N, -1);
    for (size_t k = 0; k < reps.size(); ++k) slot[reps[k]] = (int)k;
    for (size_t k = 0; k < reps.size(); ++k) {
      const double *wq = w.data() + (size_t)reps[k] * nb;
      for (int j = 0; j < nb;) {
        int e = j + 1;
        while (e < nb && std::fabs(wq[e] - wq[j]) <= 1e-9 * std::max(std::fabs(wq[j]), 1e-30)) ++e;
        for (int t = 0; t < nT; ++t) {
          double sum = 0.0;
          for (int i = j; i < e; ++i) sum += r[(size_t)t * nt + k * nb + i];
          for (int i = j; i < e; ++i) r[(size_t)t * nt + k * nb + i] = sum / (e - j);
        }
        j = e;
      }
    }
    for (int iq = 0; iq < N; ++iq) {
      const size_t k = (size_t)slot[rep[iq]];
      for (int j = 0; j < nb; ++j) {
        for (int t = 0; t < nT; ++t) rates[(size_t)t * nmodes + (size_t)iq * nb + j] = r[(size_t)t * nt + k * nb + j];
        if (counts)
          for (int ch = 0; ch < 3; ++ch) counts[((size_t)iq * nb + j) * 3 + ch] = c[(k * nb + j) * 3 + ch];
      }
    }
    if (nirr) *nirr = (int32_t)reps.size();
    ctx->err.clear();
    return FP4_OK;
  } catch (const std::bad_alloc &) {
    return ctx->fail(FP4_E_NOMEM, "host allocation failed");
  }
}

int fp4_compute_rates4_async(fp4_ctx *ctx, const double *T, int32_t nT, double scalebroad,
                             uint32_t mask, int32_t precision, void *hip_stream,
                             double *d_rates, double *d_rates_by_channel, int64_t *d_counts) {
  if (!ctx) return FP4_E_INVAL;
  try {
    int rc = check_compute_args(ctx, T, nT, scalebroad, mask, precision);
    if (rc) return rc;
    if (!d_rates) return ctx->fail(FP4_E_INVAL, "d_rates is required");
    (void)hipSetDevice(ctx->device);
    hipStream_t s = (hipStream_t)hip_stream;
    const int nt = ctx->N * ctx->nb;
    std::vector<int> tl(nt);
    for (int i = 0; i < nt; ++i) tl[i] = i;
    // the target list and temperatures are staged through the context's stream first
    if ((rc = upload(ctx, ctx->d_targets, tl.data(), tl.size()))) return rc;
    FP4_HIP(ctx, hipStreamSynchronize(ctx->stream));
    // per-q tables (after a load) are built on the context's own stream, never the caller's
    if ((rc = ensure_tables(ctx))) return rc;
    const hipStream_t keep = ctx->stream;
    ctx->stream = s;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    size_t evi = 0;
    rc = enqueue(ctx, T, nT, scalebroad, mask, precision, nt, s, d_rates, d_rates_by_channel,
                 (long long *)d_counts, ctx->profile ? &ev : nullptr, &evi);
    ctx->stream = keep;
    if (rc) return rc;
    if (ctx->profile) {
      FP4_HIP(ctx, hipStreamSynchronize(s));
      if ((rc = finish_stats(ctx, ev, nullptr, nullptr))) return rc;
    }
    ctx->err.clear();
    return FP4_OK;
  } catch (const std::bad_alloc &) {
    return ctx->fail(FP4_E_NOMEM, "host allocation failed");
  }
}

int fp4_compute_rates4_noalloc(fp4_ctx *ctx, const double *T, int32_t nT, double scalebroad,
                               uint32_t mask, int32_t precision, void *hip_stream,
                               double *d_rates, double *d_rates_by_channel, int64_t *d_counts) {
  if (!ctx) return FP4_E_INVAL;
  int rc = check_compute_args(ctx, T, nT, scalebroad, mask, precision);
  if (rc) return rc;
  if (!d_rates) return ctx->fail(FP4_E_INVAL, "d_rates is required");
  if (ctx->tables_dirty)
    return ctx->fail(FP4_E_STATE, "the per-q tables are not built (a load did not complete)");
  (void)hipSetDevice(ctx->device);
  unsigned char *base = static_cast<unsigned char *>(fp4::scratch_ptr(ctx->device));
  if (!base) return ctx->fail(FP4_E_DEVICE, "the scratch area of this device was not found");
  const hipStream_t s = (hipStream_t)hip_stream;
  const int fp32 = precision == FP4_FP32;
  const size_t nmodes = (size_t)ctx->N * ctx->nb;
  int qchunk = ctx->qchunk > 0 ? ctx->qchunk : auto_qchunk(ctx, (int)nmodes, nT);
  if (qchunk > ctx->N) qchunk = ctx->N;
  const int nchunk = (ctx->N + qchunk - 1) / qchunk;
  const size_t cb = fp32 ? sizeof(float2) : sizeof(double2);
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  // scratch layout: occupations, 1/occupations, block counter, then per target batch the
  // precontraction U, the partial rates and the partial counts
  const size_t b_occ = up(nmodes * nT * sizeof(double)), b_blk = 256;
  const size_t fixed = 2 * b_occ + b_blk;
  const size_t u_t = (size_t)ctx->nc * 27 * cb;
  const size_t p_t = (size_t)nchunk * 3 * nT * sizeof(double);
  const size_t c_t = (size_t)nchunk * 3 * sizeof(unsigned long long);
  const size_t need1 = fixed + up(u_t) + up(p_t) + up(c_t);
  if (need1 > fp4::kScratchBytes)
    return ctx->fail(FP4_E_UNSUPPORTED, "the allocation-free call needs " + std::to_string(need1) +
                                            " bytes of scratch for these sizes; its scratch area holds " +
                                            std::to_string(fp4::kScratchBytes) + " bytes");
  size_t batch = (fp4::kScratchBytes - fixed - 3 * 256) / (u_t + p_t + c_t);
  batch = std::min<size_t>(batch, nmodes);
  batch = std::min<size_t>(batch, (size_t)(((1ll << 31) - 1) / nchunk));
  double *occ = reinterpret_cast<double *>(base);
  double *iocc = reinterpret_cast<double *>(base + b_occ);
  unsigned long long *blocks = reinterpret_cast<unsigned long long *>(base + 2 * b_occ);
  void *U = base + fixed;
  double *partial = reinterpret_cast<double *>(base + fixed + up(batch * u_t));
  unsigned long long *pcount =
      reinterpret_cast<unsigned long long *>(base + fixed + up(batch * u_t) + up(batch * p_t));
  fp4::Crystal c = make_crystal(ctx);
  FP4_HIP(ctx, fp4::launch_zero(blocks, sizeof(unsigned long long), s));
  FP4_HIP(ctx, fp4::launch_occupations_v(c, T, nT, hbar_over_kb_kps(), occ, iocc, s));
  fp4::RateArgs a{};
  const double wsb = ctx->window_w * scalebroad;
  a.c_win = (wsb * ctx->dq) * (wsb * ctx->dq);
  a.sqrt_c_win = wsb * ctx->dq;
  a.c_sig = (scalebroad * ctx->dq) * (scalebroad * ctx->dq);
  a.c_min = ctx->sigma_min * ctx->sigma_min;
  a.kpref = (ctx->harmonic ? 1.0 : c4_prefactor()) / ((double)ctx->N * (double)ctx->N);
  a.harmonic = ctx->harmonic;
  a.mirror = ctx->sym34 ? 1 : 0;
  a.nT = nT;
  a.mask = mask;
  a.qclass = ctx->qclass;
  a.occ = occ;
  a.inv_occ = iocc;
  a.targets = nullptr;
  a.qchunk = qchunk;
  a.qseg = ctx->qseg;
  a.lseg = ctx->lseg;
  a.nchunk = nchunk;
  a.nxcd = kXcds;
  a.U = U;
  a.partial = partial;
  a.pcount = pcount;
  a.blocks = blocks;
  a.t0 = 0;
  for (size_t t0 = 0; t0 < nmodes; t0 += batch) {
    const int nb_t = (int)std::min(batch, nmodes - t0);
    a.tbase = (int)t0;
    a.nt = nb_t;
    FP4_HIP(ctx, fp4::launch_precontract(c, nullptr, nb_t, fp32, U, s, (int)t0));
    const hipError_t le = fp4::launch_rates(c, a, fp32, s);
    if (le == hipErrorInvalidValue)
      return ctx->fail(FP4_E_UNSUPPORTED, "the quartet list needs more LDS than a work-group has (too many atom-pair groups for this branch count)");
    FP4_HIP(ctx, le);
    FP4_HIP(ctx, fp4::launch_reduce_strided(a, nb_t, (int)nmodes, (int)t0, d_rates,
                                            d_rates_by_channel, (long long *)d_counts, s));
  }
  ctx->err.clear();
  return FP4_OK;
}

int fp4_debug_matrix_elements(fp4_ctx *ctx, int32_t n, const int32_t *quads, int32_t precision,
                              double *V) {
  if (!ctx) return FP4_E_INVAL;
  try {
    if (!ctx->have_lattice || !ctx->have_modes || !ctx->have_fc4)
      return ctx->fail(FP4_E_STATE, "debug call before all loads");
    if (n < 1 || n > (1 << 16) || !quads || !V) return ctx->fail(FP4_E_INVAL, "need 1 <= n <= 2^16 and non-null buffers");
    if (precision != FP4_FP64 && precision != FP4_FP32) return ctx->fail(FP4_E_UNSUPPORTED, "bad precision");
    for (int p = 0; p < n; ++p) {
      const int32_t *q = quads + 8 * p;
      for (int s : {0, 2, 4})
        if (q[s] < 0 || q[s] >= ctx->N) return ctx->fail(FP4_E_INVAL, "q index out of range");
      for (int s : {1, 3, 5, 6})
        if (q[s] < 0 || q[s] >= ctx->nb) return ctx->fail(FP4_E_INVAL, "branch index out of range");
      if (q[7] < 0 || q[7] > 2) return ctx->fail(FP4_E_INVAL, "channel must be 0, 1 or 2");
    }
    (void)hipSetDevice(ctx->device);
    int rc;
    if ((rc = ensure_tables(ctx))) return rc;
    // distinct targets -> slots of the precontraction buffer
    std::map<int, int> slot;
    std::vector<int> tl, ts(n);
    for (int p = 0; p < n; ++p) {
      const int mu = quads[8 * p] * ctx->nb + quads[8 * p + 1];
      auto it = slot.find(mu);
      if (it == slot.end()) {
        it = slot.emplace(mu, (int)tl.size()).first;
        tl.push_back(mu);
      }
      ts[p] = it->second;
    }
    const int fp32 = precision == FP4_FP32;
    const size_t cb = fp32 ? sizeof(float2) : sizeof(double2);
    if ((rc = upload(ctx, ctx->d_targets, tl.data(), tl.size()))) return rc;
    if ((rc = upload(ctx, ctx->d_quads, quads, (size_t)8 * n))) return rc;
    if ((rc = upload(ctx, ctx->d_tslot, ts.data(), ts.size()))) return rc;
    if ((rc = ensure(ctx, ctx->d_U, tl.size() * ctx->nc * 27 * cb))) return rc;
    if ((rc = ensure(ctx, ctx->d_V, (size_t)n * sizeof(double2)))) return rc;
    fp4::Crystal c = make_crystal(ctx);
    FP4_HIP(ctx, fp4::launch_precontract(c, (const int *)ctx->d_targets.p, (int)tl.size(), fp32, ctx->d_U.p, ctx->stream));
    FP4_HIP(ctx, fp4::launch_debug_v(c, (const int *)ctx->d_quads.p, n, (const int *)ctx->d_tslot.p, ctx->d_U.p, fp32, (double2 *)ctx->d_V.p, ctx->stream));
    FP4_HIP(ctx, hipMemcpyAsync(V, ctx->d_V.p, (size_t)n * sizeof(double2), hipMemcpyDeviceToHost, ctx->stream));
    FP4_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->err.clear();
    return FP4_OK;
  } catch (const std::bad_alloc &) {
    return ctx->fail(FP4_E_NOMEM, "host allocation failed");
  }
}

int fp4_load_fc3(fp4_ctx *ctx, int32_t ntrip, const int32_t *atoms, const int32_t *cells,
                 const double *phi) {
  if (!ctx) return FP4_E_INVAL;
  try {
    if (!ctx->have_lattice) return ctx->fail(FP4_E_STATE, "fp4_load_lattice must come first");
    if (ntrip < 1 || ntrip > (1 << 16)) return ctx->fail(FP4_E_INVAL, "need 1 <= ntrip <= 2^16");
    if (!atoms || !cells || !phi) return ctx->fail(FP4_E_INVAL, "null pointer argument");
    for (int i = 0; i < 3 * ntrip; ++i)
      if (atoms[i] < 0 || atoms[i] >= ctx->nat) return ctx->fail(FP4_E_INVAL, "triplet atom index out of range");
    for (int i = 0; i < 6 * ntrip; ++i)
      if (cells[i] < -64 || cells[i] > 64) return ctx->fail(FP4_E_INVAL, "triplet cell coordinate outside [-64, 64]");
    if (!finite_all(phi, (size_t)27 * ntrip)) return ctx->fail(FP4_E_INVAL, "force constants contain NaN or Inf");
    using V3 = std::array<int, 3>;
    std::map<V3, int> dmap, rmap;
    auto intern = [](std::map<V3, int> &m, const V3 &v) {
      auto it = m.find(v);
      if (it != m.end()) return it->second;
      const int id = (int)m.size();
      m.emplace(v, id);
      return id;
    };
    struct T3 {
      int i, j, k, d, rk, n;
    };
    std::vector<T3> ts(ntrip);
    for (int n = 0; n < ntrip; ++n) {
      const int32_t *at = atoms + 3 * n, *cl = cells + 6 * n;
      const V3 d{cl[0] - cl[3], cl[1] - cl[4], cl[2] - cl[5]};
      const V3 rk{cl[3], cl[4], cl[5]};
      ts[n] = T3{at[0], at[1], at[2], intern(dmap, d), intern(rmap, rk), n};
    }
    std::sort(ts.begin(), ts.end(), [](const T3 &x, const T3 &y) {
      return std::tie(x.j, x.k, x.d, x.i, x.rk, x.n) < std::tie(y.j, y.k, y.d, y.i, y.rk, y.n);
    });
    const int nat = ctx->nat;
    ctx->n3 = ntrip;
    ctx->jk3_start.assign(nat * nat + 1, 0);
    ctx->t3_i.resize(ntrip);
    ctx->t3_d.resize(ntrip);
    ctx->t3_rk.resize(ntrip);
    ctx->t3_phi.resize((size_t)27 * ntrip);
    for (int p = 0; p < ntrip; ++p) {
      ctx->t3_i[p] = ts[p].i;
      ctx->t3_d[p] = ts[p].d;
      ctx->t3_rk[p] = ts[p].rk;
      std::memcpy(&ctx->t3_phi[(size_t)27 * p], phi + (size_t)27 * ts[p].n, 27 * sizeof(double));
    }
    // jk3_start[jk] = first triplet whose pair index j*nat + k is >= jk
    for (int jk = 0, p = 0; jk <= nat * nat; ++jk) {
      while (p < ntrip && ts[p].j * nat + ts[p].k < jk) ++p;
      ctx->jk3_start[jk] = p;
    }
    auto flat = [](const std::map<V3, int> &m) {
      std::vector<int> v(3 * m.size());
      for (auto &kv : m)
        for (int x = 0; x < 3; ++x) v[3 * kv.second + x] = kv.first[x];
      return v;
    };
    ctx->d3vec = flat(dmap);
    ctx->rk3vec = flat(rmap);
    ctx->nd3 = (int)dmap.size();
    ctx->nrk3 = (int)rmap.size();
    (void)hipSetDevice(ctx->device);
    int rc;
    if ((rc = upload(ctx, ctx->d3_jk, ctx->jk3_start.data(), ctx->jk3_start.size()))) return rc;
    if ((rc = upload(ctx, ctx->d3_ti, ctx->t3_i.data(), ctx->t3_i.size()))) return rc;
    if ((rc = upload(ctx, ctx->d3_td, ctx->t3_d.data(), ctx->t3_d.size()))) return rc;
    if ((rc = upload(ctx, ctx->d3_trk, ctx->t3_rk.data(), ctx->t3_rk.size()))) return rc;
    if ((rc = upload(ctx, ctx->d3_phi, ctx->t3_phi.data(), ctx->t3_phi.size()))) return rc;
    if ((rc = upload(ctx, ctx->d3_dv, ctx->d3vec.data(), ctx->d3vec.size()))) return rc;
    if ((rc = upload(ctx, ctx->d3_rkv, ctx->rk3vec.data(), ctx->rk3vec.size()))) return rc;
    FP4_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->have_fc3 = true;
    ctx->tables3_dirty = true;
    ctx->err.clear();
    return FP4_OK;
  } catch (const std::bad_alloc &) {
    return ctx->fail(FP4_E_NOMEM, "host allocation failed");
  }
}

}  // extern "C"

namespace {

// Checks shared by the three-phonon rate and the feature builder; fills the target list.
int rates3_args(fp4_ctx *ctx, const double *T, int32_t nT, double scalebroad,
                const int32_t *targets, int32_t ntargets, std::vector<int> &tl) {
  if (!ctx->have_lattice || !ctx->have_modes || !ctx->have_fc3)
    return ctx->fail(FP4_E_STATE, "the three-phonon rate needs fp4_load_lattice, fp4_load_modes and fp4_load_fc3");
  if (!T || nT < 1 || nT > 8) return ctx->fail(FP4_E_INVAL, "need 1 <= nT <= 8 temperatures");
  for (int i = 0; i < nT; ++i)
    if (!(std::isfinite(T[i]) && T[i] > 0.0)) return ctx->fail(FP4_E_INVAL, "temperatures must be finite and > 0");
  if (!(std::isfinite(scalebroad) && scalebroad > 0.0)) return ctx->fail(FP4_E_INVAL, "scalebroad must be finite and > 0");
  const int nmodes = ctx->N * ctx->nb;
  if (targets) {
    if (ntargets < 1 || ntargets > nmodes) return ctx->fail(FP4_E_INVAL, "need 1 <= ntargets <= nq*nb");
    tl.assign(targets, targets + ntargets);
    for (int v : tl)
      if (v < 0 || v >= nmodes) return ctx->fail(FP4_E_INVAL, "target mode id out of range");
  } else {
    tl.resize(nmodes);
    for (int i = 0; i < nmodes; ++i) tl[i] = i;
  }
  return FP4_OK;
}

// Enqueue the three-phonon rates of the targets tl on the context stream: device outputs
// d3_rates [nT][nt], d3_counts [nt][2]; occupations left in d_occ, temperatures in d_T.
int enqueue_rates3(fp4_ctx *ctx, const double *T, int nT, double scalebroad,
                   const std::vector<int> &tl) {
  const int nmodes = ctx->N * ctx->nb;
  const int nt = (int)tl.size();
  int rc;
  if ((rc = ensure_tables(ctx))) return rc;
  if (ctx->tables3_dirty) {
    if ((rc = ensure(ctx, ctx->d3_PH3, (size_t)ctx->nd3 * ctx->N * sizeof(double2)))) return rc;
    fp4::Crystal c0 = make_crystal(ctx);
    FP4_HIP(ctx, fp4::launch_tables3(c0, (const int *)ctx->d3_dv.p, ctx->nd3, (double2 *)ctx->d3_PH3.p, ctx->stream));
    ctx->tables3_dirty = false;
  }
  if ((rc = upload(ctx, ctx->d3_targets, tl.data(), tl.size()))) return rc;
  if ((rc = upload(ctx, ctx->d_T, T, (size_t)nT))) return rc;
  if ((rc = ensure(ctx, ctx->d_occ, (size_t)nmodes * nT * sizeof(double)))) return rc;
  if ((rc = ensure(ctx, ctx->d_iocc, (size_t)nmodes * nT * sizeof(double)))) return rc;
  if ((rc = ensure(ctx, ctx->d3_rates, (size_t)nT * nt * sizeof(double)))) return rc;
  if ((rc = ensure(ctx, ctx->d3_counts, (size_t)nt * 2 * sizeof(long long)))) return rc;
  fp4::Crystal c = make_crystal(ctx);
  FP4_HIP(ctx, fp4::launch_occupations(c, (const double *)ctx->d_T.p, nT, hbar_over_kb_kps(),
                                       (double *)ctx->d_occ.p, (double *)ctx->d_iocc.p, ctx->stream));
  fp4::Fc3Dev f{};
  f.n3 = ctx->n3;
  f.nd3 = ctx->nd3;
  f.nrk = ctx->nrk3;
  f.jk_start = (const int *)ctx->d3_jk.p;
  f.t_i = (const int *)ctx->d3_ti.p;
  f.t_d = (const int *)ctx->d3_td.p;
  f.t_rk = (const int *)ctx->d3_trk.p;
  f.t_phi = (const double *)ctx->d3_phi.p;
  f.rk_vec = (const int *)ctx->d3_rkv.p;
  f.PH3 = (const double2 *)ctx->d3_PH3.p;
  fp4::Rate3Args a{};
  const double wsb = ctx->window_w * scalebroad;
  a.c_win = (wsb * ctx->dq) * (wsb * ctx->dq);
  a.c_sig = (scalebroad * ctx->dq) * (scalebroad * ctx->dq);
  a.c_min = ctx->sigma_min * ctx->sigma_min;
  a.kpref = c3_prefactor() / (double)ctx->N;
  a.nT = nT;
  a.occ = (const double *)ctx->d_occ.p;
  a.targets = (const int *)ctx->d3_targets.p;
  a.nt_total = nt;
  a.rates = (double *)ctx->d3_rates.p;
  a.counts = (long long *)ctx->d3_counts.p;
  const size_t per_target = (size_t)ctx->n3 * 9 * sizeof(double2);
  const int batch = (int)std::max<size_t>(1, std::min<size_t>((size_t)nt, ((size_t)256 << 20) / per_target));
  if ((rc = ensure(ctx, ctx->d3_U, (size_t)batch * per_target))) return rc;
  for (int t0 = 0; t0 < nt; t0 += batch) {
    const int nbt = std::min(batch, nt - t0);
    FP4_HIP(ctx, fp4::launch_precontract3(c, f, (const int *)ctx->d3_targets.p + t0, nbt,
                                          (double2 *)ctx->d3_U.p, ctx->stream));
    a.t0 = t0;
    FP4_HIP(ctx, fp4::launch_rates3(c, f, a, (const double2 *)ctx->d3_U.p, nbt, ctx->stream));
  }
  return FP4_OK;
}

}  // namespace

extern "C" {

int fp4_compute_rates3(fp4_ctx *ctx, const double *T, int32_t nT, double scalebroad,
                       const int32_t *targets, int32_t ntargets, double *rates,
                       int64_t *counts) {
  if (!ctx) return FP4_E_INVAL;
  try {
    std::vector<int> tl;
    int rc = rates3_args(ctx, T, nT, scalebroad, targets, ntargets, tl);
    if (rc) return rc;
    if (!rates) return ctx->fail(FP4_E_INVAL, "rates output is required");
    (void)hipSetDevice(ctx->device);
    const int nt = (int)tl.size();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->profile) {
      e0 = pool_event(ctx, 0);
      e1 = pool_event(ctx, 1);
      if (!e0 || !e1) return ctx->fail(FP4_E_DEVICE, "hipEventCreate failed");
      FP4_HIP(ctx, hipEventRecord(e0, ctx->stream));
    }
    if ((rc = enqueue_rates3(ctx, T, nT, scalebroad, tl))) return rc;
    if (ctx->profile) FP4_HIP(ctx, hipEventRecord(e1, ctx->stream));
    FP4_HIP(ctx, hipMemcpyAsync(rates, ctx->d3_rates.p, (size_t)nT * nt * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    if (counts)
      FP4_HIP(ctx, hipMemcpyAsync(counts, ctx->d3_counts.p, (size_t)nt * 2 * sizeof(long long), hipMemcpyDeviceToHost, ctx->stream));
    FP4_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->profile) {
      float ms = 0.f;
      FP4_HIP(ctx, hipEventElapsedTime(&ms, e0, e1));
      ctx->ms_main = ms;
      ctx->ms_total = ms;
    }
    ctx->err.clear();
    return FP4_OK;
  } catch (const std::bad_alloc &) {
    return ctx->fail(FP4_E_NOMEM, "host allocation failed");
  }
}

int fp4_surrogate_features(fp4_ctx *ctx, const double *T, int32_t nT, double scalebroad,
                           const int32_t *targets, int32_t ntargets, const float *shift,
                           const float *scale, float *X, double *rates3) {
  if (!ctx) return FP4_E_INVAL;
  try {
    std::vector<int> tl;
    int rc = rates3_args(ctx, T, nT, scalebroad, targets, ntargets, tl);
    if (rc) return rc;
    if (!ctx->have_fc4) return ctx->fail(FP4_E_STATE, "the surrogate features need fp4_load_fc4");
    if (!X) return ctx->fail(FP4_E_INVAL, "X output is required");
    if ((shift == nullptr) != (scale == nullptr)) return ctx->fail(FP4_E_INVAL, "give both shift and scale, or neither");
    if (shift) {
      for (int k = 0; k < FP4_NFEAT; ++k)
        if (!std::isfinite(shift[k]) || !std::isfinite(scale[k])) return ctx->fail(FP4_E_INVAL, "shift and scale must be finite");
    }
    (void)hipSetDevice(ctx->device);
    const int nt = (int)tl.size();
    if ((rc = enqueue_rates3(ctx, T, nT, scalebroad, tl))) return rc;
    if ((rc = ensure(ctx, ctx->df_g4, (size_t)nt * sizeof(double)))) return rc;
    if ((rc = ensure(ctx, ctx->df_X, (size_t)nT * nt * FP4_NFEAT * sizeof(float)))) return rc;
    float *d_shift = nullptr, *d_scale = nullptr;
    if (shift) {
      std::vector<float> ss(2 * FP4_NFEAT);
      std::memcpy(ss.data(), shift, FP4_NFEAT * sizeof(float));
      std::memcpy(ss.data() + FP4_NFEAT, scale, FP4_NFEAT * sizeof(float));
      if ((rc = upload(ctx, ctx->df_shift, ss.data(), ss.size()))) return rc;
      d_shift = (float *)ctx->df_shift.p;
      d_scale = d_shift + FP4_NFEAT;
    }
    fp4::Crystal c = make_crystal(ctx);
    FP4_HIP(ctx, fp4::launch_fc4_strength(c, (const int *)ctx->d3_targets.p, nt, (double *)ctx->df_g4.p, ctx->stream));
    FP4_HIP(ctx, fp4::launch_features(c, (const int *)ctx->d3_targets.p, nt, (const double *)ctx->d_T.p, nT,
                                      (const double *)ctx->d_occ.p, (const double *)ctx->d3_rates.p,
                                      (const double *)ctx->df_g4.p, d_shift, d_scale,
                                      (float *)ctx->df_X.p, ctx->stream));
    FP4_HIP(ctx, hipMemcpyAsync(X, ctx->df_X.p, (size_t)nT * nt * FP4_NFEAT * sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
    if (rates3)
      FP4_HIP(ctx, hipMemcpyAsync(rates3, ctx->d3_rates.p, (size_t)nT * nt * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    FP4_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->err.clear();
    return FP4_OK;
  } catch (const std::bad_alloc &) {
    return ctx->fail(FP4_E_NOMEM, "host allocation failed");
  }
}

int fp4_compute_kappa_rta(fp4_ctx *ctx, const double *T, int32_t nT, double scalebroad,
                          int32_t precision, double *kappa, int64_t *nskip, double *rates3,
                          double *rates4) {
  if (!ctx) return FP4_E_INVAL;
  try {
    std::vector<int> tl;
    int rc = rates3_args(ctx, T, nT, scalebroad, nullptr, 0, tl);
    if (rc) return rc;
    if ((rc = check_compute_args(ctx, T, nT, scalebroad, 7u, precision))) return rc;
    if (ctx->harmonic || ctx->qclass)
      return ctx->fail(FP4_E_UNSUPPORTED, "the conductivity needs the full rates (FP4_PARAM_PHASE_SPACE and FP4_PARAM_QCLASS must be 0)");
    if (!kappa) return ctx->fail(FP4_E_INVAL, "kappa output is required");
    (void)hipSetDevice(ctx->device);
    const int nt = (int)tl.size();
    // four-phonon rates of every mode (all channels) into d_rates, three-phonon into d3_rates
    if ((rc = upload(ctx, ctx->d_targets, tl.data(), tl.size()))) return rc;
    if ((rc = ensure(ctx, ctx->d_rates, (size_t)nT * nt * sizeof(double)))) return rc;
    if ((rc = ensure(ctx, ctx->d_counts, (size_t)nt * 3 * sizeof(long long)))) return rc;
    if ((rc = enqueue(ctx, T, nT, scalebroad, 7u, precision, nt, ctx->stream, (double *)ctx->d_rates.p,
                      nullptr, (long long *)ctx->d_counts.p, nullptr, nullptr)))
      return rc;
    if ((rc = enqueue_rates3(ctx, T, nT, scalebroad, tl))) return rc;
    if ((rc = ensure(ctx, ctx->d_kappa, (size_t)nT * 10 * sizeof(double)))) return rc;
    double *d_k = (double *)ctx->d_kappa.p;
    long long *d_skip = (long long *)(d_k + (size_t)nT * 9);
    const double *a = ctx->A;
    const double vol = std::fabs(a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                                 a[2] * (a[3] * a[7] - a[4] * a[6])) * 1e-30;   // m^3
    const double scale = 1.0 / ((double)ctx->N * vol);
    fp4::Crystal c = make_crystal(ctx);
    FP4_HIP(ctx, fp4::launch_kappa(c, (const double *)ctx->d_T.p, nT, hbar_over_kb_kps(),
                                   (const double *)ctx->d_occ.p, (const double *)ctx->d3_rates.p,
                                   (const double *)ctx->d_rates.p, scale, kKB, d_k, d_skip, ctx->stream));
    FP4_HIP(ctx, hipMemcpyAsync(kappa, d_k, (size_t)nT * 9 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    std::vector<long long> sk(nT);
    FP4_HIP(ctx, hipMemcpyAsync(sk.data(), d_skip, (size_t)nT * sizeof(long long), hipMemcpyDeviceToHost, ctx->stream));
    if (rates3)
      FP4_HIP(ctx, hipMemcpyAsync(rates3, ctx->d3_rates.p, (size_t)nT * nt * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    if (rates4)
      FP4_HIP(ctx, hipMemcpyAsync(rates4, ctx->d_rates.p, (size_t)nT * nt * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    FP4_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (nskip)
      for (int t = 0; t < nT; ++t) nskip[t] = sk[t];
    ctx->err.clear();
    return FP4_OK;
  } catch (const std::bad_alloc &) {
    return ctx->fail(FP4_E_NOMEM, "host allocation failed");
  }
}

int fp4_probe_matrix_rates(int32_t device_id, double *tflops) {
  if (!tflops) return FP4_E_INVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device_id < 0 || device_id >= ndev) {
    (void)hipGetLastError();
    return FP4_E_DEVICE;
  }
  if (hipSetDevice(device_id) != hipSuccess) return FP4_E_DEVICE;
  double *out = nullptr;
  if (hipMalloc(&out, fp4::probe_out_doubles() * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    return FP4_E_NOMEM;
  }
  for (int i = 0; i < 6; ++i) tflops[i] = 0.0;
  const hipError_t e = fp4::run_probe(out, tflops, nullptr);
  (void)hipFree(out);
  return e == hipSuccess ? FP4_OK : FP4_E_DEVICE;
}

int fp4_last_stats(const fp4_ctx *ctx, int64_t *processes, int64_t *candidates, int64_t *blocks) {
  if (!ctx) return FP4_E_INVAL;
  if (processes) *processes = ctx->st_processes;
  if (candidates) *candidates = ctx->st_candidates;
  if (blocks) *blocks = ctx->st_blocks;
  return FP4_OK;
}

int fp4_last_timing(const fp4_ctx *ctx, double *ms_main, double *ms_total) {
  if (!ctx) return FP4_E_INVAL;
  if (ms_main) *ms_main = ctx->ms_main;
  if (ms_total) *ms_total = ctx->ms_total;
  return FP4_OK;
}

}  // extern "C"

// ====================================================================== batched instances

struct fp4_batch {
  int device = 0;
  hipStream_t stream = nullptr;
  std::vector<fp4_ctx *> ctxs;
  std::string err;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::string key;
  DevBuf d_inst[4];       // instance tables of the branch-count classes nb = 3, 6, 9, 12
  DevBuf d_counter;       // work queue counters, kClassCounters per class
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double ms_last = 0.0;
  long long graph_builds = 0, graph_launches = 0;
  int fail(int code, const std::string &msg) {
    err = msg;
    return code;
  }
};

namespace {

// Eager preparation of one crystal for the persistent kernel: tables, temperatures, target
// list, buffers; fills the instance descriptor (no kernel is enqueued here).
int prepare_instance(fp4_ctx *ctx, const double *T, int nT, double sb, uint32_t mask,
                     int precision, const std::vector<int> &targets, int qchunk,
                     fp4::BatchInst *out) {
  int rc;
  const int fp32 = precision == FP4_FP32;
  const size_t nmodes = (size_t)ctx->N * ctx->nb;
  const int nt = (int)targets.size();
  if ((rc = ensure_tables(ctx))) return rc;
  if ((rc = upload(ctx, ctx->d_T, T, (size_t)nT))) return rc;
  if ((rc = upload(ctx, ctx->d_targets, targets.data(), targets.size()))) return rc;
  FP4_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if ((rc = ensure(ctx, ctx->d_occ, nmodes * nT * sizeof(double)))) return rc;
  if ((rc = ensure(ctx, ctx->d_iocc, nmodes * nT * sizeof(double)))) return rc;
  if (qchunk < 1) qchunk = 1;
  if (qchunk > ctx->N) qchunk = ctx->N;
  const int nchunk = (ctx->N + qchunk - 1) / qchunk;
  const size_t cb = fp32 ? sizeof(float2) : sizeof(double2);
  if ((rc = ensure(ctx, ctx->d_U, (size_t)nt * ctx->nc * 27 * cb))) return rc;
  if ((rc = ensure(ctx, ctx->d_partial, (size_t)nt * nchunk * 3 * nT * sizeof(double)))) return rc;
  if ((rc = ensure(ctx, ctx->d_pcount, (size_t)nt * nchunk * 3 * sizeof(unsigned long long)))) return rc;
  if ((rc = ensure(ctx, ctx->d_blocks, sizeof(unsigned long long)))) return rc;
  if ((rc = ensure(ctx, ctx->d_rates, (size_t)nT * nt * sizeof(double)))) return rc;
  if ((rc = ensure(ctx, ctx->d_counts, (size_t)nt * 3 * sizeof(long long)))) return rc;
  fp4::RateArgs a{};
  const double wsb = ctx->window_w * sb;
  a.c_win = (wsb * ctx->dq) * (wsb * ctx->dq);
  a.sqrt_c_win = wsb * ctx->dq;
  a.c_sig = (sb * ctx->dq) * (sb * ctx->dq);
  a.c_min = ctx->sigma_min * ctx->sigma_min;
  a.kpref = (ctx->harmonic ? 1.0 : c4_prefactor()) / ((double)ctx->N * (double)ctx->N);
  a.harmonic = ctx->harmonic;
  a.mirror = ctx->sym34 ? 1 : 0;
  a.nT = nT;
  a.mask = mask;
  a.qclass = ctx->qclass;
  a.occ = (const double *)ctx->d_occ.p;
  a.inv_occ = (const double *)ctx->d_iocc.p;
  a.targets = (const int *)ctx->d_targets.p;
  a.nt = nt;
  a.t0 = 0;
  a.qchunk = qchunk;
  a.qseg = ctx->qseg;
  a.lseg = ctx->lseg;
  a.nchunk = nchunk;
  a.nxcd = kXcds;
  a.U = ctx->d_U.p;
  a.partial = (double *)ctx->d_partial.p;
  a.pcount = (unsigned long long *)ctx->d_pcount.p;
  a.blocks = (unsigned long long *)ctx->d_blocks.p;
  out->c = make_crystal(ctx);
  out->a = a;
  out->item0 = 0;
  return FP4_OK;
}

int nb_class(int nb) { return nb / 3 - 1; }

// estimated relative cost of one item (one target, one q'-chunk): blocks x block cost
double item_cost(const fp4::BatchInst &b) {
  const double nb = b.c.nb;
  return (double)b.a.qchunk * nb * b.c.N * (9.0 * b.c.ng + 2.0 * nb * nb * nb);
}

// Enqueue the whole batched computation on stream s: per instance occupations and
// precontraction, counter reset, one persistent kernel per branch-count class, per
// instance ordered reduction.  Also used inside stream capture.
int enqueue_batch(fp4_batch *b, std::vector<fp4::BatchInst> (&cls)[4], int fp32, int nT,
                  const std::vector<fp4_ctx *> &ctxs, const std::vector<fp4::BatchInst> &insts,
                  hipStream_t s) {
  for (size_t i = 0; i < ctxs.size(); ++i) {
    fp4_ctx *ctx = ctxs[i];
    const fp4::BatchInst &bi = insts[i];
    FP4_HIP(b, fp4::launch_occupations(bi.c, (const double *)ctx->d_T.p, nT, hbar_over_kb_kps(),
                                       (double *)ctx->d_occ.p, (double *)ctx->d_iocc.p, s));
    FP4_HIP(b, fp4::launch_precontract(bi.c, bi.a.targets, bi.a.nt, fp32, ctx->d_U.p, s));
    FP4_HIP(b, fp4::launch_zero(ctx->d_blocks.p, sizeof(unsigned long long), s));
  }
  FP4_HIP(b, fp4::launch_zero(b->d_counter.p, 4 * fp4::kClassCounters * sizeof(unsigned long long), s));
  for (int k = 0; k < 4; ++k) {
    if (cls[k].empty()) continue;
    long long total = 0;
    size_t lds = 0;
    for (auto &bi : cls[k]) {
      total = std::max(total, bi.item0 + (long long)bi.a.nt * bi.a.nchunk);
      lds = std::max(lds, fp4::batch_lds_bytes(bi.c, fp32, nT, bi.a.qseg, bi.a.lseg));
    }
    hipError_t e = fp4::launch_batch((const fp4::BatchInst *)b->d_inst[k].p, (int)cls[k].size(), total,
                                     (unsigned long long *)b->d_counter.p + (size_t)k * fp4::kClassCounters, lds, fp32,
                                     3 * (k + 1), nT, nullptr, s);
    if (e == hipErrorInvalidValue)
      return b->fail(FP4_E_UNSUPPORTED, "an instance needs more LDS than a work-group has");
    FP4_HIP(b, e);
  }
  for (size_t i = 0; i < ctxs.size(); ++i) {
    fp4_ctx *ctx = ctxs[i];
    const fp4::BatchInst &bi = insts[i];
    FP4_HIP(b, fp4::launch_reduce(bi.a, bi.a.nt, (double *)ctx->d_rates.p, nullptr,
                                  (long long *)ctx->d_counts.p, s));
  }
  return FP4_OK;
}

// Prepare every instance, order the items of each class by cost per item, upload the
// instance tables.
int build_classes(fp4_batch *b, const std::vector<fp4_ctx *> &ctxs,
                  const std::vector<std::vector<int>> &targets, const double *T, int nT,
                  double sb, uint32_t mask, int precision, const std::vector<int> &qchunks,
                  std::vector<fp4::BatchInst> &insts, std::vector<fp4::BatchInst> (&cls)[4]) {
  insts.assign(ctxs.size(), fp4::BatchInst{});
  for (int k = 0; k < 4; ++k) cls[k].clear();
  for (size_t i = 0; i < ctxs.size(); ++i) {
    int rc = prepare_instance(ctxs[i], T, nT, sb, mask, precision, targets[i], qchunks[i], &insts[i]);
    if (rc) return b->fail(rc, std::string("instance ") + std::to_string(i) + ": " + ctxs[i]->err);
  }
  std::vector<size_t> order(ctxs.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](size_t x, size_t y) { return item_cost(insts[x]) > item_cost(insts[y]); });
  for (size_t o : order) {
    const int k = nb_class(insts[o].c.nb);
    long long item0 = 0;
    if (!cls[k].empty()) item0 = cls[k].back().item0 + (long long)cls[k].back().a.nt * cls[k].back().a.nchunk;
    insts[o].item0 = item0;
    cls[k].push_back(insts[o]);
  }
  int rc;
  if ((rc = ensure(ctxs[0], b->d_counter, 4 * fp4::kClassCounters * sizeof(unsigned long long)))) return b->fail(rc, ctxs[0]->err);
  for (int k = 0; k < 4; ++k) {
    if (cls[k].empty()) continue;
    if ((rc = ensure(ctxs[0], b->d_inst[k], cls[k].size() * sizeof(fp4::BatchInst)))) return b->fail(rc, ctxs[0]->err);
    FP4_HIP(b, hipMemcpy(b->d_inst[k].p, cls[k].data(), cls[k].size() * sizeof(fp4::BatchInst), hipMemcpyHostToDevice));
  }
  return FP4_OK;
}

}  // namespace

extern "C" {

int fp4_batch_create(fp4_batch **out, int device_id) {
  if (!out) return FP4_E_INVAL;
  *out = nullptr;
  fp4_batch *b = new (std::nothrow) fp4_batch();
  if (!b) return FP4_E_NOMEM;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device_id < 0 || device_id >= ndev ||
      hipSetDevice(device_id) != hipSuccess || hipStreamCreate(&b->stream) != hipSuccess ||
      hipEventCreate(&b->ev0) != hipSuccess || hipEventCreate(&b->ev1) != hipSuccess) {
    (void)hipGetLastError();
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return FP4_E_DEVICE;
  }
  b->device = device_id;
  *out = b;
  return FP4_OK;
}

void fp4_batch_destroy(fp4_batch *b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  (void)hipStreamSynchronize(b->stream);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (auto &d : b->d_inst) release(d);
  release(b->d_counter);
  if (b->ev0) (void)hipEventDestroy(b->ev0);
  if (b->ev1) (void)hipEventDestroy(b->ev1);
  (void)hipStreamDestroy(b->stream);
  delete b;
}

const char *fp4_batch_last_error(const fp4_batch *b) { return b ? b->err.c_str() : "null batch"; }

int fp4_batch_add(fp4_batch *b, fp4_ctx *ctx) {
  if (!b) return FP4_E_INVAL;
  if (!ctx) return b->fail(FP4_E_INVAL, "null context");
  if (ctx->device != b->device) return b->fail(FP4_E_INVAL, "context is on another device");
  if (!ctx->have_lattice || !ctx->have_modes || !ctx->have_fc4)
    return b->fail(FP4_E_STATE, "context is not fully loaded");
  if (b->ctxs.size() >= 64) return b->fail(FP4_E_UNSUPPORTED, "at most 64 instances per batch");
  for (fp4_ctx *c : b->ctxs)
    if (c == ctx) return b->fail(FP4_E_INVAL, "context already in the batch");
  b->ctxs.push_back(ctx);
  b->key.clear();
  return FP4_OK;
}

int fp4_batch_compute(fp4_batch *b, const double *T, int32_t nT, double scalebroad, uint32_t mask,
                      int32_t precision, double *rates, int64_t *counts) {
  if (!b) return FP4_E_INVAL;
  try {
    if (b->ctxs.empty()) return b->fail(FP4_E_STATE, "empty batch");
    if (!rates) return b->fail(FP4_E_INVAL, "rates output is required");
    if (nT > 4) return b->fail(FP4_E_UNSUPPORTED, "a batch takes at most 4 temperatures");
    for (fp4_ctx *ctx : b->ctxs) {
      const int rc = check_compute_args(ctx, T, nT, scalebroad, mask, precision);
      if (rc) return b->fail(rc, ctx->err);
    }
    (void)hipSetDevice(b->device);
    const int fp32 = precision == FP4_FP32;
    std::vector<std::vector<int>> targets(b->ctxs.size());
    std::vector<int> qchunks(b->ctxs.size());
    for (size_t i = 0; i < b->ctxs.size(); ++i) {
      const int nm = b->ctxs[i]->N * b->ctxs[i]->nb;
      targets[i].resize(nm);
      for (int m = 0; m < nm; ++m) targets[i][m] = m;
      qchunks[i] = b->ctxs[i]->qchunk > 0 ? b->ctxs[i]->qchunk : auto_qchunk(b->ctxs[i], nm, nT);
    }
    std::vector<fp4::BatchInst> insts;
    std::vector<fp4::BatchInst> cls[4];
    int rc = build_classes(b, b->ctxs, targets, T, nT, scalebroad, mask, precision, qchunks, insts, cls);
    if (rc) return rc;
    // graph signature: every device pointer and size the captured work uses
    std::string key = std::to_string(nT) + "/" + std::to_string(fp32);
    for (int k = 0; k < 4; ++k)
      for (auto &bi : cls[k]) {
        const unsigned char *p = reinterpret_cast<const unsigned char *>(&bi);
        key.append(reinterpret_cast<const char *>(p), sizeof(bi));
      }
    for (fp4_ctx *ctx : b->ctxs) {
      const void *ps[] = {ctx->d_T.p, ctx->d_U.p, ctx->d_rates.p, ctx->d_counts.p, ctx->d_blocks.p};
      key.append(reinterpret_cast<const char *>(ps), sizeof(ps));
    }
    if (key != b->key || !b->exec) {
      if (b->exec) (void)hipGraphExecDestroy(b->exec);
      if (b->graph) (void)hipGraphDestroy(b->graph);
      b->exec = nullptr;
      b->graph = nullptr;
      FP4_HIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed));
      rc = enqueue_batch(b, cls, fp32, nT, b->ctxs, insts, b->stream);
      hipGraph_t g = nullptr;
      const hipError_t ee = hipStreamEndCapture(b->stream, &g);
      if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      FP4_HIP(b, ee);
      b->graph = g;
      FP4_HIP(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
      b->key = key;
      b->graph_builds++;
    }
    FP4_HIP(b, hipEventRecord(b->ev0, b->stream));
    FP4_HIP(b, hipGraphLaunch(b->exec, b->stream));
    FP4_HIP(b, hipEventRecord(b->ev1, b->stream));
    b->graph_launches++;
    size_t off_r = 0, off_c = 0;
    for (size_t i = 0; i < b->ctxs.size(); ++i) {
      fp4_ctx *ctx = b->ctxs[i];
      const size_t nm = (size_t)ctx->N * ctx->nb;
      // rates of instance i: [nT][nm] at offset sum of nT*nm of the previous instances
      FP4_HIP(b, hipMemcpyAsync(rates + off_r, ctx->d_rates.p, (size_t)nT * nm * sizeof(double), hipMemcpyDeviceToHost, b->stream));
      if (counts)
        FP4_HIP(b, hipMemcpyAsync(counts + off_c, ctx->d_counts.p, nm * 3 * sizeof(long long), hipMemcpyDeviceToHost, b->stream));
      off_r += (size_t)nT * nm;
      off_c += nm * 3;
    }
    FP4_HIP(b, hipStreamSynchronize(b->stream));
    float ms = 0.f;
    FP4_HIP(b, hipEventElapsedTime(&ms, b->ev0, b->ev1));
    b->ms_last = ms;
    b->err.clear();
    return FP4_OK;
  } catch (const std::bad_alloc &) {
    return b->fail(FP4_E_NOMEM, "host allocation failed");
  }
}

int fp4_batch_last_timing(const fp4_batch *b, double *ms_graph, int64_t *graph_builds,
                          int64_t *graph_launches) {
  if (!b) return FP4_E_INVAL;
  if (ms_graph) *ms_graph = b->ms_last;
  if (graph_builds) *graph_builds = b->graph_builds;
  if (graph_launches) *graph_launches = b->graph_launches;
  return FP4_OK;
}

}  // extern "C"

namespace {

// Device time (ms) of the persistent rate pipeline on the sample targets with the given
// q'-chunk, queue segment and list segment (one untimed pass first).
int time_config(fp4_ctx *ctx, fp4_batch *b, const std::vector<int> &sample, const double *T,
                int nT, double sb, uint32_t mask, int precision, int qchunk, int qseg, int lseg,
                bool warm, float *ms) {
  const int keep_qs = ctx->qseg, keep_ls = ctx->lseg;
  ctx->qseg = qseg;
  ctx->lseg = lseg;
  std::vector<fp4::BatchInst> insts;
  std::vector<fp4::BatchInst> cls[4];
  std::vector<fp4_ctx *> one{ctx};
  int rc = build_classes(b, one, {sample}, T, nT, sb, mask, precision, {qchunk}, insts, cls);
  if (!rc && warm) rc = enqueue_batch(b, cls, precision == FP4_FP32, nT, one, insts, b->stream);
  if (!rc && hipEventRecord(b->ev0, b->stream) != hipSuccess) rc = FP4_E_DEVICE;
  if (!rc) rc = enqueue_batch(b, cls, precision == FP4_FP32, nT, one, insts, b->stream);
  if (!rc && (hipEventRecord(b->ev1, b->stream) != hipSuccess || hipStreamSynchronize(b->stream) != hipSuccess))
    rc = FP4_E_DEVICE;
  *ms = 0.f;
  if (!rc) (void)hipEventElapsedTime(ms, b->ev0, b->ev1);
  ctx->qseg = keep_qs;
  ctx->lseg = keep_ls;
  return rc;
}

// Evenly spaced active modes of the context (the autotuner's sample).
int tune_sample(fp4_ctx *ctx, int nsample, std::vector<int> &sample) {
  const int nm = ctx->N * ctx->nb;
  std::vector<double> om(nm);
  FP4_HIP(ctx, hipMemcpy(om.data(), ctx->d_omega.p, nm * sizeof(double), hipMemcpyDeviceToHost));
  std::vector<int> act;
  for (int m = 0; m < nm; ++m)
    if (om[m] > 0.0) act.push_back(m);
  if (act.empty()) return ctx->fail(FP4_E_STATE, "no active mode");
  const int ns = std::min<int>(nsample, (int)act.size());
  sample.clear();
  for (int i = 0; i < ns; ++i) sample.push_back(act[(size_t)i * act.size() / ns]);
  return FP4_OK;
}

}  // namespace

extern "C" {

int fp4_autotune(fp4_ctx *ctx, const double *T, int32_t nT, double scalebroad, uint32_t mask,
                 int32_t precision, int32_t nsample, int32_t *best_qchunk, double *ms_out,
                 int32_t *qchunk_out, int32_t ncand_max, int32_t *ncand) {
  if (!ctx) return FP4_E_INVAL;
  try {
    int rc = check_compute_args(ctx, T, nT, scalebroad, mask, precision);
    if (rc) return rc;
    if (nT > 4) return ctx->fail(FP4_E_UNSUPPORTED, "autotuning takes at most 4 temperatures");
    if (nsample < 1) return ctx->fail(FP4_E_INVAL, "nsample must be >= 1");
    (void)hipSetDevice(ctx->device);
    std::vector<int> sample;
    if ((rc = tune_sample(ctx, nsample, sample))) return rc;
    std::vector<int> cand;
    for (int q : {1, 2, 4, 8, 16, 32, 64, 128})
      if (q < ctx->N) cand.push_back(q);
    cand.push_back(ctx->N);
    fp4_batch *b = nullptr;
    if ((rc = fp4_batch_create(&b, ctx->device))) return ctx->fail(rc, "batch context creation failed");
    double best_ms = 1e300;
    int best = cand[0];
    std::vector<double> times;
    for (size_t ci = 0; ci < cand.size(); ++ci) {
      float ms = 0.f;
      rc = time_config(ctx, b, sample, T, nT, scalebroad, mask, precision, cand[ci], ctx->qseg,
                       ctx->lseg, ci == 0, &ms);
      if (rc) {
        const std::string msg = b->err;
        fp4_batch_destroy(b);
        return ctx->fail(rc, "autotune: " + msg);
      }
      times.push_back(ms);
      if (ms < best_ms) {
        best_ms = ms;
        best = cand[ci];
      }
    }
    fp4_batch_destroy(b);
    ctx->qchunk = best;
    if (best_qchunk) *best_qchunk = best;
    if (ncand) *ncand = (int)times.size();
    for (int i = 0; i < (int)times.size() && i < ncand_max; ++i) {
      if (ms_out) ms_out[i] = times[i];
      if (qchunk_out) qchunk_out[i] = cand[i];
    }
    ctx->err.clear();
    return FP4_OK;
  } catch (const std::bad_alloc &) {
    return ctx->fail(FP4_E_NOMEM, "host allocation failed");
  }
}

int fp4_autotune_shapes(fp4_ctx *ctx, const double *T, int32_t nT, double scalebroad,
                        uint32_t mask, int32_t precision, int32_t nsample, int32_t *best,
                        double *ms_out, int32_t *cand_out, int32_t ncand_max, int32_t *ncand) {
  if (!ctx) return FP4_E_INVAL;
  try {
    int rc = check_compute_args(ctx, T, nT, scalebroad, mask, precision);
    if (rc) return rc;
    if (nT > 4) return ctx->fail(FP4_E_UNSUPPORTED, "autotuning takes at most 4 temperatures");
    if (nsample < 1) return ctx->fail(FP4_E_INVAL, "nsample must be >= 1");
    (void)hipSetDevice(ctx->device);
    std::vector<int> sample;
    if ((rc = tune_sample(ctx, nsample, sample))) return rc;
    struct Cfg {
      int qchunk, qseg, lseg;
      double ms;
    };
    std::vector<Cfg> tried;
    fp4_batch *b = nullptr;
    if ((rc = fp4_batch_create(&b, ctx->device))) return ctx->fail(rc, "batch context creation failed");
    auto run = [&](int qc, int qs, int ls, bool warm, double *ms_res) {
      float ms = 0.f;
      const int r = time_config(ctx, b, sample, T, nT, scalebroad, mask, precision, qc, qs, ls, warm, &ms);
      if (!r) {
        tried.push_back(Cfg{qc, qs, ls, (double)ms});
        *ms_res = ms;
      }
      return r;
    };
    // stage 1: q'-chunk at the current segments; stage 2: queue and list segments at the
    // best chunk (configurations whose LDS does not fit a work-group are skipped)
    std::vector<int> qcs;
    for (int q : {1, 2, 4, 8, 16, 32, 64, 128})
      if (q < ctx->N) qcs.push_back(q);
    qcs.push_back(ctx->N);
    Cfg bestc{qcs[0], ctx->qseg, ctx->lseg, 1e300};
    for (size_t i = 0; i < qcs.size() && !rc; ++i) {
      double ms = 0.0;
      rc = run(qcs[i], ctx->qseg, ctx->lseg, i == 0, &ms);
      if (!rc && ms < bestc.ms) bestc = Cfg{qcs[i], ctx->qseg, ctx->lseg, ms};
    }
    const fp4::Crystal c = make_crystal(ctx);
    for (int qs : {128, 256, 512})
      for (int ls : {128, 256, 512}) {
        if (rc || (qs == bestc.qseg && ls == bestc.lseg)) continue;
        if (fp4::batch_lds_bytes(c, precision == FP4_FP32, nT, qs, ls) > 160 * 1024 - 64) continue;
        double ms = 0.0;
        rc = run(bestc.qchunk, qs, ls, false, &ms);
        if (!rc && ms < bestc.ms) bestc = Cfg{bestc.qchunk, qs, ls, ms};
      }
    if (rc) {
      const std::string msg = b->err;
      fp4_batch_destroy(b);
      return ctx->fail(rc, "autotune: " + msg);
    }
    fp4_batch_destroy(b);
    ctx->qchunk = bestc.qchunk;
    ctx->qseg = bestc.qseg;
    ctx->lseg = bestc.lseg;
    if (best) {
      best[0] = bestc.qchunk;
      best[1] = bestc.qseg;
      best[2] = bestc.lseg;
    }
    if (ncand) *ncand = (int)tried.size();
    for (int i = 0; i < (int)tried.size() && i < ncand_max; ++i) {
      if (ms_out) ms_out[i] = tried[i].ms;
      if (cand_out) {
        cand_out[3 * i] = tried[i].qchunk;
        cand_out[3 * i + 1] = tried[i].qseg;
        cand_out[3 * i + 2] = tried[i].lseg;
      }
    }
    ctx->err.clear();
    return FP4_OK;
  } catch (const std::bad_alloc &) {
    return ctx->fail(FP4_E_NOMEM, "host allocation failed");
  }
}

}  // extern "C"
