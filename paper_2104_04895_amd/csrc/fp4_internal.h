// fp4_internal.h -- structures shared by the host side and the HIP kernels of the
// four-phonon rate library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace fp4 {

// Device-resident description of one crystal: grid, modes and the regrouped quartet list.
//
// Quartet regrouping.  For quartet n with atoms (i, j, k, l) and cells (0, Rj, Rk, Rl) the
// phase of Eq. V4 for a momentum-conserving process is
//   exp(i(s' q'.Rj + s'' q''.Rk - q'''.Rl)) = exp(i q.b) exp(i s' q'.a) exp(i s'' q''.d)
// with b = -Rl, a = Rj - Rl, d = Rk - Rl.  Quartets are grouped by g = (k, l, d) ("groups")
// and inside a group by (j, a) ("combos").  Groups are ordered by (k, l, d) so that the
// groups of one (k, l) atom pair are contiguous.
struct Crystal {
  int g0, g1, g2, N;        // grid and number of q points
  int nat, nb;              // atoms, branches (3 nat)
  int ng, nc, nq4;          // groups, combos, quartets
  int na, nbv, nd;          // distinct a, b, d cell vectors
  const double *omega;      // [N*nb]
  const double *inv_omega;  // [N*nb] 1/omega (0 for inactive modes)
  const double4 *vel;       // [N*nb] (x, y, z, 0)
  const double4 *mode4;     // [N*nb] (vx, vy, vz, omega)
  const double *speed;      // [N*nb] |v|
  const double4 *qbound;    // [N] (min omega, max omega, max |v|, 0) of the active branches
  const int4 *qimg;         // [N] first-zone image of each q: n_d + m_d N_d per axis
  const int4 *qord;         // [N] (iq, n1, n2, n3) of the q points in ascending qbound.x
  const double *qord_w;     // [N] qbound.x in that order
  double w_lo, w_hi, v_hi;  // lowest and highest active frequency, highest speed
  const double2 *E64;       // [N][nb][nb]  e_{j}(atom, x) / sqrt(M_atom), column = 3 atom + x
  const float2 *E32;        // same, FP32
  const int4 *qn;           // [N] (n1, n2, n3, 0)
  const double2 *PHA64;     // [N][na]  exp(i q.a)
  const double2 *PHB64;     // [N][nbv] exp(i q.b)
  const double2 *PHD64;     // [N][nd]  exp(i q.d)
  const float2 *PHD32;      // [N][nd]
  const int *g_d;           // [ng] index of d
  const int *kl_start;      // [nat*nat + 1] first group of atom pair (k, l)
  const int *c_start;       // [ng + 1] first combo of group g
  const int *c_jat;         // [nc] slot-2 atom j of combo c
  const int *c_a;           // [nc] index of a
  const int *cq_start;      // [nc + 1] first quartet (combo order) of combo c
  const int *q_i;           // [nq4] slot-1 atom i (combo order)
  const int *q_b;           // [nq4] index of b (combo order)
  const double *q_phi;      // [nq4][81] (combo order)
};

// Per-call parameters of the rate kernel.
struct RateArgs {
  double c_win;             // ((W sb) dq)^2 : keep <=> dw^2 <= c_win s2
  double sqrt_c_win;        // W sb dq
  double c_sig;             // (sb dq)^2     : sigma^2 = c_sig s2
  double c_min;             // sigma_min^2   : delta := 1 below
  double kpref;             // C4 / N^2
  int nT;
  uint32_t mask;            // channel bits
  int qclass;               // 0 all processes, 1 normal only (Q = 0), 2 Umklapp only,
                            // 3 both classes apart: partial slot 0 normal, 1 Umklapp
                            // (all channels), 2 unused
  int harmonic;             // 0 rates; phase spaces with |V|^2 := 1: 1 WP4, 2 P4
  int mirror;               // 1: the quartet list is symmetric under the slot-3/slot-4
                            // exchange, so the redistribution blocks of q'' and q''' are
                            // transposes and one contraction serves both; 0: every block
                            // is contracted on its own
  const double *occ;        // [nT][N*nb]  n0 (0 for inactive modes)
  const double *inv_occ;    // [nT][N*nb]  1/n0 = expm1(hbar w / kT)
  const int *targets;       // [nt] mode ids, or null: target t is mode tbase + t
  int tbase;                // first mode id when targets is null
  int nt;                   // targets in this batch
  int t0;                   // index of the first target of the batch in the output
  int qchunk;               // q' points per work-group
  int qseg;                 // q'' points a wavefront queues per phase (multiple of 64)
  int lseg;                 // kept processes a wavefront evaluates per pass (>= 64)
  int nchunk;               // ceil(N / qchunk)
  int nxcd;                 // XCDs the work-groups are dealt to (blockIdx round-robin)
  const void *U;            // [nt][nc][27] complex (R) precontraction of the batch
  double *partial;          // [nt_total][nchunk][3][nT]
  unsigned long long *pcount; // [nt_total][nchunk][3]
  unsigned long long *blocks; // [1] contracted branch blocks (atomic)
};

// Work queues of a persistent batched launch: one counter per XCD range of the item list,
// 128 bytes apart, per branch-count class.
constexpr int kBatchQueues = 8;
constexpr int kQueueStride = 16;   // unsigned long long
constexpr int kClassCounters = kBatchQueues * kQueueStride;

// One crystal of a persistent batched launch; items item0 .. item0 + nt*nchunk - 1.
struct BatchInst {
  Crystal c;
  RateArgs a;
  long long item0;
};

// Device-resident regrouped third-order force constants.  Triplet n has atoms (i, j, k)
// and cells (0, Rj, Rk); triplets are ordered by the atom pair (j, k), then by d = Rj - Rk.
struct Fc3Dev {
  int n3, nd3, nrk;
  const int *jk_start;      // [nat*nat + 1] first triplet of atom pair (j, k)
  const int *t_i;           // [n3] slot-1 atom i
  const int *t_d;           // [n3] index of d
  const int *t_rk;          // [n3] index of Rk
  const double *t_phi;      // [n3][27]
  const int *rk_vec;        // [nrk][3]
  const double2 *PH3;       // [nd3][N] exp(i q.d)
};

// Per-call parameters of the three-phonon rate kernel.
struct Rate3Args {
  double c_win, c_sig, c_min;
  double kpref;             // (hbar pi / 4) / N
  int nT;
  const double *occ;        // [nT][N*nb]
  const int *targets;       // [nt_total] mode ids
  int nt_total;
  int t0;                   // first target of this launch
  double *rates;            // [nT][nt_total]
  long long *counts;        // [nt_total][2] (nullable)
};

// launchers (fp4_kernels.hip)
hipError_t launch_tables(const Crystal &c, double4 *qbound, double4 *mode4, double *speed, double *inv_omega, double2 *E64, float2 *E32,
                         const double *evec, const double *mass, int4 *qn, double2 *PHA64, double2 *PHB64,
                         double2 *PHD64, float2 *PHD32, const int *avec, const int *bvec,
                         const int *dvec, hipStream_t s);
hipError_t launch_occupations(const Crystal &c, const double *T, int nT, double hbar_over_kb,
                              double *occ, double *inv_occ, hipStream_t s);
hipError_t launch_precontract(const Crystal &c, const int *targets, int nt, int fp32,
                              void *U, hipStream_t s, int tbase = 0);
// n0 and 1/n0 with the temperatures passed by value (no device copy of T)
hipError_t launch_occupations_v(const Crystal &c, const double *T, int nT, double hbar_over_kb,
                                double *occ, double *inv_occ, hipStream_t s);
// ordered reduction writing rates [nT][stride] (and per channel [nT][3][stride]) at columns
// off .. off + nt - 1, counts [stride][3] at rows off ..
hipError_t launch_reduce_strided(const RateArgs &a, int nt, int stride, int off, double *rates,
                                 double *rates_ch, long long *counts, hipStream_t s);
size_t rate_lds_bytes_for(const Crystal &c, int fp32, int nT, int qseg, int lseg);

// Allocation-free scratch area: a file-scope device array of kScratchBytes per GPU.
// scratch_init() looks up its address on the current device (once per device) and returns
// it; scratch_ptr(dev) returns the address found for device dev (null before the lookup).
constexpr size_t kScratchBytes = (size_t)64 << 20;
hipError_t scratch_init(int dev, void **out);
void *scratch_ptr(int dev);
hipError_t launch_rates(const Crystal &c, const RateArgs &a, int fp32, hipStream_t s);
hipError_t launch_reduce(const RateArgs &a, int nt_total, double *rates, double *rates_ch,
                         long long *counts, hipStream_t s);
hipError_t launch_debug_v(const Crystal &c, const int *quads, int n, const int *tslot,
                          const void *U, int fp32, double2 *V, hipStream_t s);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);
size_t batch_lds_bytes(const Crystal &c, int fp32, int nT, int qseg, int lseg);
hipError_t launch_batch(const BatchInst *insts, int ninst, long long total,
                        unsigned long long *counter, size_t lds, int fp32, int nb, int nT,
                        int *grid_out, hipStream_t s);

// launchers (fp4_rates3.hip)
hipError_t launch_tables3(const Crystal &c, const int *dvec, int nd, double2 *PH3, hipStream_t s);
hipError_t launch_precontract3(const Crystal &c, const Fc3Dev &f, const int *targets, int nt,
                               double2 *U, hipStream_t s);
size_t rates3_lds_bytes(int nT);
hipError_t launch_rates3(const Crystal &c, const Fc3Dev &f, const Rate3Args &a,
                         const double2 *U, int nblocks, hipStream_t s);

// launcher (fp4_kappa.hip): kappa [nT][9] = scale * sum over modes of C v v tau
hipError_t launch_kappa(const Crystal &c, const double *T, int nT, double hk, const double *occ,
                        const double *r3, const double *r4, double scale, double kb,
                        double *kappa, long long *skipped, hipStream_t s);

// hardware probe (fp4_probe.hip): TFLOP/s of six timed kernels into tflops[6]
size_t probe_out_doubles();
hipError_t run_probe(double *out, double *tflops, hipStream_t s);

// launchers (fp4_features.hip)
hipError_t launch_fc4_strength(const Crystal &c, const int *targets, int nt, double *g4,
                               hipStream_t s);
hipError_t launch_features(const Crystal &c, const int *targets, int nt, const double *T, int nT,
                           const double *occ, const double *r3, const double *g4,
                           const float *shift, const float *scale, float *X, hipStream_t s);

}  // namespace fp4
