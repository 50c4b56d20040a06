/*
 * fp4.h -- C ABI of the MI355X four-phonon RTA scattering-rate library.
 *
 * The library evaluates the four-phonon bracket of the single-mode relaxation-time rate
 * (FourPhonon paper, Eq. tao0) for every mode of a Gamma-centred q-grid:
 *
 *   1/tau_4ph(lambda) = sum over lambda' = (q',j'), lambda'' = (q'',j''), j''' of
 *       1/2 G^{++} + 1/2 G^{+-} + 1/6 G^{--}     (1/N and 1/N factors included)
 *
 * with q''' = q +- q' +- q'' + Q fixed by momentum conservation (Sec. 2.2), G from
 * Eq. 4phgamma, the matrix element V from Eq. V4 and the adaptive Gaussian
 * delta(dw) = exp(-dw^2/sigma^2)/(sqrt(pi) sigma), sigma = scalebroad |v'' - v'''| |dq|
 * (Sec. 2.4 and App. B).  A process takes part only if |dw| <= W sigma (W = window width,
 * default 2; the test is evaluated squared in a fixed FP64 order), and delta is set to 1 when
 * sigma^2 < sigma_min^2 (the paper's small-sigma correction, Sec. 2.4).
 *
 * Units: omega rad/ps, v Angstrom/ps, q 1/Angstrom (2 pi included), Phi eV/Angstrom^4,
 * mass amu, T kelvin, rates 1/ps.
 *
 * Conventions of the inputs (they fix what Eq. V4 means):
 *   - lattice vectors are the ROWS of A (Angstrom); grid point iq = n1 + N1*(n2 + N2*n3) is
 *     q = sum_d (n_d/N_d) b_d, n_d in [0, N_d);
 *   - mode id mu = iq*nb + j, nb = 3*natoms;
 *   - eigenvectors diagonalise D(q) = sum_R Phi2(0a,Rb) exp(+i q.R)/sqrt(Ma Mb) (phases on
 *     lattice vectors only), are normalised to 1, and e^{-lambda} = conj(e^{lambda});
 *   - omega <= 0 marks a mode inactive: its rate is 0 and it takes part in no process.
 *
 * Error convention: every int-returning call returns FP4_OK (0) or a negative code; no
 * exception crosses the ABI; the context stays usable after an error and fp4_last_error()
 * gives the reason.  All host pointers belong to the caller and are only read (or, for
 * outputs, written) during the call; the library keeps its own device copies.  A context
 * must not be used from two host threads at once.
 */
#ifndef FP4_H
#define FP4_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FP4_OK 0
#define FP4_E_INVAL (-1)       /* bad shape, range, NaN/Inf, mask 0, T <= 0, sb <= 0 */
#define FP4_E_STATE (-2)       /* compute before load, inconsistent loads */
#define FP4_E_NOMEM (-3)       /* device or host allocation failed */
#define FP4_E_DEVICE (-4)      /* a HIP runtime call failed (text in fp4_last_error) */
#define FP4_E_UNSUPPORTED (-5) /* option not supported for these inputs */

/* arithmetic of the matrix-element contraction (the window predicate, occupations, the
 * Gaussian and all rate sums are FP64 in every mode) */
#define FP4_FP64 0   /* complex FP64 contraction */
#define FP4_FP32 1   /* complex FP32 contraction and |V|^2, promoted to FP64 */

/* keys of fp4_set_param */
#define FP4_PARAM_WINDOW_W 1      /* W of the window |dw| <= W sigma (default 2.0) */
#define FP4_PARAM_SIGMA_MIN 2     /* sigma below which delta := 1, rad/ps (default 1e-4) */
#define FP4_PARAM_QCHUNK 3        /* q' points per work-group (0 = automatic) */
#define FP4_PARAM_PROFILE 4       /* 1: time every kernel with HIP events (fp4_last_timing) */
#define FP4_PARAM_QCLASS 5        /* processes summed: 0 all (default), 1 normal only (Q = 0),
                                     2 Umklapp only (Q != 0), the classes named after Eq. tao0.
                                     Q = k(q''') - (k(q) + s' k(q') + s'' k(q'')) with k the
                                     first-zone image of a grid point: the shortest of
                                     sum_d (n_d/N_d + m_d) b_d over m_d in -2..1, ties (relative
                                     1e-10) to the first m in the order m1, m2, m3.  Rates and
                                     counts of compute calls are then those of the class. */
#define FP4_PARAM_QSEG 7          /* q'' points a wavefront queues for contraction per phase
                                     of the rate kernel (multiple of 64, 64..2048; default 256) */
#define FP4_PARAM_LSEG 8          /* kept processes a wavefront evaluates per pass of the rate
                                     kernel (multiple of 64, 64..4096; default 256) */
#define FP4_PARAM_PHASE_SPACE 6   /* 0 rates (default); otherwise compute calls return a
                                     four-phonon phase space in place of the rates, with no
                                     force constants used (|V|^2 := 1, no contraction):
                                     1 weighted phase space WP4, each kept process weighted
                                     like Eq. 4phgamma without |V|^2 and hbar^2 pi / 8
                                     (occupation factor over n0_lambda, delta, 1/(w w' w'' w'''),
                                     channel weight, 1/N^2; ps^5); 2 phase space P4, channel
                                     weight times delta over N^2 (ps).  Counts are the kept
                                     processes as for the rates. */

/* channel bits of the process mask (Eq. 4phgamma): recombination, redistribution, splitting */
/* number of surrogate input features per (temperature, mode) row */
#define FP4_NFEAT 18

#define FP4_PP 1u
#define FP4_PM 2u
#define FP4_MM 4u

typedef struct fp4_ctx fp4_ctx;
typedef struct fp4_batch fp4_batch;
typedef struct fp4_mlp fp4_mlp;

/* Create a context on HIP device `device_id`.  *out receives the handle (NULL on error).
 * Returns FP4_E_DEVICE if the device cannot be used. */
int fp4_create(fp4_ctx **out, int device_id);

/* Release every device and host resource of the context (NULL is ignored). */
void fp4_destroy(fp4_ctx *ctx);

/* Lattice and grid (Sec. 2.2: N is the number of grid points).
 *   A[9]      lattice vectors as rows, Angstrom (non-singular)
 *   grid[3]   N1, N2, N3 >= 1, N = N1 N2 N3 <= 2^20
 *   natoms    1..4 atoms in the cell (nb = 3*natoms branches); more gives FP4_E_UNSUPPORTED
 *   mass      [natoms] amu, > 0
 *   dq        |Delta q''| of the adaptive broadening (App. B), 1/Angstrom; <= 0 selects
 *             (|det B|/N)^(1/3), the cube root of the reciprocal volume per grid point.
 * Invalidates previously loaded modes and force constants. */
int fp4_load_lattice(fp4_ctx *ctx, const double A[9], const int32_t grid[3], int32_t natoms,
                     const double *mass, double dq);

/* Harmonic modes on the full grid (copied to the device).
 *   nq = N, nb = 3*natoms (else FP4_E_STATE)
 *   omega [nq][nb]                 rad/ps (omega <= 0: inactive mode)
 *   evec  [nq][nb][natoms][3]      complex, interleaved (re, im)
 *   vel   [nq][nb][3]              Angstrom/ps
 * Non-finite values give FP4_E_INVAL. */
int fp4_load_modes(fp4_ctx *ctx, int32_t nq, int32_t nb, const double *omega,
                   const double *evec, const double *vel);

/* Fourth-order force constants as a quartet list (Eq. V4, Eq. PE):
 *   atoms [n][4]      basis indices (i, j, k, l) in [0, natoms)
 *   cells [n][3][3]   integer lattice coordinates of the cells of atoms j, k, l (atom i is in
 *                     the home cell), each component in [-64, 64]
 *   phi   [n][81]     eV/Angstrom^4, index ((alpha*3 + beta)*3 + gamma)*3 + theta
 * 1 <= n <= 2^20.  The list need not be symmetric; the rate is evaluated for whatever is
 * given.  When the list is symmetric under the exchange of slots 3 and 4 (for every entry
 * (i,j,k,l; Rj,Rk,Rl) the entry (i,j,l,k; Rj,Rl,Rk) holds Phi with gamma and theta
 * exchanged, entries with equal atoms and cells summed, to 1e-12 of max |Phi|; permutation
 * symmetry of Eq. TS implies it) the redistribution matrix element is symmetric in
 * lambda'' and lambda''' and one contraction serves both members of each mirror pair;
 * otherwise every redistribution block is contracted on its own (about 1.5x the work). */
int fp4_load_fc4(fp4_ctx *ctx, int32_t nquart, const int32_t *atoms, const int32_t *cells,
                 const double *phi);

/* Set a tunable (keys FP4_PARAM_*). */
int fp4_set_param(fp4_ctx *ctx, int32_t key, double value);

/* Synchronous four-phonon rates for every mode of the grid.
 *   T[nT]                  temperatures (K), 1 <= nT <= 8, each > 0
 *   scalebroad             > 0
 *   mask                   nonzero subset of FP4_PP | FP4_PM | FP4_MM
 *   precision              FP4_FP64 or FP4_FP32
 *   rates                  host [nT][nq*nb] 1/ps (required)
 *   rates_by_channel       host [nT][3][nq*nb] or NULL
 *   counts                 host [nq*nb][3] kept processes per channel (Numprocess) or NULL
 * Inactive modes get rate 0 and count 0. */
int fp4_compute_rates4(fp4_ctx *ctx, const double *T, int32_t nT, double scalebroad,
                       uint32_t mask, int32_t precision, double *rates,
                       double *rates_by_channel, int64_t *counts);

/* Same for an explicit list of target mode ids (chunked or resumed runs, sampled checks).
 *   targets [ntargets] in [0, nq*nb), 1 <= ntargets <= nq*nb
 *   outputs as above with nq*nb replaced by ntargets (rates [nT][ntargets], ...). */
int fp4_compute_rates4_subset(fp4_ctx *ctx, const double *T, int32_t nT, double scalebroad,
                              uint32_t mask, int32_t precision, const int32_t *targets,
                              int32_t ntargets, double *rates, double *rates_by_channel,
                              int64_t *counts);

/* Normal and Umklapp parts of the rates in one pass (the two process classes named after
 * Eq. tao0, Q = 0 and Q != 0, with Q and the first-zone images as for FP4_PARAM_QCLASS; the
 * paper's outputs BTE.w_4ph_normal and BTE.w_4ph_Umklapp beside BTE.w_4ph, App. A).  Every
 * kept process is classed once per block and summed into its class; the total is their sum.
 *   targets          host [ntargets] mode ids, or NULL for every mode (ntargets ignored)
 *   rates            host [nT][nt] total (nullable), nt = ntargets or nq*nb
 *   rates_normal     host [nT][nt] normal processes (nullable)
 *   rates_umklapp    host [nT][nt] Umklapp processes (nullable; not both class outputs NULL)
 *   counts           host [nt][3] kept processes per channel, both classes, or NULL
 * Other arguments as for fp4_compute_rates4.  FP4_PARAM_QCLASS is ignored by this call; with
 * FP4_PARAM_PHASE_SPACE set it returns FP4_E_UNSUPPORTED.  Synchronous. */
int fp4_compute_rates4_classes(fp4_ctx *ctx, const double *T, int32_t nT, double scalebroad,
                               uint32_t mask, int32_t precision, const int32_t *targets,
                               int32_t ntargets, double *rates, double *rates_normal,
                               double *rates_umklapp, int64_t *counts);

/* Same on the irreducible part of the grid under a point group supplied by the caller.
 *   rot [nrot][9] integer matrices (row-major) acting on reduced q coordinates,
 *        q' = R q; in grid triples n'_d = sum_e R_de n_e N_d / N_e (mod N_d).  Every matrix
 *        must map the grid onto itself (else FP4_E_INVAL); the caller includes the identity
 *        and, for time reversal, -I.  1 <= nrot <= 96.
 *   rates [nT][nq*nb] host; counts [nq*nb][3] host or NULL; *nirr (nullable) receives the
 *        number of irreducible points.
 * The grid points are split into orbits under the matrices; one representative per orbit
 * (its lowest index) is computed with the full kernel; its rates are averaged over each set
 * of degenerate branches (frequencies equal within 1e-9 relative) and copied, branch by
 * branch, to every point of the orbit; counts are copied unaveraged.  Branches are matched by
 * their order, so the frequencies at each q must be in ascending order; a point whose
 * frequencies differ from its representative's (1e-8 relative) is reported as FP4_E_INVAL.
 * Symmetry-equivalent modes have equal rates (and degenerate sets equal sums), so this
 * equals the full-grid result averaged over degenerate branches, at a fraction of the
 * cost.  Synchronous. */
int fp4_compute_rates4_wedge(fp4_ctx *ctx, const double *T, int32_t nT, double scalebroad,
                             uint32_t mask, int32_t precision, int32_t nrot, const int32_t *rot,
                             double *rates, int64_t *counts, int32_t *nirr);

/* Asynchronous form for callers that own the stream and the output memory.
 *   hip_stream   a hipStream_t of the context's device (NULL = the null stream)
 *   d_rates      DEVICE [nT][nq*nb] doubles (required)
 *   d_rates_by_channel DEVICE [nT][3][nq*nb] or NULL;  d_counts DEVICE [nq*nb][3] or NULL
 * The rate work is enqueued on hip_stream and the call returns without waiting for it; the
 * staging of the target list, and on the first call after a load the per-q tables, run on
 * the context's own stream and are waited for.  The context's internal buffers are reused
 * by the next call, so calls on one context must not overlap on different streams. */
int fp4_compute_rates4_async(fp4_ctx *ctx, const double *T, int32_t nT, double scalebroad,
                             uint32_t mask, int32_t precision, void *hip_stream,
                             double *d_rates, double *d_rates_by_channel, int64_t *d_counts);

/* Allocation-free form of fp4_compute_rates4_async, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments and outputs as fp4_compute_rates4_async (every mode of the grid, device
 * outputs, work enqueued on hip_stream, returns without waiting).  It calls no hipMalloc,
 * hipFree or other allocating routine: its intermediates (occupations, precontraction,
 * partial sums) live in a fixed scratch area of 64 MiB per GPU, a device array of the library
 * held until the process ends, and the targets are processed in batches that fit it.
 *   - the loads must have completed (they build the per-q tables), else FP4_E_STATE;
 *   - 2 nT nq nb doubles of occupations plus one target's precontraction and partial sums
 *     must fit the 64 MiB, else FP4_E_UNSUPPORTED (the message gives the size needed);
 *   - every call on one GPU shares that GPU's scratch area, which keeps the last call's
 *     contents: calls that overlap on one GPU (other streams or host threads, any context)
 *     race and must be serialised by the caller;
 *   - fp4_last_stats and fp4_last_timing are not updated.
 * The results equal those of fp4_compute_rates4_async with the same q'-chunk. */
int fp4_compute_rates4_noalloc(fp4_ctx *ctx, const double *T, int32_t nT, double scalebroad,
                               uint32_t mask, int32_t precision, void *hip_stream,
                               double *d_rates, double *d_rates_by_channel, int64_t *d_counts);

/* Matrix elements V of Eq. V4 through the library's own contraction path.
 *   quads [n][8] = (iq, j, iq', j', iq'', j'', j''', channel) with channel 0 (++), 1 (+-),
 *                  2 (--); iq''' is q + s' q' + s'' q'' folded into the grid
 *   V     [n] complex, interleaved (re, im)
 * Test hook; 1 <= n <= 2^16. */
int fp4_debug_matrix_elements(fp4_ctx *ctx, int32_t n, const int32_t *quads,
                              int32_t precision, double *V);

/* Work counts of the last compute call: kept processes (all channels), candidate processes
 * enumerated, and branch blocks contracted. */
int fp4_last_stats(const fp4_ctx *ctx, int64_t *processes, int64_t *candidates,
                   int64_t *blocks);

/* With FP4_PARAM_PROFILE = 1: device time (ms) of the last call's kernels, from HIP events
 * recorded on the call's stream: main = the fused enumeration/contraction kernel, total =
 * first to last kernel. */
int fp4_last_timing(const fp4_ctx *ctx, double *ms_main, double *ms_total);

/* ---------------------------------------------------------------- three-phonon rate
 * Three-phonon RTA rate (Eq. tao0 three-phonon bracket, Eq. 3phgamma, Eq. V3), used as an
 * input feature of the learned surrogate:
 *   1/tau3(lambda) = (1/N) [ sum G+ + 1/2 sum G- ],  q'' = q +- q' folded into the grid,
 *   G+ = (hbar pi/4) (n' - n'') |V+|^2 delta(w + w' - w'') / (w w' w''),
 *   G- = (hbar pi/4) (n' + n'' + 1) |V-|^2 delta(w - w' - w'') / (w w' w''),
 * with the same adaptive Gaussian (sigma = scalebroad |v' - v''| dq), window, sigma floor
 * and inactive-mode rules as the four-phonon rate.  Computed in FP64. */

/* Third-order force constants (copied; the caller keeps ownership).
 *   atoms [n][3]       basis indices (i, j, k), i of the home cell
 *   cells [n][2][3]    integer lattice coordinates of the cells of atoms j and k,
 *                      each component in [-64, 64]
 *   phi   [n][27]      eV/Angstrom^3, index (alpha*3 + beta)*3 + gamma
 * 1 <= n <= 2^16.  Requires fp4_load_lattice first. */
int fp4_load_fc3(fp4_ctx *ctx, int32_t ntrip, const int32_t *atoms, const int32_t *cells,
                 const double *phi);

/* Synchronous three-phonon rates.
 *   T[nT]        temperatures (K), 1 <= nT <= 8, each > 0;  scalebroad > 0
 *   targets      host [ntargets] mode ids in [0, nq*nb), or NULL for every mode
 *                (ntargets ignored)
 *   rates        host [nT][nt] 1/ps (required), nt = ntargets or nq*nb
 *   counts       host [nt][2] kept processes of the + and - channels, or NULL
 * Requires fp4_load_lattice, fp4_load_modes and fp4_load_fc3. */
int fp4_compute_rates3(fp4_ctx *ctx, const double *T, int32_t nT, double scalebroad,
                       const int32_t *targets, int32_t ntargets, double *rates,
                       int64_t *counts);

/* Input features of the learned surrogate for every (temperature, target mode) pair:
 * row (t, i) of X [nT][nt][FP4_NFEAT] (FP32) holds
 *   0  ln w (rad/ps)            1  ln(|v| + 0.01) (A/ps)     2..13  one-hot branch j (< 12)
 *   14 ln n0(w, T)              15 ln(1/tau3 + 1e-8) (1/ps, Eq. 3phgamma, computed here)
 *   16 ln(T / 300 K)            17 ln(g4 + 1e-30), g4 = sum of |U|^2 over the slot-1
 *                                  precontraction of the fourth-order list with the mode's
 *                                  eigenvector and phase (Eq. V4), eV^2/(A^8 amu)
 * Inactive modes (w <= 0) get 0 for their logarithms.  With shift and scale (both non-NULL,
 * FP4_NFEAT floats each) every entry is standardised to (f - shift) * scale.
 *   targets  host [ntargets] mode ids, or NULL for every mode (ntargets ignored)
 *   rates3   host [nT][nt] three-phonon rates used for feature 15, or NULL
 * Requires fp4_load_lattice, fp4_load_modes, fp4_load_fc4 and fp4_load_fc3. */
int fp4_surrogate_features(fp4_ctx *ctx, const double *T, int32_t nT, double scalebroad,
                           const int32_t *targets, int32_t ntargets, const float *shift,
                           const float *scale, float *X, double *rates3);

/* RTA lattice thermal conductivity with three- and four-phonon scattering:
 *   kappa^{ab}(T) = 1/(N Omega) sum_lambda C_lambda v^a v^b tau_lambda,
 *   C_lambda = k_B x^2 n0 (n0 + 1), x = hbar w / (k_B T),  1/tau = 1/tau3 + 1/tau4,
 * i.e. Eq. tao0 without the isotope term and F = tau v (Eq. BTE in the relaxation-time
 * approximation); Omega = |det A|.  The paper takes the conductivity from ShengBTE without
 * printing it; this is the standard kinetic form.  The rates are the library's own: the
 * four-phonon rate of every mode (all channels, `precision` of the contraction) and the
 * three-phonon rate (FP64), both at `scalebroad`.  Modes with w <= 0 or with a zero total
 * rate take no part.
 *   T[nT]      1 <= nT <= 8 temperatures (K)
 *   kappa      host [nT][3][3] W/(m K) (required)
 *   nskip      host [nT] active modes left out for a zero total rate, or NULL
 *   rates3, rates4   host [nT][nq*nb] the rates used (1/ps), or NULL
 * Requires fp4_load_lattice, fp4_load_modes, fp4_load_fc4 and fp4_load_fc3; with
 * FP4_PARAM_PHASE_SPACE or FP4_PARAM_QCLASS set it returns FP4_E_UNSUPPORTED.  Synchronous. */
int fp4_compute_kappa_rta(fp4_ctx *ctx, const double *T, int32_t nT, double scalebroad,
                          int32_t precision, double *kappa, int64_t *nskip, double *rates3,
                          double *rates4);

/* ---------------------------------------------------------------- batched instances
 * Several crystals (uneven branch counts, grids, quartet lists) evaluated by one captured HIP
 * graph: per instance occupations and precontraction, one persistent kernel per branch-count
 * class whose work-groups take (instance, target, q'-chunk) items from atomic work queues
 * (one per XCD range of the item list; a work-group drains its own XCD's range, then helps
 * the others), per instance ordered reduction.  The graph is captured
 * on the first call and replayed while the instance buffers are unchanged; temperatures are
 * read from device memory at replay time. */

/* Create an empty batch on HIP device `device_id`. */
int fp4_batch_create(fp4_batch **out, int device_id);

/* Release the batch (not the contexts added to it). */
void fp4_batch_destroy(fp4_batch *b);

/* Add a fully loaded context (same device).  The caller keeps the context alive while the
 * batch is used; at most 64 instances. */
int fp4_batch_add(fp4_batch *b, fp4_ctx *ctx);

/* Rates of every mode of every instance.
 *   T[nT], 1 <= nT <= 4; scalebroad, mask, precision as in fp4_compute_rates4
 *   rates   host, concatenated in the order of fp4_batch_add: for instance i a block
 *           [nT][nq_i*nb_i] (1/ps)
 *   counts  host, concatenated blocks [nq_i*nb_i][3], or NULL
 * Each instance uses its context's q'-chunk (FP4_PARAM_QCHUNK or fp4_autotune), or the
 * automatic choice of a single call (at most 8) if unset.  Synchronous. */
int fp4_batch_compute(fp4_batch *b, const double *T, int32_t nT, double scalebroad,
                      uint32_t mask, int32_t precision, double *rates, int64_t *counts);

/* Device time (ms) of the last graph launch, and how many graphs were captured and
 * launched so far. */
int fp4_batch_last_timing(const fp4_batch *b, double *ms_graph, int64_t *graph_builds,
                          int64_t *graph_launches);

/* Reason of the last batch error. */
const char *fp4_batch_last_error(const fp4_batch *b);

/* Autotuner: times the persistent pipeline on `nsample` evenly spaced active modes of the
 * context for q'-chunk sizes 1, 2, 4, ..., 128 and N (those below N), keeps the fastest as
 * the context's FP4_PARAM_QCHUNK and returns it in *best_qchunk.  ms_out / qchunk_out
 * (nullable, ncand_max entries) receive the measured times and the candidates; *ncand the
 * number of candidates.  1 <= nT <= 4. */
int fp4_autotune(fp4_ctx *ctx, const double *T, int32_t nT, double scalebroad, uint32_t mask,
                 int32_t precision, int32_t nsample, int32_t *best_qchunk, double *ms_out,
                 int32_t *qchunk_out, int32_t ncand_max, int32_t *ncand);

/* Autotuner of the rate kernel's work shapes: first the q'-chunk as fp4_autotune, then at
 * that chunk the queue segment FP4_PARAM_QSEG and the list segment FP4_PARAM_LSEG over
 * {128, 256, 512} x {128, 256, 512} (configurations whose LDS exceeds a work-group's 160 KiB
 * are skipped), each timed on the persistent pipeline over `nsample` evenly spaced active
 * modes.  The fastest (qchunk, qseg, lseg) becomes the context's setting and is returned in
 * best[3]; cand_out [ncand_max][3] and ms_out [ncand_max] (nullable) receive the tried
 * configurations and their device times, *ncand their number.  1 <= nT <= 4. */
int fp4_autotune_shapes(fp4_ctx *ctx, const double *T, int32_t nT, double scalebroad,
                        uint32_t mask, int32_t precision, int32_t nsample, int32_t *best,
                        double *ms_out, int32_t *cand_out, int32_t ncand_max, int32_t *ncand);

/* ---------------------------------------------------------------- learned surrogate
 * A small multilayer perceptron, trained and evaluated by the library's own kernels, that
 * predicts a mode's log four-phonon rate (output 0) and the log standard deviation of that
 * prediction (output 1) from per-mode features.  Layers nin -> width -> ... -> width -> 2
 * (`depth` linear layers, SiLU between them); training minimises the Gaussian negative
 * log-likelihood 0.5 (y - mu)^2 exp(-2 s) + s with Adam in FP32; inference runs in FP32 or
 * with BF16 weights and activations (FP32 accumulation).  Parameters are one FP32 array:
 * per layer W [out][in] then b [out]. */

/* Create a network (2 <= depth <= 16, width <= 1024, nin <= 256), seeded initialisation. */
int fp4_mlp_create(fp4_mlp **out, int device_id, int32_t nin, int32_t width, int32_t depth,
                   uint64_t seed);
void fp4_mlp_destroy(fp4_mlp *m);
const char *fp4_mlp_last_error(const fp4_mlp *m);
int64_t fp4_mlp_num_params(const fp4_mlp *m);
int fp4_mlp_get_params(fp4_mlp *m, float *params);
int fp4_mlp_set_params(fp4_mlp *m, const float *params);

/* Mean loss over n samples (X [n][nin], y [n]) and its gradient with respect to every
 * parameter (grad: nullable, num_params floats). */
int fp4_mlp_loss_grad(fp4_mlp *m, const float *X, const float *y, int32_t n, double *loss,
                      float *grad);

/* `epochs` passes of Adam (lr, beta 0.9/0.999) over shuffled mini-batches of `batch` rows
 * (the last incomplete batch of an epoch is skipped).  loss_per_epoch: nullable [epochs]. */
int fp4_mlp_train(fp4_mlp *m, const float *X, const float *y, int32_t n, int32_t epochs,
                  int32_t batch, float lr, uint64_t seed, double *loss_per_epoch);

/* out [n][2] = (mu, s) for X [n][nin]; bf16 != 0 selects BF16 weights/activations.  *ms
 * (nullable) receives the device time of the forward pass. */
int fp4_mlp_predict(fp4_mlp *m, const float *X, int32_t n, int32_t bf16, float *out, double *ms);

/* Hardware probe behind the placement of the branch-block contraction (matrix cores only
 * where they pay): measured TFLOP/s on device `device_id` of six kernels, written to
 * tflops[6]: 0 FP64 MFMA 16x16x4, 1 FP64 vector FMA, 2 half of the wavefronts of each
 * work-group as 0 and half as 1, 3 BF16 MFMA 16x16x32 with FP32 accumulation, 4 FP32 vector
 * FMA, 5 half as 3 and half as 4.  Mixed kernels close to the mean of their halves mean the
 * matrix core does not run beside the vector unit.  Allocates and frees 4 MiB of device
 * memory; takes about 20 ms. */
int fp4_probe_matrix_rates(int32_t device_id, double *tflops);

/* Human-readable reason of the last error on this context ("" if none). */
const char *fp4_last_error(const fp4_ctx *ctx);

/* Static description of an error code. */
const char *fp4_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* FP4_H */
