/*
 * oracle4.c -- plain, slow FP64 CPU reference for the four-phonon RTA scattering rate.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or calls this
 * file; only the tests, the smoke check and the benchmark's CPU-baseline leg use it.
 *
 * What it computes (FourPhonon paper, Sec. 2.2 and 2.4):
 *   1/tau_4ph(lambda) = (1/N) [ sum^{++} 1/2 G^{++} + sum^{+-} 1/2 G^{+-} + sum^{--} 1/6 G^{--} ]
 *     (the four-phonon bracket of Eq. tao0), with the sums unrestricted over
 *     lambda' = (q',j'), lambda'' = (q'',j'') and j''', and q''' fixed by momentum
 *     conservation q''' = q +- q' +- q'' + Q (the definition that follows Eq. tao0);
 *   G^{(s)} from Eq. 4phgamma (prefactor hbar^2 pi / (8N), occupation factors over n0_lambda,
 *     |V|^2, delta / (w w' w'' w'''));
 *   V from Eq. V4 (sum over quartets and Cartesian indices of Phi times four eigenvector
 *     components over sqrt of the four masses, times the three lattice phases);
 *   delta from the adaptive Gaussian of Sec. 2.4 with sigma = |v'' - v'''| |dq| (App. B),
 *     scaled by scalebroad, and replaced by 1 when sigma is very small.
 *
 * Readings where the paper is silent (also used by the library; both sides implement them
 * separately):
 *   - a process is kept only if |dw| <= W sigma (evaluated squared), W = window_w;
 *   - "sigma very small" means sigma^2 < sigma_min^2, and then delta := 1 (ps);
 *   - a mode with omega <= 0 is inactive: it has rate 0 and takes part in no process;
 *   - e^{-lambda} = conj(e^{lambda}); phases exp(i q.R) use lattice vectors only and an
 *     integer reduction of q.R, so exp(i G.R) = 1 exactly;
 *   - the predicate is evaluated in a fixed FP64 order with no contraction:
 *       dw  = ((w  s0 w') s1 w'') - w'''     (s0, s1 the channel signs, left to right)
 *       d   = v'' - v'''  (component-wise),   s2 = (dx*dx + dy*dy) + dz*dz
 *       keep <=> dw*dw <= c_win * s2,         c_win = ((W*sb)*dq) * ((W*sb)*dq)
 *   - units: omega rad/ps, v A/ps, Phi eV/A^4, mass amu, T K, rates 1/ps.
 *
 * Evaluation order of V: per quartet n, the slot-1 and slot-2 factors are contracted first
 * (they are fixed while the loops over q'' and branches run) and the result is then
 * contracted with the slot-3 and slot-4 factors, which are formed once per (q'', j'') and
 * per (q''', j''') and reused across the branch loops.  Nothing is grouped across quartets.
 *
 * Compile with -O2 -ffp-contract=off so that the predicate is bit-reproducible.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <complex.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double _Complex cplx;

/* SI 2019 exact values (h, k_B, e) and CODATA 2018 (amu) */
#define HBAR (6.62607015e-34 / (2.0 * M_PI))  /* J s   */
static const double KB = 1.380649e-23;        /* J/K   */
static const double EV = 1.602176634e-19;     /* J     */
static const double AMU = 1.66053906660e-27;  /* kg    */
static const double ANG = 1.0e-10;            /* m     */

/* hbar/k_B in K*ps */
double oracle_hbar_over_kb(void) { return HBAR / KB * 1.0e12; }

/* Threads a parallel region of the oracle uses when nthreads is 0 (reported with timings). */
int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Prefactor of Eq. 4phgamma without the 1/N factors:
 *   G[1/ps] = C4 * occ * |V|^2 * delta[ps] / (w w' w'' w''')[(rad/ps)^4]
 * for V in eV / (A^4 amu^2):  C4 = hbar^2 pi / 8 * (eV/(A^4 amu^2))^2 * 1e-72. */
double oracle_c4(void) {
    const double kv = EV / (ANG * ANG * ANG * ANG * AMU * AMU);
    return HBAR * HBAR * M_PI / 8.0 * kv * kv * 1.0e-72;
}

/* Bose-Einstein occupation n0 (after Eq. 4phgamma). */
double oracle_bose(double omega, double T) {
    return 1.0 / expm1(oracle_hbar_over_kb() * omega / T);
}

/* Adaptive Gaussian delta (Sec. 2.4): exp(-dw^2/sigma^2) / (sqrt(pi) sigma), or 1 when
 * sigma^2 < sigma_min^2. */
double oracle_delta(double dw, double sigma2, double sigma_min) {
    if (sigma2 < sigma_min * sigma_min) return 1.0;
    return exp(-(dw * dw) / sigma2) / (sqrt(M_PI) * sqrt(sigma2));
}

typedef struct {
    int g[3];
    int N;
    int nat, nb;
    const double *mass, *omega, *evec, *vel;
    int nq4;
    const int32_t *atoms, *cells;
    const double *phi;
    cplx *rou;          /* exp(2 pi i k / N), exactly conjugate-symmetric */
    int ncell;          /* distinct cells of slots 2..4 in the quartet list */
    int *cid;           /* [nq4][3] cell id of slots 2, 3, 4 */
    cplx *cph;          /* [N][ncell] exp(i q.R) of every grid point and distinct cell */
} model_t;

static cplx phase(const model_t *m, int iq, const int32_t *R);

static void model_init(model_t *m, const int32_t grid[3], int32_t natoms, const double *mass,
                       const double *omega, const double *evec, const double *vel,
                       int32_t nq4, const int32_t *atoms, const int32_t *cells,
                       const double *phi) {
    m->g[0] = grid[0]; m->g[1] = grid[1]; m->g[2] = grid[2];
    m->N = grid[0] * grid[1] * grid[2];
    m->nat = natoms; m->nb = 3 * natoms;
    m->mass = mass; m->omega = omega; m->evec = evec; m->vel = vel;
    m->nq4 = nq4; m->atoms = atoms; m->cells = cells; m->phi = phi;
    m->rou = (cplx *)malloc(sizeof(cplx) * (size_t)m->N);
    for (int k = 0; k <= m->N / 2; ++k) {
        double a = 2.0 * M_PI * (double)k / (double)m->N;
        m->rou[k] = cos(a) + I * sin(a);
    }
    for (int k = m->N / 2 + 1; k < m->N; ++k) m->rou[k] = conj(m->rou[m->N - k]);
    /* table of lattice phases for the cells the quartet list uses (a lookup of the same
     * values phase() returns) */
    m->cid = (int *)malloc(sizeof(int) * 3 * (size_t)(nq4 > 0 ? nq4 : 1));
    int32_t *uniq = (int32_t *)malloc(sizeof(int32_t) * 9 * (size_t)(nq4 > 0 ? nq4 : 1));
    m->ncell = 0;
    for (int n = 0; n < nq4; ++n)
        for (int s = 0; s < 3; ++s) {
            const int32_t *R = cells + 9 * n + 3 * s;
            int found = -1;
            for (int u = 0; u < m->ncell && found < 0; ++u)
                if (uniq[3 * u] == R[0] && uniq[3 * u + 1] == R[1] && uniq[3 * u + 2] == R[2]) found = u;
            if (found < 0) {
                found = m->ncell++;
                uniq[3 * found] = R[0]; uniq[3 * found + 1] = R[1]; uniq[3 * found + 2] = R[2];
            }
            m->cid[3 * n + s] = found;
        }
    m->cph = (cplx *)malloc(sizeof(cplx) * (size_t)m->N * (m->ncell > 0 ? m->ncell : 1));
    for (int iq = 0; iq < m->N; ++iq)
        for (int u = 0; u < m->ncell; ++u) m->cph[(size_t)iq * m->ncell + u] = phase(m, iq, uniq + 3 * u);
    free(uniq);
}

static void model_free(model_t *m) { free(m->rou); free(m->cid); free(m->cph); }

static void qtriple(const model_t *m, int iq, int n[3]) {
    n[0] = iq % m->g[0];
    n[1] = (iq / m->g[0]) % m->g[1];
    n[2] = iq / (m->g[0] * m->g[1]);
}

static int imod(int a, int b) { int r = a % b; return r < 0 ? r + b : r; }

/* q''' = q + s1 q' + s2 q'' folded back into the grid (momentum conservation with the
 * Umklapp vector Q absorbed). */
static int fold(const model_t *m, int iq, int s1, int iq1, int s2, int iq2) {
    int a[3], b[3], c[3], r[3];
    qtriple(m, iq, a); qtriple(m, iq1, b); qtriple(m, iq2, c);
    for (int d = 0; d < 3; ++d) r[d] = imod(a[d] + s1 * b[d] + s2 * c[d], m->g[d]);
    return r[0] + m->g[0] * (r[1] + m->g[1] * r[2]);
}

/* Reciprocal vectors as rows of B (2 pi included): B = 2 pi inv(A)^T, A rows = lattice
 * vectors. */
static void recip(const double A[9], double B[9]) {
    const double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                       A[2] * (A[3] * A[7] - A[4] * A[6]);
    /* row i of B is 2 pi (a_j x a_k) / det for (i, j, k) cyclic */
    const double *a0 = A, *a1 = A + 3, *a2 = A + 6;
    const double *r[3][2] = {{a1, a2}, {a2, a0}, {a0, a1}};
    for (int i = 0; i < 3; ++i) {
        const double *u = r[i][0], *v = r[i][1];
        B[3 * i + 0] = 2.0 * M_PI * (u[1] * v[2] - u[2] * v[1]) / det;
        B[3 * i + 1] = 2.0 * M_PI * (u[2] * v[0] - u[0] * v[2]) / det;
        B[3 * i + 2] = 2.0 * M_PI * (u[0] * v[1] - u[1] * v[0]) / det;
    }
}

/* First-Brillouin-zone image of grid point iq: the vector sum_d (n_d / N_d + m_d) b_d of
 * smallest length over the integer shifts m_d in -2..1; among lengths equal within a
 * relative 1e-10 the first shift in the order m1, m2, m3 (m1 slowest) is kept. */
static void first_zone(const model_t *m, const double B[9], int iq, double k[3]) {
    int n[3]; qtriple(m, iq, n);
    double best = -1.0;
    for (int m1 = -2; m1 <= 1; ++m1)
        for (int m2 = -2; m2 <= 1; ++m2)
            for (int m3 = -2; m3 <= 1; ++m3) {
                const double f[3] = {(double)n[0] / m->g[0] + m1, (double)n[1] / m->g[1] + m2,
                                     (double)n[2] / m->g[2] + m3};
                double c[3], l2 = 0.0;
                for (int x = 0; x < 3; ++x) {
                    c[x] = f[0] * B[x] + f[1] * B[3 + x] + f[2] * B[6 + x];
                    l2 += c[x] * c[x];
                }
                if (best < 0.0 || l2 < best * (1.0 - 1e-10)) {
                    best = l2;
                    k[0] = c[0]; k[1] = c[1]; k[2] = c[2];
                }
            }
}

/* Public: the first-zone images of a list of grid points, k_out[n][3] Cartesian (1/Angstrom,
 * 2 pi included), as used by the normal / Umklapp split.  A[9]: lattice vectors as rows. */
int oracle_first_zone(const double A[9], const int32_t grid[3], int32_t n, const int32_t *iq,
                      double *k_out) {
    model_t m;
    m.g[0] = grid[0]; m.g[1] = grid[1]; m.g[2] = grid[2];
    m.N = grid[0] * grid[1] * grid[2];
    double B[9];
    recip(A, B);
    for (int i = 0; i < n; ++i) {
        if (iq[i] < 0 || iq[i] >= m.N) return -1;
        first_zone(&m, B, iq[i], k_out + 3 * i);
    }
    return 0;
}

/* exp(i q.R) for grid point iq and integer cell R (lattice coordinates). */
static cplx phase(const model_t *m, int iq, const int32_t *R) {
    int n[3]; qtriple(m, iq, n);
    long k = 0;
    for (int d = 0; d < 3; ++d) k += (long)imod(n[d] * R[d], m->g[d]) * (m->N / m->g[d]);
    return m->rou[k % m->N];
}

static cplx ev(const model_t *m, int iq, int j, int atom, int x) {
    const double *p = m->evec + 2 * ((((size_t)iq * m->nb + j) * m->nat + atom) * 3 + x);
    return p[0] + I * p[1];
}

/* Factor of one slot of Eq. V4: e_x^{+-lambda}(atom) exp(+-i q.R) / sqrt(M_atom). */
static cplx slot_factor(const model_t *m, int sign, int iq, int j, int atom, const int32_t *R,
                        int x) {
    cplx f = ev(m, iq, j, atom, x) * phase(m, iq, R) / sqrt(m->mass[atom]);
    return sign > 0 ? f : conj(f);
}

static const int32_t ZERO_CELL[3] = {0, 0, 0};

/* The same factor with the phase taken from the per-cell table (slot = 1, 2, 3 for the
 * quartet's atoms j, k, l). */
static cplx slot_factor_n(const model_t *m, int sign, int iq, int j, int n, int slot, int x) {
    const int atom = m->atoms[4 * n + slot];
    cplx f = ev(m, iq, j, atom, x) * m->cph[(size_t)iq * m->ncell + m->cid[3 * n + slot - 1]] /
             sqrt(m->mass[atom]);
    return sign > 0 ? f : conj(f);
}

/* V of Eq. V4 for four modes with slot signs sg[0..3] (slot 1 is the target, sign +1 in
 * the rate; the general form is used by the permutation tests).  The quartet's slot-1
 * atom sits in the home cell. */
static cplx v4_general(const model_t *m, const int mode[4], const int sg[4]) {
    cplx V = 0.0;
    for (int n = 0; n < m->nq4; ++n) {
        const int32_t *at = m->atoms + 4 * n;
        const int32_t *cl = m->cells + 9 * n;
        const double *ph = m->phi + 81 * (size_t)n;
        cplx X[4][3];
        for (int s = 0; s < 4; ++s) {
            const int32_t *R = s == 0 ? ZERO_CELL : cl + 3 * (s - 1);
            int iq = mode[s] / m->nb, j = mode[s] % m->nb;
            for (int x = 0; x < 3; ++x) X[s][x] = slot_factor(m, sg[s], iq, j, at[s], R, x);
        }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                for (int c = 0; c < 3; ++c)
                    for (int d = 0; d < 3; ++d)
                        V += ph[((a * 3 + b) * 3 + c) * 3 + d] * X[0][a] * X[1][b] * X[2][c] * X[3][d];
    }
    return V;
}

/* Public: V for n explicit processes.  modes4[n][4] are mode ids iq*nb + j, signs4[n][4]
 * are the slot signs (+1: e^{lambda} e^{+iq.R}; -1: the complex conjugate).  Output V
 * interleaved (re, im). */
int oracle_v4(const int32_t grid[3], int32_t natoms, const double *mass, const double *omega,
              const double *evec, const double *vel, int32_t nq4, const int32_t *atoms,
              const int32_t *cells, const double *phi, int32_t n, const int32_t *modes4,
              const int32_t *signs4, double *V) {
    model_t m;
    model_init(&m, grid, natoms, mass, omega, evec, vel, nq4, atoms, cells, phi);
    for (int i = 0; i < n; ++i) {
        int md[4], sg[4];
        for (int s = 0; s < 4; ++s) { md[s] = modes4[4 * i + s]; sg[s] = signs4[4 * i + s]; }
        cplx v = v4_general(&m, md, sg);
        V[2 * i] = creal(v); V[2 * i + 1] = cimag(v);
    }
    model_free(&m);
    return 0;
}

/* The three channels of Eq. 4phgamma: signs of lambda' and lambda'' and the weight of
 * each in Eq. tao0. */
static const int CH_S1[3] = {+1, +1, -1};
static const int CH_S2[3] = {+1, -1, -1};
static const double CH_W[3] = {0.5, 0.5, 1.0 / 6.0};

/* Energy-window predicate (fixed FP64 order, see header). */
static int keep_process(const model_t *m, int ch, int mu, int mu1, int mu2, int mu3,
                        double c_win, double *dw_out, double *s2_out) {
    const double w = m->omega[mu], w1 = m->omega[mu1], w2 = m->omega[mu2], w3 = m->omega[mu3];
    double a = CH_S1[ch] > 0 ? w + w1 : w - w1;
    double b = CH_S2[ch] > 0 ? a + w2 : a - w2;
    double dw = b - w3;
    const double *v2 = m->vel + 3 * (size_t)mu2, *v3 = m->vel + 3 * (size_t)mu3;
    double dx = v2[0] - v3[0], dy = v2[1] - v3[1], dz = v2[2] - v3[2];
    double s2 = (dx * dx + dy * dy) + dz * dz;
    *dw_out = dw; *s2_out = s2;
    return dw * dw <= c_win * s2;
}

static void neumaier(double *sum, double *comp, double x) {
    double t = *sum + x;
    if (fabs(*sum) >= fabs(x)) *comp += (*sum - t) + x;
    else *comp += (x - t) + *sum;
    *sum = t;
}

/*
 * Public: four-phonon RTA rates for a list of target modes.
 *   rates[nT][ntargets]            1/ps  (required)
 *   rates_ch[nT][3][ntargets]      per channel (++, +-, --), optional
 *   counts[ntargets][3]            number of kept processes per channel, optional
 * If want_rates == 0 only the counts are produced (no matrix elements are evaluated).
 * Returns 0, or -1 on invalid arguments.
 */
static int rates_core(const int32_t grid[3], int32_t natoms, const double *mass,
                      const double *omega, const double *evec, const double *vel, int32_t nq4,
                      const int32_t *atoms, const int32_t *cells, const double *phi,
                      const double *T, int32_t nT, double scalebroad, uint32_t mask,
                      double window_w, double sigma_min, double dq, int32_t ntargets,
                      const int32_t *targets, int32_t nq1, const int32_t *q1list,
                      const double *A, int32_t qclass,
                      int32_t want_rates, double *rates, double *rates_ch, int64_t *counts,
                      int32_t nthreads);

int oracle_rates4(const int32_t grid[3], int32_t natoms, const double *mass,
                  const double *omega, const double *evec, const double *vel, int32_t nq4,
                  const int32_t *atoms, const int32_t *cells, const double *phi,
                  const double *T, int32_t nT, double scalebroad, uint32_t mask,
                  double window_w, double sigma_min, double dq, int32_t ntargets,
                  const int32_t *targets, int32_t want_rates, double *rates,
                  double *rates_ch, int64_t *counts, int32_t nthreads) {
    return rates_core(grid, natoms, mass, omega, evec, vel, nq4, atoms, cells, phi, T, nT,
                      scalebroad, mask, window_w, sigma_min, dq, ntargets, targets, -1, NULL,
                      NULL, 0, want_rates, rates, rates_ch, counts, nthreads);
}

/* Public: four-phonon phase spaces, the rate sum of Eq. tao0 with the anharmonic strength
 * taken out (no force constants are used; the channel weights 1/2, 1/2, 1/6 and 1/N^2 stay):
 *   kind 1, weighted phase space WP4: each process contributes its occupation factor of
 *     Eq. 4phgamma (over n0_lambda) times delta / (w w' w'' w''')   [ps^5];
 *   kind 2, phase space P4: each process contributes delta          [ps].
 * The paper defines the weighting in a reference it cites without printing it; these are
 * the Eq. 4phgamma terms with |V|^2 and the prefactor hbar^2 pi / 8 set to 1.  Outputs as
 * for oracle_rates4 (counts are the same kept-process counts). */
int oracle_phase_space4(const int32_t grid[3], int32_t natoms, const double *mass,
                        const double *omega, const double *evec, const double *vel,
                        int32_t nq4, const int32_t *atoms, const int32_t *cells,
                        const double *phi, const double *T, int32_t nT, double scalebroad,
                        uint32_t mask, double window_w, double sigma_min, double dq,
                        int32_t ntargets, const int32_t *targets, int32_t kind, double *rates,
                        double *rates_ch, int64_t *counts, int32_t nthreads) {
    if (kind < 1 || kind > 2) return -1;
    return rates_core(grid, natoms, mass, omega, evec, vel, nq4, atoms, cells, phi, T, nT,
                      scalebroad, mask, window_w, sigma_min, dq, ntargets, targets, -1, NULL,
                      NULL, 0, kind + 1, rates, rates_ch, counts, nthreads);
}

/* Public: the same sum restricted to normal processes (qclass 1: Q = 0) or to Umklapp
 * processes (qclass 2: Q != 0), the two classes named after Eq. tao0.  Q is
 * k(q''') - (k(q) + s' k(q') + s'' k(q'')) with k(q) the first-Brillouin-zone image of each
 * grid point (the Cartesian image of smallest length; among images of equal length within a
 * relative 1e-10, the first in the order of the integer shift m = (m1, m2, m3), each from
 * -2 to 1, m1 slowest).  A[9]: lattice vectors as rows (Angstrom). */
int oracle_rates4_class(const int32_t grid[3], int32_t natoms, const double *mass,
                        const double *omega, const double *evec, const double *vel,
                        int32_t nq4, const int32_t *atoms, const int32_t *cells,
                        const double *phi, const double *T, int32_t nT, double scalebroad,
                        uint32_t mask, double window_w, double sigma_min, double dq,
                        int32_t ntargets, const int32_t *targets, const double *A,
                        int32_t qclass, int32_t want_rates, double *rates, double *rates_ch,
                        int64_t *counts, int32_t nthreads) {
    if (!A || qclass < 0 || qclass > 2) return -1;
    return rates_core(grid, natoms, mass, omega, evec, vel, nq4, atoms, cells, phi, T, nT,
                      scalebroad, mask, window_w, sigma_min, dq, ntargets, targets, -1, NULL,
                      A, qclass, want_rates, rates, rates_ch, counts, nthreads);
}

/* Public: the same sum restricted to the partner points q' listed in q1list[nq1] (a sample of
 * the work of the full sum, used to time the oracle on a bounded part of a workload). */
int oracle_rates4_partners(const int32_t grid[3], int32_t natoms, const double *mass,
                           const double *omega, const double *evec, const double *vel,
                           int32_t nq4, const int32_t *atoms, const int32_t *cells,
                           const double *phi, const double *T, int32_t nT, double scalebroad,
                           uint32_t mask, double window_w, double sigma_min, double dq,
                           int32_t ntargets, const int32_t *targets, int32_t nq1,
                           const int32_t *q1list, int32_t want_rates, double *rates,
                           double *rates_ch, int64_t *counts, int32_t nthreads) {
    if (nq1 < 1 || !q1list) return -1;
    for (int i = 0; i < nq1; ++i)
        if (q1list[i] < 0 || q1list[i] >= grid[0] * grid[1] * grid[2]) return -1;
    return rates_core(grid, natoms, mass, omega, evec, vel, nq4, atoms, cells, phi, T, nT,
                      scalebroad, mask, window_w, sigma_min, dq, ntargets, targets, nq1, q1list,
                      NULL, 0, want_rates, rates, rates_ch, counts, nthreads);
}

static int rates_core(const int32_t grid[3], int32_t natoms, const double *mass,
                      const double *omega, const double *evec, const double *vel, int32_t nq4,
                      const int32_t *atoms, const int32_t *cells, const double *phi,
                      const double *T, int32_t nT, double scalebroad, uint32_t mask,
                      double window_w, double sigma_min, double dq, int32_t ntargets,
                      const int32_t *targets, int32_t nq1, const int32_t *q1list,
                      const double *A, int32_t qclass,
                      int32_t want_rates, double *rates, double *rates_ch, int64_t *counts,
                      int32_t nthreads) {
    if (natoms <= 0 || nT <= 0 || ntargets < 0 || scalebroad <= 0.0 || dq <= 0.0) return -1;
    model_t m;
    model_init(&m, grid, natoms, mass, omega, evec, vel, nq4, atoms, cells, phi);
    const int N = m.N, nb = m.nb, nmodes = N * nb;
    /* first-zone Cartesian image of every grid point (only for a class-restricted sum) */
    double *kimg = NULL, Bm[9];
    if (qclass) {
        recip(A, Bm);
        kimg = (double *)malloc(sizeof(double) * 3 * (size_t)N);
        for (int iq = 0; iq < N; ++iq) first_zone(&m, Bm, iq, kimg + 3 * iq);
    }
    const int NQ1 = q1list ? nq1 : N;   /* partner points q' in the sum */
    const double c_win = ((window_w * scalebroad) * dq) * ((window_w * scalebroad) * dq);
    const double c_sig = (scalebroad * dq) * (scalebroad * dq);
    const double C4 = oracle_c4();
    const double inv_n2 = 1.0 / ((double)N * (double)N);
    const double hk = oracle_hbar_over_kb();

    /* n0 for every mode and temperature (0 for inactive modes, never used) */
    double *occ = (double *)calloc((size_t)nT * nmodes, sizeof(double));
    for (int t = 0; t < nT; ++t)
        for (int mu = 0; mu < nmodes; ++mu)
            if (omega[mu] > 0.0) occ[(size_t)t * nmodes + mu] = 1.0 / expm1(hk * omega[mu] / T[t]);

    /* partial sums per (target, q') so that the parallel loop has a fixed summation order */
    const size_t npart = (size_t)ntargets * NQ1;
    double *part = (double *)calloc(npart * nT * 3 * 2, sizeof(double)); /* sum, comp */
    int64_t *pcnt = (int64_t *)calloc(npart * 3, sizeof(int64_t));

#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        const size_t nq4a = (size_t)(m.nq4 > 0 ? m.nq4 : 1);
        cplx *W = (cplx *)malloc(sizeof(cplx) * nq4a * 9);
        cplx *X3 = (cplx *)malloc(sizeof(cplx) * nq4a * 3);
        cplx *X4all = (cplx *)malloc(sizeof(cplx) * nq4a * 3 * (size_t)nb);
        int *have4 = (int *)malloc(sizeof(int) * (size_t)nb);
#pragma omp for schedule(dynamic, 1)
        for (long long task = 0; task < (long long)npart; ++task) {
            const int it = (int)(task / NQ1), k1 = (int)(task % NQ1);
            const int iq1 = q1list ? q1list[k1] : k1;
            const int mu = targets[it];
            const int iq = mu / nb, j = mu % nb;
            double *P = part + (size_t)task * nT * 3 * 2;
            int64_t *C = pcnt + (size_t)task * 3;
            if (omega[mu] <= 0.0) continue;
            for (int ch = 0; ch < 3; ++ch) {
                if (!(mask & (1u << ch))) continue;
                const int s1 = CH_S1[ch], s2 = CH_S2[ch];
                for (int j1 = 0; j1 < nb; ++j1) {
                    const int mu1 = iq1 * nb + j1;
                    if (omega[mu1] <= 0.0) continue;
                    /* slot-1 x slot-2 partial contraction per quartet:
                     * W_n^{gt} = sum_{ab} Phi_n^{abgt} X1_n^a X2_n^b */
                    if (want_rates == 1) {
                        for (int n = 0; n < m.nq4; ++n) {
                            const int32_t *at = m.atoms + 4 * n;
                            const int32_t *cl = m.cells + 9 * n;
                            const double *ph = m.phi + 81 * (size_t)n;
                            cplx X1[3], X2[3];
                            for (int x = 0; x < 3; ++x) {
                                X1[x] = slot_factor(&m, +1, iq, j, at[0], ZERO_CELL, x);
                                X2[x] = slot_factor_n(&m, s1, iq1, j1, n, 1, x);
                            }
                            for (int c = 0; c < 3; ++c)
                                for (int d = 0; d < 3; ++d) {
                                    cplx acc = 0.0;
                                    for (int a = 0; a < 3; ++a)
                                        for (int b = 0; b < 3; ++b)
                                            acc += ph[((a * 3 + b) * 3 + c) * 3 + d] * X1[a] * X2[b];
                                    W[9 * n + 3 * c + d] = acc;
                                }
                        }
                    }
                    for (int iq2 = 0; iq2 < N; ++iq2) {
                        const int iq3 = fold(&m, iq, s1, iq1, s2, iq2);
                        if (qclass) {
                            /* Q = k(q''') - (k(q) + s' k(q') + s'' k(q'')), Cartesian */
                            double q2 = 0.0, bl = 0.0;
                            for (int x = 0; x < 3; ++x) {
                                const double Qx = kimg[3 * iq3 + x] - (kimg[3 * iq + x] + s1 * kimg[3 * iq1 + x] +
                                                                      s2 * kimg[3 * iq2 + x]);
                                q2 += Qx * Qx;
                                bl += Bm[x] * Bm[x];
                            }
                            const int umklapp = q2 > 1e-12 * bl;
                            if ((qclass == 1 && umklapp) || (qclass == 2 && !umklapp)) continue;
                        }
                        /* slot-4 factors of this q''' for each j''' (formed on first use) */
                        memset(have4, 0, sizeof(int) * (size_t)nb);
                        for (int j2 = 0; j2 < nb; ++j2) {
                            const int mu2 = iq2 * nb + j2;
                            if (omega[mu2] <= 0.0) continue;
                            int have3 = 0;
                            for (int j3 = 0; j3 < nb; ++j3) {
                                const int mu3 = iq3 * nb + j3;
                                if (omega[mu3] <= 0.0) continue;
                                double dw, s2v;
                                if (!keep_process(&m, ch, mu, mu1, mu2, mu3, c_win, &dw, &s2v)) continue;
                                C[ch] += 1;
                                if (!want_rates) continue;
                                double v2 = 1.0;   /* phase-space sums: |V|^2 := 1 */
                                if (want_rates == 1) {
                                if (!have3) {
                                    for (int n = 0; n < m.nq4; ++n)
                                        for (int x = 0; x < 3; ++x)
                                            X3[3 * n + x] = slot_factor_n(&m, s2, iq2, j2, n, 2, x);
                                    have3 = 1;
                                }
                                cplx *X4 = X4all + (size_t)j3 * nq4a * 3;
                                if (!have4[j3]) {
                                    for (int n = 0; n < m.nq4; ++n)
                                        for (int x = 0; x < 3; ++x)
                                            X4[3 * n + x] = slot_factor_n(&m, -1, iq3, j3, n, 3, x);
                                    have4[j3] = 1;
                                }
                                /* V = sum_n sum_{gt} W_n^{gt} X3_n^g X4_n^t  (Eq. V4) */
                                cplx V = 0.0;
                                for (int n = 0; n < m.nq4; ++n)
                                    for (int c = 0; c < 3; ++c) {
                                        cplx y = 0.0;
                                        for (int d = 0; d < 3; ++d) y += W[9 * n + 3 * c + d] * X4[3 * n + d];
                                        V += X3[3 * n + c] * y;
                                    }
                                v2 = creal(V) * creal(V) + cimag(V) * cimag(V);
                                }
                                const double delta = oracle_delta(dw, c_sig * s2v, sigma_min);
                                const double wprod = omega[mu] * omega[mu1] * omega[mu2] * omega[mu3];
                                for (int t = 0; t < nT; ++t) {
                                    const double *n0 = occ + (size_t)t * nmodes;
                                    double f;
                                    /* occupation factors of Eq. 4phgamma */
                                    if (ch == 0) f = (1.0 + n0[mu1]) * (1.0 + n0[mu2]) * n0[mu3] / n0[mu];
                                    else if (ch == 1) f = (1.0 + n0[mu1]) * n0[mu2] * n0[mu3] / n0[mu];
                                    else f = n0[mu1] * n0[mu2] * n0[mu3] / n0[mu];
                                    double G = C4 * inv_n2 * f * v2 * delta / wprod;
                                    if (want_rates == 2) G = inv_n2 * f * delta / wprod;    /* WP4 */
                                    else if (want_rates == 3) G = inv_n2 * delta;          /* P4 */
                                    neumaier(&P[(t * 3 + ch) * 2], &P[(t * 3 + ch) * 2 + 1], CH_W[ch] * G);
                                }
                            }
                        }
                    }
                }
            }
        }
        free(W);
        free(X3);
        free(X4all);
        free(have4);
    }

    /* ordered reduction over q' */
    for (int it = 0; it < ntargets; ++it) {
        int64_t cc[3] = {0, 0, 0};
        for (int t = 0; t < nT; ++t) {
            double tot = 0.0, totc = 0.0;
            for (int ch = 0; ch < 3; ++ch) {
                double s = 0.0, c = 0.0;
                for (int k1 = 0; k1 < NQ1; ++k1) {
                    const double *P = part + ((size_t)it * NQ1 + k1) * nT * 3 * 2;
                    neumaier(&s, &c, P[(t * 3 + ch) * 2]);
                    c += P[(t * 3 + ch) * 2 + 1];
                }
                if (rates_ch) rates_ch[((size_t)t * 3 + ch) * ntargets + it] = s + c;
                neumaier(&tot, &totc, s + c);
            }
            rates[(size_t)t * ntargets + it] = tot + totc;
        }
        for (int k1 = 0; k1 < NQ1; ++k1)
            for (int ch = 0; ch < 3; ++ch) cc[ch] += pcnt[((size_t)it * NQ1 + k1) * 3 + ch];
        if (counts) for (int ch = 0; ch < 3; ++ch) counts[3 * (size_t)it + ch] = cc[ch];
    }
    free(part); free(pcnt); free(occ); free(kimg);
    model_free(&m);
    return 0;
}

/* Default |dq| reading: (|det B| / N)^(1/3), B the reciprocal vectors (2 pi included).
 * A holds the lattice vectors as rows (Angstrom). */
double oracle_default_dq(const double A[9], const int32_t grid[3]) {
    const double detA = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                        A[2] * (A[3] * A[7] - A[4] * A[6]);
    const double detB = pow(2.0 * M_PI, 3) / fabs(detA);
    const double N = (double)grid[0] * grid[1] * grid[2];
    return cbrt(detB / N);
}

/* ======================================================================= three-phonon
 * Three-phonon RTA rate (Eq. tao0, 3ph bracket; Eq. 3phgamma; Eq. V3), used as an input
 * feature of the learned surrogate:
 *   1/tau_3ph(lambda) = (1/N) [ sum^{+} G^{+} + sum^{-} 1/2 G^{-} ]
 *   G^{+} = hbar pi/4 (n' - n'') / (w w' w'') |V^{+}|^2 delta(w + w' - w''),  q'' = q + q'
 *   G^{-} = hbar pi/4 (n' + n'' + 1) / (w w' w'') |V^{-}|^2 delta(w - w' - w''), q'' = q - q'
 *   V^{+-} = sum_{ijk} sum_{abg} Phi e_a^{l}(i) e_b^{+-l'}(j) e_g^{-l''}(k) / sqrt(MMM)
 *            exp(+-i q'.r_j) exp(-i q''.r_k)
 * Readings (same as for four phonons): the adaptive Gaussian with sigma = sb |v' - v''| |dq|
 * (derivative of the energy mismatch with respect to q' with q'' fixed by momentum), the
 * window |dw| <= W sigma evaluated squared in the fixed order dw = (w +- w') - w'',
 * s2 = (dx*dx + dy*dy) + dz*dz with d = v' - v'', delta := 1 below sigma_min, inactive modes
 * excluded.  Triplets: atoms[n][3], cells[n][2][3] (atoms j, k; atom i in the home cell),
 * phi[n][27] eV/A^3 with index (a*3+b)*3+g. */

/* hbar pi / 4 for V in eV/(A^3 amu^1.5), delta in ps, omega in rad/ps, rate in 1/ps */
double oracle_c3(void) {
    const double kv = EV / (ANG * ANG * ANG * AMU * sqrt(AMU));
    return HBAR * M_PI / 4.0 * kv * kv * 1.0e-60;
}

static cplx v3_general(const model_t *m, int n3, const int32_t *atoms, const int32_t *cells,
                       const double *phi, const int mode[3], const int sg[3]) {
    cplx V = 0.0;
    for (int n = 0; n < n3; ++n) {
        const int32_t *at = atoms + 3 * n;
        cplx X[3][3];
        for (int s = 0; s < 3; ++s) {
            const int32_t *R = s == 0 ? ZERO_CELL : cells + 6 * n + 3 * (s - 1);
            const int iq = mode[s] / m->nb, j = mode[s] % m->nb;
            for (int x = 0; x < 3; ++x) X[s][x] = slot_factor(m, sg[s], iq, j, at[s], R, x);
        }
        const double *ph = phi + 27 * (size_t)n;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                for (int c = 0; c < 3; ++c) V += ph[(a * 3 + b) * 3 + c] * X[0][a] * X[1][b] * X[2][c];
    }
    return V;
}

/* Public: V of Eq. V3 for explicit (mode, sign) triples. */
int oracle_v3(const int32_t grid[3], int32_t natoms, const double *mass, const double *omega,
              const double *evec, const double *vel, int32_t n3, const int32_t *atoms,
              const int32_t *cells, const double *phi, int32_t n, const int32_t *modes3,
              const int32_t *signs3, double *V) {
    model_t m;
    model_init(&m, grid, natoms, mass, omega, evec, vel, 0, NULL, NULL, NULL);
    for (int i = 0; i < n; ++i) {
        int md[3], sg[3];
        for (int s = 0; s < 3; ++s) { md[s] = modes3[3 * i + s]; sg[s] = signs3[3 * i + s]; }
        const cplx v = v3_general(&m, n3, atoms, cells, phi, md, sg);
        V[2 * i] = creal(v); V[2 * i + 1] = cimag(v);
    }
    model_free(&m);
    return 0;
}

/* Public: three-phonon rates rates[nT][ntargets] and kept counts counts[ntargets][2]
 * (channel +, channel -). */
int oracle_rates3(const int32_t grid[3], int32_t natoms, const double *mass,
                  const double *omega, const double *evec, const double *vel, int32_t n3,
                  const int32_t *atoms, const int32_t *cells, const double *phi,
                  const double *T, int32_t nT, double scalebroad, double window_w,
                  double sigma_min, double dq, int32_t ntargets, const int32_t *targets,
                  double *rates, int64_t *counts, int32_t nthreads) {
    if (natoms <= 0 || nT <= 0 || ntargets < 0 || scalebroad <= 0.0 || dq <= 0.0) return -1;
    model_t m;
    model_init(&m, grid, natoms, mass, omega, evec, vel, 0, NULL, NULL, NULL);
    const int N = m.N, nb = m.nb, nmodes = N * nb;
    const double c_win = ((window_w * scalebroad) * dq) * ((window_w * scalebroad) * dq);
    const double c_sig = (scalebroad * dq) * (scalebroad * dq);
    const double C3 = oracle_c3();
    const double hk = oracle_hbar_over_kb();
    double *occ = (double *)calloc((size_t)nT * nmodes, sizeof(double));
    for (int t = 0; t < nT; ++t)
        for (int mu = 0; mu < nmodes; ++mu)
            if (omega[mu] > 0.0) occ[(size_t)t * nmodes + mu] = 1.0 / expm1(hk * omega[mu] / T[t]);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int it = 0; it < ntargets; ++it) {
        const int mu = targets[it];
        double sum[8], comp[8];
        for (int t = 0; t < nT && t < 8; ++t) { sum[t] = 0.0; comp[t] = 0.0; }
        int64_t cnt[2] = {0, 0};
        if (omega[mu] > 0.0) {
            const int iq = mu / nb;
            for (int ch = 0; ch < 2; ++ch) {
                const int s1 = ch == 0 ? +1 : -1;
                for (int iq1 = 0; iq1 < N; ++iq1) {
                    /* q'' = q +- q' folded into the grid */
                    int a[3], b[3], r[3];
                    qtriple(&m, iq, a); qtriple(&m, iq1, b);
                    for (int d = 0; d < 3; ++d) r[d] = imod(a[d] + s1 * b[d], m.g[d]);
                    const int iq2 = r[0] + m.g[0] * (r[1] + m.g[1] * r[2]);
                    for (int j1 = 0; j1 < nb; ++j1) {
                        const int mu1 = iq1 * nb + j1;
                        if (omega[mu1] <= 0.0) continue;
                        for (int j2 = 0; j2 < nb; ++j2) {
                            const int mu2 = iq2 * nb + j2;
                            if (omega[mu2] <= 0.0) continue;
                            const double w = omega[mu], w1 = omega[mu1], w2 = omega[mu2];
                            const double aw = s1 > 0 ? w + w1 : w - w1;
                            const double dw = aw - w2;
                            const double *v1 = vel + 3 * (size_t)mu1, *v2 = vel + 3 * (size_t)mu2;
                            const double dx = v1[0] - v2[0], dy = v1[1] - v2[1], dz = v1[2] - v2[2];
                            const double s2 = (dx * dx + dy * dy) + dz * dz;
                            if (!(dw * dw <= c_win * s2)) continue;
                            cnt[ch] += 1;
                            const int md[3] = {mu, mu1, mu2};
                            const int sg[3] = {+1, s1, -1};
                            const cplx V = v3_general(&m, n3, atoms, cells, phi, md, sg);
                            const double v2abs = creal(V) * creal(V) + cimag(V) * cimag(V);
                            const double delta = oracle_delta(dw, c_sig * s2, sigma_min);
                            for (int t = 0; t < nT && t < 8; ++t) {
                                const double *n0 = occ + (size_t)t * nmodes;
                                const double f = ch == 0 ? n0[mu1] - n0[mu2] : n0[mu1] + n0[mu2] + 1.0;
                                const double G = C3 * f * v2abs * delta / (w * w1 * w2);
                                neumaier(&sum[t], &comp[t], (ch == 0 ? 1.0 : 0.5) * G / (double)N);
                            }
                        }
                    }
                }
            }
        }
        for (int t = 0; t < nT && t < 8; ++t) rates[(size_t)t * ntargets + it] = sum[t] + comp[t];
        if (counts) { counts[2 * (size_t)it] = cnt[0]; counts[2 * (size_t)it + 1] = cnt[1]; }
    }
    free(occ);
    model_free(&m);
    return 0;
}

/* ======================================================================= thermal conductivity
 * Public: RTA lattice thermal conductivity with three- and four-phonon scattering (the
 * single-mode relaxation time of Eq. tao0 without the isotope term, F = tau v from Eq. BTE
 * in the relaxation-time approximation).  The paper takes the conductivity expression from
 * ShengBTE without printing it; the reading used here is the standard kinetic one:
 *   kappa^{ab} = 1/(N Omega) sum_lambda C_lambda v_lambda^a v_lambda^b tau_lambda,
 *   C_lambda = k_B x^2 n0 (n0 + 1),  x = hbar w / (k_B T),
 *   1/tau_lambda = 1/tau3 + 1/tau4,
 * with Omega the cell volume |det A|.  Modes with w <= 0 or with zero total rate take no part
 * (their count is returned in nskip[t]).  Inputs rates3/rates4 [nT][nmodes] in 1/ps, omega
 * rad/ps, vel [nmodes][3] A/ps, A [9] Angstrom; output kappa [nT][3][3] in W/(m K). */
int oracle_kappa_rta(const int32_t grid[3], int32_t natoms, const double *omega,
                     const double *vel, const double A[9], const double *T, int32_t nT,
                     const double *rates3, const double *rates4, double *kappa,
                     int64_t *nskip) {
    if (natoms <= 0 || nT <= 0) return -1;
    const long N = (long)grid[0] * grid[1] * grid[2];
    const long nmodes = N * 3 * natoms;
    const double omega_cell = fabs(A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                                   A[2] * (A[3] * A[7] - A[4] * A[6])) * 1e-30;   /* m^3 */
    const double hk = oracle_hbar_over_kb();
    for (int t = 0; t < nT; ++t) {
        double s[9], c[9];
        for (int e = 0; e < 9; ++e) { s[e] = 0.0; c[e] = 0.0; }
        int64_t skipped = 0;
        for (long mu = 0; mu < nmodes; ++mu) {
            const double w = omega[mu];
            const double rate = rates3[(size_t)t * nmodes + mu] + rates4[(size_t)t * nmodes + mu];
            if (!(w > 0.0) || !(rate > 0.0)) { skipped += w > 0.0; continue; }
            const double x = hk * w / T[t];
            const double n0 = oracle_bose(w, T[t]);
            const double cap = KB * x * x * n0 * (n0 + 1.0);          /* J/K */
            const double tau = 1e-12 / rate;                            /* s */
            const double *v = vel + 3 * (size_t)mu;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    neumaier(&s[3 * a + b], &c[3 * a + b], cap * (v[a] * 100.0) * (v[b] * 100.0) * tau);
        }
        for (int e = 0; e < 9; ++e) kappa[(size_t)t * 9 + e] = (s[e] + c[e]) / ((double)N * omega_cell);
        if (nskip) nskip[t] = skipped;
    }
    return 0;
}
