/* Test driver for the oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU test
 * infrastructure; built and run by tests/test_oracle_sanitizers.py).  Reads the arguments of
 * oracle_rates4 from raw little-endian files in a directory, runs it, writes the rates and
 * counts back, and frees everything, so that the sanitizers see every access the oracle makes
 * and every allocation it leaves behind. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_rates4(const int32_t grid[3], int32_t natoms, const double *mass,
                  const double *omega, const double *evec, const double *vel, int32_t nq4,
                  const int32_t *atoms, const int32_t *cells, const double *phi,
                  const double *T, int32_t nT, double scalebroad, uint32_t mask,
                  double window_w, double sigma_min, double dq, int32_t ntargets,
                  const int32_t *targets, int32_t want_rates, double *rates,
                  double *rates_ch, int64_t *counts, int32_t nthreads);

static void *read_all(const char *dir, const char *name, size_t *bytes) {
  char path[4096];
  snprintf(path, sizeof path, "%s/%s", dir, name);
  FILE *f = fopen(path, "rb");
  if (!f) { fprintf(stderr, "cannot open %s\n", path); exit(2); }
  fseek(f, 0, SEEK_END);
  const long n = ftell(f);
  fseek(f, 0, SEEK_SET);
  void *p = malloc(n > 0 ? (size_t)n : 1);
  if (n > 0 && fread(p, 1, (size_t)n, f) != (size_t)n) { fprintf(stderr, "short read %s\n", path); exit(2); }
  fclose(f);
  *bytes = (size_t)n;
  return p;
}

static void write_all(const char *dir, const char *name, const void *p, size_t bytes) {
  char path[4096];
  snprintf(path, sizeof path, "%s/%s", dir, name);
  FILE *f = fopen(path, "wb");
  if (!f || fwrite(p, 1, bytes, f) != bytes) { fprintf(stderr, "cannot write %s\n", path); exit(2); }
  fclose(f);
}

int main(int argc, char **argv) {
  if (argc != 2) { fprintf(stderr, "usage: %s DIR\n", argv[0]); return 2; }
  const char *d = argv[1];
  size_t nb;
  int32_t *grid = read_all(d, "grid.i32", &nb);
  int32_t *ints = read_all(d, "ints.i32", &nb);     /* natoms, nq4, nT, mask, ntargets */
  double *scal = read_all(d, "scal.f64", &nb);      /* scalebroad, window_w, sigma_min, dq */
  double *mass = read_all(d, "mass.f64", &nb);
  double *omega = read_all(d, "omega.f64", &nb);
  double *evec = read_all(d, "evec.f64", &nb);
  double *vel = read_all(d, "vel.f64", &nb);
  int32_t *atoms = read_all(d, "atoms.i32", &nb);
  int32_t *cells = read_all(d, "cells.i32", &nb);
  double *phi = read_all(d, "phi.f64", &nb);
  double *T = read_all(d, "T.f64", &nb);
  int32_t *targets = read_all(d, "targets.i32", &nb);
  const int32_t nT = ints[2], nt = ints[4];
  double *rates = calloc((size_t)nT * nt, sizeof(double));
  double *rch = calloc((size_t)nT * 3 * nt, sizeof(double));
  int64_t *counts = calloc((size_t)nt * 3, sizeof(int64_t));
  const int rc = oracle_rates4(grid, ints[0], mass, omega, evec, vel, ints[1], atoms, cells, phi,
                               T, nT, scal[0], (uint32_t)ints[3], scal[1], scal[2], scal[3], nt,
                               targets, 1, rates, rch, counts, 0);
  write_all(d, "rates.f64", rates, (size_t)nT * nt * sizeof(double));
  write_all(d, "counts.i64", counts, (size_t)nt * 3 * sizeof(int64_t));
  free(grid); free(ints); free(scal); free(mass); free(omega); free(evec); free(vel);
  free(atoms); free(cells); free(phi); free(T); free(targets);
  free(rates); free(rch); free(counts);
  return rc;
}
