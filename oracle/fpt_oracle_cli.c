/*
 * fpt_oracle_cli.c -- command-line driver of the oracle, used to time the
 * plain FP64 method on host cores (CPU baseline of the benchmark).
 * TEST INFRASTRUCTURE ONLY.
 *
 * usage: fpt_oracle_cli model alpha T V0 gamma0 ramp dt phi0 v0 threshold
 *                       max_steps seed first n
 * (use "nan" for defaulted phi0 / v0 / threshold).  Prints one line:
 *   first n replica_steps n_escaped seconds
 * and then one escape step per replica.
 */
#define _POSIX_C_SOURCE 199309L
#include <stdio.h>
#include <stdlib.h>
#include <time.h>

#include "fpt_oracle.h"

static double now_s(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

int main(int argc, char** argv) {
  if (argc != 15) {
    fprintf(stderr,
            "usage: %s model alpha T V0 gamma0 ramp dt phi0 v0 threshold "
            "max_steps seed first n\n",
            argv[0]);
    return 2;
  }
  oracle_params p;
  p.model = atoi(argv[1]);
  p.scheme = 0;
  p.rng = 0;
  p.reserved = 0;
  p.alpha = strtod(argv[2], NULL);
  p.T = strtod(argv[3], NULL);
  p.V0 = strtod(argv[4], NULL);
  p.gamma0 = strtod(argv[5], NULL);
  p.ramp = strtod(argv[6], NULL);
  p.dt = strtod(argv[7], NULL);
  p.phi0 = strtod(argv[8], NULL);
  p.v0 = strtod(argv[9], NULL);
  p.threshold = strtod(argv[10], NULL);
  p.max_steps = strtoll(argv[11], NULL, 10);
  p.seed = strtoull(argv[12], NULL, 10);
  const uint64_t first = strtoull(argv[13], NULL, 10);
  const uint64_t n = strtoull(argv[14], NULL, 10);
  int64_t* steps = (int64_t*)malloc(sizeof(int64_t) * (n ? n : 1));
  if (!steps) return 3;
  const double t0 = now_s();
  oracle_run(&p, first, n, steps, NULL);
  const double t1 = now_s();
  uint64_t n_esc = 0;
  for (uint64_t i = 0; i < n; ++i) n_esc += steps[i] >= 1;
  printf("%llu %llu %llu %llu %.9f\n", (unsigned long long)first,
         (unsigned long long)n,
         (unsigned long long)oracle_replica_steps(steps, n, p.max_steps),
         (unsigned long long)n_esc, t1 - t0);
  for (uint64_t i = 0; i < n; ++i) printf("%lld\n", (long long)steps[i]);
  free(steps);
  return 0;
}
