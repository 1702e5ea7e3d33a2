/*
 * fpt_oracle.h -- reference (oracle) implementation of the first-passage-time
 * method of Pierro, Troiano, Mejuto, Filatrella, "Stochastic first passage time
 * accelerated with CUDA" (arXiv:1802.05065).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded FP64
 * program that the tests and the CPU-baseline leg of the benchmark use to
 * check the GPU library.  It shares no code, header, table or constant with
 * the GPU library, and the GPU library never calls it.
 *
 * Conventions (all readings of the paper are listed in the design notes):
 *   - model 0 = underdamped Josephson junction, the Euler update of
 *     Algorithm 1 (EscapeTime) and Algorithm 3 (SwitchingCurrent), Sect. III.B;
 *     scheme 1 replaces it by the semi-implicit (symplectic) Euler variant,
 *     v first and then phi with the new v (an extension, not in the paper);
 *     model 1 = overdamped washboard, the first-order analogue mentioned in
 *     Sect. II.B (the paper prints no algorithm for it):
 *     phi' = -V0 sin(phi) + gamma + noise, potential -V0 cos(phi) - gamma phi,
 *     whose well is at arcsin(gamma / V0); the NaN defaults of phi0 and of
 *     the threshold (pi - phi0) follow it (V0 = 0 is the plain drift-diffusion
 *     walk and needs explicit values).
 *   - noise amplitude D = alpha*T (Eq. (9): D = beta*theta with beta -> alpha,
 *     theta -> T); per-step noise sigma*r with sigma = sqrt(2*D*h) as in
 *     Algorithm 1.  Overdamped: sigma = sqrt(2*T*h).
 *   - bias at step k: gamma_k = gamma0 + ramp*dt*k (Algorithm 3, delta-gamma =
 *     ramp*dt; ramp = 0 gives the fixed bias of Algorithm 1).
 *   - Gaussian draws: Box-Muller on Philox4x32-10 words keyed by
 *     (seed, replica, block), replacing the paper's Mersenne Twister
 *     (Algorithm 2) by a counter-based generator; rng = 1 selects the paper's
 *     generator instead: one MT19937 per replica seeded with seed + replica
 *     (Sect. III.B), its words taken 4 per block in stream order.
 */
#ifndef FPT_ORACLE_H
#define FPT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t model;       /* 0 underdamped, 1 overdamped */
  int32_t scheme;      /* underdamped: 0 explicit (Algorithm 1), 1 semi-implicit */
  int32_t rng;         /* 0 Philox4x32-10; 1 MT19937 per replica (Algorithm 2) */
  int32_t reserved;
  double alpha;        /* damping (beta of Eq. (10)) */
  double T;            /* temperature (theta of Eq. (9)) */
  double V0;           /* potential amplitude of Eq. (10) */
  double gamma0;       /* bias at t = 0 */
  double ramp;         /* d gamma / dt (per unit time); 0 = fixed bias */
  double dt;           /* Euler step h */
  double phi0;         /* initial phase; NaN -> arcsin(gamma0) */
  double v0;           /* initial velocity; NaN -> 0 */
  double threshold;    /* escape when phi > threshold; NaN -> pi - phi0 */
  int64_t max_steps;   /* klim: steps k = 1..max_steps are tried */
  uint64_t seed;       /* Philox key */
} oracle_params;

typedef struct {
  uint64_t n_escaped, n_censored, n_overflow;
  uint64_t sum_k;
  uint64_t sum_k2_lo, sum_k2_hi;  /* 128-bit sum of k^2 */
  double mean_t, se_t;            /* over escaped replicas, in time units */
} oracle_moments;

/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11).
 * ctr[0..3], key[0..1] -> out[0..3]. */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                          uint32_t out[4]);

/* Words for (seed, replica, block): key = (seed lo, seed hi),
 * counter = (block lo, block hi, replica lo, replica hi). */
void oracle_rng_words(uint64_t seed, uint64_t replica, uint64_t block,
                      uint32_t out[4]);

/* The four standard normals of one block (Box-Muller, both outputs of each
 * pair): z[0], z[1] from words 0,1 and z[2], z[3] from words 2,3. */
void oracle_normals(uint64_t seed, uint64_t replica, uint64_t block,
                    double z[4]);

/* MT19937 (Matsumoto, Nishimura 1998): the first n outputs of the generator
 * seeded by the standard initialization with the 32-bit seed. */
void oracle_mt19937(uint32_t seed, uint64_t n, uint32_t* out);

/* Resolve NaN defaults and the per-step constants of the plan.
 * sigma_out, dgamma_out, phi0_out, v0_out, th_out may be NULL. */
void oracle_derived(const oracle_params* p, double* sigma_out,
                    double* dgamma_out, double* phi0_out, double* v0_out,
                    double* th_out);

/* First passage step of one replica: the smallest k in [1, max_steps] with
 * phi_k > threshold, or -1.  phi_end/v_end (nullable) receive the state at
 * that step (or at max_steps). */
int64_t oracle_escape_step(const oracle_params* p, uint64_t replica,
                           double* phi_end, double* v_end);

/* Replicas first .. first+n-1; steps[i] and (nullable) phi_end[i]. */
void oracle_run(const oracle_params* p, uint64_t first, uint64_t n,
                int64_t* steps, double* phi_end);

/* Free trajectory (no threshold) of one replica for n_steps steps:
 * phi[k-1], v[k-1] are the state after step k.  v may be NULL. */
void oracle_trajectory(const oracle_params* p, uint64_t replica,
                       int64_t n_steps, double* phi, double* v);

/* Histogram of escape steps over [1, k_hist] in n_bins uniform integer bins:
 * bin(k) = ((k-1)*n_bins) div k_hist; k > k_hist counts as overflow, k = -1
 * as censored.  Moments over escaped replicas (k >= 1), times = k*dt. */
void oracle_histogram(const int64_t* steps, uint64_t n, int32_t n_bins,
                      int64_t k_hist, double dt, uint64_t* hist,
                      oracle_moments* m);

/* Total replica-steps of a result array: sum of k, censored replicas counted
 * at max_steps. */
uint64_t oracle_replica_steps(const int64_t* steps, uint64_t n,
                              int64_t max_steps);

#ifdef __cplusplus
}
#endif
#endif /* FPT_ORACLE_H */
