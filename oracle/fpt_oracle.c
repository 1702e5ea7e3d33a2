/*
 * fpt_oracle.c -- the oracle: a plain single-threaded FP64 implementation of
 * the escape-time / switching-current method of arXiv:1802.05065.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU
 * baseline of the benchmark.  It is written from the paper, shares nothing
 * with the GPU library and is never linked into it.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared (no fast-math), so
 * every expression below is evaluated in IEEE double in source order.
 */
#include "fpt_oracle.h"

#include <math.h>
#include <stddef.h>

/* pi rounded to double */
static const double PI = 3.14159265358979323846;

/* ---------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon et al., SC'11, "Parallel random numbers: as easy as
 * 1, 2, 3").  One round maps (x0, x1, x2, x3) with key (k0, k1) to
 *   (hi(B*x2) ^ x1 ^ k0,  lo(B*x2),  hi(A*x0) ^ x3 ^ k1,  lo(A*x0))
 * with A = 0xD2511F53, B = 0xCD9E8D57; the key is bumped by the Weyl
 * constants (0x9E3779B9, 0xBB67AE85) between rounds.                      */

static void philox_round(uint32_t x[4], uint32_t k0, uint32_t k1) {
  const uint64_t pa = (uint64_t)0xD2511F53u * (uint64_t)x[0];
  const uint64_t pb = (uint64_t)0xCD9E8D57u * (uint64_t)x[2];
  const uint32_t y0 = (uint32_t)(pb >> 32) ^ x[1] ^ k0;
  const uint32_t y1 = (uint32_t)pb;
  const uint32_t y2 = (uint32_t)(pa >> 32) ^ x[3] ^ k1;
  const uint32_t y3 = (uint32_t)pa;
  x[0] = y0;
  x[1] = y1;
  x[2] = y2;
  x[3] = y3;
}

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                          uint32_t out[4]) {
  uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    philox_round(x, k0, k1);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  for (int i = 0; i < 4; ++i) out[i] = x[i];
}

void oracle_rng_words(uint64_t seed, uint64_t replica, uint64_t block,
                      uint32_t out[4]) {
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  const uint32_t ctr[4] = {(uint32_t)block, (uint32_t)(block >> 32),
                           (uint32_t)replica, (uint32_t)(replica >> 32)};
  oracle_philox4x32_10(ctr, key, out);
}

/* ---------------------------------------------------------------------- */
/* Algorithm 2's generator, MT19937 (Matsumoto and Nishimura, ACM TOMACS 8,
 * 1998), taken straight from its defining linear recurrence over words of
 * w = 32 bits with degree n = 624, middle distance m = 397, separation r = 31:
 *   x_{k+n} = x_{k+m} xor A(upper bit of x_k | lower 31 bits of x_{k+1}),
 *   A(y) = (y >> 1) xor (0x9908b0df if y is odd else 0),
 * started from x_0 = seed, x_i = 1812433253 (x_{i-1} xor (x_{i-1} >> 30)) + i
 * for i = 1 .. n-1.  Output number t (t = 0, 1, ...) is x_{n+t} passed through
 * the tempering map (shifts 11, 7, 15, 18 with masks 0x9d2c5680 and
 * 0xefc60000).  The state keeps the last n terms of the sequence; each call
 * computes the next term from three of them, so no batch regeneration is
 * needed.                                                                   */

enum { MT_N = 624, MT_M = 397 };

typedef struct {
  uint32_t x[MT_N]; /* x[t mod n] holds term t for the n most recent terms */
  uint64_t k;       /* index of the oldest stored term */
} mt_state;

static void mt_seed(mt_state* s, uint32_t seed) {
  uint32_t prev = seed;
  s->x[0] = seed;
  for (uint32_t i = 1; i < MT_N; ++i) {
    prev = 1812433253u * (prev ^ (prev >> 30)) + i;
    s->x[i] = prev;
  }
  s->k = 0;
}

static uint32_t mt_temper(uint32_t y) {
  y ^= y >> 11;
  y ^= (y << 7) & 0x9d2c5680u;
  y ^= (y << 15) & 0xefc60000u;
  return y ^ (y >> 18);
}

static uint32_t mt_next(mt_state* s) {
  static const uint32_t odd_term[2] = {0u, 0x9908b0dfu};
  const uint32_t xk = s->x[s->k % MT_N];
  const uint32_t xk1 = s->x[(s->k + 1) % MT_N];
  const uint32_t xkm = s->x[(s->k + MT_M) % MT_N];
  const uint32_t y = (xk & 0x80000000u) | (xk1 & 0x7fffffffu);
  const uint32_t next = xkm ^ (y >> 1) ^ odd_term[y & 1u];
  /* term k + n replaces term k, which is no longer needed */
  s->x[s->k % MT_N] = next;
  s->k += 1;
  return mt_temper(next);
}

void oracle_mt19937(uint32_t seed, uint64_t n, uint32_t* out) {
  mt_state s;
  mt_seed(&s, seed);
  for (uint64_t i = 0; i < n; ++i) out[i] = mt_next(&s);
}

/* ---------------------------------------------------------------------- */
/* nrand() of Sect. III.B: Box-Muller on uniforms.  A 32-bit word x maps to
 * u = (x + 1/2) 2^-32, which lies strictly inside (0, 1) so log(u) is finite.
 * Each pair of uniforms (a, b) gives two normals
 *   sqrt(-2 ln a) cos(2 pi b),  sqrt(-2 ln a) sin(2 pi b).               */

static double word_to_uniform(uint32_t x) {
  return ((double)x + 0.5) * 0x1p-32;
}

static void box_muller4(const uint32_t w[4], double z[4]) {
  for (int pair = 0; pair < 2; ++pair) {
    const double a = word_to_uniform(w[2 * pair]);
    const double b = word_to_uniform(w[2 * pair + 1]);
    const double radius = sqrt(-2.0 * log(a));
    const double angle = 2.0 * PI * b;
    z[2 * pair] = radius * cos(angle);
    z[2 * pair + 1] = radius * sin(angle);
  }
}

void oracle_normals(uint64_t seed, uint64_t replica, uint64_t block,
                    double z[4]) {
  uint32_t w[4];
  oracle_rng_words(seed, replica, block, w);
  box_muller4(w, z);
}

/* Source of the 4 words of each block of one replica. */
typedef struct {
  int rng;
  uint64_t seed, replica;
  mt_state mt;
} word_source;

static void source_init(word_source* src, const oracle_params* p, uint64_t replica) {
  src->rng = p->rng;
  src->seed = p->seed;
  src->replica = replica;
  if (p->rng == 1) mt_seed(&src->mt, (uint32_t)(p->seed + replica));
}

static void source_normals(word_source* src, uint64_t block, double z[4]) {
  uint32_t w[4];
  if (src->rng == 1) {
    for (int i = 0; i < 4; ++i) w[i] = mt_next(&src->mt);
  } else {
    oracle_rng_words(src->seed, src->replica, block, w);
  }
  box_muller4(w, z);
}

/* ---------------------------------------------------------------------- */
/* Plan constants (Algorithm 1 / Algorithm 3 preamble).                    */

void oracle_derived(const oracle_params* p, double* sigma_out,
                    double* dgamma_out, double* phi0_out, double* v0_out,
                    double* th_out) {
  double sigma;
  if (p->model == 0) {
    /* sigma = sqrt(2 D h), D = beta*theta (Eq. (9)) = alpha*T */
    const double D = p->alpha * p->T;
    sigma = sqrt(2.0 * D * p->dt);
  } else {
    sigma = sqrt(2.0 * p->T * p->dt);
  }
  /* phi0 = the bottom of the well: arcsin(gamma) for Eq. (10), where V0
   * multiplies the bias as well; arcsin(gamma / V0) for the overdamped
   * potential -V0 cos(phi) - gamma phi */
  const double well_sin = p->model == 0 ? p->gamma0 : p->gamma0 / p->V0;
  const double phi0 = isnan(p->phi0) ? asin(well_sin) : p->phi0;
  const double v0 = isnan(p->v0) ? 0.0 : p->v0;
  /* th = pi - phi0: the top of the barrier of the tilted washboard */
  const double th = isnan(p->threshold) ? PI - phi0 : p->threshold;
  if (sigma_out) *sigma_out = sigma;
  if (dgamma_out) *dgamma_out = p->ramp * p->dt;
  if (phi0_out) *phi0_out = phi0;
  if (v0_out) *v0_out = v0;
  if (th_out) *th_out = th;
}

/* ---------------------------------------------------------------------- */
/* The replica loop of Algorithms 1 and 3.
 *
 * Underdamped (Algorithm 1, Eq. (10) with V0):
 *   phi_k = phi_{k-1} + h v_{k-1}
 *   v_k   = v_{k-1} + h (-alpha v_{k-1} - V0 sin phi_{k-1} + V0 gamma_k)
 *           + sigma r_k
 * Both updates read the state of step k-1 (explicit Euler-Maruyama).
 * Overdamped (first-order analogue, potential -V0 cos(phi) - gamma phi):
 *   phi_k = phi_{k-1} + h (-V0 sin phi_{k-1} + gamma_k) + sigma r_k
 * Escape: first k with phi_k > th (strict); none within max_steps -> -1.
 * r_k is normal number (k-1) mod 4 of block (k-1) div 4.                  */

typedef struct {
  double sigma, dgamma, phi, v, th;
} run_state;

static void load_state(const oracle_params* p, run_state* s) {
  oracle_derived(p, &s->sigma, &s->dgamma, &s->phi, &s->v, &s->th);
}

/* One Euler step k (k >= 1) with normal r; updates phi, v. */
static void euler_step(const oracle_params* p, run_state* s, int64_t k,
                       double r) {
  const double gamma_k = p->gamma0 + s->dgamma * (double)k;
  if (p->model == 0) {
    const double phi_new = s->phi + p->dt * s->v;
    const double force =
        -p->alpha * s->v - p->V0 * sin(s->phi) + p->V0 * gamma_k;
    const double v_new = s->v + p->dt * force + s->sigma * r;
    /* explicit: phi moves with v_{k-1}; semi-implicit: with v_k */
    s->phi = p->scheme == 1 ? s->phi + p->dt * v_new : phi_new;
    s->v = v_new;
  } else {
    const double drift = -p->V0 * sin(s->phi) + gamma_k;
    s->phi = s->phi + p->dt * drift + s->sigma * r;
  }
}

int64_t oracle_escape_step(const oracle_params* p, uint64_t replica,
                           double* phi_end, double* v_end) {
  run_state s;
  load_state(p, &s);
  word_source src;
  source_init(&src, p, replica);
  double z[4] = {0, 0, 0, 0};
  int64_t result = -1;
  for (int64_t k = 1; k <= p->max_steps; ++k) {
    const int64_t j = (k - 1) / 4;
    const int q = (int)((k - 1) % 4);
    if (q == 0) source_normals(&src, (uint64_t)j, z);
    euler_step(p, &s, k, z[q]);
    if (s.phi > s.th) {
      result = k;
      break;
    }
  }
  if (phi_end) *phi_end = s.phi;
  if (v_end) *v_end = s.v;
  return result;
}

void oracle_run(const oracle_params* p, uint64_t first, uint64_t n,
                int64_t* steps, double* phi_end) {
  for (uint64_t i = 0; i < n; ++i) {
    double phi = 0.0;
    steps[i] = oracle_escape_step(p, first + i, &phi, NULL);
    if (phi_end) phi_end[i] = phi;
  }
}

void oracle_trajectory(const oracle_params* p, uint64_t replica,
                       int64_t n_steps, double* phi, double* v) {
  run_state s;
  load_state(p, &s);
  word_source src;
  source_init(&src, p, replica);
  double z[4] = {0, 0, 0, 0};
  for (int64_t k = 1; k <= n_steps; ++k) {
    const int64_t j = (k - 1) / 4;
    const int q = (int)((k - 1) % 4);
    if (q == 0) source_normals(&src, (uint64_t)j, z);
    euler_step(p, &s, k, z[q]);
    phi[k - 1] = s.phi;
    if (v) v[k - 1] = s.v;
  }
}

/* ---------------------------------------------------------------------- */
/* Histogram and moments of the recorded escape steps (the escape-time and
 * switching-current histograms of Sect. II.B and IV.B).                   */

void oracle_histogram(const int64_t* steps, uint64_t n, int32_t n_bins,
                      int64_t k_hist, double dt, uint64_t* hist,
                      oracle_moments* m) {
  for (int32_t b = 0; b < n_bins; ++b) hist[b] = 0;
  uint64_t n_esc = 0, n_cens = 0, n_over = 0, sum_k = 0;
  unsigned __int128 sum_k2 = 0;
  for (uint64_t i = 0; i < n; ++i) {
    const int64_t k = steps[i];
    if (k < 1) {
      ++n_cens;
      continue;
    }
    ++n_esc;
    sum_k += (uint64_t)k;
    sum_k2 += (unsigned __int128)k * (unsigned __int128)k;
    if (k > k_hist) {
      ++n_over;
    } else {
      const int64_t b = ((k - 1) * (int64_t)n_bins) / k_hist;
      hist[b] += 1;
    }
  }
  m->n_escaped = n_esc;
  m->n_censored = n_cens;
  m->n_overflow = n_over;
  m->sum_k = sum_k;
  m->sum_k2_lo = (uint64_t)sum_k2;
  m->sum_k2_hi = (uint64_t)(sum_k2 >> 64);
  m->mean_t = NAN;
  m->se_t = NAN;
  if (n_esc > 0) m->mean_t = dt * ((double)sum_k / (double)n_esc);
  if (n_esc > 1) {
    /* n*sum(k^2) - (sum k)^2 = n^2 * (population variance), exact */
    const unsigned __int128 nn = (unsigned __int128)n_esc;
    const unsigned __int128 m2 =
        nn * sum_k2 - (unsigned __int128)sum_k * (unsigned __int128)sum_k;
    const double var_mean =
        (double)m2 / ((double)n_esc * (double)n_esc * (double)(n_esc - 1));
    m->se_t = dt * sqrt(var_mean);
  }
}

uint64_t oracle_replica_steps(const int64_t* steps, uint64_t n,
                              int64_t max_steps) {
  uint64_t total = 0;
  for (uint64_t i = 0; i < n; ++i)
    total += steps[i] >= 1 ? (uint64_t)steps[i] : (uint64_t)max_steps;
  return total;
}
