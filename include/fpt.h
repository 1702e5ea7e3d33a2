/*
 * fpt.h -- C ABI of the MI355X (gfx950) first-passage-time library.
 *
 * The library integrates many independent Langevin replicas of a Josephson
 * junction in a tilted washboard potential, each until its phase crosses a
 * threshold, records every first-passage step and bins the steps into
 * escape-time / switching-current histograms.  The method is that of
 * Pierro, Troiano, Mejuto, Filatrella, "Stochastic first passage time
 * accelerated with CUDA" (arXiv:1802.05065):
 *   - Eq. (10): phi'' + beta phi' = V0 (-sin phi + gamma + gamma_N), with the
 *     noise strength of Eqs. (11)-(12), D = beta theta (Eq. (9));
 *   - Algorithm 1 (EscapeTime): explicit Euler-Maruyama from
 *     (phi0, v0) = (arcsin gamma, 0) until phi > pi - phi0, recording k*h or
 *     -1 after klim steps;
 *   - Algorithm 3 (SwitchingCurrent): the same with the bias ramped by
 *     delta-gamma per step, recording the bias at the crossing;
 *   - Sect. III.B: one realization per thread, a finished thread takes the
 *     next job (the streaming figure), the escape times land in an array.
 *
 * Conventions shared by every call:
 *   - Units are the paper's normalized units with the damping called alpha
 *     (beta in Eq. (10)) and the temperature called T (theta in Eq. (9)).
 *     Underdamped step k (k = 1, 2, ...), both updates from step k-1 values:
 *       phi_k = phi_{k-1} + dt v_{k-1}
 *       v_k   = v_{k-1} + dt (-alpha v_{k-1} - V0 sin phi_{k-1} + V0 gamma_k)
 *               + sqrt(2 alpha T dt) r_k
 *     Overdamped (first-order analogue, Sect. II.B; potential
 *     -V0 cos(phi) - gamma phi):
 *       phi_k = phi_{k-1} + dt (-V0 sin phi_{k-1} + gamma_k) + sqrt(2 T dt) r_k
 *     with gamma_k = gamma0 + ramp*dt*k evaluated in FP64 from the integer k.
 *   - r_k is standard normal number (k-1) mod 4 of block (k-1) div 4 of the
 *     replica: Philox4x32-10 with key = seed and counter = (block, replica
 *     index within its parameter set), mapped u = (x + 1/2) 2^-32 and
 *     Box-Muller (cos, sin) on word pairs (0,1) and (2,3).  Results therefore
 *     depend only on (parameters, seed, replica index), never on the lane,
 *     launch shape, tuning or on other sets running at the same time.
 *   - Escape: the first k in [1, max_steps] with phi_k > threshold (strict).
 *     None: the replica is censored and recorded as -1.
 *   - Escape steps are int64; time = k*dt and switching bias = gamma_k are
 *     derived by the caller in FP64.
 *   - Device pointers are plain HIP device addresses (e.g. torch tensors'
 *     data_ptr()); streams are hipStream_t passed as void* (NULL = default).
 *     The caller owns every buffer it passes; the library never frees them.
 *   - Errors are negative fpt_status values; fpt_last_error() returns the
 *     calling thread's last message.  No call aborts or throws across the ABI.
 */
#ifndef FPT_H
#define FPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FPT_API_VERSION 2
#define FPT_MAX_BINS 4096

typedef enum {
  FPT_OK = 0,
  FPT_PENDING = 1,      /* fpt_poll: job admitted or queued, not finished */
  FPT_E_INVAL = -1,     /* bad argument; nothing was launched */
  FPT_E_NOMEM = -2,     /* workspace / pool too small for the request */
  FPT_E_DEVICE = -3,    /* a HIP call failed (message names it) */
  FPT_E_BUSY = -4,      /* server queue full */
  FPT_E_NOTFOUND = -5,  /* unknown job id */
  FPT_E_STATE = -6      /* call out of order (e.g. histogram before simulate) */
} fpt_status;

typedef enum { FPT_UNDERDAMPED = 0, FPT_OVERDAMPED = 1 } fpt_model;

/* FPT_EXPLICIT: Algorithm 1's update, both phi and v from step k-1 values
 * (small oscillations grow by 1 - h alpha + h^2 per step: unstable when
 * dt cos(phi*) > alpha).  FPT_SEMI_IMPLICIT: v_k first, then
 * phi_k = phi_{k-1} + dt v_k (symplectic Euler, per-step factor 1 - h alpha;
 * same cost).  Underdamped model only. */
typedef enum { FPT_EXPLICIT = 0, FPT_SEMI_IMPLICIT = 1 } fpt_scheme;

/* FPT_FP64: every replica operation in FP64 (the plain path); sin, the
 * Box-Muller log and sin/cos within about 2 ulp of their correctly rounded
 * values.
 * FPT_FP32C: replica state in FP32 with a compensated phase (a float pair
 * between 4-step blocks; each block's advance, summed in FP32, is added with
 * Kahan's compensation); FP64 is kept for gamma_k from the exact integer
 * step and for the threshold test near the threshold.  The same Philox words
 * feed both. */
typedef enum { FPT_FP64 = 0, FPT_FP32C = 1 } fpt_precision;

/* Normal-number source.  FPT_RNG_PHILOX: the counter-based generator above.
 * FPT_RNG_MT19937: Algorithm 2's generator, one MT19937 per replica seeded
 * by the standard 32-bit initialization with (seed + replica index) mod 2^32
 * (Sect. III.B); block j of a replica takes its outputs 4j .. 4j+3 and the
 * same Box-Muller map.  Its 2.5 KB state per resident lane lives in the
 * workspace.  MT19937 plans take one parameter set and one replica per lane;
 * the server accepts only FPT_RNG_PHILOX jobs. */
typedef enum { FPT_RNG_PHILOX = 0, FPT_RNG_MT19937 = 1 } fpt_rng;

/* FPT_SCHED_REFILL: persistent lanes; a lane whose replica escaped or was
 * censored takes the next undrawn replica (the paper's "assign a new job to
 * the processor that has just completed", done on the device).
 * FPT_SCHED_ONE_PER_LANE: replica i is bound to lane i for its whole run
 * (Algorithm 1's one-realization-per-thread launch). */
typedef enum { FPT_SCHED_REFILL = 0, FPT_SCHED_ONE_PER_LANE = 1 } fpt_schedule;

/* One parameter set ("job").  NaN phi0 / v0 / threshold select Algorithm 1's
 * defaults: the bottom of the well at rest and the barrier top, phi0 =
 * arcsin(gamma0), v0 = 0, threshold = pi - phi0.  For the overdamped model
 * the well of -V0 cos(phi) - gamma phi is at arcsin(gamma0 / V0), which is
 * the default phi0 there (the threshold stays pi - phi0).  A NaN phi0 needs
 * |gamma0| <= 1 (underdamped) or V0 != 0 and |gamma0| <= |V0| (overdamped). */
typedef struct fpt_params {
  int32_t model;        /* fpt_model */
  int32_t n_bins;       /* histogram bins, 1..FPT_MAX_BINS */
  int32_t scheme;       /* fpt_scheme (underdamped only; 0 for overdamped) */
  int32_t rng;          /* fpt_rng */
  double alpha;         /* damping (underdamped), >= 0 */
  double T;             /* temperature, >= 0 (T = 0: noise-free) */
  double V0;            /* potential amplitude (1 in plasma units) */
  double gamma0;        /* bias at t = 0 */
  double ramp;          /* d gamma / dt per unit time (0: fixed bias) */
  double dt;            /* Euler step h, > 0 */
  double phi0, v0;      /* initial state (NaN: defaults) */
  double threshold;     /* escape when phi > threshold (NaN: pi - phi0) */
  int64_t max_steps;    /* klim, >= 1 */
  int64_t n_replicas;   /* >= 0 */
  int64_t hist_k_max;   /* bins cover steps [1, hist_k_max]; 0: max_steps.
                           bin(k) = ((k-1) n_bins) div hist_k_max;
                           k > hist_k_max counts as overflow */
  uint64_t seed;        /* Philox key, or MT19937 base seed */
} fpt_params;

/* Launch tuning.  Zero fields are filled by the autotuner (cached per GPU
 * architecture, precision, model and set-count bucket). */
typedef struct fpt_tuning {
  int32_t schedule;          /* fpt_schedule */
  int32_t replicas_per_lane; /* 1 or 2 (0: autotune) */
  int32_t waves_per_simd;    /* 1..8 resident waves per SIMD (0: autotune); capped
                                at the kernel's occupancy (fpt_plan_stats reports
                                the value used) */
  int32_t steps_per_launch;  /* multiple of 4 (0: autotune) */
  int32_t use_graph;         /* 1: replay launches through a captured hipGraph */
  int32_t no_compaction;     /* 1: keep the launch width to the end.  Otherwise a
                                refill plan (Philox) whose queue is drained and
                                whose active replicas fill at most 80% of the
                                slots moves them to a dense prefix and narrows
                                later launches; results do not change */
  int32_t no_regroup;        /* Multi-set refill plans (and the server) keep each
                                wavefront to one set: after every launch while
                                undrawn replicas remain, the active replicas'
                                state moves into set order (each set starting a
                                wavefront) and the free slots past them take the
                                next replicas; inside a launch only wavefronts
                                free in every lane draw.  1: no regrouping, and
                                every free slot draws at once (wavefronts then
                                mix sets and a block takes one pass per set).
                                Results do not change */
  int32_t reserved;
} fpt_tuning;

/* Per-set results.  Moments are over escaped replicas; times in units of t. */
typedef struct fpt_moments {
  uint64_t n_escaped, n_censored, n_overflow;
  uint64_t sum_k;                 /* sum of escape steps (exact while
                                     n_escaped * max_steps < 2^64) */
  uint64_t sum_k2_lo, sum_k2_hi;  /* 128-bit sum of squared escape steps */
  double mean_t, se_t;            /* dt*mean(k), dt*stddev(k)/sqrt(n) */
} fpt_moments;

typedef struct fpt_run_stats {
  uint64_t replica_steps;     /* sum of k over escaped + max_steps per censored */
  uint64_t lane_steps;        /* lane-steps issued (idle lanes included) */
  int64_t n_launches;         /* integrator launches of the last simulate */
  double kernel_ms;           /* sum of their durations (HIP events) */
  double wall_ms;             /* fpt_simulate entry to last launch done */
  fpt_tuning tuning;          /* tuning actually used */
  int64_t n_compactions;      /* tail compactions of the last simulate */
  int64_t n_regroups;         /* moves of the active state into set order */
  uint64_t extra_passes;      /* multi-set blocks: passes beyond one per
                                 wavefront and slot (lane_steps / 256 is the
                                 number of wavefront-slot blocks) */
} fpt_run_stats;

typedef struct fpt_plan_s* fpt_plan_t;
typedef struct fpt_server_s* fpt_server_t;

/* ---- plans: a fixed batch of parameter sets ------------------------------ */

/* Validate n_sets parameter sets (1 .. 2^20 - 1, all of one model) and
 * derive the per-set constants of Algorithm 1 / 3's preamble:
 * sigma = sqrt(2 alpha T dt) (overdamped sqrt(2 T dt)), delta-gamma =
 * ramp*dt, phi0, v0, threshold.
 * tuning may be NULL (all fields autotuned).  Host-only; no device memory.
 * Errors: FPT_E_INVAL (message names the set and field). */
fpt_status fpt_plan(const fpt_params* sets, int32_t n_sets, int32_t precision,
                    const fpt_tuning* tuning, fpt_plan_t* out);

/* Bytes of device workspace fpt_simulate needs for this plan (caller
 * allocates, 256-byte aligned, and may reuse it across calls). */
fpt_status fpt_plan_workspace(fpt_plan_t plan, size_t* bytes);

/* Run every replica of every set: the replica loop of Algorithm 1 (fixed
 * bias) and Algorithm 3 (ramped bias) -- Euler steps from (phi0, v0) until
 * phi > threshold, recording the step k (the escape time k*h, or the
 * switching bias gamma_k) or -1 after max_steps -- with the replicas spread
 * over persistent lanes as in Sect. III.B (one realization per thread, a
 * finished thread takes the next one).  Asynchronous on `stream`.
 *   workspace : device, >= fpt_plan_workspace bytes
 *   out_steps : host array of n_sets device pointers (int64[n_replicas] each,
 *               entries may be NULL), or NULL: escape step per replica, -1 if
 *               censored
 *   out_hist  : device uint64[sum of n_bins], sets in plan order, or NULL
 *               (then kept in the workspace); zeroed by the call
 * Results are identical for every tuning.  Errors: FPT_E_INVAL, FPT_E_DEVICE. */
fpt_status fpt_simulate(fpt_plan_t plan, void* workspace,
                        int64_t* const* out_steps, uint64_t* out_hist,
                        void* stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): fpt_simulate with
 * the workspace in a static device array of the library, of
 * FPT_NOALLOC_SCRATCH_BYTES, which each GPU the library runs on holds from
 * its first use until the process ends.  The call allocates nothing: no
 * device or pinned memory, no events, no graphs; the caller still passes the
 * outputs (as for fpt_simulate; out_hist NULL keeps the histograms in the
 * static array until the next call on that GPU).
 *   - the plan's tuning must be complete (replicas_per_lane, waves_per_simd,
 *     steps_per_launch non-zero; no autotuning trials) with use_graph 0,
 *     else FPT_E_INVAL;
 *   - the workspace of the plan at that launch shape (laid out for the shape
 *     itself, not for the largest one fpt_plan_workspace reports) must fit
 *     the array, else FPT_E_NOMEM;
 *   - every call on one GPU shares that GPU's array, which keeps the last
 *     call's contents (each call clears what it needs at zero): calls that
 *     overlap on one GPU, from several threads or streams, race;
 *   - results equal fpt_simulate's for the same plan; fpt_histogram(_all)
 *     and fpt_plan_stats read this run (kernel_ms stays 0: no events);
 *   - like fpt_simulate, the call drives its launches from the host and
 *     returns when the run has finished (it waits on `stream` between
 *     launch groups), so it is not itself recorded into a stream capture:
 *     what it spares its caller is every allocation and handle creation. */
#define FPT_NOALLOC_SCRATCH_BYTES (48ull << 20)
fpt_status fpt_simulate_noalloc(fpt_plan_t plan, int64_t* const* out_steps,
                                uint64_t* out_hist, void* stream);

/* Copy set `set`'s histogram (n_bins counts) and moments of the last
 * fpt_simulate to host memory: the escape-time histogram of Sect. II.B and
 * the switching-current histogram / CDF of Sect. IV.B (bins over escape
 * steps; gamma_k is monotone in k), and the mean first-passage time with
 * its standard error that Sect. IV.A fits against the Kramers law.
 * Synchronizes that call's stream.  Either pointer may be NULL.
 * Errors: FPT_E_STATE before a simulate. */
fpt_status fpt_histogram(fpt_plan_t plan, int32_t set, uint64_t* host_counts,
                         fpt_moments* host_m);

/* Every set at once (the same histograms and moments as fpt_histogram:
 * Sect. II.B, IV.A, IV.B), with one device-to-host copy of the histograms and
 * one of the moments (plans of many sets):
 *   host_counts : host uint64[sum of n_bins], sets in plan order, or NULL
 *   host_m      : host fpt_moments[n_sets], or NULL
 * Synchronizes the last fpt_simulate's stream.  Errors: FPT_E_STATE before
 * a simulate. */
fpt_status fpt_histogram_all(fpt_plan_t plan, uint64_t* host_counts, fpt_moments* host_m);

/* Counters and timing of the last fpt_simulate (synchronizes). */
fpt_status fpt_plan_stats(fpt_plan_t plan, fpt_run_stats* out);

void fpt_plan_destroy(fpt_plan_t plan);

/* ---- serving: jobs admitted continuously -------------------------------- */

/* Continuous form of the streaming scheme of Sect. III.B (its three steps:
 * integrate until the threshold, hand the escape time back, give the freed
 * processor the next realization) for jobs, parameter sets that arrive over
 * time.  A request loop on its own host thread owns `stream` and the
 * caller's device pool (`pool_bytes` at `device_pool`, which must stay
 * allocated until fpt_server_destroy).  Jobs are admitted as set slots and pool memory free
 * up; their replicas share the resident persistent lanes with the jobs
 * already running.  While every admitted replica has been drawn, the loop
 * packs the running ones into fewer lanes as they finish (tail compaction),
 * which speeds up each remaining replica; an admission restores the full
 * width.  While replicas wait, each launch is followed by a regroup into set
 * order as for plans (tuning->no_regroup).  Every job of a server shares its
 * model and scheme (fpt_scheme: explicit, or semi-implicit for the
 * underdamped model), since every launch runs one integrator.  Pool memory
 * beyond the fixed lane state holds the work ring (at least 4096 chunks of
 * 64 replicas, up to half the rest) and the jobs' histograms (the rest); a
 * job is admitted once a set slot, ring room for its replicas and room for
 * its bins are free.  Errors: FPT_E_NOMEM if the pool cannot hold the fixed
 * lane state, the minimal ring and FPT_MAX_BINS bins. */
fpt_status fpt_server_create(void* device_pool, size_t pool_bytes,
                             int32_t precision, int32_t model, int32_t scheme,
                             const fpt_tuning* tuning, void* stream,
                             fpt_server_t* out);

/* Queue one job: one parameter set whose replicas become new realizations
 * for freed lanes (Sect. III.B, third step) once pool memory and a set slot
 * are free (non-blocking, thread-safe).  FPT_E_NOMEM if the job could never
 * fit the pool, FPT_E_INVAL for bad parameters, FPT_E_BUSY if the queue is
 * full. */
fpt_status fpt_submit(fpt_server_t server, const fpt_params* params,
                      uint64_t* job_id);

/* Result of one job: the histogram and moments of its escape steps
 * (Sect. II.B, IV.A, IV.B, as fpt_histogram), gathered from the escape times
 * the lanes hand back (Sect. III.B, second step) once its last realization
 * has finished.  FPT_PENDING while queued or running; FPT_OK once finished,
 * filling host_counts (n_bins), moments and the submit-to-finish latency
 * (any may be NULL).  A finished job is forgotten after its first FPT_OK. */
fpt_status fpt_poll(fpt_server_t server, uint64_t job_id,
                    uint64_t* host_counts, fpt_moments* host_m,
                    double* latency_s);

typedef struct fpt_server_stats {
  uint64_t submitted, admitted, finished, queued, running;
  uint64_t replica_steps;   /* of finished jobs */
  int64_t n_launches;
  double busy_s;            /* time with at least one job running */
  int64_t n_compactions;    /* narrowings of the launch to the active slots
                               while every admitted replica was drawn */
  int64_t n_regroups;       /* moves of the active state into set order */
} fpt_server_stats;

fpt_status fpt_server_stats_get(fpt_server_t server, fpt_server_stats* out);

/* Stops the loop after the running launch, drops unfinished jobs. */
void fpt_server_destroy(fpt_server_t server);

/* ---- diagnostics (same device code as the integrator) ------------------- */

/* Philox words of replicas [replica0, replica0+n_rep) x blocks
 * [block0, block0+n_blk): out[((r*n_blk)+b)*4 + w], device uint32. */
fpt_status fpt_rng_words(uint64_t seed, uint64_t replica0, int64_t n_rep,
                         uint64_t block0, int64_t n_blk, uint32_t* out,
                         void* stream);

/* The MT19937 words the integrator draws in FPT_RNG_MT19937 mode: outputs
 * 4b .. 4b+3 of the generator seeded with (seed + r) mod 2^32 for replicas
 * r in [replica0, replica0+n_rep) and blocks b in [block0, block0+n_blk),
 * laid out as fpt_rng_words; n_rep <= 2^24 and block0 + n_blk <= 2^24 (each
 * lane generates every word up to the last block).  Allocates and frees
 * n_rep * 2496 bytes of temporary device state and synchronizes `stream`. */
fpt_status fpt_mt_words(uint64_t seed, uint64_t replica0, int64_t n_rep,
                        uint64_t block0, int64_t n_blk, uint32_t* out,
                        void* stream);

/* The four normals of the same blocks, as the integrator of `precision`
 * computes them: out is device double (FPT_FP64) or float (FPT_FP32C). */
fpt_status fpt_normals(uint64_t seed, uint64_t replica0, int64_t n_rep,
                       uint64_t block0, int64_t n_blk, int32_t precision,
                       void* out, void* stream);

/* State (phi, v) after each of n_steps steps of one replica, no threshold:
 * out_phi / out_v device double[n_steps] (FP32C: phi_hi - c and v widened).
 * With params->rng = FPT_RNG_MT19937 the call allocates 2496 bytes of
 * temporary device state and synchronizes `stream`. */
fpt_status fpt_trajectory(const fpt_params* params, uint64_t replica,
                          int64_t n_steps, int32_t precision, double* out_phi,
                          double* out_v, void* stream);

const char* fpt_last_error(void);
int32_t fpt_api_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FPT_H */
