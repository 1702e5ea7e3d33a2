/*
 * fpt_c_client.c -- a plain C program that drives libfpt through include/fpt.h
 * alone (device memory from the HIP runtime's C API, no Python, no torch).
 * The GPU tests run it and compare what it prints with the Python binding's
 * results for the same parameters.
 *
 *   fpt_c_client plan  <fp64|fp32c> <steps.bin> <params...>
 *       one plan of one parameter set: escape steps written to steps.bin
 *       (int64, n_replicas), then one "moments" line and one "counts" line
 *   fpt_c_client noalloc <fp64|fp32c> <steps.bin> <params...>
 *       the same through fpt_simulate_noalloc (fixed tuning R 1, W 2, 4096
 *       steps per launch)
 *   fpt_c_client serve <fp64|fp32c> <n_jobs> <params...>
 *       a server on a 256 MiB pool, n_jobs jobs with seeds seed .. seed+n-1
 *       submitted at once and polled to the end: one "job" line each
 *
 * <params...> = model alpha T V0 gamma0 ramp dt phi0 v0 threshold max_steps
 *               n_replicas n_bins hist_k_max seed   (fpt_params fields;
 *               "nan" selects a default)
 * Exit status 0 on success, 1 on a usage error, 2 on a library or HIP error
 * (its message on stderr).
 */
#include <hip/hip_runtime_api.h>
#include <inttypes.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#include "fpt.h"

#define N_PARAM_ARGS 15

static int fail_fpt(const char* what, fpt_status st) {
  fprintf(stderr, "%s: status %d: %s\n", what, (int)st, fpt_last_error());
  return 2;
}

static int fail_hip(const char* what, hipError_t e) {
  fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
  return 2;
}

static int parse_params(char** v, fpt_params* p) {
  memset(p, 0, sizeof(*p));
  p->model = (int32_t)strtol(v[0], NULL, 10);
  p->alpha = strtod(v[1], NULL);
  p->T = strtod(v[2], NULL);
  p->V0 = strtod(v[3], NULL);
  p->gamma0 = strtod(v[4], NULL);
  p->ramp = strtod(v[5], NULL);
  p->dt = strtod(v[6], NULL);
  p->phi0 = strtod(v[7], NULL);
  p->v0 = strtod(v[8], NULL);
  p->threshold = strtod(v[9], NULL);
  p->max_steps = strtoll(v[10], NULL, 10);
  p->n_replicas = strtoll(v[11], NULL, 10);
  p->n_bins = (int32_t)strtol(v[12], NULL, 10);
  p->hist_k_max = strtoll(v[13], NULL, 10);
  p->seed = strtoull(v[14], NULL, 10);
  p->scheme = FPT_EXPLICIT;
  p->rng = FPT_RNG_PHILOX;
  return p->n_bins >= 1 && p->n_bins <= FPT_MAX_BINS && p->n_replicas >= 0 ? 0 : 1;
}

static void print_moments(const char* tag, const fpt_moments* m) {
  printf("%s %" PRIu64 " %" PRIu64 " %" PRIu64 " %" PRIu64 " %" PRIu64 " %" PRIu64 " %.17g\n",
         tag, m->n_escaped, m->n_censored, m->n_overflow, m->sum_k, m->sum_k2_lo,
         m->sum_k2_hi, m->mean_t);
}

static void print_counts(const char* tag, const uint64_t* c, int32_t n) {
  printf("%s", tag);
  for (int32_t i = 0; i < n; ++i) printf(" %" PRIu64, c[i]);
  printf("\n");
}

static int run_plan(int precision, const char* path, const fpt_params* p, int noalloc) {
  fpt_plan_t plan = NULL;
  fpt_tuning tune;
  memset(&tune, 0, sizeof(tune));
  tune.replicas_per_lane = 1;
  tune.waves_per_simd = 2;
  tune.steps_per_launch = 4096;
  fpt_status st = fpt_plan(p, 1, precision, noalloc ? &tune : NULL, &plan);
  if (st != FPT_OK) return fail_fpt("fpt_plan", st);

  const size_t n = (size_t)p->n_replicas;
  void* ws = NULL;
  int64_t* steps = NULL;
  uint64_t* hist = NULL;
  hipError_t e;
  int rc = 0;
  if (!noalloc) {
    size_t bytes = 0;
    st = fpt_plan_workspace(plan, &bytes);
    if (st != FPT_OK) { rc = fail_fpt("fpt_plan_workspace", st); goto done; }
    if ((e = hipMalloc(&ws, bytes)) != hipSuccess) { rc = fail_hip("hipMalloc ws", e); goto done; }
  }
  if ((e = hipMalloc((void**)&steps, (n ? n : 1) * sizeof(int64_t))) != hipSuccess) {
    rc = fail_hip("hipMalloc steps", e);
    goto done;
  }
  if ((e = hipMalloc((void**)&hist, (size_t)p->n_bins * sizeof(uint64_t))) != hipSuccess) {
    rc = fail_hip("hipMalloc hist", e);
    goto done;
  }
  {
    int64_t* const outs[1] = {steps};
    st = noalloc ? fpt_simulate_noalloc(plan, outs, hist, NULL)
                 : fpt_simulate(plan, ws, outs, hist, NULL);
    if (st != FPT_OK) { rc = fail_fpt("fpt_simulate", st); goto done; }
  }
  {
    uint64_t* counts = (uint64_t*)calloc((size_t)p->n_bins, sizeof(uint64_t));
    uint64_t* dev_counts = (uint64_t*)calloc((size_t)p->n_bins, sizeof(uint64_t));
    int64_t* host_steps = (int64_t*)malloc((n ? n : 1) * sizeof(int64_t));
    fpt_moments m;
    fpt_run_stats rs;
    if (!counts || !dev_counts || !host_steps) {
      fprintf(stderr, "host allocation failed\n");
      rc = 2;
    } else if ((st = fpt_histogram(plan, 0, counts, &m)) != FPT_OK) {
      rc = fail_fpt("fpt_histogram", st);
    } else if ((st = fpt_plan_stats(plan, &rs)) != FPT_OK) {
      rc = fail_fpt("fpt_plan_stats", st);
    } else if ((e = hipMemcpy(host_steps, steps, n * sizeof(int64_t), hipMemcpyDeviceToHost)) !=
                   hipSuccess ||
               (e = hipMemcpy(dev_counts, hist, (size_t)p->n_bins * sizeof(uint64_t),
                              hipMemcpyDeviceToHost)) != hipSuccess) {
      rc = fail_hip("hipMemcpy", e);
    } else {
      FILE* f = fopen(path, "wb");
      if (!f || fwrite(host_steps, sizeof(int64_t), n, f) != n) {
        fprintf(stderr, "cannot write %s\n", path);
        rc = 2;
      }
      if (f) fclose(f);
      if (rc == 0) {
        print_moments("moments", &m);
        print_counts("counts", counts, p->n_bins);
        print_counts("device_counts", dev_counts, p->n_bins);
        printf("stats %" PRIu64 " %" PRId64 "\n", rs.replica_steps, rs.n_launches);
      }
    }
    free(counts);
    free(dev_counts);
    free(host_steps);
  }
done:
  if (hist) (void)hipFree(hist);
  if (steps) (void)hipFree(steps);
  if (ws) (void)hipFree(ws);
  fpt_plan_destroy(plan);
  return rc;
}

static int run_serve(int precision, int n_jobs, const fpt_params* p) {
  const size_t pool_bytes = (size_t)256 << 20;
  void* pool = NULL;
  hipError_t e = hipMalloc(&pool, pool_bytes);
  if (e != hipSuccess) return fail_hip("hipMalloc pool", e);
  fpt_server_t srv = NULL;
  int rc = 0;
  uint64_t* ids = (uint64_t*)calloc((size_t)n_jobs, sizeof(uint64_t));
  int* done = (int*)calloc((size_t)n_jobs, sizeof(int));
  uint64_t* counts = (uint64_t*)calloc((size_t)p->n_bins, sizeof(uint64_t));
  fpt_status st = fpt_server_create(pool, pool_bytes, precision, p->model, p->scheme, NULL,
                                    NULL, &srv);
  if (st != FPT_OK) {
    rc = fail_fpt("fpt_server_create", st);
    goto out;
  }
  if (!ids || !done || !counts) {
    fprintf(stderr, "host allocation failed\n");
    rc = 2;
    goto out;
  }
  for (int i = 0; i < n_jobs; ++i) {
    fpt_params job = *p;
    job.seed = p->seed + (uint64_t)i;
    if ((st = fpt_submit(srv, &job, &ids[i])) != FPT_OK) {
      rc = fail_fpt("fpt_submit", st);
      goto out;
    }
  }
  {
    int left = n_jobs;
    const time_t t0 = time(NULL);
    while (left > 0) {
      for (int i = 0; i < n_jobs; ++i) {
        if (done[i]) continue;
        fpt_moments m;
        double latency = 0.0;
        st = fpt_poll(srv, ids[i], counts, &m, &latency);
        if (st == FPT_PENDING) continue;
        if (st != FPT_OK) {
          rc = fail_fpt("fpt_poll", st);
          goto out;
        }
        done[i] = 1;
        --left;
        char tag[32];
        snprintf(tag, sizeof(tag), "job %d", i);
        print_moments(tag, &m);
        snprintf(tag, sizeof(tag), "job_counts %d", i);
        print_counts(tag, counts, p->n_bins);
      }
      if (left > 0) {
        if (time(NULL) - t0 > 120) {
          fprintf(stderr, "jobs not finished within 120 s\n");
          rc = 2;
          goto out;
        }
        const struct timespec pause = {0, 2000000};
        nanosleep(&pause, NULL);
      }
    }
  }
out:
  if (srv) fpt_server_destroy(srv);
  free(ids);
  free(done);
  free(counts);
  (void)hipFree(pool);
  return rc;
}

int main(int argc, char** argv) {
  if (argc != 4 + N_PARAM_ARGS) {
    fprintf(stderr, "usage: %s plan|noalloc|serve fp64|fp32c <steps.bin|n_jobs> <%d params>\n",
            argv[0], N_PARAM_ARGS);
    return 1;
  }
  if (fpt_api_version() != FPT_API_VERSION) {
    fprintf(stderr, "library API %d, header %d\n", (int)fpt_api_version(), FPT_API_VERSION);
    return 2;
  }
  const int precision = strcmp(argv[2], "fp32c") == 0 ? FPT_FP32C : FPT_FP64;
  fpt_params p;
  if (parse_params(argv + 4, &p) != 0) {
    fprintf(stderr, "bad parameters\n");
    return 1;
  }
  if (strcmp(argv[1], "plan") == 0) return run_plan(precision, argv[3], &p, 0);
  if (strcmp(argv[1], "noalloc") == 0) return run_plan(precision, argv[3], &p, 1);
  if (strcmp(argv[1], "serve") == 0) {
    const int n_jobs = (int)strtol(argv[3], NULL, 10);
    if (n_jobs < 1 || n_jobs > 64) {
      fprintf(stderr, "n_jobs must be 1..64\n");
      return 1;
    }
    return run_serve(precision, n_jobs, &p);
  }
  fprintf(stderr, "unknown mode %s\n", argv[1]);
  return 1;
}
