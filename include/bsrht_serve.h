/*
 * bsrht_serve.h -- serving runtime for block SRHT sketch, randomized SVD and
 * Nystrom jobs on one GPU (continuous batching of independent jobs).
 *
 * Each job is one call of bsrht.h: BSRHT_JOB_SKETCH is bsrht_apply (the
 * sketch Y = Omega A of section 2, eq. (2.4)), BSRHT_JOB_RSVD is rsvd
 * (section 3.1, Algorithm 1, which sketches first), BSRHT_JOB_NYSTROM is
 * nystrom (section 3.2, Algorithm 2 with Remark 3.1's fallback).  The server owns no
 * device memory of its own: the caller hands it one device arena at
 * creation, and every byte a job needs beyond its inputs and outputs (the
 * call's workspace and, on a plan-cache miss, the plan's sign/index tables)
 * is carved from that arena.  A job is admitted only when its bytes fit, so
 * the arena size is the HBM budget.  A job's result is the same as the same
 * call made alone (every kernel of the library reduces in a fixed order that
 * does not depend on what else runs).
 *
 * Execution: admitted jobs run concurrently, one per stream slot.  A job is a
 * coroutine that queues its kernels on its slot's stream and suspends where
 * the algorithm needs a value from the device (a Cholesky flag, a Jacobi
 * sweep count); the server resumes it once the event recorded there has
 * completed.  Small FP32 sketch jobs (blocks of >= 64 rows, A of at most
 * 64 MiB) that are ready together run as one batched launch on one slot
 * (bsrht_apply_batch: persistent kernels replayed from a captured HIP graph;
 * each result is bitwise the single call's); up to BSRHT_BATCH_MAX such jobs
 * are admitted beyond the slot count, and each slot keeps its descriptor
 * table in the arena (bsrht_batch_table_bytes bytes).  There are no worker
 * threads: jobs advance inside
 * bsrht_server_submit, bsrht_server_poll and bsrht_server_drain, which make
 * every HIP call of the server, so a client keeps polling while jobs run.
 *
 * Scheduling: jobs are admitted in arrival order; while the oldest waiting
 * job does not fit, a younger job among the next 8 that fits may be admitted
 * ahead of it ("backfill"), until the oldest has waited 100 ms, after which
 * nothing bypasses it.  Plans are cached by (n, p, l, seed, sampling,
 * precision) and evicted least-recently-used when an admission needs their
 * bytes and no admitted job uses them.
 *
 * Timestamps are seconds on the server's monotonic clock
 * (bsrht_server_clock); t_done is taken when the server observes the job's
 * completion event, so its resolution is the client's polling interval.
 * Every function is thread-safe (one lock).  Errors are the BSRHT_* status
 * codes of bsrht.h.
 */
#ifndef BSRHT_SERVE_H
#define BSRHT_SERVE_H

#include <stddef.h>
#include <stdint.h>

#include "bsrht.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bsrht_server_s *bsrht_server_t;

#define BSRHT_JOB_SKETCH 0  /* Y = Omega A            (bsrht_apply) */
#define BSRHT_JOB_RSVD 1    /* sketch + Algorithm 1   (rsvd)        */
#define BSRHT_JOB_NYSTROM 2 /* sketch + Algorithm 2   (nystrom)     */

/* One job.  Device pointers are caller-owned and must stay valid (inputs
 * unchanged, outputs untouched) from submission until the job's result has
 * been returned by bsrht_server_poll.  The plan is (n, p, l, seed, sampling,
 * precision) exactly as for bsrht_plan. */
typedef struct {
  int64_t id;        /* caller's tag, returned with the result */
  int kind;          /* BSRHT_JOB_SKETCH, BSRHT_JOB_RSVD or BSRHT_JOB_NYSTROM */
  int64_t n, m, p, l;  /* NYSTROM: m == n (A is n x n, symmetric PSD) */
  int64_t k;         /* RSVD / NYSTROM target rank (ignored for SKETCH) */
  uint64_t seed;
  int sampling, precision;
  const float *A;    /* device, n x m, leading dimension lda */
  int64_t lda;
  float *Y;          /* SKETCH: device l x m, leading dimension ldy */
  int64_t ldy;
  float *U;          /* RSVD: device outputs as for rsvd(): U n x k, */
  double *S;         /*   S k, V m x k (row-major), info int32;      */
  float *V;          /* NYSTROM: as for nystrom(): U n x k, S = lambda */
  int32_t *info;     /*   (k, descending), info; V is not used       */
} bsrht_job_t;

typedef struct {
  int64_t id;
  int status;            /* status of the job's library call */
  int64_t arena_bytes;   /* arena bytes held while the job ran */
  double t_submit;       /* bsrht_server_submit returned (arrival) */
  double t_start;        /* admitted and taken by a worker */
  double t_done;         /* the job's stream had finished its work */
} bsrht_job_result_t;

typedef struct {
  int64_t submitted, completed, rejected;
  int64_t plan_hits, plan_misses, plan_evictions;
  int64_t backfilled;        /* admissions ahead of an older waiting job */
  int64_t peak_arena_bytes;  /* high-water mark of arena bytes in use */
  int peak_running;          /* high-water mark of concurrently running jobs */
  int64_t queued;            /* waiting for admission now */
  int64_t batches;           /* batched launches of small sketch jobs */
  int64_t batched_jobs;      /* jobs that ran in them */
} bsrht_server_stats_t;

/* Arena bytes a job needs when its plan is not cached (workspace + tables);
 * 0 for invalid sizes. */
size_t bsrht_job_bytes(const bsrht_job_t *job);

/*
 * Creates a server on the current device with `streams` concurrent job slots
 * (1..64), each a non-blocking HIP stream of default priority with an event
 * and 128 KiB of pinned staging.  arena: device memory of arena_bytes
 * (caller-owned, 256-byte aligned, freed by the caller after
 * bsrht_server_destroy).
 */
int bsrht_server_create(void *arena, size_t arena_bytes, int streams, bsrht_server_t *out);

/*
 * Same scheduler with a host-only executor, for testing admission and
 * ordering without a GPU: no HIP call is made, the arena is a byte budget,
 * and a job "runs" by sleeping seconds_per_gb * (4 n m / 1e9) seconds on one
 * of `workers` threads.  Job pointers are not dereferenced.
 */
int bsrht_server_create_fake(size_t arena_bytes, int workers, double seconds_per_gb,
                             bsrht_server_t *out);

/* Queues a job (copied).  BSRHT_EINVAL for invalid sizes, kind or pointers;
 * BSRHT_ENOMEM when the job alone needs more than the whole arena. */
int bsrht_server_submit(bsrht_server_t srv, const bsrht_job_t *job);

/*
 * Submits jobs[0 .. count) in order under one lock, then admits and starts
 * what fits (a burst of jobs arrives together, which is what lets small
 * sketch jobs be batched).  Each job is checked as by bsrht_server_submit;
 * the first rejected job stops the call: *accepted receives the number of
 * jobs submitted before it, and its status is returned.
 */
int bsrht_server_submit_many(bsrht_server_t srv, const bsrht_job_t *jobs, int count,
                             int *accepted);

/* Advances running jobs, then moves up to max finished results into out
 * (completion order) and stores their number in *count; waits up to
 * timeout_s seconds for the first one when none is ready (0 = do not wait). */
int bsrht_server_poll(bsrht_server_t srv, bsrht_job_result_t *out, int max, double timeout_s,
                      int *count);

/* Turns the batched launches of small sketch jobs on (default) or off; off,
 * every job runs alone on a slot.  Applies to jobs started afterwards. */
int bsrht_server_set_batching(bsrht_server_t srv, int on);

/* Runs / waits until every submitted job has finished. */
int bsrht_server_drain(bsrht_server_t srv);

int bsrht_server_stats(bsrht_server_t srv, bsrht_server_stats_t *out);

/* Seconds on the server's clock (the clock of the result timestamps). */
double bsrht_server_clock(bsrht_server_t srv);

/* Drains, then releases the streams, events, staging and cached plans. */
int bsrht_server_destroy(bsrht_server_t srv);

#ifdef __cplusplus
}
#endif

#endif /* BSRHT_SERVE_H */
