/*
 * librpca -- batched Split-SPCP: many independent instances of uneven shape
 * solved together on one GPU.
 *
 * Each instance is the problem of rpca.h (f(U,V) = phi(U V^T) +
 * lam_L/2 (||U||^2 + ||V||^2), Sec. 1 eq. PhiDef and eq. smoothNC; L-BFGS with
 * memory `mem`, Sec. 5.1; certificate of Sec. 3.4), fully observed.  The
 * batch runs every solver step as one launch for all instances: the
 * reductions and L-BFGS passes cover all instances in one grid each, and the
 * sweep is one persistent kernel per tile class (k <= 16 or <= 32, tiles per
 * column chunk) present in the batch, pulling (instance, row group, column
 * chunk) items from a queue sorted by decreasing cost.  Instances that have converged skip every
 * kernel.  Groups of solver slots are captured once in a hipGraph and
 * replayed until all instances are done; certificates then run per instance.
 *
 * Results are bitwise identical to solving each instance alone with
 * rpca_solve (same kernels, same fixed reduction orders).
 *
 * Conventions are those of rpca.h.  Arrays named "host array" hold one entry
 * per instance in host memory; their elements are device pointers where the
 * single-instance call takes device pointers.
 */
#ifndef RPCA_BATCH_H
#define RPCA_BATCH_H

#include <stdint.h>

#include "rpca.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rpca_batch rpca_batch;

typedef struct rpca_batch_layout {
  int32_t count;            /* instances */
  int32_t sweep_items;      /* (instance, row group, chunk) items of one sweep */
  int32_t sweep_grid_fp32;  /* persistent workgroups of the FP32 sweeps (all classes) */
  int32_t sweep_grid_bf16;  /* persistent workgroups of the BF16 sweeps (all classes) */
  int32_t lds_bytes;        /* largest dynamic LDS per workgroup of a sweep */
  int32_t graphs;           /* captured slot groups so far */
  int32_t sweep_classes;    /* persistent sweep launches per pass (one per tile class) */
} rpca_batch_layout;

/* Create a batch of `count` (1..65536) instances; m, n, k, lam_s, lam_l are
 * host arrays of `count` values with the constraints of rpca_create.  The
 * batch owns one workspace per instance and its own non-blocking stream. */
int rpca_batch_create(int32_t count, const int64_t* m, const int64_t* n, const int32_t* k,
                      const double* lam_s, const double* lam_l, rpca_batch** out);

/* Objective and gradient of every instance in one batched pass (the
 * persistent sweep plus two batched reductions).  X, U, V, f, gU, gV: host
 * arrays of device pointers with the layouts of rpca_objgrad.  precision:
 * RPCA_PREC_FP32 or RPCA_PREC_BF16.  Ordered after earlier work on `stream`;
 * later work on `stream` is ordered after it. */
int rpca_batch_objgrad(rpca_batch* b, const float* const* X, const float* const* U,
                       const float* const* V, double* const* f, float* const* gU,
                       float* const* gV, int32_t precision, void* stream);

/* Solve every instance.  X: host array of device pointers (column-major
 * m_i x n_i); U, V: host arrays of device pointers, the starting factors on
 * input (unless opts->init is RPCA_INIT_RSVD) and the solutions on output.
 * opts applies to all instances (NULL = defaults).  info: host array of
 * `count` records, or NULL.  Blocks until every instance is done.  Returns
 * the largest per-instance status (warnings > 0), or the first error < 0.
 * The solver slots run batched on the batch's stream; the per-instance steps
 * that synchronise with the host (rSVD start, preconditioner refresh and
 * restart between cycles, certificates) run on up to 16 host worker threads,
 * each with its own stream of the batch, so a batch must not be used from
 * two host threads at once.  The worker count is the host's hardware thread
 * count capped at 16; RPCA_BATCH_WORKERS=1..16 in the environment (read at the
 * first batched solve) sets it. */
int rpca_batch_solve(rpca_batch* b, const float* const* X, float* const* U, float* const* V,
                     const rpca_opts* opts, rpca_info* info, void* stream);

/* 1 (default): replay captured slot groups; 0: launch the same kernels eagerly. */
int rpca_batch_set_graphs(rpca_batch* b, int32_t on);

/* Decomposition of the batch (for reports and tests). */
int rpca_batch_info(rpca_batch* b, rpca_batch_layout* out);

/* Wave target of instance i's sweep decomposition.  A batch shares one
 * chip's worth of waves (16 per compute unit) over its instances in
 * proportion to m n (k > 16 weighs 1.6 times), at least 4 each, so its items
 * stay long enough to stream; a context made by rpca_create_waves with this
 * value computes instance i's objective and gradient bit for bit as the
 * batch does.  RPCA_EINVAL for a bad index or null pointer. */
int rpca_batch_instance_waves(rpca_batch* b, int32_t i, int32_t* waves);

void rpca_batch_destroy(rpca_batch* b);

/* Sweep decomposition table (process-wide), keyed by (k bucket: k <= 8, 16,
 * 24, 32; n bucket: n <= 64, 128, 256, 512, larger).  An entry holds the
 * number of waves the row strips of one sweep are spread over and the
 * divisor of the widest column chunk that fits the LDS budget.  Contexts and
 * batches read the table when they are created, so tune first.
 *
 * rpca_autotune: for every entry, time rpca_objgrad on a synthetic probe
 * instance (m_probe rows in [32, 2^24], the bucket's largest k and n) for
 * each candidate (1024, 2048 or 4096 waves x divisor 1 or 2), `reps` calls
 * each (1..10000) on `stream`, and keep the fastest.  Blocks until done.
 * A batch reads both parts of an entry: the chunk divisor as is, and the wave
 * count as a factor (entry / 1024) on the instance's share of the chip's waves.
 * rpca_tune_get / rpca_tune_set read or overwrite the entry that covers
 * (k, n) (for saving and restoring a tuned table). */
int rpca_autotune(int64_t m_probe, int32_t reps, void* stream);
int rpca_tune_get(int32_t k, int64_t n, int32_t* target_waves, int32_t* chunk_div);
int rpca_tune_set(int32_t k, int64_t n, int32_t target_waves, int32_t chunk_div);

#ifdef __cplusplus
}
#endif

#endif /* RPCA_BATCH_H */
