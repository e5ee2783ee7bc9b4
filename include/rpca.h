/*
 * librpca -- Split-SPCP (Burer-Monteiro robust PCA with the sparse part
 * marginalised) on AMD Instinct MI355X (gfx950).
 *
 * The method (Driggs, Becker & Aravkin, "Adapting Regularized Low-Rank Models
 * for Parallel Architectures"):
 *
 *   phi(L)  = min_S 1/2 ||P_Omega(L + S - X)||_F^2 + lam_S ||S||_1
 *           = sum_{(i,j) in Omega} huber_{lam_S}(L_ij - X_ij)            (Sec. 1, eq. PhiDef)
 *   f(U,V)  = phi(U V^T) + lam_L/2 (||U||_F^2 + ||V||_F^2)               (eq. smoothNC, eq. Thm5)
 *   G       = Omega .* clip(U V^T - X, -lam_S, lam_S)                    (Sec. 3.2, eq. diff)
 *   df/dU   = G V + lam_L U,   df/dV = G^T U + lam_L V
 *
 * minimised by L-BFGS (memory 10, Sec. 5.1) and checked by the convergence
 * certificate of Sec. 3.4 (gap bound eq. Fbound).
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - X is FP32, column-major, m x n, leading dimension m (one video frame per
 *    column, as in Sec. 5.4).  Unobserved entries may hold any finite value.
 *  - U is m x k and V is n x k, FP32, row-major (row i of U is U[i*k .. i*k+k)).
 *    Gradients use the same layout.
 *  - Pointers documented as "device" must be HIP device allocations on the
 *    context's device.  "host" pointers are ordinary host memory.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *    asynchronous on `stream` unless documented otherwise.
 *  - The caller owns every buffer it passes in; the context owns its workspace.
 *    A context must not be used from two streams or two threads at once.
 *  - Return codes: 0 = success; > 0 = warning, outputs valid; < 0 = error,
 *    outputs unspecified.  All argument checks happen before any HIP call.
 */
#ifndef RPCA_H
#define RPCA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum rpca_status {
  RPCA_OK = 0,
  RPCA_ENOTCONV = 1,      /* iteration budget spent; outputs are the last iterate */
  RPCA_ELINESEARCH = 2,   /* no strong-Wolfe step found after a restart; outputs valid */
  RPCA_ENOTCERT = 3,      /* converged but the certificate does not reach the target gap */
  RPCA_EINVAL = -1,       /* bad argument (checked before any HIP call) */
  RPCA_ENOMEM = -2,       /* device or pinned allocation failed */
  RPCA_EHIP = -3,         /* a HIP runtime call failed */
  RPCA_ENONFINITE = -4,   /* objective or gradient became NaN/Inf */
  RPCA_ETOOBIG = -5       /* the instance exceeds the fixed scratch of rpca_objgrad_noalloc */
};

enum rpca_precision {
  RPCA_PREC_FP32 = 0,         /* FP32 products on MFMA, FP32 residual, FP64 reductions */
  RPCA_PREC_BF16_POLISH = 1,  /* BF16 MFMA products until a loose tolerance, then FP32 */
  RPCA_PREC_BF16 = 2          /* BF16 MFMA products throughout */
};

enum rpca_init {
  RPCA_INIT_GIVEN = 0,        /* start from the U, V the caller passes */
  RPCA_INIT_RSVD = 1          /* randomized-SVD cold start (Sec. 4.2), overwrites U, V */
};

typedef struct rpca_ctx rpca_ctx;

/* Solver options.  rpca_default_opts() fills the defaults listed here. */
typedef struct rpca_opts {
  int32_t precision;        /* rpca_precision, default RPCA_PREC_FP32 */
  int32_t mem;              /* L-BFGS pairs kept, 1..15, default 10 (Sec. 5.1) */
  int32_t max_iter;         /* L-BFGS iterations, default 5000 */
  int32_t init;             /* rpca_init, default RPCA_INIT_GIVEN */
  double gtol;              /* stop: ||g||_inf <= gtol * max(1,|f|), default 1e-6 */
  double ftol;              /* stop: relative f decrease over 5 iterations < ftol, default 1e-9;
                               0 switches the test off (certification rounds always do) */
  double bf16_gtol;         /* RPCA_PREC_BF16_POLISH: the BF16 phase ends once ||g||_inf has
                               fallen to bf16_gtol times its value at the phase's first
                               iteration (a test that does not grow with m n), when f stops
                               decreasing (ftol) or when the line search stalls at the BF16
                               rounding level; then the FP32 polish runs.  Default 1e-3 */
  double c1, c2;            /* strong-Wolfe constants, default 1e-4, 0.9 */
  int32_t certify;          /* 1 (default): run the certificate at the end; while rel_gap > cert_tol
                               continue from the point reached (one more preconditioner cycle
                               with the stopping tests off, or a tenfold tighter gtol in plain
                               variables) and certify again, at most 8 certificates */
  double cert_tol;          /* certified threshold on gap/F, default 1e-3 */
  int32_t rsvd_oversample;  /* p, default 10 */
  int32_t rsvd_power;       /* q, default 2 */
  uint64_t seed;            /* seed of the counter-based generator (rSVD sketch, power start) */
  int32_t slots_per_sync;   /* line-search trials per host poll, default 16 */
  int32_t precond;          /* 1 (default): iterate on A = U P_U^{-1}, B = V P_V^{-1} with
                               P_U = (V^T V + lam_L I)^{-1/2}, P_V = (U^T U + lam_L I)^{-1/2},
                               refreshed every precond_cycle iterations (same minimisers;
                               far fewer iterations for ill-conditioned factors); 0: plain */
  int32_t precond_cycle;    /* iterations per preconditioner refresh, default 50 */
} rpca_opts;

typedef struct rpca_info {
  int32_t status;           /* rpca_status of the solve */
  int32_t iters;            /* accepted L-BFGS iterations (all phases) */
  int32_t evals;            /* objective+gradient evaluations */
  int32_t iters_bf16;       /* iterations done in the BF16 phase */
  double f;                 /* final objective f(U,V) */
  double gnorm_inf;         /* final ||grad f||_inf */
  double rel_gap;           /* certificate gap/F (NaN when not certified) */
  int32_t certified;        /* rel_gap <= cert_tol */
  int32_t cert_rounds;      /* certificate evaluations performed */
  double seconds;           /* wall time of the call */
} rpca_info;

typedef struct rpca_cert {
  double T1, T2, T3, T4;    /* the four terms of ||E||_F^2 (Sec. 3.4), normalised by lam_L */
  double E;                 /* ||E||_F including the rank-truncation correction */
  double F;                 /* F(L) = lam_L ||L||_* + phi(L) (eq. genConvex) */
  double phi;               /* phi(L) */
  double phi0;              /* phi(0) = sum_Omega huber(X) */
  double F_bound;           /* min(F, phi0, best F known to the context) */
  double normL;             /* ||L||_F */
  double gap;               /* E * (lam_L ||L||_F + F_bound)  (eq. Fbound) */
  double rel_gap;           /* gap / F */
  double normM2;            /* ||P_U^perp D P_V^perp||_F^2 */
  double theta[32];         /* leading singular values of P_U^perp D P_V^perp (Ritz estimates) */
  double sigma[64];         /* singular values of L (first min(k,64)) */
  int32_t r;                /* numerical rank of L used by the certificate */
  int32_t power_iters;      /* block power iterations run for T4 */
  int32_t block;            /* block size of the power iteration */
  int32_t certified;        /* rel_gap <= cert_tol */
} rpca_cert;

/* Fill `opts` with the defaults.  Never fails. */
void rpca_default_opts(rpca_opts* opts);

/* Create a context for m x n data, factor rank k (1 <= k <= 32, k <= min(m,n)),
 * weights lam_S > 0, lam_L > 0 (eq. lag / eq. Thm5).
 * mask: NULL for full observation, else m x n column-major bytes (nonzero =
 * observed, the sampling operator P_Omega of Sec. 6.2) in HOST memory; it is
 * packed into a device bitmask, the caller keeps ownership.
 * Allocates the device workspace on the current HIP device.
 * Returns RPCA_EINVAL, RPCA_ENOMEM or RPCA_EHIP on failure (*out untouched). */
int rpca_create(int64_t m, int64_t n, int32_t k, double lam_S, double lam_L,
                const uint8_t* mask, rpca_ctx** out);

/* rpca_create with the sweep's decomposition fixed by a wave count:
 * target_waves (0..2^20) is the number of wavefronts the row strips of one
 * sweep are spread over (0: the tuning table's value for this k and n).  A
 * context that shares the GPU with others (or that must reproduce an
 * instance of a batch bit for bit, see rpca_batch_instance_waves) uses it.
 * Same errors as rpca_create; target_waves out of range is RPCA_EINVAL. */
int rpca_create_waves(int64_t m, int64_t n, int32_t k, double lam_S, double lam_L,
                      const uint8_t* mask, int32_t target_waves, rpca_ctx** out);

/* rpca_create_waves with the observation mask P_Omega (Sec. 6.2) given as a
 * DEVICE bitmask, the layout rpca_objgrad_noalloc reads: column-major, entry
 * (i, j) observed when bit i % 32 of word j * ceil(m / 32) + i / 32 is set (bits
 * past row m - 1 are cleared in the copy).  The context copies it (device to
 * device, on the null stream, synchronously) and the caller keeps ownership.  mask_bits NULL is RPCA_EINVAL (use rpca_create for
 * full observation); otherwise the errors of rpca_create_waves. */
int rpca_create_device_mask(int64_t m, int64_t n, int32_t k, double lam_S, double lam_L,
                            const uint32_t* mask_bits, int32_t target_waves, rpca_ctx** out);

/* Solver slots replayed from captured HIP graphs (on) or launched one by one
 * (off, the default: on the 76,800 x 200 video the graphs took 15.85 ms per
 * solve against 15.57 ms eager, the launch queue already running ahead of the
 * GPU).  With graphs, rpca_solve replays a captured group of
 * slots_per_sync slots (direction, trial sweep, finishing reduction, pair
 * update) on a stream the context owns, ordered after the caller's stream; the
 * graphs are kept per (X, preconditioner, regulariser, memory, group size,
 * precision) and freed by rpca_destroy.  Results are bitwise the same either
 * way.  With kernel timing on (rpca_profile_enable) the slots are launched one
 * by one.  RPCA_EINVAL for a null context. */
int rpca_set_graphs(rpca_ctx* ctx, int32_t on);

/* The sweep decomposition a context took when it was created (from the
 * tuning table, or from rpca_create_waves): out[0] workgroup rows, out[1]
 * strips of 16 rows per wave, out[2] columns per chunk, out[3] chunks.
 * Host only; RPCA_EINVAL for null arguments. */
int rpca_sweep_layout(const rpca_ctx* ctx, int32_t out[4]);

/* Elastic-net regulariser (Sec. 1 lists it among the structures r(S) that
 * marginalise like the l1 norm): r(S) = lam_S ||S||_1 + mu/2 ||S||_F^2.  The
 * per-entry marginal keeps rho(r) = r^2/2 for |r| <= lam_S and becomes
 * lam_S |r| - lam_S^2/2 + kappa/2 (|r| - lam_S)^2 beyond, kappa = mu / (1 + mu), so
 * grad phi = Omega .* (c + kappa (R - c)), c = clip(R, +-lam_S), still 1-Lipschitz:
 * the solver, the certificate and the rank-growth step apply unchanged.  Every
 * later objective, gradient, solve and certificate of the context uses it.
 * mu = 0 (the default) is the l1 regulariser, bit for bit.  With mu > 0 the
 * products run in FP32 only: rpca_objgrad_ex and rpca_solve return RPCA_EINVAL
 * for the BF16 precisions.  mu >= 0 and finite, else RPCA_EINVAL.  Changing mu
 * forgets the certificate's cached values. */
int rpca_set_elastic(rpca_ctx* ctx, double mu);

/* Objective and gradient at (U, V) (Sec. 1 eq. PhiDef/eq. smoothNC, Sec. 3.2 eq. diff).
 * X, U, V, gU, gV: device.  f: device pointer to one double receiving f(U,V).
 * Deterministic: the same inputs give bitwise identical outputs. */
int rpca_objgrad(rpca_ctx* ctx, const float* X, const float* U, const float* V,
                 double* f, float* gU, float* gV, void* stream);

/* rpca_objgrad with a choice of product precision: RPCA_PREC_FP32 (same as
 * rpca_objgrad) or RPCA_PREC_BF16 (U, V and G rounded to bf16 for the MFMA
 * products, FP32 accumulation and residual, FP64 sums). */
int rpca_objgrad_ex(rpca_ctx* ctx, const float* X, const float* U, const float* V,
                    double* f, float* gU, float* gV, int32_t precision, void* stream);

/* Bytes of the device array behind rpca_objgrad_noalloc (per GPU). */
#define RPCA_NOALLOC_SCRATCH_MB 64

/* rpca_objgrad for callers that cannot allocate: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  No context: the
 * instance is described by its arguments (the same rules as rpca_create:
 * 1 <= k <= 32, k <= min(m, n), lam_S, lam_L > 0 and finite), the l1
 * regulariser and FP32 products.  X, U, V, gU, gV, f: device, as in
 * rpca_objgrad.  mask_bits: NULL (every entry observed) or a DEVICE bitmask,
 * column-major: entry (i, j) is observed when bit i % 32 of word
 * j * ceil(m / 32) + i / 32 is set.  The same kernels and the same sweep
 * decomposition as a context made by rpca_create for these sizes, so the
 * outputs are bitwise those of rpca_objgrad on such a context.
 * Allocates nothing (no hipMalloc, hipFree or allocating library call): the
 * partial sums live in one library-owned device array of
 * RPCA_NOALLOC_SCRATCH_MB MiB per GPU, resolved on the first call on each
 * device and held until the process ends.  Every call on a GPU shares that
 * GPU's array: calls in stream order are safe, calls that overlap on one GPU
 * (two streams or two threads at once) race.  Call with the device that holds
 * the buffers current.  Returns RPCA_EINVAL for bad arguments, RPCA_ETOOBIG when
 * the instance's partials do not fit the array (they take
 * 4 R n k + 8 ceil(R / 16) n k bytes for the R <= 256 workgroup rows of the
 * default decomposition, plus 4 C m k when the n columns span C > 1 chunks of
 * a few hundred; 2.1 MB at 76,800 x 200, k = 10), RPCA_EHIP when the array's address cannot be
 * resolved or a launch fails. */
int rpca_objgrad_noalloc(int64_t m, int64_t n, int32_t k, double lam_S, double lam_L,
                         const uint32_t* mask_bits, const float* X, const float* U,
                         const float* V, double* f, float* gU, float* gV, void* stream);

/* Minimise f from (U, V) with L-BFGS + strong-Wolfe line search (Sec. 5.1).
 * X: device.  U, V: device, in = start (ignored with RPCA_INIT_RSVD), out =
 * solution.  opts: host, NULL = defaults.  info: host, may be NULL.
 * Blocks the calling thread until the solve ends (the iteration runs on the
 * device; the host only polls a status word between batches of trials). */
int rpca_solve(rpca_ctx* ctx, const float* X, float* U, float* V,
               const rpca_opts* opts, rpca_info* info, void* stream);

/* Convergence certificate at L = U V^T (Sec. 3.4): T1..T3 from the factor
 * SVD (footnote of Sec. 3.4) and one gradient sweep; T4 by projected block
 * power iteration on P_U^perp D P_V^perp (from Ritz values: exact when the
 * block holds every singular value above 1, an over-estimate otherwise); gap
 * bound eq. Fbound.  X, U, V: device.  out: host.
 * Blocks until the result is in `out`. */
int rpca_certificate(rpca_ctx* ctx, const float* X, const float* U, const float* V,
                     rpca_cert* out, void* stream);

/* Rank-growth direction at L = U V^T (Sec. 4.1, which adds one column to U
 * and V when the solver stops).  The column is read from the certificate's last
 * block: (sigma, u, v) is the top singular triplet of P_U^perp D P_V^perp
 * (D = grad phi(L) / lam_L; v from the certificate's block power iteration, u =
 * P_U^perp D v / sigma, so u^T D v = sigma).  L is optimal only if sigma <= 1.
 * When sigma > 1, the factors [U, u_col], [V, v_col] with u_col = sqrt(t) u,
 * v_col = -sqrt(t) v and t = lam_L (sigma - 1) lower f by at least
 * lam_L^2 (sigma - 1)^2 / 2 (phi's curvature along the unit-Frobenius u v^T is at
 * most 1); when sigma <= 1 both columns are zero and t = 0.
 * X, U, V: device (as rpca_solve).  u_col (m floats), v_col (n floats): device,
 * written.  sigma, t: host.  Blocks until done.  RPCA_EINVAL on null pointers. */
int rpca_rank_direction(rpca_ctx* ctx, const float* X, const float* U, const float* V,
                        float* u_col, float* v_col, double* sigma, double* t, void* stream);

/* rpca_solve with the rank grown on demand (Sec. 4.1): start at rank k0; below
 * k_max each rank is solved without certification rounds and then certified
 * once: certified -> done; not certified and the growth direction
 * (rpca_rank_direction) has sigma > 1 -> append that column pair and continue
 * from the grown factors at rank k + 1; otherwise (and at k_max) the solve
 * continues with certification rounds as rpca_solve.  Each rank uses its own
 * context (made and destroyed inside); the call blocks until done.  m, n,
 * lam_S, lam_L, mask: as rpca_create; 1 <= k0 <= k_max <= 32, k_max <=
 * min(m, n).  X: device.  U, V: device buffers of m * k_max and n * k_max
 * floats; in: the start at rank k0 (the first m * k0 and n * k0 floats,
 * row-major; ignored with RPCA_INIT_RSVD), out: the solution at rank *k_out
 * (the first m * k_out and n * k_out floats).  opts as rpca_solve (certify is
 * forced on).  info: status, f, gradient and certificate of the last rank;
 * iters, evals and cert_rounds summed over all ranks.  Returns that status
 * (RPCA_EINVAL on bad arguments before any HIP call). */
int rpca_solve_grow(int64_t m, int64_t n, int32_t k0, int32_t k_max, double lam_S, double lam_L,
                    const uint8_t* mask, const float* X, float* U, float* V, int32_t* k_out,
                    const rpca_opts* opts, rpca_info* info, void* stream);

/* Convex baseline: accelerated proximal gradient (FISTA with function-value
 * restart) on F(L) = lam_L ||L||_* + phi(L) (eq. genConvex), the class of solvers
 * the paper compares against (Sec. 6.1: SVT steps with a randomized SVD).  Each
 * step takes the singular-value threshold of Z = Y - grad phi(Y) at the
 * extrapolated point Y from a randomized SVD of Z (sketch of width rank +
 * oversample, warm-started with the last step's right singular vectors and
 * widened while every sketched value exceeds lam_L; power_steps subspace
 * iterations), computed through thin products that form Z tile by tile from Y's
 * factors and X.  Step size 1 (grad phi is 1-Lipschitz).  Stops when the
 * relative change of F between steps is at most tol, or after max_iter steps.
 * ctx: its k bounds the rank of an iterate (momentum needs the ranks of two
 * iterates to fit in k, else that step is a plain one; a rank above k is
 * truncated and reported); every entry observed (a context made with a mask:
 * RPCA_EINVAL).  X: device.  U, V: device outputs (m x k, n x k row-major), the
 * balanced factors L = U V^T, zero beyond the rank; start L = 0.  1 <= max_iter,
 * tol >= 0, 0 <= oversample <= 32, 0 <= power_steps <= 8.  Blocks until done.
 * Returns RPCA_OK (converged) or RPCA_ENOTCONV, RPCA_EINVAL, RPCA_ENOMEM, RPCA_EHIP. */
typedef struct rpca_prox_info {
  int32_t status;           /* RPCA_OK or RPCA_ENOTCONV */
  int32_t iters;            /* proximal steps accepted */
  int32_t restarts;         /* momentum restarts */
  int32_t rank;             /* rank of the returned L */
  int32_t sketch;           /* last sketch width */
  int32_t truncated;        /* 1 if some step had more than k values above lam_L */
  double F;                 /* F(L) of the returned L */
  double rel_change;        /* last relative change of F */
  double seconds;           /* wall time of the call */
} rpca_prox_info;
int rpca_prox_solve(rpca_ctx* ctx, const float* X, float* U, float* V, int32_t max_iter, double tol,
                    int32_t oversample, int32_t power_steps, uint64_t seed, rpca_prox_info* info, void* stream);

/* Randomized-SVD start (Sec. 4.2): U0 = U_k S_k^{1/2}, V0 = V_k S_k^{1/2} from
 * the sketch Y = P_Omega(X) Omega_s, q power steps, B = Q^T P_Omega(X).
 * Omega_s: device, n x (k+p) row-major FP32 test matrix (p = oversample);
 * pass NULL to draw it on the device from `seed` (SplitMix64 + Box-Muller).
 * U, V: device outputs.  Synchronous. */
int rpca_init_rsvd(rpca_ctx* ctx, const float* X, const float* Omega_s, int32_t oversample,
                   int32_t power_steps, uint64_t seed, float* U, float* V, void* stream);

/* Kernel classes reported by the profiler. */
enum rpca_kernel_class {
  RPCA_K_SWEEP = 0,       /* fused objective/gradient sweep over X (plain evaluations) */
  RPCA_K_FINISH = 1,      /* finishing reduction + line-search step */
  RPCA_K_UPDATE = 2,      /* L-BFGS history update (FP64 dots) */
  RPCA_K_DIRECTION = 3,   /* L-BFGS direction */
  RPCA_K_TRIAL = 4,       /* the same sweep at line-search trial points */
  RPCA_K_LEFT = 5,        /* thin product Op W of the certificate, the rSVD and the proximal baseline */
  RPCA_K_RIGHT = 6,       /* thin product Op^T Y (the same users) */
  RPCA_K_GRAM = 7,        /* fused thin product Op^T (Op W) in one pass, per-workgroup sums (certificate
                             and rSVD power steps; the FP64 sum over workgroups is not counted) */
  RPCA_K_NCLASS = 8
};

typedef struct rpca_profile {
  int64_t launches[8];      /* launches per rpca_kernel_class since the last reset */
  double ms[8];             /* summed device time (HIP events on the launch stream) */
} rpca_profile;

/* Turn per-launch HIP-event timing of the solver kernels on (1) or off (0).
 * When on, rpca_objgrad and rpca_solve record an event pair around each kernel
 * on the stream it runs on; times are collected at the next synchronisation.
 * Meant for measurement; it adds a little host overhead per launch. */
int rpca_profile_enable(rpca_ctx* ctx, int32_t on);

/* Copy the accumulated profile into `out` (host); reset it when `reset` != 0.
 * Synchronises the context's pending events. */
int rpca_profile_read(rpca_ctx* ctx, rpca_profile* out, int32_t reset);

/* Release the context and its device workspace. NULL is ignored. */
void rpca_destroy(rpca_ctx* ctx);

/* Human-readable name of a status code (static storage). */
const char* rpca_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* RPCA_H */
