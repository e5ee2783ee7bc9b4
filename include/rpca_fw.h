/* Frank-Wolfe with the sparse part marginalised (Sec. 6.2, Alg. 1) on the GPU.
 *
 * Problem: over (L, t) with ||L||_* <= t, minimise lam_L t + phi(L), with phi
 * the Huber marginal of rpca.h (the program of Sec. 6.2, equivalent to SPCP).
 * One iteration from (L_k, t_k):
 *   G_k = P_Omega(clip(L_k - X, -lam_S, lam_S)) (the gradient of phi);
 *   (sigma, u, v) = top singular triplet of G_k (block power iteration on
 *   G_k^T G_k with 8 vectors and Rayleigh-Ritz, warm-started from the previous
 *   iteration's block);
 *   vertex (V, Vt) = (0, 0) if lam_L >= sigma, else (-B_k u v^T, B_k) with the
 *   bound B_k = (phi(L_k) + lam_L t_k) / lam_L (B_0 = phi(0) / lam_L at L = 0);
 *   eta = minimiser over [0, 1] of 1/2 ||G_k + eta P_Omega(V - L_k)||^2 +
 *   lam_L ((1 - eta) t_k + eta Vt) (closed form; the model majorises the
 *   objective, which therefore never increases);
 *   L_{k+1} = (1 - eta) L_k + eta V, t_{k+1} = (1 - eta) t_k + eta Vt.
 * The Frank-Wolfe gap <G_k, L_k - V> + lam_L (t_k - Vt) bounds the distance of
 * lam_L t_k + phi(L_k) to the optimum (up to the power iteration's accuracy).
 *
 * Storage: L, G and X are m x n FP32 column-major in HBM (X as in rpca.h); the
 * solver keeps L dense because its rank grows by one per step.  Sums in FP64.
 * The power steps' Rayleigh-Ritz, the step size and the stop test run on the
 * device; the host waits only on the power steps' stop flags.
 */
#ifndef RPCA_FW_H
#define RPCA_FW_H

#include <stdint.h>

#include "rpca.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rpca_fw rpca_fw;

typedef struct rpca_fw_info {
  int32_t status;        /* RPCA_OK: gap <= tol * F; RPCA_ENOTCONV: max_iter reached */
  int32_t iters;         /* Frank-Wolfe steps taken */
  int32_t power_iters;   /* power-iteration steps, all iterations */
  int32_t last_step;     /* 1 if the last vertex was nonzero */
  double F;              /* lam_L t + phi(L) at the returned (L, t) */
  double phi;            /* phi(L) */
  double gap;            /* Frank-Wolfe gap at the returned (L, t) */
  double sigma;          /* top singular value of G at the returned L */
  double eta;            /* last step size taken */
  double seconds;        /* wall time of the call */
} rpca_fw_info;

/* Workspace for m x n problems: G (m x n FP32), the power-iteration vectors and
 * the reduction partials (about 4 m n + 8 (m + n) bytes plus partials).  mask:
 * NULL (every entry observed) or m x n column-major host bytes, nonzero =
 * observed; copied, the caller keeps ownership.  lam_S, lam_L > 0 and finite.
 * RPCA_EINVAL on bad arguments (before any HIP call), RPCA_ENOMEM, RPCA_EHIP. */
int rpca_fw_create(int64_t m, int64_t n, double lam_S, double lam_L, const uint8_t* mask, rpca_fw** out);

/* Alg. 1 from (L, *t) until the gap is at most tol * F or max_iter steps.
 * X: device, m x n FP32 column-major.  L: device, m x n FP32 column-major, in:
 * the start (all zeros with *t = 0 is the cold start of Alg. 1; any start needs
 * ||L||_* <= *t), out: the last iterate.  t: host, in/out.  max_iter >= 0
 * (0 evaluates the start only), tol >= 0.  power_tol: the power iteration stops
 * when the top Ritz pair's relative residual ||G^T G x - theta x|| / theta is at
 * most this (at most 100 steps per iteration); 0 selects 1e-4.  info: may be
 * NULL.  Blocks until done.  The power-iteration block is kept as the next
 * call's warm start.  Returns
 * RPCA_OK / RPCA_ENOTCONV as in info->status, RPCA_EINVAL on bad arguments,
 * RPCA_ENONFINITE when phi(L) or <G, L> is NaN/Inf (an observed NaN/Inf in X
 * or L; *t is then the t of that iterate, L holds it, info is not written and
 * the next call starts the power iteration cold), RPCA_EHIP. */
int rpca_fw_solve(rpca_fw* fw, const float* X, float* L, double* t, int32_t max_iter, double tol,
                  double power_tol, rpca_fw_info* info, void* stream);

void rpca_fw_destroy(rpca_fw* fw);

/* Kernel timing.  When on, rpca_fw_solve records an event pair around each
 * streaming kernel (classes below; the small finishing kernels are not
 * counted); rpca_fw_profile_read collects them (synchronising on the events)
 * and optionally resets the counters.  RPCA_EINVAL on a null handle or out. */
enum rpca_fw_kernel {
  RPCA_FW_K_UPDATE = 0,    /* L <- a L + b y v^T and G: reads L, X; writes L, G */
  RPCA_FW_K_LEFT = 1,      /* partial Y = G Xb over column chunks: reads G */
  RPCA_FW_K_RIGHT = 2,     /* the power step: for n <= 256 the per-workgroup sums of
                              G^T (G Xb) in one pass over G (reads G), else the
                              partial Z = G^T Y over row chunks (reads G and Y) */
  RPCA_FW_K_BILINEAR = 3   /* u^T P_Omega(L) v: reads L */
};
typedef struct rpca_fw_profile {
  int64_t launches[4];
  double ms[4];
} rpca_fw_profile;
int rpca_fw_profile_enable(rpca_fw* fw, int32_t on);
int rpca_fw_profile_read(rpca_fw* fw, rpca_fw_profile* out, int32_t reset);

#ifdef __cplusplus
}
#endif

#endif
