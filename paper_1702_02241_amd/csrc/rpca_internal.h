// Internal declarations shared by the HIP translation units of librpca.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <chrono>
#include <vector>

#include "../../include/rpca.h"

#define RPCA_MEMMAX 16      // ring slots for (s, y): up to 15 pairs plus one spare
#define RPCA_NSCAL 8        // scalar partial slots per workgroup of a sweep

// Control phases of the device-resident L-BFGS state machine.  Every kernel of
// a solver slot reads `phase` first and does nothing unless the phase is its own.
enum {
  PH_TRIAL = 0,     // evaluate f, grad at x + alpha d (line-search trial)
  PH_UPDATE = 1,    // trial accepted: store the (s, y) pair, form the compact matrices
  PH_DIRECTION = 2, // form d = -H g
  PH_DONE = 3
};

// Reasons the device loop stops (state.stop).
enum {
  STOP_NONE = 0,
  STOP_GTOL = 1,
  STOP_FTOL = 2,
  STOP_MAXITER = 3,
  STOP_LINESEARCH = 4,
  STOP_NONFINITE = 5
};

// Device-resident solver state.  One instance per context (in device memory);
// the host initialises it and reads it back between batches of trials.
struct SolverState {
  int phase;
  int cur;              // which x/g buffer holds the current iterate
  int stop;
  int iter;             // accepted iterations
  int evals;            // objective+gradient evaluations
  int max_iter;
  int mem;              // pairs to keep
  int count;            // pairs stored
  int newest;           // ring slot of the newest pair (-1 if none)
  int spare;            // ring slot written by the next update
  int order[RPCA_MEMMAX];   // ring slots from oldest to newest
  int ls_stage;         // 0 = bracketing, 1 = zoom
  int ls_trials;        // trials in the current search
  int restarted;        // memory already reset once in this search
  int first_iter;       // the next direction's first trial step is min(1, 1/||g||_1), not 1
  int mode_bf16;        // products in BF16 for the current phase
  int dir_pending;      // PH_TRIAL set up by the update (g^T d known): the direction pass still has to form d
  double c1, c2, gtol, ftol;
  double eps_f;         // relative rounding level of f for the approximate-Wolfe test
  double f;             // objective at the current iterate
  double dphi0;         // g^T d at the current iterate
  double gnorm_inf, gnorm1, gg;
  double alpha;         // step of the pending trial
  double a_prev, f_prev, d_prev;
  double a_lo, f_lo, d_lo, a_hi, f_hi, d_hi;
  double f_t, dphi_t;   // last trial
  double dd;            // d^T d
  double gamma;
  double fhist[8];
  double best_f;
  double gref;          // gtol < 0: the gradient test is ||g||_inf <= -gtol * gref, gref = ||g||_inf
                        // at the phase's first iteration (0 until then)
  // --- everything above is the state head (what the line search reads and writes) ---
  double SY[RPCA_MEMMAX][RPCA_MEMMAX];  // s_i^T y_j by slot
  double YY[RPCA_MEMMAX][RPCA_MEMMAX];  // y_i^T y_j by slot
  double coef_s[RPCA_MEMMAX];           // d = -(gamma g + sum coef_s[slot] s_slot + sum coef_y[slot] y_slot)
  double coef_y[RPCA_MEMMAX];
};

// Block-cooperative copy of the solver state in 8-byte words (used to stage the
// state in LDS before one thread runs the scalar algebra on it).
__device__ __forceinline__ void copy_state_block(SolverState* dst, const SolverState* src) {
  static_assert(sizeof(SolverState) % 8 == 0, "state size");
  const unsigned long long* s = reinterpret_cast<const unsigned long long*>(src);
  unsigned long long* d = reinterpret_cast<unsigned long long*>(dst);
  for (int i = threadIdx.x; i < (int)(sizeof(SolverState) / 8); i += blockDim.x) d[i] = s[i];
}

// The same for the state head only (the fields before the (s, y) Gram matrices).
__device__ __forceinline__ void copy_state_head(SolverState* dst, const SolverState* src) {
  static_assert(offsetof(SolverState, SY) % 8 == 0, "state head size");
  const unsigned long long* s = reinterpret_cast<const unsigned long long*>(src);
  unsigned long long* d = reinterpret_cast<unsigned long long*>(dst);
  for (int i = threadIdx.x; i < (int)(offsetof(SolverState, SY) / 8); i += blockDim.x) d[i] = s[i];
}

// Arguments of the fused objective/gradient sweep.
struct SweepArgs {
  const float* X;
  const uint32_t* mask;   // column-major bitmask, word (j*mw + i/32), or null
  int64_t m, n;
  int32_t k, mw;
  float lam_s, lam_l;
  float kappa;            // slope of rho' beyond lam_s: mu / (1 + mu) (elastic net), 0 for l1
  int32_t xvec;           // 1: X is 16-byte aligned and m % 4 == 0 (vector loads allowed)
  // base point: U[cur], V[cur]; trial point = base + alpha * d
  const float* U[2];
  const float* V[2];
  const float* dU;
  const float* dV;
  SolverState* st;        // null for a plain evaluation (alpha = 0, cur = 0)
  float* Ut[2];           // trial point written to Ut[1-cur] (solver) or nothing
  float* Vt[2];
  float* gU[2];           // gradient output for the evaluated point (index: out slot)
  float* gupart;          // [chunks][m*k] partial G V when n spans several chunks
  float* gvpart;          // [row_groups][n*k] partial G^T U (one per workgroup row)
  double* spart;          // [row_groups*chunks][RPCA_NSCAL] scalar partials
  const float* pc;        // preconditioner [W | M_U | M_V] (k x k each) or null (plain variables)
  int32_t strips_per_wave;  // most 16-row strips of one wave (row group rg of R owns strips [rg S/R, (rg+1) S/R))
  int32_t chunk_w;        // columns per chunk (multiple of 16)
  int32_t nchunks;
  int32_t row_groups;     // workgroups along the rows (grid.x)
};

// One work item of the batched sweep: workgroup row rg, column chunk ch of instance inst.
struct SweepItem {
  int32_t inst, rg, ch, kb, tmax;
};

// Arguments of the finishing reduction (gV, f, g^T d, line-search step).
struct FinishArgs {
  int64_t m, n;
  int32_t k;
  float lam_l;
  const float* U[2];      // point that was evaluated (index = out slot)
  const float* V[2];
  const float* dU;
  const float* dV;
  SolverState* st;
  const float* gupart;
  const float* gvpart;
  const double* spart;
  float* gU[2];
  float* gV[2];
  double* level2;         // [segs][n*k] first-level sums of the G^T U partials
  double* fpart;          // [blocks][3] partials of the second reduction
  unsigned int* counter;  // last-block counter (zero between launches)
  double* f_out;          // plain mode: receives f (null: not stored)
  double* aux_out;        // plain mode, optional: phi, ||U||^2, ||V||^2, ||G||_F^2
  int32_t nchunks, row_groups, sweep_wgs;
  int32_t segs, rows_per_seg;  // workgroup rows are summed in segs segments
  int32_t gv_blocks;      // set by the launcher
  const float* pc;        // preconditioner [W | M_U | M_V] or null (see SweepArgs)
};

// Flat N-vector kernels of L-BFGS.  x, g, d, S, Y all hold N = (m+n)k floats,
// the U part first (row-major) then the V part.
struct LbfgsArgs {
  int64_t N;
  SolverState* st;
  float* x[2];
  float* g[2];
  float* d;
  float* S;               // [RPCA_MEMMAX][N]
  float* Y;               // [RPCA_MEMMAX][N]
  double* part;           // [blocks][RPCA_NDOT]
  unsigned int* counter;
};

#define RPCA_NDOT (4 * RPCA_MEMMAX + 8)
#define RPCA_LBFGS_MAX_BLOCKS 1024  // blocks of an L-BFGS pass; its partials take RPCA_NDOT each

// Host-side launchers (defined in the .hip files).
namespace rpca {
// Sweep decomposition per (k bucket, n bucket) (see rpca_autotune).
constexpr int TUNE_KB = 4;   // k <= 8, 16, 24, 32
constexpr int TUNE_NB = 5;   // n <= 64, 128, 256, 512, larger
struct SweepTune {
  int target_waves;  // waves the strips of one sweep are spread over
  int chunk_div;     // widest LDS-fitting chunk divided by this
};
int tune_k_bucket(int k);
int tune_n_bucket(int64_t n);
SweepTune tune_get(int k, int64_t n);
void tune_set(int kbucket, int nbucket, SweepTune t);
// Sweep decomposition of an m x n, rank-k instance; target_waves > 0 replaces
// the table's wave target (a batch spreads one chip's waves over many instances).
int sweep_blocks_for(int64_t m, int64_t n, int k, int* row_groups, int* strips_per_wg, int* chunk_w,
                     int* nchunks, int target_waves = 0);
// rpca_create with the sweep's wave target given (0: the tuning table's).
int create_ctx(int64_t m, int64_t n, int32_t k, double lam_s, double lam_l, const uint8_t* mask,
               int target_waves, rpca_ctx** out, const uint32_t* mask_bits_dev = nullptr);
hipError_t launch_objgrad(const SweepArgs& sa, const FinishArgs& fa, bool trial, bool bf16,
                          hipStream_t stream);
hipError_t launch_sweep(const SweepArgs& sa, bool trial, bool bf16, hipStream_t stream);
hipError_t launch_finish(const FinishArgs& fa, bool trial, hipStream_t stream);
hipError_t launch_lbfgs_update(const LbfgsArgs& a, int mem, hipStream_t stream);
hipError_t launch_lbfgs_direction(const LbfgsArgs& a, int mem, hipStream_t stream, bool with_final = true);
int lbfgs_blocks(int64_t N);
// Batched launches: arrays of per-instance arguments in device memory, block
// offsets off[0..count] (device) of each instance in the flattened grid.
hipError_t launch_sweep_batch(int kb, int tmax, const SweepArgs* args, const SweepItem* items, int nitems,
                              unsigned* head, int grid, int lds_floats, bool masked, bool trial, bool bf16,
                              hipStream_t s);
int sweep_batch_grid(int kb, int tmax, int lds_floats, bool masked, bool trial, bool bf16);
int sweep_lds_floats(int kb, int k, int cwp);
int sweep_tmax_class(int kb, int ntiles);
hipError_t launch_finish_batch(const FinishArgs* fa, const int* off1, int total1, const int* off2, int total2,
                               int count, unsigned* queue_heads, int nheads, bool trial, hipStream_t s);
hipError_t launch_lbfgs_update_batch(const LbfgsArgs* la, const int* off, int count, int total_blocks, int mem,
                                    hipStream_t s);
hipError_t launch_lbfgs_direction_batch(const LbfgsArgs* la, const int* off, int count, int total_blocks,
                                       int mem, hipStream_t s, bool with_final = true);
int finish_blocks(int64_t m, int64_t n, int k, int nchunks, int* gv_blocks);
}  // namespace rpca

// Context internals needed by the certificate / initialisation module.
struct rpca_ctx;
namespace rpca {
struct CtxView {
  int64_t m, n;
  int k;
  double lam_s, lam_l;
  double kappa;          // elastic-net slope (0: l1)
  const uint32_t* mask;
  int mw;
  double* best_F;
  rpca_ctx* ctx;         // for kernel timing (prof_begin / prof_end)
  double* phi0;          // phi(0) of the current solve (NaN: unknown)
  const void** phi0_X;   // the X it belongs to
};
CtxView ctx_view(rpca_ctx* c);
// Event pair around one launch when the context's kernel timing is on: begin
// records the first event (token null when timing is off), end the second and
// files the pair under class cls.
hipError_t prof_begin(rpca_ctx* c, hipStream_t s, void** token);
hipError_t prof_end(rpca_ctx* c, int cls, hipStream_t s, void* token);
bool prof_enabled(const rpca_ctx* c);  // kernel timing on
// Optional outputs of the certificate's power iteration: the top Ritz vector v of
// M^T M (n values, P_V^perp-projected, unit norm) and the k x r map T_U with
// U1 = U T_U (the left singular vectors of L).
struct CertExtra {
  std::vector<double> v;
  std::vector<double> TU;
  int r = 0;
};
int certificate_impl(rpca_ctx* c, const float* X, const float* U, const float* V, rpca_cert* out,
                     double quick_tol, hipStream_t s, CertExtra* extra = nullptr);
int growth_direction_impl(rpca_ctx* c, const float* X, const float* U, const float* V, float* u_col,
                          float* v_col, double* sigma, double* t, hipStream_t s,
                          rpca_cert* cert_out = nullptr);
int ctx_objgrad_aux(rpca_ctx* c, const float* X, const float* U, const float* V, double* f_dev,
                    double* aux_dev, float* gU, float* gV, hipStream_t s);
// Device workspace owned by the context, grown on demand; *fresh = 1 when newly allocated.
void* ctx_workspace(rpca_ctx* c, size_t bytes, int* fresh);
// Pinned host staging owned by the context (at least 256 KB, grown on demand;
// null on failure).  Callers synchronise their copies through it before returning.
void* ctx_pinned(rpca_ctx* c, size_t bytes);
// hipHostFree that leaves no pending error behind when the free fails.
void host_free(void* p);

// Solve steps shared by rpca_solve and the batched solver.
struct SolvePhase {
  bool bf16;
  double gtol;
};
struct InstanceArgs {
  SweepArgs sa_loop, sa_eval;
  FinishArgs fa_loop, fa_eval;
  LbfgsArgs lu, ld;
  int fin1_blocks, fin2_blocks, lb_blocks;
  int row_groups, nchunks, chunk_w, spw;
  bool masked;
  SolverState* state_dev;
  SolverState* state_host;
};
bool valid_opts(const rpca_opts& o);
int solve_phases(const rpca_opts& o, SolvePhase* ph);
int solve_setup(rpca_ctx* c, const float* X, float* U, float* V, const rpca_opts& o, double gtol0,
                hipStream_t s);
int eval_current(rpca_ctx* c, const float* X, int cur, bool bf16, hipStream_t s);
int run_lbfgs(rpca_ctx* c, const float* X, const rpca_opts* o, bool bf16, hipStream_t s);
int resume_state(rpca_ctx* c, double gtol, double ftol, hipStream_t s);
int restart_state(rpca_ctx* c, double gtol, double ftol, int max_iter, bool reset_memory, hipStream_t s);
int run_cycles(rpca_ctx* c, const float* X, const rpca_opts& o, bool bf16, double gtol, double ftol,
               bool keep_memory, int budget, hipStream_t s);
void instance_args(rpca_ctx* c, const float* X, int cur, InstanceArgs* out);
// Preconditioned variables (precond.hip).
constexpr int PC_GRAM_BLOCKS = 256;
int precond_refresh(rpca_ctx* c, int cur, hipStream_t s);
int precond_to_plain(rpca_ctx* c, int cur, hipStream_t s);
SolverState* ctx_state_host(rpca_ctx* c);
// Certificates a solve takes at most (each but the last followed by a round).
constexpr int CERT_ROUNDS = 8;
int copy_out(rpca_ctx* c, float* U, float* V, hipStream_t s);
int round_tolerances(const rpca_opts& o, double* gtol, double* ftol);
void end_round(rpca_ctx* c, const rpca_opts& o);
int finish_status(rpca_ctx* c, const rpca_opts& o, int certified, double rel_gap, int rounds, int iters_bf16,
                  std::chrono::steady_clock::time_point t0, rpca_info* info);
int solve_finish(rpca_ctx* c, const float* X, float* U, float* V, const rpca_opts& o, bool final_bf16,
                 double gtol, int iters_bf16, std::chrono::steady_clock::time_point t0, rpca_info* info,
                 hipStream_t s);
// Fused thin Gram product Z = Op^T (Op W) in one pass over X (gram_apply.hip):
// Op = Omega .* rho'(U V^T - X) (resid) or Omega .* X; rank k <= 16, n <= 256.
struct GramApplyArgs {
  const float* X;
  const uint32_t* mask;   // column-major bitmask (word j*mw + i/32) or null
  int64_t m, n;
  int32_t k, mw;
  float lam_s, kappa;
  const float* U;         // m x k row-major (residual source)
  const float* V;         // n x k row-major (residual source)
  const float* W;         // n x 16 row-major FP32, columns past the block zero
  float* part;            // [row_groups][n * 16] per-workgroup sums
  int32_t row_groups;     // workgroups (grid)
  int32_t xvec;           // 1: X is 16-byte aligned and m % 4 == 0
  const double* skip;     // null, or a device flag: when nonzero the pass and its sum do nothing
};
bool gram_apply_fits(int64_t n, int k);
size_t gram_apply_lds_bytes(int64_t n);
// The pass: per-workgroup FP32 sums into a.part.
hipError_t launch_gram_apply_pass(const GramApplyArgs& a, bool resid, hipStream_t s);
// The sum over workgroups (FP64, fixed order):
// Z[j * ldz + col0 + p] = scale * (Op^T Op W)[j][p] for p < b.
hipError_t launch_gram_apply_sum(const GramApplyArgs& a, double* Z, int ldz, int col0, int b, double scale,
                                 hipStream_t s);
// Both.
hipError_t launch_gram_apply(const GramApplyArgs& a, bool resid, double* Z, int ldz, int col0, int b, double scale,
                             hipStream_t s);
}  // namespace rpca
