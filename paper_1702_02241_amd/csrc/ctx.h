// The context object behind rpca_ctx* (shared by the translation units that
// manage its buffers: api.hip and precond.hip).
#pragma once

#include <math.h>

#include <vector>

#include "rpca_internal.h"

struct rpca_ctx {
  int64_t m = 0, n = 0;
  int k = 0;
  double lam_s = 0, lam_l = 0;
  double mu = 0;             // elastic-net weight of ||S||_F^2 / 2 (0: the l1 regulariser)
  uint32_t* mask = nullptr;  // device bitmask or null
  int mw = 0;
  // sweep configuration
  int row_groups = 0, spw = 0, chunk_w = 0, nchunks = 0, sweep_wgs = 0, segs = 0, rps = 16;
  float* gvpart = nullptr;
  float* gupart = nullptr;
  double* spart = nullptr;
  double* fpart = nullptr;
  double* level2 = nullptr;
  unsigned int* counters = nullptr;  // [0] finish, [1] update, [2] direction, [3..] spare
  // solver workspace
  int64_t N = 0;  // (m + n) k padded to a multiple of 256
  float* x[2] = {nullptr, nullptr};
  float* g[2] = {nullptr, nullptr};
  float* d = nullptr;
  float* S = nullptr;
  float* Y = nullptr;
  double* lpart = nullptr;
  SolverState* st = nullptr;       // device
  SolverState* st_host = nullptr;  // pinned host mirror
  double* dscratch = nullptr;      // device doubles for small results
  double best_F = INFINITY;        // best convex objective seen by certificates
  double phi0 = NAN;               // phi(0) cached for the certificates of one solve
  const void* phi0_X = nullptr;    // ... and the X it was computed from
  // preconditioned variables A = U P_U^{-1}, B = V P_V^{-1} (see precond.hip)
  bool pc_on = false;
  float* pc_dev = nullptr;         // [W | M_U | M_V | P_U | P_V | P_U^{-1} | P_V^{-1}], k x k each
  double* pc_gram = nullptr;       // Gram partials
  // certificate / rSVD workspace (allocated on first use)
  void* cert_ws = nullptr;
  size_t cert_ws_bytes = 0;
  void* cert_pin = nullptr;  // pinned host staging of the certificate's small copies
  size_t cert_pin_bytes = 0;
  // captured groups of solver slots (see run_lbfgs), keyed by what the launches read
  struct SlotGraph {
    const float* X;
    const float* pc;
    float kappa;
    int mem, slots;
    bool bf16;
    hipGraphExec_t exec;
  };
  std::vector<SlotGraph> graphs;
  hipStream_t gstream = nullptr;   // the graphs' stream (non-blocking, default priority)
  hipEvent_t gev = nullptr;        // orders gstream after the caller's stream
  bool use_graphs = false;        // off by default: measured no faster (see rpca_set_graphs)
  // optional per-launch timing
  struct Pending {
    int cls;
    hipEvent_t a, b;
  };
  bool prof_on = false;
  std::vector<hipEvent_t> ev_free;
  std::vector<Pending> pending;
  int64_t prof_launches[RPCA_K_NCLASS] = {0};
  double prof_ms[RPCA_K_NCLASS] = {0};
};
