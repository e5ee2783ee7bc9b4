// C ABI of librpca: context and workspace management, objective/gradient,
// the device-resident L-BFGS solve loop, certificate and rSVD entry points.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <chrono>
#include <new>
#include <vector>

#include "ctx.h"
#include "rpca_internal.h"
#include "smalllinalg.h"


namespace {

bool hip_ok(hipError_t e) { return e == hipSuccess; }

#define HIPCHK(expr)                          \
  do {                                        \
    if (!hip_ok(expr)) return RPCA_EHIP;      \
  } while (0)

template <typename T>
int dalloc(T** p, size_t count) {
  void* q = nullptr;
  if (count == 0) count = 1;
  if (hipMalloc(&q, count * sizeof(T)) != hipSuccess) return RPCA_ENOMEM;
  *p = static_cast<T*>(q);
  return RPCA_OK;
}

void dfree(void* p) {
  if (p) (void)hipFree(p);
}

SweepArgs make_sweep_args(const rpca_ctx* c, const float* X) {
  SweepArgs a;
  memset(&a, 0, sizeof(a));
  a.X = X;
  a.mask = c->mask;
  a.m = c->m;
  a.n = c->n;
  a.k = c->k;
  a.mw = c->mw;
  a.lam_s = (float)c->lam_s;
  a.lam_l = (float)c->lam_l;
  a.kappa = (float)(c->mu / (1.0 + c->mu));
  // vector (buffer) loads: 16-byte aligned columns, lane offsets within 32 bits
  a.xvec = (c->m % 4 == 0) && (((uintptr_t)X & 15u) == 0) && c->m < ((int64_t)1 << 26);
  a.gupart = c->gupart;
  a.gvpart = c->gvpart;
  a.spart = c->spart;
  a.strips_per_wave = c->spw;
  a.chunk_w = c->chunk_w;
  a.nchunks = c->nchunks;
  a.row_groups = c->row_groups;
  return a;
}

FinishArgs make_finish_args(const rpca_ctx* c) {
  FinishArgs f;
  memset(&f, 0, sizeof(f));
  f.m = c->m;
  f.n = c->n;
  f.k = c->k;
  f.lam_l = (float)c->lam_l;
  f.gupart = c->gupart;
  f.gvpart = c->gvpart;
  f.spart = c->spart;
  f.fpart = c->fpart;
  f.level2 = c->level2;
  f.segs = c->segs;
  f.rows_per_seg = c->rps;
  f.counter = c->counters + 0;
  f.nchunks = c->nchunks;
  f.row_groups = c->row_groups;
  f.sweep_wgs = c->sweep_wgs;
  return f;
}

void solver_views(const rpca_ctx* c, SweepArgs* sa, FinishArgs* fa, LbfgsArgs* la) {
  const int64_t mk = c->m * c->k;
  for (int i = 0; i < 2; ++i) {
    sa->U[i] = c->x[i];
    sa->V[i] = c->x[i] + mk;
    sa->Ut[i] = c->x[i];
    sa->Vt[i] = c->x[i] + mk;
    sa->gU[i] = c->g[i];
    fa->U[i] = c->x[i];
    fa->V[i] = c->x[i] + mk;
    fa->gU[i] = c->g[i];
    fa->gV[i] = c->g[i] + mk;
  }
  sa->dU = c->d;
  sa->dV = c->d + mk;
  sa->st = c->st;
  sa->pc = c->pc_on ? c->pc_dev : nullptr;
  fa->pc = sa->pc;
  fa->dU = c->d;
  fa->dV = c->d + mk;
  fa->st = c->st;
  memset(la, 0, sizeof(*la));
  la->N = c->N;
  la->st = c->st;
  for (int i = 0; i < 2; ++i) {
    la->x[i] = c->x[i];
    la->g[i] = c->g[i];
  }
  la->d = c->d;
  la->S = c->S;
  la->Y = c->Y;
  la->part = c->lpart;
}

hipEvent_t take_event(rpca_ctx* c) {
  if (!c->ev_free.empty()) {
    hipEvent_t e = c->ev_free.back();
    c->ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Collect the elapsed times of recorded event pairs (synchronises on them).
void prof_collect(rpca_ctx* c) {
  for (auto& p : c->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      c->prof_launches[p.cls] += 1;
      c->prof_ms[p.cls] += ms;
    }
    c->ev_free.push_back(p.a);
    c->ev_free.push_back(p.b);
  }
  c->pending.clear();
}

// Launch wrapper that brackets one launch with an event pair when profiling is on.
template <typename F>
hipError_t timed(rpca_ctx* c, int cls, hipStream_t s, F&& launch) {
  if (!c->prof_on) return launch();
  hipEvent_t a = take_event(c), b = take_event(c);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, s);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, s);
  if (e != hipSuccess) return e;
  c->pending.push_back({cls, a, b});
  if (c->pending.size() >= 4096) prof_collect(c);
  return hipSuccess;
}

hipError_t objgrad_launch(rpca_ctx* c, const SweepArgs& sa, const FinishArgs& fa, bool trial,
                          bool bf16, hipStream_t s) {
  hipError_t e = timed(c, trial ? RPCA_K_TRIAL : RPCA_K_SWEEP, s, [&] { return rpca::launch_sweep(sa, trial, bf16, s); });
  if (e != hipSuccess) return e;
  return timed(c, RPCA_K_FINISH, s, [&] { return rpca::launch_finish(fa, trial, s); });
}

}  // namespace

namespace {
// word mw - 1 of every column of a packed mask &= keep
__global__ void k_clear_tail_bits(uint32_t* mask, int64_t n, int mw, uint32_t keep) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j < n) mask[j * mw + mw - 1] &= keep;
}
}  // namespace

int rpca::create_ctx(int64_t m, int64_t n, int32_t k, double lam_s, double lam_l, const uint8_t* mask,
                     int target_waves, rpca_ctx** out, const uint32_t* mask_bits_dev) {
  if (!out) return RPCA_EINVAL;
  if (m < 1 || n < 1 || k < 1 || k > 32 || k > m || k > n) return RPCA_EINVAL;
  if (!(lam_s > 0) || !(lam_l > 0) || !isfinite(lam_s) || !isfinite(lam_l)) return RPCA_EINVAL;
  if (m > (int64_t)1 << 31 || n > (int64_t)1 << 24) return RPCA_EINVAL;
  rpca_ctx* c = new (std::nothrow) rpca_ctx();
  if (!c) return RPCA_ENOMEM;
  c->m = m;
  c->n = n;
  c->k = k;
  c->lam_s = lam_s;
  c->lam_l = lam_l;
  int rc = RPCA_OK;
#define TRY(expr)                   \
  do {                              \
    rc = (expr);                    \
    if (rc != RPCA_OK) {            \
      rpca_destroy(c);              \
      return rc;                    \
    }                               \
  } while (0)
  if (mask) {
    c->mw = (int)((m + 31) / 32);
    std::vector<uint32_t> bits((size_t)c->mw * (size_t)n, 0u);
    for (int64_t j = 0; j < n; ++j) {
      const uint8_t* col = mask + j * m;
      uint32_t* w = bits.data() + j * c->mw;
      for (int64_t i = 0; i < m; ++i)
        if (col[i]) w[i >> 5] |= 1u << (i & 31);
    }
    TRY(dalloc(&c->mask, bits.size()));
    if (hipMemcpy(c->mask, bits.data(), bits.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
      rpca_destroy(c);
      return RPCA_EHIP;
    }
  } else if (mask_bits_dev) {
    // already packed on the device: the context keeps its own copy
    c->mw = (int)((m + 31) / 32);
    const size_t words = (size_t)c->mw * (size_t)n;
    TRY(dalloc(&c->mask, words));
    if (hipMemcpy(c->mask, mask_bits_dev, words * 4, hipMemcpyDeviceToDevice) != hipSuccess) {
      rpca_destroy(c);
      return RPCA_EHIP;
    }
    if (m % 32) {  // clear the bits past row m - 1 (as the host packing leaves them)
      hipLaunchKernelGGL(k_clear_tail_bits, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, 0, c->mask, n, c->mw,
                         (uint32_t)((1u << (m % 32)) - 1u));
      if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        rpca_destroy(c);
        return RPCA_EHIP;
      }
    }
  }
  c->sweep_wgs =
      rpca::sweep_blocks_for(m, n, k, &c->row_groups, &c->spw, &c->chunk_w, &c->nchunks, target_waves);
  TRY(dalloc(&c->gvpart, (size_t)c->row_groups * n * k));
  if (c->nchunks > 1) TRY(dalloc(&c->gupart, (size_t)c->nchunks * m * k));
  TRY(dalloc(&c->spart, (size_t)c->sweep_wgs * RPCA_NSCAL));
  TRY(dalloc(&c->fpart, (size_t)rpca::finish_blocks(m, n, k, c->nchunks, nullptr) * 3 + 16));
  c->rps = 16;
  c->segs = (c->row_groups + c->rps - 1) / c->rps;
  TRY(dalloc(&c->level2, (size_t)c->segs * n * k));
  TRY(dalloc(&c->counters, 16));
  if (hipMemset(c->counters, 0, 16 * sizeof(unsigned)) != hipSuccess) {
    rpca_destroy(c);
    return RPCA_EHIP;
  }
  const int64_t raw = (m + n) * k;
  c->N = ((raw + 255) / 256) * 256;
  for (int i = 0; i < 2; ++i) {
    TRY(dalloc(&c->x[i], c->N));
    TRY(dalloc(&c->g[i], c->N));
  }
  TRY(dalloc(&c->d, c->N));
  TRY(dalloc(&c->S, (size_t)RPCA_MEMMAX * c->N));
  TRY(dalloc(&c->Y, (size_t)RPCA_MEMMAX * c->N));
  TRY(dalloc(&c->lpart, (size_t)RPCA_NDOT * (RPCA_LBFGS_MAX_BLOCKS + 1)));  // partials, then the combined dots
  TRY(dalloc(&c->st, 1));
  TRY(dalloc(&c->dscratch, 64));
  TRY(dalloc(&c->pc_dev, (size_t)7 * k * k));
  TRY(dalloc(&c->pc_gram, (size_t)(rpca::PC_GRAM_BLOCKS + 1) * k * k));  // partials + their sum
  void* hp = nullptr;
  if (hipHostMalloc(&hp, sizeof(SolverState), hipHostMallocDefault) != hipSuccess) {
    rpca_destroy(c);
    return RPCA_ENOMEM;
  }
  c->st_host = static_cast<SolverState*>(hp);
  // zero the padded tails once; kernels never write past (m+n)k
  for (int i = 0; i < 2; ++i) {
    if (hipMemset(c->x[i], 0, c->N * 4) != hipSuccess || hipMemset(c->g[i], 0, c->N * 4) != hipSuccess) {
      rpca_destroy(c);
      return RPCA_EHIP;
    }
  }
  if (hipMemset(c->d, 0, c->N * 4) != hipSuccess ||
      hipMemset(c->S, 0, (size_t)RPCA_MEMMAX * c->N * 4) != hipSuccess ||
      hipMemset(c->Y, 0, (size_t)RPCA_MEMMAX * c->N * 4) != hipSuccess) {
    rpca_destroy(c);
    return RPCA_EHIP;
  }
#undef TRY
  *out = c;
  return RPCA_OK;
}

extern "C" {

int rpca_profile_enable(rpca_ctx* c, int32_t on) {
  if (!c) return RPCA_EINVAL;
  c->prof_on = on != 0;
  return RPCA_OK;
}

int rpca_profile_read(rpca_ctx* c, rpca_profile* out, int32_t reset) {
  if (!c || !out) return RPCA_EINVAL;
  prof_collect(c);
  for (int i = 0; i < RPCA_K_NCLASS; ++i) {
    out->launches[i] = c->prof_launches[i];
    out->ms[i] = c->prof_ms[i];
    if (reset) {
      c->prof_launches[i] = 0;
      c->prof_ms[i] = 0.0;
    }
  }
  return RPCA_OK;
}

void rpca_default_opts(rpca_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->precision = RPCA_PREC_FP32;
  o->mem = 10;
  o->max_iter = 5000;
  o->precond = 1;
  o->precond_cycle = 50;
  o->init = RPCA_INIT_GIVEN;
  o->gtol = 1e-6;
  o->ftol = 1e-9;
  o->bf16_gtol = 1e-3;
  o->c1 = 1e-4;
  o->c2 = 0.9;
  o->certify = 1;
  o->cert_tol = 1e-3;
  o->rsvd_oversample = 10;
  o->rsvd_power = 2;
  o->seed = 12345;
  o->slots_per_sync = 16;
}

const char* rpca_status_string(int s) {
  switch (s) {
    case RPCA_OK: return "ok";
    case RPCA_ENOTCONV: return "iteration budget spent";
    case RPCA_ELINESEARCH: return "line search failed";
    case RPCA_ENOTCERT: return "converged but not certified";
    case RPCA_EINVAL: return "invalid argument";
    case RPCA_ENOMEM: return "out of memory";
    case RPCA_EHIP: return "HIP runtime error";
    case RPCA_ENONFINITE: return "non-finite objective or gradient";
    case RPCA_ETOOBIG: return "instance too large for the fixed scratch array";
    default: return "unknown status";
  }
}

void rpca_destroy(rpca_ctx* c) {
  if (!c) return;
  dfree(c->mask);
  dfree(c->gvpart);
  dfree(c->gupart);
  dfree(c->spart);
  dfree(c->fpart);
  dfree(c->level2);
  dfree(c->counters);
  dfree(c->x[0]);
  dfree(c->x[1]);
  dfree(c->g[0]);
  dfree(c->g[1]);
  dfree(c->d);
  dfree(c->S);
  dfree(c->Y);
  dfree(c->lpart);
  dfree(c->st);
  dfree(c->dscratch);
  dfree(c->pc_dev);
  dfree(c->pc_gram);
  dfree(c->cert_ws);
  for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
  if (c->gev) (void)hipEventDestroy(c->gev);
  if (c->gstream) (void)hipStreamDestroy(c->gstream);
  rpca::host_free(c->cert_pin);
  rpca::host_free(c->st_host);
  prof_collect(c);
  for (hipEvent_t e : c->ev_free) (void)hipEventDestroy(e);
  delete c;
}

int rpca_create(int64_t m, int64_t n, int32_t k, double lam_s, double lam_l, const uint8_t* mask,
                rpca_ctx** out) {
  return rpca::create_ctx(m, n, k, lam_s, lam_l, mask, 0, out);
}

int rpca_create_waves(int64_t m, int64_t n, int32_t k, double lam_s, double lam_l, const uint8_t* mask,
                      int32_t target_waves, rpca_ctx** out) {
  if (target_waves < 0 || target_waves > (1 << 20)) return RPCA_EINVAL;
  return rpca::create_ctx(m, n, k, lam_s, lam_l, mask, target_waves, out);
}

int rpca_create_device_mask(int64_t m, int64_t n, int32_t k, double lam_s, double lam_l,
                            const uint32_t* mask_bits, int32_t target_waves, rpca_ctx** out) {
  if (!mask_bits || target_waves < 0 || target_waves > (1 << 20)) return RPCA_EINVAL;
  return rpca::create_ctx(m, n, k, lam_s, lam_l, nullptr, target_waves, out, mask_bits);
}


int rpca_set_graphs(rpca_ctx* c, int32_t on) {
  if (!c) return RPCA_EINVAL;
  c->use_graphs = on != 0;
  return RPCA_OK;
}

int rpca_sweep_layout(const rpca_ctx* c, int32_t out[4]) {
  if (!c || !out) return RPCA_EINVAL;
  out[0] = c->row_groups;
  out[1] = c->spw;
  out[2] = c->chunk_w;
  out[3] = c->nchunks;
  return RPCA_OK;
}

int rpca_set_elastic(rpca_ctx* c, double mu) {
  if (!c || !(mu >= 0) || !isfinite(mu)) return RPCA_EINVAL;
  if (mu != c->mu) {  // a different objective: forget what the certificates cached
    c->mu = mu;
    c->best_F = INFINITY;
    c->phi0 = NAN;
    c->phi0_X = nullptr;
  }
  return RPCA_OK;
}

int rpca_objgrad(rpca_ctx* c, const float* X, const float* U, const float* V, double* f, float* gU,
                 float* gV, void* stream) {
  return rpca_objgrad_ex(c, X, U, V, f, gU, gV, RPCA_PREC_FP32, stream);
}

int rpca_objgrad_ex(rpca_ctx* c, const float* X, const float* U, const float* V, double* f,
                    float* gU, float* gV, int32_t precision, void* stream) {
  if (!c || !X || !U || !V || !f || !gU || !gV) return RPCA_EINVAL;
  if (precision != RPCA_PREC_FP32 && precision != RPCA_PREC_BF16) return RPCA_EINVAL;
  if (c->mu != 0 && precision != RPCA_PREC_FP32) return RPCA_EINVAL;  // elastic net: FP32 products only
  SweepArgs sa = make_sweep_args(c, X);
  FinishArgs fa = make_finish_args(c);
  sa.U[0] = sa.U[1] = U;
  sa.V[0] = sa.V[1] = V;
  sa.gU[0] = sa.gU[1] = gU;
  fa.U[0] = fa.U[1] = U;
  fa.V[0] = fa.V[1] = V;
  fa.gU[0] = fa.gU[1] = gU;
  fa.gV[0] = fa.gV[1] = gV;
  fa.f_out = f;
  HIPCHK(objgrad_launch(c, sa, fa, false, precision == RPCA_PREC_BF16, (hipStream_t)stream));
  return RPCA_OK;
}

}  // extern "C"

namespace rpca {

CtxView ctx_view(rpca_ctx* c) {
  CtxView v;
  v.m = c->m;
  v.n = c->n;
  v.k = c->k;
  v.lam_s = c->lam_s;
  v.lam_l = c->lam_l;
  v.kappa = c->mu / (1.0 + c->mu);
  v.mask = c->mask;
  v.mw = c->mw;
  v.best_F = &c->best_F;
  v.ctx = c;
  v.phi0 = &c->phi0;
  v.phi0_X = &c->phi0_X;
  return v;
}

bool prof_enabled(const rpca_ctx* c) { return c && c->prof_on; }

hipError_t prof_begin(rpca_ctx* c, hipStream_t s, void** token) {
  *token = nullptr;
  if (!c->prof_on) return hipSuccess;
  hipEvent_t a = take_event(c);
  if (!a) return hipErrorOutOfMemory;
  *token = (void*)a;
  return hipEventRecord(a, s);
}

hipError_t prof_end(rpca_ctx* c, int cls, hipStream_t s, void* token) {
  if (!token) return hipSuccess;
  hipEvent_t b = take_event(c);
  if (!b) return hipErrorOutOfMemory;
  const hipError_t e = hipEventRecord(b, s);
  if (e != hipSuccess) return e;
  c->pending.push_back({cls, (hipEvent_t)token, b});
  if (c->pending.size() >= 4096) prof_collect(c);
  return hipSuccess;
}

int ctx_objgrad_aux(rpca_ctx* c, const float* X, const float* U, const float* V, double* f_dev,
                    double* aux_dev, float* gU, float* gV, hipStream_t s) {
  SweepArgs sa = make_sweep_args(c, X);
  FinishArgs fa = make_finish_args(c);
  sa.U[0] = sa.U[1] = U;
  sa.V[0] = sa.V[1] = V;
  sa.gU[0] = sa.gU[1] = gU;
  fa.U[0] = fa.U[1] = U;
  fa.V[0] = fa.V[1] = V;
  fa.gU[0] = fa.gU[1] = gU;
  fa.gV[0] = fa.gV[1] = gV;
  fa.f_out = f_dev;
  fa.aux_out = aux_dev;
  HIPCHK(objgrad_launch(c, sa, fa, false, false, s));
  return RPCA_OK;
}

SolverState* ctx_state_host(rpca_ctx* c) { return c->st_host; }

void host_free(void* p) {
  // a failed free must not stay pending: the next hipGetLastError would report it
  if (p && hipHostFree(p) != hipSuccess) (void)hipGetLastError();
}

void* ctx_pinned(rpca_ctx* c, size_t bytes) {
  if (c->cert_pin && c->cert_pin_bytes >= bytes) return c->cert_pin;
  host_free(c->cert_pin);
  c->cert_pin = nullptr;
  c->cert_pin_bytes = 0;
  // one allocation covers the preconditioner's k x k and the certificate's
  // 2 n x 32 staging for n up to 512
  if (bytes < ((size_t)256 << 10)) bytes = (size_t)256 << 10;
  void* p = nullptr;
  if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
  c->cert_pin = p;
  c->cert_pin_bytes = bytes;
  return p;
}

void* ctx_workspace(rpca_ctx* c, size_t bytes, int* fresh) {
  *fresh = 0;
  if (c->cert_ws && c->cert_ws_bytes >= bytes) return c->cert_ws;
  dfree(c->cert_ws);
  c->cert_ws = nullptr;
  c->cert_ws_bytes = 0;
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  c->cert_ws = p;
  c->cert_ws_bytes = bytes;
  *fresh = 1;
  return p;
}

// One solver slot: direction, trial sweep, finishing reduction, pair update.  The
// direction pass's own finish (needed only when the state enters PH_DIRECTION: a
// restart, or a dropped memory) runs in the first slot of a group.
hipError_t launch_slot(const SweepArgs& sa, const FinishArgs& fa, const LbfgsArgs& lu, const LbfgsArgs& ld, int mem,
                       bool bf16, hipStream_t s, bool first) {
  hipError_t e = launch_lbfgs_direction(ld, mem, s, first);
  if (e != hipSuccess) return e;
  if ((e = launch_sweep(sa, true, bf16, s)) != hipSuccess) return e;
  if ((e = launch_finish(fa, true, s)) != hipSuccess) return e;
  return launch_lbfgs_update(lu, mem, s);
}

// The captured group of `slots` slots for these arguments (built on first use, on
// the context's own stream: a caller's stream may be the null stream, which cannot
// be captured).  The launches of a group read only buffers the context owns, X,
// the preconditioner and the mask, so the key is X, the preconditioner pointer,
// the regulariser's slope, the memory, the group size and the product precision.
hipError_t slot_graph(rpca_ctx* c, const SweepArgs& sa, const FinishArgs& fa, const LbfgsArgs& lu,
                      const LbfgsArgs& ld, int mem, bool bf16, int slots, hipGraphExec_t* out) {
  for (auto& g : c->graphs)
    if (g.X == sa.X && g.pc == sa.pc && g.kappa == sa.kappa && g.mem == mem && g.slots == slots &&
        g.bf16 == bf16) {
      *out = g.exec;
      return hipSuccess;
    }
  hipError_t e;
  if (!c->gstream) {
    if ((e = hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&c->gev, hipEventDisableTiming)) != hipSuccess) return e;
  }
  if ((e = hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
  hipError_t le = hipSuccess;
  for (int q = 0; q < slots && le == hipSuccess; ++q) le = launch_slot(sa, fa, lu, ld, mem, bf16, c->gstream, q == 0);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(c->gstream, &graph);
  if (le != hipSuccess || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return le != hipSuccess ? le : e;
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return e;
  if (c->graphs.size() >= 8) {  // keep the cache small: drop the oldest
    (void)hipGraphExecDestroy(c->graphs.front().exec);
    c->graphs.erase(c->graphs.begin());
  }
  c->graphs.push_back({sa.X, sa.pc, sa.kappa, mem, slots, bf16, exec});
  *out = exec;
  return hipSuccess;
}

// Run the device-resident L-BFGS from x[cur] (whose f and g are valid) until the
// device reports PH_DONE.  Returns an rpca_status.  Groups of slots are replayed
// from a captured graph on the context's stream (ordered after the caller's), or,
// with kernel timing on, launched one by one on the caller's stream.
int run_lbfgs(rpca_ctx* c, const float* X, const rpca_opts* o, bool bf16, hipStream_t s) {
  SweepArgs sa = make_sweep_args(c, X);
  FinishArgs fa = make_finish_args(c);
  LbfgsArgs la;
  solver_views(c, &sa, &fa, &la);
  LbfgsArgs lu = la, ld = la;
  lu.counter = c->counters + 1;
  ld.counter = c->counters + 2;
  const int slots = o->slots_per_sync > 0 ? o->slots_per_sync : 16;
  if (c->use_graphs && !c->prof_on) {
    hipGraphExec_t exec = nullptr;
    HIPCHK(slot_graph(c, sa, fa, lu, ld, o->mem, bf16, slots, &exec));
    for (int guard = 0; guard < 1000000; ++guard) {
      HIPCHK(hipEventRecord(c->gev, s));
      HIPCHK(hipStreamWaitEvent(c->gstream, c->gev, 0));
      HIPCHK(hipGraphLaunch(exec, c->gstream));
      HIPCHK(hipMemcpyAsync(c->st_host, c->st, sizeof(SolverState), hipMemcpyDeviceToHost, c->gstream));
      HIPCHK(hipStreamSynchronize(c->gstream));
      if (c->st_host->phase == PH_DONE) break;
    }
    return RPCA_OK;
  }
  for (int guard = 0; guard < 1000000; ++guard) {
    for (int q = 0; q < slots; ++q) {
      HIPCHK(timed(c, RPCA_K_DIRECTION, s, [&] { return launch_lbfgs_direction(ld, o->mem, s, q == 0); }));
      HIPCHK(objgrad_launch(c, sa, fa, true, bf16, s));
      HIPCHK(timed(c, RPCA_K_UPDATE, s, [&] { return launch_lbfgs_update(lu, o->mem, s); }));
    }
    HIPCHK(hipMemcpyAsync(c->st_host, c->st, sizeof(SolverState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (c->prof_on) prof_collect(c);
    if (c->st_host->phase == PH_DONE) break;
  }
  return RPCA_OK;
}

}  // namespace rpca

namespace rpca {

// Plain evaluation at the current iterate x[cur]: g[cur] and state.f (device).
int eval_current(rpca_ctx* c, const float* X, int cur, bool bf16, hipStream_t s) {
  const int64_t mk = c->m * c->k;
  SweepArgs sa = make_sweep_args(c, X);
  FinishArgs fa = make_finish_args(c);
  sa.U[0] = sa.U[1] = c->x[cur];
  sa.V[0] = sa.V[1] = c->x[cur] + mk;
  sa.gU[0] = sa.gU[1] = c->g[cur];
  fa.U[0] = fa.U[1] = c->x[cur];
  fa.V[0] = fa.V[1] = c->x[cur] + mk;
  fa.gU[0] = fa.gU[1] = c->g[cur];
  fa.gV[0] = fa.gV[1] = c->g[cur] + mk;
  fa.f_out = &c->st->f;
  sa.pc = c->pc_on ? c->pc_dev : nullptr;
  fa.pc = sa.pc;
  HIPCHK(objgrad_launch(c, sa, fa, false, bf16, s));
  return RPCA_OK;
}

// Restart the device loop from the current iterate after a phase change:
// keep the L-BFGS memory, clear the stop flag and the f history.
int resume_state(rpca_ctx* c, double gtol, double ftol, hipStream_t s) {
  return restart_state(c, gtol, ftol, -1, false, s);
}

// Restart with an iteration cap (max_iter < 0: keep it) and optionally an empty
// memory (after a change of variables the stored pairs no longer apply).
int restart_state(rpca_ctx* c, double gtol, double ftol, int max_iter, bool reset_memory, hipStream_t s) {
  SolverState* h = c->st_host;
  HIPCHK(hipMemcpyAsync(h, c->st, sizeof(SolverState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  h->phase = PH_DIRECTION;
  h->dir_pending = 0;
  h->stop = STOP_NONE;
  h->gtol = gtol;
  h->ftol = ftol;
  h->restarted = 0;
  if (max_iter >= 0) h->max_iter = max_iter;
  if (reset_memory) {
    // the first step after a restart is 1 (first_iter stays as it was: only the
    // very first iteration of a solve scales its step by 1/||g||_1)
    h->count = 0;
    h->newest = -1;
    h->spare = 0;
  }
  for (int i = 0; i < 8; ++i) h->fhist[i] = INFINITY;
  HIPCHK(hipMemcpyAsync(c->st, h, sizeof(SolverState), hipMemcpyHostToDevice, s));
  return RPCA_OK;
}

// One solver phase from the plain iterate in x[cur]: in preconditioned
// variables, cycles of o.precond_cycle iterations, each with a preconditioner
// refreshed from the current point and an empty memory; plain, one cycle that
// keeps the memory.  Ends with x[cur] plain again.
int run_cycles(rpca_ctx* c, const float* X, const rpca_opts& o, bool bf16, double gtol, double ftol,
               bool keep_memory, int budget, hipStream_t s) {
  int rc;
  const int it0 = c->st_host->iter;
  const int limit = (budget > 0 && o.max_iter - it0 > budget) ? it0 + budget : o.max_iter;
  for (;;) {
    const int cur = c->st_host->cur;
    int cap = limit;
    if (o.precond) {
      if ((rc = precond_refresh(c, cur, s))) return rc;
      const int it = c->st_host->iter;
      cap = (limit - it > o.precond_cycle) ? it + o.precond_cycle : limit;
    }
    if ((rc = restart_state(c, gtol, ftol, cap, o.precond || !keep_memory, s))) return rc;
    if ((rc = eval_current(c, X, cur, bf16, s))) return rc;
    if ((rc = run_lbfgs(c, X, &o, bf16, s))) return rc;
    const SolverState* h = c->st_host;
    if (!(o.precond && h->stop == STOP_MAXITER && h->iter < limit)) break;
  }
  return precond_to_plain(c, c->st_host->cur, s);
}

// Everything a batched launch needs to run this context's solver slots:
// arguments of the loop kernels and of a plain evaluation at x[cur], the
// sweep's work decomposition and the block counts of the other kernels.
void instance_args(rpca_ctx* c, const float* X, int cur, InstanceArgs* out) {
  const int64_t mk = c->m * c->k;
  out->sa_loop = make_sweep_args(c, X);
  out->fa_loop = make_finish_args(c);
  LbfgsArgs la;
  solver_views(c, &out->sa_loop, &out->fa_loop, &la);
  out->lu = la;
  out->ld = la;
  out->lu.counter = c->counters + 1;
  out->ld.counter = c->counters + 2;
  out->sa_eval = make_sweep_args(c, X);
  out->fa_eval = make_finish_args(c);
  SweepArgs& sa = out->sa_eval;
  FinishArgs& fa = out->fa_eval;
  sa.U[0] = sa.U[1] = c->x[cur];
  sa.V[0] = sa.V[1] = c->x[cur] + mk;
  sa.gU[0] = sa.gU[1] = c->g[cur];
  fa.U[0] = fa.U[1] = c->x[cur];
  fa.V[0] = fa.V[1] = c->x[cur] + mk;
  fa.gU[0] = fa.gU[1] = c->g[cur];
  fa.gV[0] = fa.gV[1] = c->g[cur] + mk;
  fa.f_out = &c->st->f;
  sa.pc = c->pc_on ? c->pc_dev : nullptr;
  fa.pc = sa.pc;
  int gvb = 0;
  out->fin2_blocks = finish_blocks(c->m, c->n, c->k, c->nchunks, &gvb);
  out->fa_loop.gv_blocks = gvb;
  out->fa_eval.gv_blocks = gvb;
  out->fin1_blocks = (int)((c->n * c->k + 255) / 256) * c->segs;  // reduce1: 256 elements per block
  out->lb_blocks = lbfgs_blocks(c->N);
  out->row_groups = c->row_groups;
  out->nchunks = c->nchunks;
  out->chunk_w = c->chunk_w;
  out->spw = c->spw;
  out->masked = c->mask != nullptr;
  out->state_dev = c->st;
  out->state_host = c->st_host;
}

}  // namespace rpca

namespace rpca {

bool valid_opts(const rpca_opts& o) {
  return !(o.mem < 1 || o.mem > RPCA_MEMMAX - 1 || o.max_iter < 0 || !(o.c1 > 0) || !(o.c2 > o.c1) ||
           !(o.c2 < 1) || !(o.gtol >= 0) || !(o.ftol >= 0) || o.precision < 0 || o.precision > 2 ||
           !(o.bf16_gtol >= 0) || !(o.cert_tol > 0) || o.precond < 0 || o.precond > 1 ||
           (o.precond && o.precond_cycle < 1));
}

int solve_phases(const rpca_opts& o, SolvePhase* ph) {
  int nph = 0;
  if (o.precision == RPCA_PREC_FP32) ph[nph++] = {false, o.gtol};
  else if (o.precision == RPCA_PREC_BF16) ph[nph++] = {true, o.gtol};
  else {
    // the BF16 phase's gradient test is relative to its first iteration's gradient
    ph[nph++] = {true, -o.bf16_gtol};
    ph[nph++] = {false, o.gtol};
  }
  return nph;
}

// Start of a solve: optional cold start, iterate x[0] = (U, V), fresh device state
// (phase DIRECTION; the caller evaluates f and g at x[0] next).
int solve_setup(rpca_ctx* c, const float* X, float* U, float* V, const rpca_opts& o, double gtol0,
                hipStream_t s) {
  const int64_t mk = c->m * c->k, nk = c->n * c->k;
  if (o.init == RPCA_INIT_RSVD) {
    const int rc = rpca_init_rsvd(c, X, nullptr, o.rsvd_oversample, o.rsvd_power, o.seed, U, V, s);
    if (rc != RPCA_OK) return rc;
  }
  HIPCHK(hipMemcpyAsync(c->x[0], U, mk * 4, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(c->x[0] + mk, V, nk * 4, hipMemcpyDeviceToDevice, s));
  c->phi0 = NAN;  // X may have changed since the last solve
  c->phi0_X = nullptr;
  SolverState* h = c->st_host;
  memset(h, 0, sizeof(*h));
  h->phase = PH_DIRECTION;
  h->cur = 0;
  h->max_iter = o.max_iter;
  h->mem = o.mem;
  h->newest = -1;
  // First trial step of the solve: in plain variables 1/||g||_1 (the scale of g
  // says nothing about the curvature); in preconditioned variables the Hessian is
  // close to the identity on the factors' span, so the unit step along -g is the
  // natural first trial (over sketch seeds 1-8 on the 76,800 x 200 video it took
  // the evaluations per solve from 78-194 to 64-90 for the same iterations).
  h->first_iter = o.precond ? 0 : 1;
  h->c1 = o.c1;
  h->c2 = o.c2;
  h->gtol = gtol0;
  h->ftol = o.ftol;
  h->eps_f = 1e-7;
  for (int i = 0; i < 8; ++i) h->fhist[i] = INFINITY;
  h->best_f = INFINITY;
  h->gamma = 1.0;
  h->evals = 1;
  HIPCHK(hipMemcpyAsync(c->st, h, sizeof(SolverState), hipMemcpyHostToDevice, s));
  return RPCA_OK;
}

// U, V <- the plain iterate x[cur] (host state current).
int copy_out(rpca_ctx* c, float* U, float* V, hipStream_t s) {
  const int cur = c->st_host->cur;
  HIPCHK(hipMemcpyAsync(U, c->x[cur], c->m * c->k * 4, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(V, c->x[cur] + c->m * c->k, c->n * c->k * 4, hipMemcpyDeviceToDevice, s));
  return RPCA_OK;
}

// Tolerances of a certification round: near the optimum f changes by less than
// its FP32 evaluation noise per iteration while the gradient still carries the
// structure the certificate measures, so a round runs with the f test off and,
// in preconditioned variables, the gradient test off too for half a cycle
// (plain variables: a tenfold tighter gradient test, no budget).
int round_tolerances(const rpca_opts& o, double* gtol, double* ftol) {
  *gtol = o.precond ? 0.0 : *gtol * 0.1;
  *ftol = 0.0;
  return o.precond ? (o.precond_cycle > 1 ? o.precond_cycle / 2 : 1) : 0;
}

// A round that ran out of its budget (not of max_iter) ends like a gradient stop.
void end_round(rpca_ctx* c, const rpca_opts& o) {
  if (c->st_host->stop == STOP_MAXITER && c->st_host->iter < o.max_iter) c->st_host->stop = STOP_GTOL;
}

// Status and info of a finished solve (host state current).
int finish_status(rpca_ctx* c, const rpca_opts& o, int certified, double rel_gap, int rounds, int iters_bf16,
                  std::chrono::steady_clock::time_point t0, rpca_info* info) {
  const SolverState fin = *c->st_host;
  int status;
  switch (fin.stop) {
    case STOP_MAXITER: status = RPCA_ENOTCONV; break;
    case STOP_LINESEARCH: status = RPCA_ELINESEARCH; break;
    case STOP_NONFINITE: status = RPCA_ENONFINITE; break;
    default: status = RPCA_OK;
  }
  if (o.certify && status != RPCA_ENONFINITE) {
    // the certificate decides: a search that stalled at the rounding level of
    // the objective is a normal end when the point is certified
    if (certified) status = RPCA_OK;
    else if (status == RPCA_OK) status = RPCA_ENOTCERT;
  }
  if (info) {
    info->status = status;
    info->iters = fin.iter;
    info->evals = fin.evals;
    info->iters_bf16 = iters_bf16;
    info->f = fin.f;
    info->gnorm_inf = fin.gnorm_inf;
    info->rel_gap = rel_gap;
    info->certified = certified;
    info->cert_rounds = rounds;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return status;
}

// End of a solve: copy the iterate out, certify (continuing with the stopping
// tests off, or tightened, while the gap is above the target, at most
// CERT_ROUNDS certificates), and fill `info`.  Returns the rpca_status of the solve.
int solve_finish(rpca_ctx* c, const float* X, float* U, float* V, const rpca_opts& o, bool final_bf16,
                 double gtol, int iters_bf16, std::chrono::steady_clock::time_point t0, rpca_info* info,
                 hipStream_t s) {
  double rel_gap = NAN;
  int certified = 0, rounds = 0, rc;
  double ftol = o.ftol;
  HIPCHK(hipMemcpyAsync(c->st_host, c->st, sizeof(SolverState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (;;) {
    if ((rc = copy_out(c, U, V, s))) return rc;
    const int stop = c->st_host->stop;
    if (!o.certify || stop == STOP_NONFINITE) break;
    rpca_cert cert;
    const int crc = certificate_impl(c, X, U, V, &cert, o.cert_tol, s);
    if (crc < 0) return crc;
    ++rounds;
    rel_gap = cert.rel_gap;
    certified = rel_gap <= o.cert_tol;
    if (certified || stop == STOP_MAXITER || rounds >= CERT_ROUNDS) break;
    // not certified yet: continue from here
    const int budget = round_tolerances(o, &gtol, &ftol);
    if ((rc = run_cycles(c, X, o, final_bf16, gtol, ftol, true, budget, s))) return rc;
    end_round(c, o);
  }
  HIPCHK(hipStreamSynchronize(s));
  return finish_status(c, o, certified, rel_gap, rounds, iters_bf16, t0, info);
}

}  // namespace rpca

extern "C" int rpca_solve(rpca_ctx* c, const float* X, float* U, float* V, const rpca_opts* opts,
                          rpca_info* info, void* stream) {
  if (!c || !X || !U || !V) return RPCA_EINVAL;
  rpca_opts o;
  if (opts) o = *opts;
  else rpca_default_opts(&o);
  if (!rpca::valid_opts(o)) return RPCA_EINVAL;
  if (c->mu != 0 && o.precision != RPCA_PREC_FP32) return RPCA_EINVAL;  // elastic net: FP32 products only
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = (hipStream_t)stream;
  rpca::SolvePhase phases[2];
  const int nph = rpca::solve_phases(o, phases);
  int rc = rpca::solve_setup(c, X, U, V, o, phases[0].gtol, s);
  if (rc) return rc;
  if ((rc = rpca::run_cycles(c, X, o, phases[0].bf16, phases[0].gtol, o.ftol, true, 0, s))) return rc;
  int iters_bf16 = phases[0].bf16 ? c->st_host->iter : 0;
  bool final_bf16 = phases[0].bf16;
  for (int ph = 1; ph < nph; ++ph) {
    if (c->st_host->stop == STOP_NONFINITE || c->st_host->stop == STOP_MAXITER) break;
    if ((rc = rpca::run_cycles(c, X, o, phases[ph].bf16, phases[ph].gtol, o.ftol, true, 0, s))) return rc;
    final_bf16 = phases[ph].bf16;
  }
  return rpca::solve_finish(c, X, U, V, o, final_bf16, phases[nph - 1].gtol, iters_bf16, t0, info, s);
}

// Rank grown on demand (Sec. 4.1): one context per rank.  Below k_max a rank is
// solved without certification rounds, then one certificate decides: certified
// -> done; growth column with sigma > 1 -> widen the factors in place and go on
// at k + 1; otherwise the full certified solve continues at this rank.
extern "C" int rpca_solve_grow(int64_t m, int64_t n, int32_t k0, int32_t k_max, double lam_s, double lam_l,
                               const uint8_t* mask, const float* X, float* U, float* V, int32_t* k_out,
                               const rpca_opts* opts, rpca_info* info, void* stream) {
  if (!X || !U || !V || !k_out) return RPCA_EINVAL;
  if (k0 < 1 || k_max < k0 || k_max > 32 || k_max > m || k_max > n) return RPCA_EINVAL;
  rpca_opts o;
  if (opts) o = *opts;
  else rpca_default_opts(&o);
  o.certify = 1;
  if (!rpca::valid_opts(o)) return RPCA_EINVAL;
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = (hipStream_t)stream;
  // staging for the widened factors and the column pair
  float* stage = nullptr;
  const size_t wide = (size_t)(m + n) * (size_t)k_max, cols = (size_t)(m + n);
  if (k_max > k0 && hipMalloc(&stage, (wide + cols) * sizeof(float)) != hipSuccess) return RPCA_ENOMEM;
  int k = k0, rc = RPCA_OK;
  int32_t iters = 0, evals = 0, iters_bf16 = 0, rounds = 0;
  rpca_info last{};
  auto tally = [&] {
    iters += last.iters;
    evals += last.evals;
    iters_bf16 += last.iters_bf16;
    rounds += last.cert_rounds;
  };
  for (;;) {
    rpca_ctx* c = nullptr;
    if ((rc = rpca_create(m, n, k, lam_s, lam_l, mask, &c))) break;
    if (k == k_max) {
      rc = rpca_solve(c, X, U, V, &o, &last, stream);
      if (rc >= 0) tally();
      rpca_destroy(c);
      break;
    }
    rpca_opts quick = o;
    quick.certify = 0;
    rc = rpca_solve(c, X, U, V, &quick, &last, stream);
    if (rc >= 0) tally();
    if (rc < 0 || rc == RPCA_ENOTCONV) {
      rpca_destroy(c);
      break;
    }
    rpca_cert cert;
    double sigma = 0.0, t = 0.0;
    float* Ug = stage;
    float* Vg = stage + (size_t)m * (k + 1);
    float* ucol = stage + wide;
    float* vcol = ucol + m;
    rc = rpca::growth_direction_impl(c, X, U, V, ucol, vcol, &sigma, &t, s, &cert);
    if (rc) {
      rpca_destroy(c);
      break;
    }
    ++rounds;
    if (cert.rel_gap <= o.cert_tol) {  // certified at this rank
      rpca_destroy(c);
      last.status = rc = RPCA_OK;
      last.certified = 1;
      last.rel_gap = cert.rel_gap;
      break;
    }
    if (!(sigma > 1.0)) {  // no descent column: the gap is not from the rank bound
      rpca_opts more = o;
      more.init = RPCA_INIT_GIVEN;
      rc = rpca_solve(c, X, U, V, &more, &last, stream);
      if (rc >= 0) tally();
      rpca_destroy(c);
      break;
    }
    rpca_destroy(c);
    const size_t f4 = sizeof(float), wk = (size_t)k * f4, wk1 = (size_t)(k + 1) * f4;
    if (hipMemcpy2DAsync(Ug, wk1, U, wk, wk, (size_t)m, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpy2DAsync(Ug + k, wk1, ucol, f4, f4, (size_t)m, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpy2DAsync(Vg, wk1, V, wk, wk, (size_t)n, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpy2DAsync(Vg + k, wk1, vcol, f4, f4, (size_t)n, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(U, Ug, (size_t)m * wk1, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(V, Vg, (size_t)n * wk1, hipMemcpyDeviceToDevice, s) != hipSuccess) {
      rc = RPCA_EHIP;
      break;
    }
    ++k;
    o.init = RPCA_INIT_GIVEN;
  }
  if (stage) {
    if (hipStreamSynchronize(s) != hipSuccess && rc >= 0) rc = RPCA_EHIP;
    (void)hipFree(stage);
  }
  *k_out = k;
  if (info && rc >= 0) {
    *info = last;
    info->iters = iters;
    info->evals = evals;
    info->iters_bf16 = iters_bf16;
    info->cert_rounds = rounds;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return rc;
}
