// Device-resident L-BFGS (memory <= 15) for the flat vector x = [vec(U); vec(V)].
//
// The paper's solver is L-BFGS with 10 pairs in memory (Sec. 5.1, Table 1).  On
// the GPU the two-loop recursion would need 2*mem dependent grid-wide
// reductions per iteration, so the direction uses the equivalent compact form
// of the inverse Hessian (Byrd, Nocedal & Schnabel 1994, Thm. 2.2) with H0 = gamma I:
//
//   H g = gamma g + S p + gamma Y q,   q = -R^{-1} a,
//   p   = R^{-T} ( (Dg + gamma Y^T Y) R^{-1} a - gamma b ),   a = S^T g, b = Y^T g,
//
// where R is the upper triangle of S^T Y and Dg its diagonal.  One pass over
// the history ("update") computes every inner product the small matrices need
// in FP64; its finishing kernel combines the block partials (one block per
// value, the last to arrive runs the mem x mem algebra in one wave) and, since
// g^T d = -(gamma g^T g + p^T a - gamma u^T b) follows from the same inner
// products, also sets up the line search.  A second pass ("direction") then
// only forms d = -H g.  Only after a restart (no pairs, d = -g) does the
// direction pass end in a one-block kernel that sums g^T d itself.  The whole
// iteration stays on the device.
#include "rpca_internal.h"
#include "linesearch.h"

#include <math.h>

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int THREADS = 256;
constexpr int WAVES = THREADS / 64;
constexpr int LBFGS_MAX_BLOCKS = RPCA_LBFGS_MAX_BLOCKS;  // blocks of a streaming pass; the combined dots follow their partials

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ double dot4(f4 a, f4 b) {
  return (double)a[0] * b[0] + (double)a[1] * b[1] + (double)a[2] * b[2] + (double)a[3] * b[3];
}

// Reduce NV per-thread values over the block (value IMAX, if in range, is a
// max, the others sums) and write them value-major to part[v*nb + block].
template <int NV, int IMAX>
__device__ void block_partials(const double (&acc)[NV], double* part, int bx, int nb) {
  __shared__ double sh[WAVES][NV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double r = (v == IMAX) ? wave_max(acc[v]) : wave_sum(acc[v]);
    if (lane == 0) sh[wave][v] = r;
  }
  __syncthreads();
  for (int v = threadIdx.x; v < NV; v += THREADS) {
    double r = sh[0][v];
    for (int w = 1; w < WAVES; ++w) r = (v == IMAX) ? fmax(r, sh[w][v]) : r + sh[w][v];
    part[(int64_t)v * nb + bx] = r;
  }
}

// One block: combine the nb block partials of NV values in a fixed order into out[]
// (LDS).  Thread t sums partials t, t + THREADS, ... of every value (all loads
// independent, so they are in flight together), then wave reductions and the
// waves in a fixed order.
template <int NV, int IMAX>
__device__ void combine_partials(const double* part, int nb, double* out) {
  __shared__ double sh[WAVES][NV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double r[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) r[v] = 0.0;  // the max value (|g|) is >= 0: 0 is its identity too
  for (int b = threadIdx.x; b < nb; b += THREADS) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double x = part[(int64_t)v * nb + b];
      r[v] = (v == IMAX) ? fmax(r[v], x) : r[v] + x;
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double q = (v == IMAX) ? wave_max(r[v]) : wave_sum(r[v]);
    if (lane == 0) sh[wave][v] = q;
  }
  __syncthreads();
  for (int v = threadIdx.x; v < NV; v += THREADS) {
    double q = sh[0][v];
    for (int w = 1; w < WAVES; ++w) q = (v == IMAX) ? fmax(q, sh[w][v]) : q + sh[w][v];
    out[v] = q;
  }
  __syncthreads();
}

// Layout of the dot vector of the update pass: 4 per stored pair (s_i.g, y_i.g,
// s_i.y, y_i.y), then the new pair's scalars.
template <int MEM>
struct DotIdx {
  static constexpr int SY = 4 * MEM + 0;  // s_new . y_new
  static constexpr int YY = SY + 1;       // y_new . y_new
  static constexpr int SG = SY + 2;       // s_new . g_new
  static constexpr int YG = SY + 3;       // y_new . g_new
  static constexpr int GG = SY + 4;       // g_new . g_new
  static constexpr int GINF = SY + 5;     // max |g_new|
  static constexpr int G1 = SY + 6;       // sum |g_new|
  static constexpr int SS = SY + 7;       // s_new . s_new
  static constexpr int NV = SY + 8;
};

// Value of lane `src` (a constant) to every lane, through the scalar unit.
__device__ __forceinline__ double bcast(double v, int src) {
  const unsigned long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffull), src);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), src);
  return __longlong_as_double(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ int bcast_int(int v, int src) { return __builtin_amdgcn_readlane(v, src); }

// The small algebra of an update, by one wave on the LDS copy of the state; lane
// i owns stored pair i (in age order).  Pair bookkeeping: norms, the keep test,
// the new pair's inner products into the slot matrices, the ring order, gamma.
// Then the compact-form coefficients from R[i][j] = s_i^T y_j and Q[i][j] =
// y_i^T y_j (ordered), with a = S^T g, b = Y^T g:
//   u = R^{-1} a                               (back substitution)
//   w_i = R_ii u_i - gamma b_i + gamma (Q u)_i
//   p = R^{-T} w                               (forward substitution)
//   coef_s = p, coef_y = -gamma u              (scattered to the slots)
// Both substitutions run column by column: the solved entry is broadcast from
// its lane through the scalar unit and every lane updates its own entry, so a
// step costs one broadcast and one FMA.
// Returns g^T d for the next direction d = -(gamma g + S coef_s + Y coef_y):
//   g^T d = -(gamma g^T g + sum_i coef_s_i a_i + coef_y_i b_i)   (every lane).
template <int MEM>
__device__ double update_wave(SolverState* st, const double* D) {
  using I = DotIdx<MEM>;
  const int lane = threadIdx.x & 63;
  const int cnt = st->count;
  const double sy = D[I::SY], yy = D[I::YY], ss = D[I::SS];
  if (lane == 0) {
    st->iter += 1;
    st->gnorm_inf = D[I::GINF];
    st->gnorm1 = D[I::G1];
    st->gg = D[I::GG];
  }
  double av = (lane < cnt) ? D[4 * lane + 0] : 0.0;
  double bv = (lane < cnt) ? D[4 * lane + 1] : 0.0;
  int ord = (lane < cnt) ? st->order[lane] : 0;
  int h = cnt;
  const bool keep = sy > 1e-10 * sqrt(ss * yy) && isfinite(sy) && isfinite(yy);
  if (keep) {
    const int sn = st->spare;
    if (lane < cnt) {
      st->SY[ord][sn] = D[4 * lane + 2];
      st->YY[ord][sn] = D[4 * lane + 3];
      st->YY[sn][ord] = D[4 * lane + 3];
    }
    if (lane == 0) {
      st->SY[sn][sn] = sy;
      st->YY[sn][sn] = yy;
    }
    int next_spare;
    if (h < st->mem) {
      if (lane == h) {
        ord = sn;
        av = D[I::SG];
        bv = D[I::YG];
      }
      h += 1;
      next_spare = h;
    } else {
      // full: the oldest pair leaves, the others move down one place
      next_spare = bcast_int(ord, 0);
      const int ord_up = __shfl_down(ord, 1, 64);
      const double av_up = __shfl_down(av, 1, 64), bv_up = __shfl_down(bv, 1, 64);
      if (lane < h - 1) {
        ord = ord_up;
        av = av_up;
        bv = bv_up;
      } else if (lane == h - 1) {
        ord = sn;
        av = D[I::SG];
        bv = D[I::YG];
      }
    }
    if (lane < h) st->order[lane] = ord;
    if (lane == 0) {
      st->count = h;
      st->spare = next_spare;
      st->newest = sn;
      st->gamma = sy / yy;
    }
  }
  if (h == 0) return -D[I::GG];  // steepest descent (gamma 1 without pairs)
  const double gamma = keep ? sy / yy : st->gamma;
  // this lane's row and column of R and row of Q (ordered pairs)
  double rowR[MEM], colR[MEM], rowQ[MEM];
  double diag = 1.0;
#pragma unroll
  for (int i = 0; i < MEM; ++i) {
    const int oi = bcast_int(ord, i);
    const bool in = lane < h && i < h;
    rowR[i] = in ? st->SY[ord][oi] : 0.0;
    colR[i] = in ? st->SY[oi][ord] : 0.0;
    rowQ[i] = in ? st->YY[ord][oi] : 0.0;
    if (i == lane) diag = in ? rowR[i] : 1.0;
  }
  const double dinv = 1.0 / diag;
  double u = (lane < h) ? av : 0.0;
#pragma unroll
  for (int i = MEM - 1; i >= 0; --i) {
    if (i < h) {
      const double ui = bcast(u * dinv, i);
      if (lane == i) u = ui;
      else if (lane < i) u = fma(-rowR[i], ui, u);
    }
  }
  double qu = 0.0;
#pragma unroll
  for (int j = 0; j < MEM; ++j)
    if (j < h) qu = fma(rowQ[j], bcast(u, j), qu);
  double p = (lane < h) ? diag * u - gamma * bv + gamma * qu : 0.0;
#pragma unroll
  for (int i = 0; i < MEM; ++i) {
    if (i < h) {
      const double pi = bcast(p * dinv, i);
      if (lane == i) p = pi;
      else if (lane > i && lane < h) p = fma(-colR[i], pi, p);
    }
  }
  if (lane < RPCA_MEMMAX) {
    st->coef_s[lane] = 0.0;
    st->coef_y[lane] = 0.0;
  }
  if (lane < h) {
    st->coef_s[ord] = p;
    st->coef_y[ord] = -gamma * u;
  }
  const double gdl = (lane < h) ? p * av - gamma * u * bv : 0.0;
  return -(gamma * D[I::GG] + wave_sum(gdl));
}

// Stopping tests after an update (one thread).
template <int MEM>
__device__ void update_stops(SolverState* st, const double* D, double gd) {
  using I = DotIdx<MEM>;
  const double f = st->f;
  for (int i = 0; i < 7; ++i) st->fhist[i] = st->fhist[i + 1];
  st->fhist[7] = f;
  if (f < st->best_f) st->best_f = f;
  // gradient threshold: relative to max(1, |f|), or (gtol < 0) to the gradient at
  // the phase's first iteration, a test whose scale does not grow with m n
  double gthr;
  if (st->gtol < 0.0) {
    if (!(st->gref > 0.0)) st->gref = D[I::GINF];
    gthr = -st->gtol * st->gref;
  } else {
    gthr = st->gtol * fmax(1.0, fabs(f));
  }
  int stop = STOP_NONE;
  if (!isfinite(f) || !isfinite(D[I::GG])) stop = STOP_NONFINITE;
  else if (D[I::GINF] <= gthr) stop = STOP_GTOL;
  else if (st->ftol > 0.0 && st->iter >= 5 && (st->fhist[2] - f) <= st->ftol * fmax(1.0, fabs(f)))
    stop = STOP_FTOL;
  else if (st->iter >= st->max_iter) stop = STOP_MAXITER;
  st->stop = stop;
  if (stop == STOP_NONE) {
    // the next direction's slope is known from the inner products: the line search
    // starts now and the direction pass of the next slot only forms d
    rpca_ls::setup_trial(st, gd, D[I::G1], 1);
  } else {
    st->phase = PH_DONE;
  }
}

template <int MEM>
__device__ __forceinline__ void lbfgs_update_body(const LbfgsArgs& a, int bx, int nb) {
  // The block's four waves walk the same elements (lane l: bx*64 + l, then every
  // nb*64-th); wave w owns the stored pairs w, w + 4, w + 8, ... and wave 0 also
  // the new pair (its store and scalars).  Every value is summed by one wave, so
  // the block partial is that wave's sum and few accumulators stay live.
  using I = DotIdx<MEM>;
  constexpr int PW = (MEM + WAVES - 1) / WAVES;
  SolverState* st = a.st;
  if (st->phase != PH_UPDATE) return;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int cur = st->cur;
  const int64_t n4 = a.N >> 2;
  const f4* gn = reinterpret_cast<const f4*>(a.g[cur]);
  const f4* go = reinterpret_cast<const f4*>(a.g[1 - cur]);
  const f4* dd = reinterpret_cast<const f4*>(a.d);
  const float alpha = (float)st->alpha;
  const int cnt = st->count;
  const f4* Sp[PW];
  const f4* Yp[PW];
#pragma unroll
  for (int j = 0; j < PW; ++j) {
    const int i = w + WAVES * j;
    const int slot = (i < cnt) ? st->order[i] : 0;  // unused pairs read slot 0 (ignored)
    Sp[j] = reinterpret_cast<const f4*>(a.S + (int64_t)slot * a.N);
    Yp[j] = reinterpret_cast<const f4*>(a.Y + (int64_t)slot * a.N);
  }
  f4* Ssp = reinterpret_cast<f4*>(a.S + (int64_t)st->spare * a.N);
  f4* Ysp = reinterpret_cast<f4*>(a.Y + (int64_t)st->spare * a.N);
  double acc[4 * PW], nw[8];
#pragma unroll
  for (int v = 0; v < 4 * PW; ++v) acc[v] = 0.0;
#pragma unroll
  for (int v = 0; v < 8; ++v) nw[v] = 0.0;
  const int64_t stride = (int64_t)nb * 64;
  for (int64_t e = (int64_t)bx * 64 + lane; e < n4; e += stride) {
    // the pair loads are issued before the new pair is stored (the spare slot may
    // alias a stored one as far as the compiler knows), so they are in flight together
    f4 Sv[PW], Yv[PW];
#pragma unroll
    for (int j = 0; j < PW; ++j) {
      if (w + WAVES * j < MEM) {
        Sv[j] = Sp[j][e];
        Yv[j] = Yp[j][e];
      }
    }
    const f4 g1 = gn[e];
    const f4 y = g1 - go[e];
    if (w == 0) {
      const f4 sv = alpha * dd[e];
      Ssp[e] = sv;
      Ysp[e] = y;
      nw[0] += dot4(sv, y);
      nw[1] += dot4(y, y);
      nw[2] += dot4(sv, g1);
      nw[3] += dot4(y, g1);
      nw[4] += dot4(g1, g1);
      const double m4 = fmax(fmax(fabs((double)g1[0]), fabs((double)g1[1])),
                             fmax(fabs((double)g1[2]), fabs((double)g1[3])));
      nw[5] = fmax(nw[5], m4);
      nw[6] += fabs((double)g1[0]) + fabs((double)g1[1]) + fabs((double)g1[2]) + fabs((double)g1[3]);
      nw[7] += dot4(sv, sv);
    }
#pragma unroll
    for (int j = 0; j < PW; ++j) {
      if (w + WAVES * j < MEM) {
        acc[4 * j + 0] += dot4(Sv[j], g1);
        acc[4 * j + 1] += dot4(Yv[j], g1);
        acc[4 * j + 2] += dot4(Sv[j], y);
        acc[4 * j + 3] += dot4(Yv[j], y);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < PW; ++j) {
    const int i = w + WAVES * j;
    if (i < MEM) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double r = wave_sum(acc[4 * j + q]);
        if (lane == 0) a.part[(int64_t)(4 * i + q) * nb + bx] = r;
      }
    }
  }
  if (w == 0) {
    static_assert(I::SY + 5 == I::GINF && I::SY + 7 == I::SS, "new-pair value order");
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const double r = (v == 5) ? wave_max(nw[v]) : wave_sum(nw[v]);
      if (lane == 0) a.part[(int64_t)(I::SY + v) * nb + bx] = r;
    }
  }
}

template <int MEM>
__global__ __launch_bounds__(THREADS) void k_lbfgs_update(LbfgsArgs a) {
  lbfgs_update_body<MEM>(a, blockIdx.x, gridDim.x);
}

// One block: combine the update partials and run the small (mem x mem) algebra on
// an LDS copy of the state (global latency per access would dominate otherwise).
template <int MEM>
__device__ __forceinline__ void lbfgs_update_final_body(const LbfgsArgs& a, int nb) {
  using I = DotIdx<MEM>;
  constexpr int NV = I::NV;
  SolverState* st = a.st;
  if (st->phase != PH_UPDATE) return;
  __shared__ double D[NV];
  combine_partials<NV, I::GINF>(a.part, nb, D);
  __shared__ SolverState sst;
  copy_state_block(&sst, st);
  __syncthreads();
  if (threadIdx.x < 64) {
    const double gd = update_wave<MEM>(&sst, D);
    if (threadIdx.x == 0) update_stops<MEM>(&sst, D, gd);
  }
  __syncthreads();
  copy_state_block(st, &sst);
}

// The same with the combine spread over one block per value: block v sums value v
// of the nb partials in a fixed order into dots[v]; the last block to arrive
// (thread-0 fence + counter over NV blocks) runs the algebra.
template <int MEM>
__global__ __launch_bounds__(THREADS) void k_lbfgs_update_final_mb(LbfgsArgs a, int nb) {
  using I = DotIdx<MEM>;
  constexpr int NV = I::NV;
  SolverState* st = a.st;
  if (st->phase != PH_UPDATE) return;
  const int v = blockIdx.x;
  const bool is_max = v == I::GINF;
  double* dots = a.part + (int64_t)RPCA_NDOT * LBFGS_MAX_BLOCKS;
  __shared__ double sh[WAVES];
  __shared__ int s_last;
  double r = 0.0;
  for (int b = threadIdx.x; b < nb; b += THREADS) {
    const double x = a.part[(int64_t)v * nb + b];
    r = is_max ? fmax(r, x) : r + x;
  }
  r = is_max ? wave_max(r) : wave_sum(r);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = r;
  __syncthreads();
  if (threadIdx.x == 0) {
    double q = sh[0];
    for (int w = 1; w < WAVES; ++w) q = is_max ? fmax(q, sh[w]) : q + sh[w];
    dots[v] = q;
    __threadfence();
    const unsigned prev = atomicAdd(a.counter, 1u);
    s_last = prev == (unsigned)NV - 1u;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  __shared__ double D[NV];
  for (int t = threadIdx.x; t < NV; t += THREADS) D[t] = dots[t];
  __shared__ SolverState sst;
  copy_state_block(&sst, st);
  __syncthreads();
  if (threadIdx.x < 64) {
    const double gd = update_wave<MEM>(&sst, D);
    if (threadIdx.x == 0) {
      update_stops<MEM>(&sst, D, gd);
      *a.counter = 0u;
    }
  }
  __syncthreads();
  copy_state_block(st, &sst);
}


template <int MEM>
__device__ __forceinline__ void lbfgs_direction_body(const LbfgsArgs& a, int bx, int nb) {
  SolverState* st = a.st;
  if (st->phase != PH_DIRECTION && !(st->phase == PH_TRIAL && st->dir_pending)) return;
  const int cur = st->cur;
  const int64_t n4 = a.N >> 2;
  const f4* g = reinterpret_cast<const f4*>(a.g[cur]);
  f4* d = reinterpret_cast<f4*>(a.d);
  const int cnt = st->count;
  const float gamma = cnt > 0 ? (float)st->gamma : 1.0f;
  int slot[MEM];
  float cs[MEM], cy[MEM];
#pragma unroll
  for (int i = 0; i < MEM; ++i) {
    slot[i] = (i < cnt) ? st->order[i] : 0;
    cs[i] = (i < cnt) ? (float)st->coef_s[slot[i]] : 0.f;
    cy[i] = (i < cnt) ? (float)st->coef_y[slot[i]] : 0.f;
  }
  double acc[3] = {0.0, 0.0, 0.0};
  const int64_t stride = (int64_t)nb * THREADS;
  for (int64_t e = (int64_t)bx * THREADS + threadIdx.x; e < n4; e += stride) {
    // unused slots carry zero coefficients; no branch around the loads, all of
    // which are issued before the first is used
    f4 Sv[MEM], Yv[MEM];
#pragma unroll
    for (int i = 0; i < MEM; ++i) {
      Sv[i] = *(reinterpret_cast<const f4*>(a.S + (int64_t)slot[i] * a.N) + e);
      Yv[i] = *(reinterpret_cast<const f4*>(a.Y + (int64_t)slot[i] * a.N) + e);
    }
    const f4 gv = g[e];
    __builtin_amdgcn_sched_barrier(0);  // keep every load ahead of the arithmetic
    f4 h = gamma * gv;
#pragma unroll
    for (int i = 0; i < MEM; ++i) h += cs[i] * Sv[i] + cy[i] * Yv[i];
    const f4 dv = -h;
    d[e] = dv;
    acc[0] += dot4(gv, dv);
    acc[1] += dot4(dv, dv);
    acc[2] += fabs((double)gv[0]) + fabs((double)gv[1]) + fabs((double)gv[2]) + fabs((double)gv[3]);
  }
  block_partials<3, -1>(acc, a.part, bx, nb);
}

template <int MEM>
__global__ __launch_bounds__(THREADS) void k_lbfgs_direction(LbfgsArgs a) {
  lbfgs_direction_body<MEM>(a, blockIdx.x, gridDim.x);
}

// One block: g^T d, d^T d, ||g||_1 from the direction partials; first trial step.
__device__ __forceinline__ void lbfgs_direction_final_body(const LbfgsArgs& a, int nb) {
  SolverState* st = a.st;
  if (st->phase != PH_DIRECTION) return;
  __shared__ double D[3];
  combine_partials<3, -1>(a.part, nb, D);
  if (threadIdx.x == 0) {
    st->dd = D[1];
    rpca_ls::setup_trial(st, D[0], D[2], 0);
  }
}

__global__ __launch_bounds__(THREADS) void k_lbfgs_direction_final(LbfgsArgs a, int nb) {
  lbfgs_direction_final_body(a, nb);
}

// ---------------------------------------------------------------------------
// Batched forms: one launch serves every instance of a batch.  off[i] ..
// off[i+1] are the blocks of instance i (off[count] = grid size); the final
// kernels run one block per instance.
__device__ __forceinline__ int batch_instance(const int* off, int count, int b) {
  int lo = 0, hi = count;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <int MEM>
__global__ __launch_bounds__(THREADS) void k_lbfgs_update_batch(const LbfgsArgs* la, const int* off, int count) {
  const int i = batch_instance(off, count, blockIdx.x);
  lbfgs_update_body<MEM>(la[i], blockIdx.x - off[i], off[i + 1] - off[i]);
}

template <int MEM>
__global__ __launch_bounds__(THREADS) void k_lbfgs_update_final_batch(const LbfgsArgs* la, const int* off) {
  const int i = blockIdx.x;
  lbfgs_update_final_body<MEM>(la[i], off[i + 1] - off[i]);
}

template <int MEM>
__global__ __launch_bounds__(THREADS) void k_lbfgs_direction_batch(const LbfgsArgs* la, const int* off, int count) {
  const int i = batch_instance(off, count, blockIdx.x);
  lbfgs_direction_body<MEM>(la[i], blockIdx.x - off[i], off[i + 1] - off[i]);
}

__global__ __launch_bounds__(THREADS) void k_lbfgs_direction_final_batch(const LbfgsArgs* la, const int* off) {
  const int i = blockIdx.x;
  lbfgs_direction_final_body(la[i], off[i + 1] - off[i]);
}

}  // namespace

namespace rpca {

int lbfgs_blocks(int64_t N) {
  // about one float4 per thread of the direction pass (four per lane of the update
  // pass, whose waves split the pairs), at most RPCA_LBFGS_MAX_BLOCKS
  int64_t b = (N / 4 + THREADS - 1) / THREADS;
  if (b < 1) b = 1;
  if (b > LBFGS_MAX_BLOCKS) b = LBFGS_MAX_BLOCKS;
  return (int)b;
}

#define RPCA_MEM_CASES(X) \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15)

hipError_t launch_lbfgs_update(const LbfgsArgs& a, int mem, hipStream_t stream) {
  const int nb = lbfgs_blocks(a.N);
  const dim3 grid(nb);
  switch (mem) {
#define CASE(M)                                                                              \
  case M:                                                                                    \
    hipLaunchKernelGGL((k_lbfgs_update<M>), grid, dim3(THREADS), 0, stream, a);             \
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;                      \
    hipLaunchKernelGGL((k_lbfgs_update_final_mb<M>), dim3(DotIdx<M>::NV), dim3(THREADS), 0, stream, a, nb); \
    break;
    RPCA_MEM_CASES(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_lbfgs_update_batch(const LbfgsArgs* la, const int* off, int count, int total_blocks,
                                    int mem, hipStream_t stream) {
  switch (mem) {
#define CASE(M)                                                                                         \
  case M:                                                                                               \
    hipLaunchKernelGGL((k_lbfgs_update_batch<M>), dim3(total_blocks), dim3(THREADS), 0, stream, la, off, \
                       count);                                                                          \
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;                                 \
    hipLaunchKernelGGL((k_lbfgs_update_final_batch<M>), dim3(count), dim3(THREADS), 0, stream, la, off); \
    break;
    RPCA_MEM_CASES(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_lbfgs_direction_batch(const LbfgsArgs* la, const int* off, int count, int total_blocks,
                                       int mem, hipStream_t stream, bool with_final) {
  switch (mem) {
#define CASE(M)                                                                                            \
  case M:                                                                                                  \
    hipLaunchKernelGGL((k_lbfgs_direction_batch<M>), dim3(total_blocks), dim3(THREADS), 0, stream, la, off, \
                       count);                                                                             \
    break;
    RPCA_MEM_CASES(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
  if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
  if (with_final) hipLaunchKernelGGL(k_lbfgs_direction_final_batch, dim3(count), dim3(THREADS), 0, stream, la, off);
  return hipGetLastError();
}

hipError_t launch_lbfgs_direction(const LbfgsArgs& a, int mem, hipStream_t stream, bool with_final) {
  const int nb = lbfgs_blocks(a.N);
  const dim3 grid(nb);
  switch (mem) {
#define CASE(M)                                                                        \
  case M:                                                                              \
    hipLaunchKernelGGL((k_lbfgs_direction<M>), grid, dim3(THREADS), 0, stream, a);    \
    break;
    RPCA_MEM_CASES(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
  if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
  if (with_final) hipLaunchKernelGGL(k_lbfgs_direction_final, dim3(1), dim3(THREADS), 0, stream, a, nb);
  return hipGetLastError();
}

}  // namespace rpca
