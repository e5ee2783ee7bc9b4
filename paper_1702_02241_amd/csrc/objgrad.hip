// Objective/gradient: launch of the fused sweep (sweep_kernel.h) and the finishing
// reduction with the device-side line-search step.

#include <math.h>

#include <mutex>

#include "linesearch.h"

#include "rpca_internal.h"
#include "sweep_kernel.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

constexpr int FIN_THREADS = 256;

__device__ __forceinline__ f4 mfma_f32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f4 mfma_bf16(s4 a, s4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  constexpr int W = NT / 64;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < W; ++w) r += sh[w];
  return r;
}

// ---------------------------------------------------------------------------
// Finishing reduction, two launches (no grid-wide fence in the wide one):
//   k_reduce1: grid (ceil(nk/256), segs); thread o of block (bx, by) sums the
//     G^T U partials of workgroup rows [by*rps, (by+1)*rps) -> level2[by][o].
//   k_reduce2: blocks < gv_blocks (whole rows of V each): gV = sum_by level2 +
//     lam_l V_t (fixed order), or its preconditioned form;
//     further blocks (several chunks only): gU = sum over chunks + lam_l U_t.
//     Each block publishes three scalar partials; the last block to arrive
//     (thread-0 fence + counter over a handful of blocks) forms f and g^T d
//     and, in solver mode, runs one step of the line search.
__device__ __forceinline__ void reduce1_body(const FinishArgs& a, int bx, int by) {
  // arm the second kernel's last-block counter (it also returns to zero after
  // every completed reduction; this covers memory that starts undefined)
  if (bx == 0 && by == 0 && threadIdx.x == 0) *a.counter = 0u;
  const int64_t nk = a.n * a.k;
  const int64_t o = (int64_t)bx * FIN_THREADS + threadIdx.x;
  if (o >= nk) return;
  const int r0 = by * a.rows_per_seg;
  int r1 = r0 + a.rows_per_seg;
  if (r1 > a.row_groups) r1 = a.row_groups;
  const float* src = a.gvpart + o;
  double s = 0.0;
  int r = r0;
  // eight loads in flight, summed in row order
  for (; r + 7 < r1; r += 8) {
    float x[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) x[e] = src[(int64_t)(r + e) * nk];
#pragma unroll
    for (int e = 0; e < 8; ++e) s += (double)x[e];
  }
  for (; r < r1; ++r) s += (double)src[(int64_t)r * nk];
  a.level2[(int64_t)by * nk + o] = s;
}

__global__ __launch_bounds__(FIN_THREADS) void k_reduce1(FinishArgs a) { reduce1_body(a, blockIdx.x, blockIdx.y); }

// Block bx of the nblk blocks of one instance.
template <bool TRIAL>
__device__ __forceinline__ void reduce2_body(const FinishArgs& a, const int bx, const int nblk) {
  __shared__ double sh[FIN_THREADS / 64];
  __shared__ int s_last;
  int outi = 0;
  SolverState* st = a.st;
  if (TRIAL) {
    if (st->phase != PH_TRIAL) return;
    outi = 1 - st->cur;
  }
  const int64_t nk = a.n * a.k, mk = a.m * a.k;
  const float lam_l = a.lam_l;
  const float* Vt = a.V[outi];
  const float* Ut = a.U[outi];
  const int tid = threadIdx.x;
  double vv = 0.0, gvd = 0.0, gud = 0.0;
  const int k = a.k;
  if (bx < a.gv_blocks) {
    // whole rows per block: thread (jr, c) of row j = bx * rpb + jr
    const int rpb = FIN_THREADS / k;
    const int jr = tid / k, c = tid % k;
    const int64_t j = (int64_t)bx * rpb + jr;
    const bool ok = jr < rpb && j < a.n;
    const int64_t o = j * k + c;
    double s = 0.0;
    if (ok) {
      int q = 0;
      for (; q + 7 < a.segs; q += 8) {  // eight loads in flight, summed in segment order
        double x[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = a.level2[(int64_t)(q + e) * nk + o];
#pragma unroll
        for (int e = 0; e < 8; ++e) s += x[e];
      }
      for (; q < a.segs; ++q) s += a.level2[(int64_t)q * nk + o];
    }
    if (!a.pc) {
      if (ok) {
        const float v = Vt[o];
        const float gvv = (float)(s + (double)lam_l * (double)v);
        a.gV[outi][o] = gvv;
        vv = (double)v * (double)v;
        if (TRIAL) gvd = (double)gvv * (double)a.dV[o];
      }
    } else {
      // preconditioned variables: grad_B = (G^T A) W + lam_l B M_V, ||V||^2 = sum B M_V B^T
      __shared__ double sS[FIN_THREADS];
      sS[tid] = s;
      __syncthreads();
      if (ok) {
        const float* W = a.pc;
        const float* MV = a.pc + 2 * k * k;
        double t1 = 0.0, t2 = 0.0;
        for (int t = 0; t < k; ++t) {
          t1 += sS[jr * k + t] * (double)W[t * k + c];
          t2 += (double)Vt[j * k + t] * (double)MV[t * k + c];
        }
        const float gvv = (float)(t1 + (double)lam_l * t2);
        a.gV[outi][o] = gvv;
        vv = (double)Vt[o] * t2;
        if (TRIAL) gvd = (double)gvv * (double)a.dV[o];
      }
    }
  } else {
    const float* MU = a.pc ? a.pc + k * k : nullptr;
    const int64_t stride = (int64_t)(nblk - a.gv_blocks) * FIN_THREADS;
    for (int64_t o = (int64_t)(bx - a.gv_blocks) * FIN_THREADS + tid; o < mk; o += stride) {
      double s = 0.0;
      int cc = 0;
      for (; cc + 7 < a.nchunks; cc += 8) {  // eight loads in flight, summed in chunk order
        float x[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = a.gupart[(int64_t)(cc + e) * mk + o];
#pragma unroll
        for (int e = 0; e < 8; ++e) s += (double)x[e];
      }
      for (; cc < a.nchunks; ++cc) s += (double)a.gupart[(int64_t)cc * mk + o];
      double reg = Ut[o];
      if (MU) {  // A M_U
        const int64_t i = o / k;
        const int c = (int)(o % k);
        reg = 0.0;
        for (int t = 0; t < k; ++t) reg += (double)Ut[i * k + t] * (double)MU[t * k + c];
      }
      const float gu = (float)(s + (double)lam_l * reg);
      a.gU[outi][o] = gu;
      if (TRIAL) gud += (double)gu * (double)a.dU[o];
    }
  }
  const double b0 = block_sum<FIN_THREADS>(vv, sh);
  const double b1 = block_sum<FIN_THREADS>(gvd, sh);
  const double b2 = block_sum<FIN_THREADS>(gud, sh);
  if (tid == 0) {
    a.fpart[bx * 3 + 0] = b0;
    a.fpart[bx * 3 + 1] = b1;
    a.fpart[bx * 3 + 2] = b2;
    __threadfence();
    const unsigned prev = atomicAdd(a.counter, 1u);
    s_last = (prev == (unsigned)nblk - 1u);
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  double fd = 0.0, uu = 0.0, gd1 = 0.0, g2 = 0.0, p0 = 0.0, p1 = 0.0, p2 = 0.0;
  for (int q = tid; q < a.sweep_wgs; q += FIN_THREADS) {
    fd += a.spart[(int64_t)q * RPCA_NSCAL + 0];
    uu += a.spart[(int64_t)q * RPCA_NSCAL + 1];
    gd1 += a.spart[(int64_t)q * RPCA_NSCAL + 2];
    g2 += a.spart[(int64_t)q * RPCA_NSCAL + 3];
  }
  for (int b = tid; b < nblk; b += FIN_THREADS) {
    p0 += a.fpart[b * 3 + 0];
    p1 += a.fpart[b * 3 + 1];
    p2 += a.fpart[b * 3 + 2];
  }
  {
    // the seven sums in one pass: wave reductions, then the waves in a fixed order
    __shared__ double sh7[FIN_THREADS / 64][7];
    double v[7] = {fd, uu, gd1, g2, p0, p1, p2};
#pragma unroll
    for (int e = 0; e < 7; ++e)
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) v[e] += __shfl_xor(v[e], o, 64);
    if ((tid & 63) == 0)
#pragma unroll
      for (int e = 0; e < 7; ++e) sh7[tid >> 6][e] = v[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 7; ++e) {
      double r = 0.0;
      for (int w = 0; w < FIN_THREADS / 64; ++w) r += sh7[w][e];
      v[e] = r;
    }
    fd = v[0];
    uu = v[1];
    gd1 = v[2];
    g2 = v[3];
    p0 = v[4];
    p1 = v[5];
    p2 = v[6];
  }
  if (!TRIAL) {
    if (tid == 0) {
      if (a.f_out) *a.f_out = fd + 0.5 * (double)lam_l * (uu + p0);
      if (a.aux_out) {
        a.aux_out[0] = fd;  // phi(U V^T)
        a.aux_out[1] = uu;  // ||U||^2
        a.aux_out[2] = p0;  // ||V||^2
        a.aux_out[3] = g2;  // ||G||_F^2
      }
      *a.counter = 0u;
    }
    return;
  }
  // line-search step on an LDS copy of the state head (one thread), written back by the block
  __shared__ SolverState sst;
  copy_state_head(&sst, st);
  __syncthreads();
  if (tid == 0) {
    sst.dir_pending = 0;  // this trial's direction has been formed
    rpca_ls::line_search_step(&sst, fd + 0.5 * (double)lam_l * (uu + p0), gd1 + p1 + p2);
    *a.counter = 0u;
  }
  __syncthreads();
  copy_state_head(st, &sst);
}

template <bool TRIAL>
__global__ __launch_bounds__(FIN_THREADS) void k_reduce2(FinishArgs a) {
  reduce2_body<TRIAL>(a, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// Batched forms (one launch for every instance of a batch).  off1/off2: block
// offsets of each instance in the reduce1 / reduce2 grids; reduce1 also
// re-arms the work queue of the batched sweep that preceded it.
__device__ __forceinline__ int batch_instance(const int* off, int count, int b) {
  int lo = 0, hi = count;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(FIN_THREADS) void k_reduce1_batch(const FinishArgs* fa, const int* off, int count,
                                                              unsigned* queue_heads, int nheads) {
  if (blockIdx.x == 0 && (int)threadIdx.x < nheads) queue_heads[threadIdx.x] = 0u;
  const int i = batch_instance(off, count, blockIdx.x);
  const FinishArgs& a = fa[i];
  const int gvb = (int)((a.n * a.k + FIN_THREADS - 1) / FIN_THREADS);
  const int lb = blockIdx.x - off[i];
  reduce1_body(a, lb % gvb, lb / gvb);
}

template <bool TRIAL>
__global__ __launch_bounds__(FIN_THREADS) void k_reduce2_batch(const FinishArgs* fa, const int* off, int count) {
  const int i = batch_instance(off, count, blockIdx.x);
  reduce2_body<TRIAL>(fa[i], blockIdx.x - off[i], off[i + 1] - off[i]);
}

}  // namespace

namespace rpca {

hipError_t launch_sweep_f32_plain(const SweepArgs&, bool, hipStream_t);
hipError_t launch_sweep_f32_trial(const SweepArgs&, bool, hipStream_t);
hipError_t launch_sweep_bf16_plain(const SweepArgs&, bool, hipStream_t);
hipError_t launch_sweep_bf16_trial(const SweepArgs&, bool, hipStream_t);
hipError_t launch_sweep_f32_elastic(const SweepArgs&, bool, bool, hipStream_t);

// Sweep decomposition table, keyed by (k bucket, n bucket): the number of
// waves the strips are spread over and the divisor of the widest chunk.
// Defaults are what measurements at the benchmark shapes favoured; rpca_autotune
// replaces entries by timing the candidates on the device.
// The table is process-wide: reads and writes hold its mutex (contexts of a
// batch are set up from several host threads).
namespace {
struct TuneTable {
  std::mutex mu;
  SweepTune t[TUNE_KB][TUNE_NB];
  TuneTable() {
    // k <= 16: two workgroups per CU (the k16 sweep); k > 16: one, and for more
    // than 512 columns (many chunks, few rows each) four times as many row groups
    // (8192 x 8192, k = 25, Bernoulli(0.3) mask: 444 -> 369 us)
    for (int a = 0; a < TUNE_KB; ++a)
      for (int b = 0; b < TUNE_NB; ++b)
        t[a][b] = SweepTune{a < 2 ? 2048 : (b == TUNE_NB - 1 ? 4096 : 1024), 1};
  }
};
TuneTable& tune_table() {
  static TuneTable tt;  // initialised once, thread-safely
  return tt;
}
}  // namespace

int tune_k_bucket(int k) { return k <= 8 ? 0 : k <= 16 ? 1 : k <= 24 ? 2 : 3; }
int tune_n_bucket(int64_t n) { return n <= 64 ? 0 : n <= 128 ? 1 : n <= 256 ? 2 : n <= 512 ? 3 : 4; }

SweepTune tune_get(int k, int64_t n) {
  TuneTable& tt = tune_table();
  std::lock_guard<std::mutex> lock(tt.mu);
  return tt.t[tune_k_bucket(k)][tune_n_bucket(n)];
}

void tune_set(int kbucket, int nbucket, SweepTune t) {
  TuneTable& tt = tune_table();
  std::lock_guard<std::mutex> lock(tt.mu);
  tt.t[kbucket][nbucket] = t;
}

// Column chunks (each fitting the sweep's LDS budget) and the wave/workgroup
// split of the rows, from the tuning table.
int sweep_blocks_for(int64_t m, int64_t n, int k, int* row_groups, int* strips_per_wave, int* chunk_w,
                     int* nchunks, int target_waves) {
  SweepTune t = tune_get(k, n);
  if (target_waves > 0) t.target_waves = target_waves;
  const int kb = (k + 15) / 16;
  int cmax = rpca_sweep::max_chunk(kb, k);
  if (t.chunk_div > 1) cmax = ((cmax / t.chunk_div + 15) / 16) * 16;
  if (cmax < 16) cmax = 16;
  int nch = (int)((n + cmax - 1) / cmax);
  int cw = (int)(((n + nch - 1) / nch + 15) / 16) * 16;
  if (cw > cmax) cw = cmax;
  nch = (int)((n + cw - 1) / cw);
  const int64_t nstrips = (m + 15) / 16;
  // the waves of all chunks together make up the table's target
  int64_t target = (t.target_waves + nch - 1) / nch;
  if (target > nstrips) target = nstrips;
  if (target < 1) target = 1;
  // workgroup rows split the strips as evenly as integers allow (the kernel
  // gives row rg the strips [rg S / R, (rg + 1) S / R))
  int64_t wgs = (target + rpca_sweep::WAVES - 1) / rpca_sweep::WAVES;
  if (wgs > nstrips) wgs = nstrips;
  const int64_t per_wg = (nstrips + wgs - 1) / wgs;
  *row_groups = (int)wgs;
  *strips_per_wave = (int)((per_wg + rpca_sweep::WAVES - 1) / rpca_sweep::WAVES);
  *chunk_w = cw;
  *nchunks = nch;
  return (int)(wgs * nch);
}

hipError_t launch_sweep(const SweepArgs& sa, bool trial, bool bf16, hipStream_t stream) {
  const bool masked = sa.mask != nullptr;
  if (sa.kappa != 0.f) {  // elastic-net marginal: FP32 products only (callers reject BF16 first)
    if (bf16) return hipErrorInvalidValue;
    return launch_sweep_f32_elastic(sa, trial, masked, stream);
  }
  if (bf16)
    return trial ? launch_sweep_bf16_trial(sa, masked, stream) : launch_sweep_bf16_plain(sa, masked, stream);
  return trial ? launch_sweep_f32_trial(sa, masked, stream) : launch_sweep_f32_plain(sa, masked, stream);
}

int finish_blocks(int64_t m, int64_t n, int k, int nchunks, int* gv_blocks) {
  const int rpb = FIN_THREADS / k;  // whole rows of V per block
  const int gvb = (int)((n + rpb - 1) / rpb);
  int gub = 0;
  if (nchunks > 1) {
    // one output per thread (all chunks' partials of it in flight eight at a time)
    gub = (int)((m * k + FIN_THREADS - 1) / FIN_THREADS);
    if (gub > 4096) gub = 4096;
  }
  if (gv_blocks) *gv_blocks = gvb;
  return gvb + gub;
}

hipError_t launch_finish(const FinishArgs& fa, bool trial, hipStream_t stream) {
  FinishArgs f2 = fa;
  const int blocks = finish_blocks(fa.m, fa.n, fa.k, fa.nchunks, &f2.gv_blocks);
  const int gvb = (int)((fa.n * fa.k + FIN_THREADS - 1) / FIN_THREADS);
  hipLaunchKernelGGL(k_reduce1, dim3(gvb, fa.segs), dim3(FIN_THREADS), 0, stream, f2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (trial)
    hipLaunchKernelGGL((k_reduce2<true>), dim3(blocks), dim3(FIN_THREADS), 0, stream, f2);
  else
    hipLaunchKernelGGL((k_reduce2<false>), dim3(blocks), dim3(FIN_THREADS), 0, stream, f2);
  return hipGetLastError();
}

hipError_t launch_sweep_batch_f32(int, int, const SweepArgs*, const SweepItem*, int, unsigned*, int, int, bool, bool,
                                  hipStream_t);
hipError_t launch_sweep_batch_bf16(int, int, const SweepArgs*, const SweepItem*, int, unsigned*, int, int, bool,
                                   bool, hipStream_t);
int sweep_batch_grid_f32(int, int, int, bool, bool);
int sweep_batch_grid_bf16(int, int, int, bool, bool);

hipError_t launch_sweep_batch(int kb, int tmax, const SweepArgs* args, const SweepItem* items, int nitems,
                              unsigned* head, int grid, int lds_floats, bool masked, bool trial, bool bf16,
                              hipStream_t s) {
  return bf16 ? launch_sweep_batch_bf16(kb, tmax, args, items, nitems, head, grid, lds_floats, masked, trial, s)
              : launch_sweep_batch_f32(kb, tmax, args, items, nitems, head, grid, lds_floats, masked, trial, s);
}

int sweep_batch_grid(int kb, int tmax, int lds_floats, bool masked, bool trial, bool bf16) {
  return bf16 ? sweep_batch_grid_bf16(kb, tmax, lds_floats, masked, trial)
              : sweep_batch_grid_f32(kb, tmax, lds_floats, masked, trial);
}

int sweep_lds_floats(int kb, int k, int cwp) { return rpca_sweep::lds_floats(kb, k, cwp); }
int sweep_tmax_class(int kb, int ntiles) { return rpca_sweep::tmax_class(kb, ntiles); }

hipError_t launch_finish_batch(const FinishArgs* fa, const int* off1, int total1, const int* off2, int total2,
                               int count, unsigned* queue_heads, int nheads, bool trial, hipStream_t stream) {
  if (nheads > FIN_THREADS) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reduce1_batch, dim3(total1), dim3(FIN_THREADS), 0, stream, fa, off1, count, queue_heads,
                     nheads);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (trial)
    hipLaunchKernelGGL((k_reduce2_batch<true>), dim3(total2), dim3(FIN_THREADS), 0, stream, fa, off2, count);
  else
    hipLaunchKernelGGL((k_reduce2_batch<false>), dim3(total2), dim3(FIN_THREADS), 0, stream, fa, off2, count);
  return hipGetLastError();
}

hipError_t launch_objgrad(const SweepArgs& sa, const FinishArgs& fa, bool trial, bool bf16,
                          hipStream_t stream) {
  const hipError_t e = launch_sweep(sa, trial, bf16, stream);
  if (e != hipSuccess) return e;
  return launch_finish(fa, trial, stream);
}

}  // namespace rpca
