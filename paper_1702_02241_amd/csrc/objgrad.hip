// Fused Split-SPCP objective/gradient sweep for gfx950.
//
// One pass over X computes, per 16 x 16 tile held in registers,
//   R = U V^T - X                 (Sec. 5 eq. Thm5, the residual of the marginal phi)
//   rho(R), G = Omega .* clip(R)  (Huber value and derivative, Sec. 1 eq. PhiDef, Sec. 3.2 eq. diff)
//   G^T U  (MFMA, accumulated per workgroup -> partial)  and  G V (VALU, complete rows)
// so neither R nor G is ever written to memory.  A workgroup owns a range of
// 16-row strips and one chunk of columns; the four waves of a workgroup take
// interleaved strips.  The MFMA tile layout (v_mfma_f32_16x16x4_f32, wave64):
//   A[i][kk] lane = i + 16*kk,  B[kk][j] lane = j + 16*kk,  D[i][j] lane = j + 16*(i/4), reg i%4.
// Seeding the accumulator with -X makes the MFMA produce the residual tile
// directly; its register layout (column j = lane%16, rows 4*(lane/16)+r) is
// exactly the A operand layout that G^T U needs with the K index running over
// rows, so G feeds the second MFMA without any shuffle.
#include "rpca_internal.h"

#include <math.h>

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int WAVES = 4;
constexpr int THREADS = 64 * WAVES;

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum `v` over the 256 threads of the block in a fixed order; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < WAVES; ++w) r += sh[w];
  return r;
}

// ---------------------------------------------------------------------------
// Main sweep.
//   KB = number of 16-wide blocks of the factor rank (k <= 16*KB)
//   JT = 16-column tiles per chunk (chunk width 16*JT)
template <int KB, int JT, bool MASKED, bool TRIAL, bool VEC4>
__global__ __launch_bounds__(THREADS) void k_objgrad_sweep(SweepArgs a) {
  constexpr int KMAX = 16 * KB;
  __shared__ float sV[JT * 16 * KMAX];
  __shared__ float sC[JT * 16 * KMAX];
  __shared__ double sRed[WAVES][4];

  int cur = 0;
  float alpha = 0.f;
  int outi = 0;
  if (TRIAL) {
    const SolverState* st = a.st;
    if (st->phase != PH_TRIAL) return;
    cur = st->cur;
    alpha = (float)st->alpha;
    outi = 1 - cur;
  }
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int rg = blockIdx.x, ch = blockIdx.y;
  const int64_t m = a.m, n = a.n;
  const int k = a.k;
  const float lam_s = a.lam_s, lam_l = a.lam_l;
  const float* __restrict__ U = a.U[cur];
  const float* __restrict__ V = a.V[cur];
  const float* __restrict__ X = a.X;

  const int64_t j_begin = (int64_t)ch * a.chunk_w;
  const int ncols = (int)((n - j_begin) < a.chunk_w ? (n - j_begin) : a.chunk_w);
  const int ntiles = (ncols + 15) >> 4;

  // Stage the (trial) V rows of this chunk in LDS, rows padded to KMAX.
  for (int idx = tid; idx < JT * 16 * KMAX; idx += THREADS) {
    const int jl = idx / KMAX, kk = idx % KMAX;
    float v = 0.f;
    if (jl < ncols && kk < k) {
      const int64_t o = (j_begin + jl) * k + kk;
      v = V[o];
      if (TRIAL) {
        v = fmaf(alpha, a.dV[o], v);
        if (rg == 0) a.Vt[outi][o] = v;
      }
    }
    sV[idx] = v;
  }
  __syncthreads();

  const int KS = (k + 3) >> 2;
  f4 gv[JT][KB];
#pragma unroll
  for (int t = 0; t < JT; ++t)
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) gv[t][kb] = f4{0.f, 0.f, 0.f, 0.f};
  double f_acc = 0.0, uu_acc = 0.0, gud_acc = 0.0, gg_acc = 0.0;

  const int64_t nstrips = (m + 15) >> 4;
  const int64_t s_begin = (int64_t)rg * a.strips_per_wg;
  int64_t s_end = s_begin + a.strips_per_wg;
  if (s_end > nstrips) s_end = nstrips;

  for (int64_t s = s_begin + wave; s < s_end; s += WAVES) {
    const int64_t i0 = s * 16;
    // Trial U rows of this strip in the two operand layouts.
    float ua[4 * KB];
#pragma unroll
    for (int q = 0; q < 4 * KB; ++q) {
      const int kk = 4 * q + g;
      const int64_t i = i0 + c;
      float v = 0.f;
      if (q < KS && kk < k && i < m) {
        v = U[i * k + kk];
        if (TRIAL) v = fmaf(alpha, a.dU[i * k + kk], v);
      }
      ua[q] = v;
    }
    float ub[4][KB], dub[4][KB];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        const int kk = 16 * kb + c;
        const int64_t i = i0 + 4 * g + r;
        float v = 0.f, dv = 0.f;
        if (kk < k && i < m) {
          v = U[i * k + kk];
          if (TRIAL) {
            dv = a.dU[i * k + kk];
            v = fmaf(alpha, dv, v);
          }
        }
        ub[r][kb] = v;
        dub[r][kb] = dv;
      }

    float accu[4][KMAX];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int kk = 0; kk < KMAX; ++kk) accu[r][kk] = 0.f;

    const bool full_rows = (i0 + 16 <= m);
#pragma unroll
    for (int t = 0; t < JT; ++t) {
      if (t < ntiles) {
        const int jl = t * 16 + c;
        const int64_t j = j_begin + jl;
        const bool jok = jl < ncols;
        float x[4];
        const float* xp = X + j * m + i0 + 4 * g;
        if (VEC4 && full_rows && jok) {
          const f4 xv = *reinterpret_cast<const f4*>(xp);
          x[0] = xv[0]; x[1] = xv[1]; x[2] = xv[2]; x[3] = xv[3];
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r) x[r] = (jok && i0 + 4 * g + r < m) ? xp[r] : 0.f;
        }
        uint32_t bits = 0xFu;
        if (MASKED) {
          bits = 0u;
          if (jok) {
            const uint32_t w = a.mask[j * a.mw + (i0 >> 5)];
            bits = (w >> ((int)(i0 & 31) + 4 * g)) & 0xFu;
          }
        }
        f4 acc = f4{-x[0], -x[1], -x[2], -x[3]};
#pragma unroll
        for (int q = 0; q < 4 * KB; ++q)
          if (q < KS) acc = mfma4(ua[q], sV[jl * KMAX + 4 * q + g], acc);
        float G[4];
        float ftile = 0.f, gtile = 0.f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float R = acc[r];
          const float ar = fabsf(R);
          float rho = (ar <= lam_s) ? 0.5f * R * R : lam_s * (ar - 0.5f * lam_s);
          float gr = fminf(fmaxf(R, -lam_s), lam_s);
          if (MASKED && !((bits >> r) & 1u)) {
            rho = 0.f;
            gr = 0.f;
          }
          ftile += rho;
          gtile = fmaf(gr, gr, gtile);
          G[r] = gr;
        }
        f_acc += (double)ftile;
        gg_acc += (double)gtile;
        // G^T U on MFMA: K runs over the 16 rows of the strip (rows 4*g + r).
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
#pragma unroll
          for (int r = 0; r < 4; ++r) gv[t][kb] = mfma4(G[r], ub[r][kb], gv[t][kb]);
        // G V on the vector ALUs: each lane accumulates its 4 rows against V row j.
#pragma unroll
        for (int kk = 0; kk < KMAX; ++kk) {
          if (kk < k) {
            const float vv = sV[jl * KMAX + kk];
#pragma unroll
            for (int r = 0; r < 4; ++r) accu[r][kk] = fmaf(G[r], vv, accu[r][kk]);
          }
        }
      }
    }
    // Sum the G V partials over the 16 lanes (columns) that share rows.
#pragma unroll
    for (int kk = 0; kk < KMAX; ++kk) {
      if (kk < k) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float v = accu[r][kk];
          v += __shfl_xor(v, 1, 64);
          v += __shfl_xor(v, 2, 64);
          v += __shfl_xor(v, 4, 64);
          v += __shfl_xor(v, 8, 64);
          accu[r][kk] = v;
        }
      }
    }
    // Lane (g, c) writes rows i0+4g+r, column kk = 16*kb + c.
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t i = i0 + 4 * g + r;
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        const int kk = 16 * kb + c;
        float sel = 0.f;
#pragma unroll
        for (int q = 0; q < 16; ++q) sel = (q == c) ? accu[r][16 * kb + q] : sel;
        if (kk < k && i < m) {
          const int64_t o = i * k + kk;
          if (a.nchunks == 1) {
            const float gu = fmaf(lam_l, ub[r][kb], sel);
            a.gU[outi][o] = gu;
            if (TRIAL) gud_acc += (double)gu * (double)dub[r][kb];
          } else {
            a.gupart[(int64_t)ch * m * k + o] = sel;
          }
          if (ch == 0) {
            uu_acc += (double)ub[r][kb] * (double)ub[r][kb];
            if (TRIAL) a.Ut[outi][o] = ub[r][kb];
          }
        }
      }
    }
  }

  // Combine the waves' G^T U tiles in LDS in a fixed order (deterministic).
  for (int w = 0; w < WAVES; ++w) {
    if (wave == w) {
#pragma unroll
      for (int t = 0; t < JT; ++t)
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int idx = (t * 16 + 4 * g + r) * KMAX + 16 * kb + c;
            sC[idx] = (w == 0 ? 0.f : sC[idx]) + gv[t][kb][r];
          }
    }
    __syncthreads();
  }
  float* gvp = a.gvpart + (int64_t)rg * n * k;
  for (int idx = tid; idx < ncols * k; idx += THREADS) {
    const int jl = idx / k, kk = idx - jl * k;
    gvp[(j_begin + jl) * k + kk] = sC[jl * KMAX + kk];
  }

  // Scalar partials: data term of f, ||U_t||^2, gU^T dU, sum G^2.
  double v0 = wave_sum(f_acc), v1 = wave_sum(uu_acc), v2 = wave_sum(gud_acc),
         v3 = wave_sum(gg_acc);
  if (lane == 0) {
    sRed[wave][0] = v0;
    sRed[wave][1] = v1;
    sRed[wave][2] = v2;
    sRed[wave][3] = v3;
  }
  __syncthreads();
  if (tid < 4) {
    double s = 0.0;
    for (int w = 0; w < WAVES; ++w) s += sRed[w][tid];
    a.spart[((int64_t)rg * a.nchunks + ch) * RPCA_NSCAL + tid] = s;
  }
}

// ---------------------------------------------------------------------------
// Strong-Wolfe line search, one step of the state machine (Nocedal & Wright
// Alg. 3.5 bracketing + Alg. 3.6 zoom, cubic interpolation), run by one thread
// after each trial evaluation.

__device__ bool cubic_min(double a0, double f0, double d0, double a1, double f1, double d1,
                          double* out) {
  if (a0 == a1) return false;
  const double e1 = d0 + d1 - 3.0 * (f0 - f1) / (a0 - a1);
  const double disc = e1 * e1 - d0 * d1;
  if (!(disc >= 0.0) || !isfinite(disc)) return false;
  const double e2 = copysign(sqrt(disc), a1 - a0);
  const double den = d1 - d0 + 2.0 * e2;
  if (den == 0.0 || !isfinite(den)) return false;
  *out = a1 - (a1 - a0) * (d1 + e2 - e1) / den;
  return isfinite(*out);
}

__device__ void zoom_next(SolverState* st) {
  const double lo = st->a_lo, hi = st->a_hi;
  const double left = fmin(lo, hi), right = fmax(lo, hi), w = right - left;
  double a;
  if (!cubic_min(lo, st->f_lo, st->d_lo, hi, st->f_hi, st->d_hi, &a) || a < left + 0.01 * w ||
      a > right - 0.01 * w)
    a = 0.5 * (lo + hi);
  st->alpha = a;
}

__device__ void search_failed(SolverState* st) {
  if (st->count > 0 && !st->restarted) {
    // drop the memory once and retry along steepest descent
    st->count = 0;
    st->spare = 0;
    st->newest = -1;
    st->restarted = 1;
    st->phase = PH_DIRECTION;
  } else {
    st->stop = STOP_LINESEARCH;
    st->phase = PH_DONE;
  }
}

__device__ void accept_trial(SolverState* st, double ft) {
  st->cur = 1 - st->cur;
  st->f = ft;
  st->restarted = 0;
  st->phase = PH_UPDATE;
}

__device__ void line_search_step(SolverState* st, double ft, double dt) {
  st->evals += 1;
  st->ls_trials += 1;
  st->f_t = ft;
  st->dphi_t = dt;
  const double a = st->alpha, f0 = st->f, d0 = st->dphi0, c1 = st->c1, c2 = st->c2;
  const bool finite = isfinite(ft) && isfinite(dt);
  // Approximate Wolfe (Hager & Zhang): once f-differences reach the rounding level of
  // the evaluation, accept a step whose slope satisfies
  // -c2|d0| <= dphi <= (1 - 2 c1)|d0| and whose value is within eps_f |f0| of f0.
  if (finite && ft <= f0 + st->eps_f * fabs(f0) && dt >= c2 * d0 && dt <= (2.0 * c1 - 1.0) * d0 &&
      ft > f0 + c1 * a * d0) {
    accept_trial(st, ft);
    return;
  }
  const bool armijo_fail = !finite || ft > f0 + c1 * a * d0;
  if (st->ls_stage == 0) {
    if (armijo_fail || (st->ls_trials > 1 && ft >= st->f_prev)) {
      st->a_lo = st->a_prev; st->f_lo = st->f_prev; st->d_lo = st->d_prev;
      st->a_hi = a; st->f_hi = finite ? ft : INFINITY; st->d_hi = finite ? dt : 0.0;
      st->ls_stage = 1;
      zoom_next(st);
    } else if (fabs(dt) <= -c2 * d0) {
      accept_trial(st, ft);
      return;
    } else if (dt >= 0.0) {
      st->a_lo = a; st->f_lo = ft; st->d_lo = dt;
      st->a_hi = st->a_prev; st->f_hi = st->f_prev; st->d_hi = st->d_prev;
      st->ls_stage = 1;
      zoom_next(st);
    } else {
      double an;
      const double lo_b = a + 0.01 * (a - st->a_prev), hi_b = 10.0 * a;
      if (!cubic_min(st->a_prev, st->f_prev, st->d_prev, a, ft, dt, &an) || an < lo_b || an > hi_b)
        an = fmin(fmax(2.0 * a, lo_b), hi_b);
      st->a_prev = a; st->f_prev = ft; st->d_prev = dt;
      st->alpha = an;
    }
  } else {
    if (armijo_fail || ft >= st->f_lo) {
      st->a_hi = a; st->f_hi = finite ? ft : INFINITY; st->d_hi = finite ? dt : 0.0;
    } else {
      if (fabs(dt) <= -c2 * d0) {
        accept_trial(st, ft);
        return;
      }
      if (dt * (st->a_hi - st->a_lo) >= 0.0) {
        st->a_hi = st->a_lo; st->f_hi = st->f_lo; st->d_hi = st->d_lo;
      }
      st->a_lo = a; st->f_lo = ft; st->d_lo = dt;
    }
    if (fabs(st->a_hi - st->a_lo) <= 1e-12 * fmax(1.0, fabs(st->a_hi))) {
      search_failed(st);
      return;
    }
    zoom_next(st);
  }
  if (st->ls_trials >= 30 || !(st->alpha > 0.0)) search_failed(st);
}

// ---------------------------------------------------------------------------
// Finishing reduction, two levels in one launch.
//   blocks (bx < gv_blocks, by < segs): sum the G^T U partials of row groups
//       [by*rps, (by+1)*rps) for 256 outputs -> level2[by][o];
//   blocks bx >= gv_blocks (by == 0): multi-chunk G V rows -> gU (+ lam_l U_t);
//   the last block to finish: gV = sum_by level2 + lam_l V_t, f, g^T d, and in
//   solver mode one step of the line search.  All sums run in a fixed order.
template <bool TRIAL>
__global__ __launch_bounds__(THREADS) void k_objgrad_finish(FinishArgs a) {
  __shared__ double sh[WAVES];
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
  const int bx = blockIdx.x, by = blockIdx.y;
  double gud = 0.0;
  if (bx < a.gv_blocks) {
    const int64_t o = (int64_t)bx * THREADS + threadIdx.x;
    if (o < nk) {
      const int r0 = by * a.rows_per_seg;
      int r1 = r0 + a.rows_per_seg;
      if (r1 > a.row_groups) r1 = a.row_groups;
      double s = 0.0;
      for (int r = r0; r < r1; ++r) s += (double)a.gvpart[(int64_t)r * nk + o];
      a.level2[(int64_t)by * nk + o] = s;
    }
  } else if (by == 0) {
    const int64_t stride = (int64_t)(gridDim.x - a.gv_blocks) * THREADS;
    for (int64_t o = (int64_t)(bx - a.gv_blocks) * THREADS + threadIdx.x; o < mk; o += stride) {
      double s = 0.0;
      for (int c = 0; c < a.nchunks; ++c) s += (double)a.gupart[(int64_t)c * mk + o];
      const float gu = (float)(s + (double)lam_l * (double)Ut[o]);
      a.gU[outi][o] = gu;
      if (TRIAL) gud += (double)gu * (double)a.dU[o];
    }
  }
  const int nblocks = gridDim.x * gridDim.y;
  const int bid = by * gridDim.x + bx;
  const double b2 = block_sum(gud, sh);
  if (threadIdx.x == 0) a.fpart[bid] = b2;
  // every writer publishes its level2 / gU / fpart stores before the count
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned prev = atomicAdd(a.counter, 1u);
    s_last = (prev == (unsigned)nblocks - 1u);
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  // Last block.
  double vv = 0.0, gvd = 0.0;
  for (int64_t o = threadIdx.x; o < nk; o += THREADS) {
    double s = 0.0;
    for (int q = 0; q < a.segs; ++q) s += a.level2[(int64_t)q * nk + o];
    const float v = Vt[o];
    const float gvv = (float)(s + (double)lam_l * (double)v);
    a.gV[outi][o] = gvv;
    vv += (double)v * (double)v;
    if (TRIAL) gvd += (double)gvv * (double)a.dV[o];
  }
  double fd = 0.0, uu = 0.0, gd1 = 0.0, gd2 = 0.0, g2 = 0.0;
  for (int w = threadIdx.x; w < a.sweep_wgs; w += THREADS) {
    fd += a.spart[(int64_t)w * RPCA_NSCAL + 0];
    uu += a.spart[(int64_t)w * RPCA_NSCAL + 1];
    gd1 += a.spart[(int64_t)w * RPCA_NSCAL + 2];
    g2 += a.spart[(int64_t)w * RPCA_NSCAL + 3];
  }
  for (int b = threadIdx.x; b < nblocks; b += THREADS) gd2 += a.fpart[b];
  fd = block_sum(fd, sh);
  uu = block_sum(uu, sh);
  gd1 = block_sum(gd1, sh);
  gd2 = block_sum(gd2, sh);
  vv = block_sum(vv, sh);
  gvd = block_sum(gvd, sh);
  g2 = block_sum(g2, sh);
  if (threadIdx.x == 0) {
    const double f = fd + 0.5 * (double)lam_l * (uu + vv);
    const double dphi = gd1 + gd2 + gvd;
    if (!TRIAL) {
      *a.f_out = f;
      if (a.aux_out) {
        a.aux_out[0] = fd;   // phi(U V^T)
        a.aux_out[1] = uu;   // ||U||^2
        a.aux_out[2] = vv;   // ||V||^2
        a.aux_out[3] = g2;   // ||G||_F^2
      }
    } else {
      line_search_step(st, f, dphi);
    }
    *a.counter = 0u;
  }
}

template <int KB, bool MASKED, bool TRIAL>
hipError_t launch_sweep_v(const SweepArgs& sa, bool vec4, dim3 grid, hipStream_t stream) {
  constexpr int JT = 16 / KB;
  if (vec4)
    hipLaunchKernelGGL((k_objgrad_sweep<KB, JT, MASKED, TRIAL, true>), grid, dim3(THREADS), 0,
                       stream, sa);
  else
    hipLaunchKernelGGL((k_objgrad_sweep<KB, JT, MASKED, TRIAL, false>), grid, dim3(THREADS), 0,
                       stream, sa);
  return hipGetLastError();
}

template <bool MASKED, bool TRIAL>
hipError_t launch_sweep_m(const SweepArgs& sa, bool vec4, dim3 grid, hipStream_t stream) {
  if (sa.k <= 16) return launch_sweep_v<1, MASKED, TRIAL>(sa, vec4, grid, stream);
  return launch_sweep_v<2, MASKED, TRIAL>(sa, vec4, grid, stream);
}

}  // namespace

namespace rpca {

int sweep_blocks_for(int64_t m, int64_t n, int k, int* row_groups, int* strips_per_wg,
                     int* chunk_w, int* nchunks) {
  const int cw = (k <= 16) ? 256 : 128;
  const int nch = (int)((n + cw - 1) / cw);
  const int64_t nstrips = (m + 15) / 16;
  int64_t target = (1024 + nch - 1) / nch;
  if (target < 1) target = 1;
  int64_t spw = (nstrips + target - 1) / target;
  spw = ((spw + WAVES - 1) / WAVES) * WAVES;
  if (spw < WAVES) spw = WAVES;
  const int64_t rgs = (nstrips + spw - 1) / spw;
  *row_groups = (int)rgs;
  *strips_per_wg = (int)spw;
  *chunk_w = cw;
  *nchunks = nch;
  return (int)(rgs * nch);
}

hipError_t launch_sweep(const SweepArgs& sa, bool trial, bool bf16, hipStream_t stream) {
  (void)bf16;
  const dim3 grid(sa.row_groups, sa.nchunks);
  const bool vec4 = (sa.m % 4) == 0;
  if (sa.mask)
    return trial ? launch_sweep_m<true, true>(sa, vec4, grid, stream)
                 : launch_sweep_m<true, false>(sa, vec4, grid, stream);
  return trial ? launch_sweep_m<false, true>(sa, vec4, grid, stream)
               : launch_sweep_m<false, false>(sa, vec4, grid, stream);
}

hipError_t launch_finish(const FinishArgs& fa, bool trial, hipStream_t stream) {
  const int gvb = (int)((fa.n * fa.k + THREADS - 1) / THREADS);
  int gub = 0;
  if (fa.nchunks > 1) {
    gub = (int)((fa.m * fa.k + THREADS * 8 - 1) / (THREADS * 8));
    if (gub > 1024) gub = 1024;
  }
  FinishArgs f2 = fa;
  f2.gv_blocks = gvb;
  const dim3 fgrid(gvb + gub, fa.segs);
  if (trial)
    hipLaunchKernelGGL((k_objgrad_finish<true>), fgrid, dim3(THREADS), 0, stream, f2);
  else
    hipLaunchKernelGGL((k_objgrad_finish<false>), fgrid, dim3(THREADS), 0, stream, f2);
  return hipGetLastError();
}

hipError_t launch_objgrad(const SweepArgs& sa, const FinishArgs& fa, bool trial, bool bf16,
                          hipStream_t stream) {
  const hipError_t e = launch_sweep(sa, trial, bf16, stream);
  if (e != hipSuccess) return e;
  return launch_finish(fa, trial, stream);
}

}  // namespace rpca
