// Fused thin Gram product Z = Op^T (Op W) in one pass over X, for rank k <= 16
// and n <= 256 columns (one chunk of at most 16 column tiles).
//
// Op is the certificate's gradient operator G = Omega .* rho'(U V^T - X) (the
// residual source; its power iteration on M^T M needs D^T D x = G^T G x / lam_L^2,
// Sec. 3.4) or the data Omega .* X (the randomized-SVD start's subspace iteration
// on A^T A, Sec. 4.2).  The separate left and right sweeps read X twice and
// carry FP64 vectors; here each 16-row strip of a wave
//   1. forms its G tiles exactly as the objective sweep does (MFMA with the
//      accumulator seeded by X and the A operand -U, then the clip), keeps them
//      in registers and accumulates Y_s = G_s W (16 x 16, through the per-wave
//      transpose tile, W staged in LDS in the objective sweep's G V layout);
//   2. once the strip's Y_s is complete, adds G_s^T Y_s to the per-tile Z
//      accumulators: Y_s is already in the B-operand layout of that product
//      (rows 4g + r of column c in lane (g, c)) and the G tiles in its A layout.
// Products and the per-workgroup sums are FP32 (MFMA), the sums over workgroups
// FP64 in a fixed order (two small kernels).  With the residual source the
// kernel computes (-G)^T (-G W) = G^T G W, so no negation is needed.
#include "sweep_kernel.h"

namespace {

using rpca_sweep::BUF_DWORD3;
using rpca_sweep::f4;
using rpca_sweep::mfma_f32;
using rpca_sweep::NT;
using rpca_sweep::WAVES;
using namespace rpca_sweep::k16;

constexpr int GA_TMAX = 16;  // column tiles (n <= 256)
constexpr int GA_PF = 4;     // tiles per load group
constexpr int GA_NG = GA_TMAX / GA_PF;

template <bool RESID, bool MASKED>
__global__ __launch_bounds__(NT, 1) void k_gram_apply(rpca::GramApplyArgs a) {
  if (a.skip && *a.skip != 0.0) return;
  extern __shared__ float lds[];
  constexpr int TMAX = GA_TMAX, PF = GA_PF, NG = GA_NG, NBUF = 4, D = NBUF - 1;  // three groups in flight
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c = lane & 15, g = lane >> 4;
  const int64_t m = a.m, n = a.n;
  const int k = a.k;
  const float lam_s = a.lam_s, kappa = a.kappa;
  const float* __restrict__ U = a.U;
  const float* __restrict__ X = a.X;
  const int ncols = (int)n;
  const int ntiles = (ncols + 15) >> 4;
  const int cwp = ntiles * 16;
  float* sVr = lds;                    // [cwp][RS]   residual operand: V[col][4q + g]
  float* sWg = lds + cwp * RS;         // [ntiles][256] W[16t + 4q + g][c]
  float* sT = sWg + ntiles * 256;      // per-wave transpose tiles
  float* myT = sT + w * NTB * 16 * TS;

  // strips of this workgroup: whole pairs of strips, waves interleaved (as the sweep)
  const int64_t nstrips = (m + 15) >> 4;
  const int64_t R = gridDim.x, rg = blockIdx.x;
  const int64_t npairs = (nstrips + 1) >> 1;
  const int64_t s_lo = 2 * (rg * npairs / R);
  const int64_t s_hi_p = 2 * ((rg + 1) * npairs / R);
  const int64_t s_hi = s_hi_p < nstrips ? s_hi_p : nstrips;
  const int64_t s_first = s_lo + w;
  int64_t n_all = 0;
  if (s_first < s_hi) n_all = (s_hi - s_first + WAVES - 1) / WAVES;
  const bool vec = a.xvec != 0 && (int64_t)cwp * m * 4 < ((int64_t)1 << 31);
  const int64_t full_lim = vec ? (m >> 4) : 0;
  int64_t n_pipe = 0;
  if (s_first < full_lim) {
    n_pipe = (full_lim - s_first + WAVES - 1) / WAVES;
    if (n_pipe > n_all) n_pipe = n_all;
  }

  // residual A operand of the strip: -U[row c][4q + g] (rows past m and ranks past k: 0)
  auto load_ua = [&](int64_t s, float (&ua)[4]) {
    if (!RESID) return;
    const int64_t i0 = s * 16;
    const int rows_in = (i0 + 16 <= m) ? 16 : (int)(m - i0);
    const bool row_ok = c < rows_in;
    const int rc = row_ok ? c : rows_in - 1;
    const float* __restrict__ Us = U + i0 * k;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int kk = 4 * q + g;
      const float v = Us[(uint32_t)(rc * k + (kk < k ? kk : k - 1))];
      ua[q] = (kk < k && row_ok) ? -v : 0.f;
    }
  };

  const __amdgpu_buffer_rsrc_t xrs =
      __builtin_amdgcn_make_buffer_rsrc((void*)X, (short)0, (int)((int64_t)ncols * m * 4), BUF_DWORD3);
  const uint32_t lane_off = (uint32_t)(c * m * 4 + 16 * g);
  auto load_group = [&](int64_t s, int gi, f4(&xr)[PF], uint32_t(&br)[PF], bool live) {
    // column offset in the VGPR offset (covered by the buffer range check)
    const uint32_t voff = live ? lane_off + (uint32_t)(s * 64) : 0xC0000000u;
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int t = gi * PF + u;
      xr[u] = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(xrs, voff + (uint32_t)(64 * t * m), 0, 0));
      if (MASKED && 16 * t < ncols) {
        const int jl = 16 * t + c;
        const int64_t i0 = s * 16;
        const uint32_t* __restrict__ mrow = a.mask + (int64_t)(16 * t) * a.mw + (i0 >> 5);
        const uint32_t moff = (uint32_t)(((jl < ncols) ? c : (ncols - 1 - 16 * t)) * a.mw);
        br[u] = (mrow[moff] >> ((int)(i0 & 31) + 4 * g)) & 0xFu;
      }
    }
  };

  float Gs[TMAX][4];
  f4 za[TMAX];
#pragma unroll
  for (int t = 0; t < TMAX; ++t) za[t] = f4{0.f, 0.f, 0.f, 0.f};

  // One group of PF tiles of the current strip: operator values into Gs and the
  // transpose tiles, then Y += G W.
  auto tile_group = [&](int gi, const float (&ua)[4], f4(&xr)[PF], const uint32_t(&br)[PF], f4& y) {
    if (RESID) {
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int t = gi * PF + u;
        if (t >= ntiles) continue;
        const f4 vr = *reinterpret_cast<const f4*>(sVr + (16 * t + c) * RS + g * 4);
        xr[u] = mfma_f32(ua[0], vr[0], xr[u]);
        xr[u] = mfma_f32(ua[1], vr[1], xr[u]);
        xr[u] = mfma_f32(ua[2], vr[2], xr[u]);
        if (k > 12) xr[u] = mfma_f32(ua[3], vr[3], xr[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int t = gi * PF + u;
      if (t >= ntiles) continue;
      const int jl = 16 * t + c;
      const uint32_t bits = MASKED ? ((jl < ncols) ? br[u] : 0u) : 0xFu;
      float* tT = myT + u * 16 * TS;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float v = xr[u][r];
        if (RESID) {
          // -rho'(R) from the negated residual (clip, elastic slope beyond it)
          const float cl = __builtin_amdgcn_fmed3f(v, -lam_s, lam_s);
          v = kappa != 0.f ? fmaf(kappa, v - cl, cl) : cl;
        }
        if (MASKED && !((bits >> r) & 1u)) v = 0.f;
        Gs[t][r] = v;
        tT[(4 * g + r) * TS + (c & 3) * 4 + (c >> 2)] = v;
      }
    }
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int t = gi * PF + u;
      if (t >= ntiles) continue;
      const f4 gt = *reinterpret_cast<const f4*>(myT + u * 16 * TS + c * TS + g * 4);
      const f4 wg = *reinterpret_cast<const f4*>(sWg + t * 256 + g * 64 + c * 4);
#pragma unroll
      for (int q = 0; q < 4; ++q) y = mfma_f32(gt[q], wg[q], y);
    }
  };

  // Z_t += G_t^T Y for every tile of the strip
  auto strip_end = [&](const f4& y) {
#pragma unroll
    for (int t = 0; t < TMAX; ++t) {
      if (t >= ntiles) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) za[t] = mfma_f32(Gs[t][r], y[r], za[t]);
    }
  };

  float ua[4] = {0.f, 0.f, 0.f, 0.f}, nua[4] = {0.f, 0.f, 0.f, 0.f};
  f4 xbuf[NBUF][PF];
  uint32_t bbuf[NBUF][PF] = {};
  if (n_pipe > 0) {
    load_ua(s_first, ua);
#pragma unroll
    for (int d = 0; d < D; ++d) load_group(s_first, d, xbuf[d], bbuf[d], true);
  }

  // ---- stage V (residual operand) and W ----
  if (RESID) {
    for (int idx = tid; idx < cwp * 4; idx += NT) {
      const int jl = idx >> 2, gg = idx & 3;
      f4 v4;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int kk = 4 * q + gg;
        v4[q] = (jl < ncols && kk < k) ? a.V[(int64_t)jl * k + kk] : 0.f;
      }
      *reinterpret_cast<f4*>(sVr + jl * RS + gg * 4) = v4;
    }
  }
  for (int idx = tid; idx < ntiles * 64; idx += NT) {
    const int t = idx >> 6, gg = (idx >> 4) & 3, cc = idx & 15;
    f4 w4;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = 16 * t + 4 * q + gg;
      w4[q] = j < ncols ? a.W[(int64_t)j * 16 + cc] : 0.f;
    }
    *reinterpret_cast<f4*>(sWg + idx * 4) = w4;
  }
  __syncthreads();

  for (int64_t j = 0; j < n_pipe; ++j) {
    const int64_t s = s_first + WAVES * j;
    const bool more = j + 1 < n_pipe;
    const int64_t sn = more ? s + WAVES : s;
    f4 y = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
      const int ga = gi + D;
      if (ga < NG) {
        if (ga * PF < ntiles) load_group(s, ga, xbuf[ga % NBUF], bbuf[ga % NBUF], true);
      } else {
        if (ga == NG) load_ua(sn, nua);
        load_group(sn, ga - NG, xbuf[ga % NBUF], bbuf[ga % NBUF], more);
      }
      __builtin_amdgcn_sched_barrier(0);
      if (gi * PF < ntiles) tile_group(gi, ua, xbuf[gi % NBUF], bbuf[gi % NBUF], y);
    }
    strip_end(y);
#pragma unroll
    for (int q = 0; q < 4; ++q) ua[q] = nua[q];
  }
  // remaining strips (ragged last strip, or X without vector alignment): element loads
  for (int64_t j = n_pipe; j < n_all; ++j) {
    const int64_t s = s_first + WAVES * j;
    float ub[4];
    load_ua(s, ub);
    f4 y = f4{0.f, 0.f, 0.f, 0.f};
    const int64_t i0 = s * 16;
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
      if (gi * PF >= ntiles) continue;
      f4 xr[PF];
      uint32_t br[PF] = {};
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int t = gi * PF + u;
        xr[u] = f4{0.f, 0.f, 0.f, 0.f};
        if (t < ntiles) {
          const int jl = 16 * t + c;
          const int64_t jc = jl < ncols ? jl : ncols - 1;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t i = i0 + 4 * g + r;
            const float xv = X[jc * m + (i < m ? i : m - 1)];
            xr[u][r] = (i < m && jl < ncols) ? xv : 0.f;
          }
          if (MASKED) br[u] = (a.mask[jc * a.mw + (i0 >> 5)] >> ((int)(i0 & 31) + 4 * g)) & 0xFu;
        }
      }
      tile_group(gi, ub, xr, br, y);
    }
    strip_end(y);
  }

  // ---- the waves' Z accumulators through LDS (over the start layout), fixed order ----
  __syncthreads();
  float* sZ = lds + w * cwp * 16;
#pragma unroll
  for (int t = 0; t < TMAX; ++t) {
    if (t < ntiles) {
#pragma unroll
      for (int r = 0; r < 4; ++r) sZ[(16 * t + 4 * g + r) * 16 + c] = za[t][r];
    }
  }
  __syncthreads();
  float* zp = a.part + rg * n * 16;
  for (int idx = tid; idx < ncols * 16; idx += NT) {
    float acc = 0.f;
#pragma unroll
    for (int ww = 0; ww < WAVES; ++ww) acc += lds[ww * cwp * 16 + idx];
    zp[idx] = acc;
  }
}

// Z[j * ldz + col0 + p] = scale * (sum over workgroups r of part[r][j * 16 + p]), p < b.
// One pass: a block takes GR_OUT consecutive outputs; its GR_SL row slices sum
// workgroups sl, sl + GR_SL, ... in FP64 (all loads of a slice in flight at
// once), then one thread per output adds the slices in slice order.  The order
// depends only on the number of workgroups.
constexpr int GR_OUT = 16, GR_SL = 16, GR_INF = 16;
__global__ __launch_bounds__(256) void k_ga_reduce(const float* __restrict__ part, int64_t n, int rows, int b,
                                                   double scale, double* __restrict__ Z, int ldz, int col0,
                                                   const double* __restrict__ skip) {
  if (skip && *skip != 0.0) return;
  __shared__ double sh[GR_SL][GR_OUT + 1];
  const int oo = threadIdx.x & (GR_OUT - 1), sl = threadIdx.x / GR_OUT;
  const int64_t outs = n * b;
  const int64_t o = (int64_t)blockIdx.x * GR_OUT + oo;
  const int64_t oc = o < outs ? o : outs - 1;
  const int64_t j = oc / b;
  const int64_t src = j * 16 + (oc - j * b);
  const int64_t stride = n * 16;
  double s = 0.0;
  for (int r0 = sl; r0 < rows; r0 += GR_SL * GR_INF) {
    float x[GR_INF];
#pragma unroll
    for (int e = 0; e < GR_INF; ++e) {  // clamped rows: every load issued before the first use
      const int r = r0 + e * GR_SL;
      x[e] = part[(int64_t)(r < rows ? r : rows - 1) * stride + src];
    }
#pragma unroll
    for (int e = 0; e < GR_INF; ++e) s += r0 + e * GR_SL < rows ? (double)x[e] : 0.0;
  }
  sh[sl][oo] = s;
  __syncthreads();
  if (sl == 0 && o < outs) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < GR_SL; ++q) t += sh[q][oo];
    Z[j * ldz + col0 + (o - j * b)] = scale * t;
  }
}

}  // namespace

namespace rpca {

size_t gram_apply_lds_bytes(int64_t n) {
  const int ntiles = (int)((n + 15) / 16), cwp = ntiles * 16;
  const int start = cwp * RS + ntiles * 256 + WAVES * NTB * 16 * TS;
  const int end = WAVES * cwp * 16;
  return (size_t)(start > end ? start : end) * sizeof(float);
}

bool gram_apply_fits(int64_t n, int k) { return n >= 1 && n <= 16 * GA_TMAX && k >= 0 && k <= 16; }

hipError_t launch_gram_apply_pass(const GramApplyArgs& a, bool resid, hipStream_t s) {
  if (!gram_apply_fits(a.n, resid ? a.k : 0) || a.row_groups < 1) return hipErrorInvalidValue;
  const size_t lb = gram_apply_lds_bytes(a.n);
  const dim3 grid((unsigned)a.row_groups);
  if (resid) {
    if (a.mask) hipLaunchKernelGGL((k_gram_apply<true, true>), grid, dim3(NT), lb, s, a);
    else hipLaunchKernelGGL((k_gram_apply<true, false>), grid, dim3(NT), lb, s, a);
  } else {
    if (a.mask) hipLaunchKernelGGL((k_gram_apply<false, true>), grid, dim3(NT), lb, s, a);
    else hipLaunchKernelGGL((k_gram_apply<false, false>), grid, dim3(NT), lb, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_gram_apply_sum(const GramApplyArgs& a, double* Z, int ldz, int col0, int b, double scale,
                                 hipStream_t s) {
  if (a.n < 1 || b < 1 || b > 16 || a.row_groups < 1) return hipErrorInvalidValue;
  const int64_t outs = a.n * b;
  hipLaunchKernelGGL(k_ga_reduce, dim3((unsigned)((outs + GR_OUT - 1) / GR_OUT)), dim3(GR_OUT * GR_SL), 0, s,
                     (const float*)a.part, a.n, a.row_groups, b, scale, Z, ldz, col0, a.skip);
  return hipGetLastError();
}

hipError_t launch_gram_apply(const GramApplyArgs& a, bool resid, double* Z, int ldz, int col0, int b, double scale,
                             hipStream_t s) {
  if (b < 1 || b > 16) return hipErrorInvalidValue;
  const hipError_t e = launch_gram_apply_pass(a, resid, s);
  if (e != hipSuccess) return e;
  return launch_gram_apply_sum(a, Z, ldz, col0, b, scale, s);
}

}  // namespace rpca
