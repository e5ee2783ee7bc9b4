// Convergence certificate (Sec. 3.4) and randomized-SVD start (Sec. 4.2).
//
// Both need thin products with the m x n operator G = Omega .* clip(U V^T - X)
// (the certificate, D = G / lam_L) or with A = P_Omega(X) (the rSVD).  Two
// sweeps cover every case, in FP64 for the vectors and the accumulation:
//   left : Y = Op W    (W is n x b, Y is m x b; rows of a strip complete in-wave)
//   right: Z = Op^T Y  (Y is m x b, Z is n x b; per-row-group partials, fixed-order sum)
// The residual tile is recomputed in registers exactly as in the objective
// sweep (MFMA with the accumulator seeded by -X), so nothing of size m x n is
// ever stored.
//
// Certificate terms.  With the factor SVD of the footnote of Sec. 3.4 written
// as U1 = U T_U, V1 = V T_V (T from the eigen-decompositions of U^T U, V^T V
// and the SVD of R_U R_V^T), every term except the last needs only k x k
// Gram matrices of [U, G V] and [V, G^T U], which one objective sweep provides:
//   T1 = ||I + U1^T D V1||^2,   T2 = ||D^T U1 - V1 C^T||^2,   T3 = ||D V1 - U1 C||^2
// (C = U1^T D V1; T2 and T3 summed entry by entry over the n x r and m x r blocks
// in FP64 by one thin pass each), and ||P_U^perp D P_V^perp||_F^2 follows from
// ||G||_F^2 and the Gram traces.  T4 =
// sum (sigma_i(P_U^perp D P_V^perp) - 1)_+^2 replaces the (m-r) x (n-r) SVD of the
// paper by block power iteration on M^T M with M = P_U^perp D P_V^perp, applied
// as P_V^perp (D^T D x' - B B^T x'), x' = P_V^perp x, B = D^T U1: one left and one
// right sweep per iteration.  Ritz values are lower bounds of the singular
// values; T4 is reported as an estimate with the iteration count.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "rpca_internal.h"
#include "ritz_kernel.h"
#include "smalllinalg.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int THREADS = 256;
constexpr int WAVES = 4;
constexpr int BP = 8;      // columns per pass of a thin product
constexpr int RJT = 4;     // 16-column tiles per chunk of the right sweep
constexpr size_t LEFT_LDS_MAX = 48 * 1024;  // W and V staged in LDS up to this size

// Operator sources: the gradient G = Omega .* rho'(U V^T - X) (residual), the data
// Omega .* X, or the proximal-gradient point Z = U V^T - G (every entry observed).
enum { SRC_RESID = 0, SRC_DATA = 1, SRC_PROX = 2 };

struct GArgs {
  const float* X;
  const uint32_t* mask;
  int64_t m, n;
  int32_t k, mw;
  float lam_s;
  float kappa;     // elastic-net slope beyond lam_s (0: l1)
  const float* U;  // residual source only
  const float* V;
  const double* W;  // left: n x ldw
  int32_t ldw;
  double* Y;        // left: output m x ldy; right: input m x ldy
  int32_t ldy;
  int32_t col0, bw;  // columns [col0, col0 + bw) of this pass (bw <= BP)
  double* part;      // right: [row_groups][n * BP]
  int32_t strips_per_wg, nchunks, row_groups;
};

// rho'(R): clip(R, +-lam_s), continued with slope kappa beyond the threshold
// (elastic net; kappa = 0 is the l1 clip).
__device__ __forceinline__ float grad_rho(float R, float lam_s, float kappa) {
  const float c = fminf(fmaxf(R, -lam_s), lam_s);
  return kappa != 0.f ? fmaf(kappa, R - c, c) : c;
}

// Operator value of one entry from the residual r = (U V^T - X)_ij and x = X_ij.
template <int SRC>
__device__ __forceinline__ float op_value(float r, float x, float lam_s, float kappa) {
  const float g = grad_rho(r, lam_s, kappa);
  return SRC == SRC_PROX ? (x + r) - g : g;
}

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Loads of one 16-column tile of the operator for the 4 rows i0+4g+r of column
// j (held by lane (g, c)): X (one 16-byte load when the strip lies inside X and
// X allows vector loads), the residual's V operands and the mask bits.  Split
// from the arithmetic (tile_op) so that the next tile's loads are in flight
// while the current tile is computed.  Columns past n load column n-1 (in
// bounds) and are zeroed by tile_op.
struct TileIn {
  f4 x;
  float vb[8];
  uint32_t bits;
};

template <int SRC, bool MASKED>
__device__ __forceinline__ void tile_load(const GArgs& a, int64_t i0, int64_t j, bool jok, bool vec, int KS,
                                          TileIn& t) {
  const int lane = threadIdx.x & 63, g = lane >> 4;
  const int64_t jc = jok ? j : a.n - 1;
  const float* col = a.X + jc * a.m;
  if (vec) {
    t.x = *reinterpret_cast<const f4*>(col + i0 + 4 * g);
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t i = i0 + 4 * g + r;
      t.x[r] = col[i < a.m ? i : a.m - 1];
    }
  }
  t.bits = 0xFu;
  if (MASKED) t.bits = (a.mask[jc * a.mw + (i0 >> 5)] >> ((int)(i0 & 31) + 4 * g)) & 0xFu;
  if (SRC != SRC_DATA) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (q < KS) {
        const int kk = 4 * q + g;
        t.vb[q] = a.V[jc * a.k + (kk < a.k ? kk : a.k - 1)];
      }
    }
  }
}

// Operator values of a loaded tile: G = Omega .* clip(U V^T - X) (residual) or
// Omega .* X (data), zero outside the matrix.
template <int SRC, bool MASKED>
__device__ __forceinline__ void tile_op(const GArgs& a, const TileIn& t, int64_t i0, bool jok, const float (&ua)[8],
                                        int KS, float (&G)[4]) {
  const int lane = threadIdx.x & 63, g = lane >> 4;
  float x[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) x[r] = (jok && i0 + 4 * g + r < a.m) ? t.x[r] : 0.f;
  if (SRC != SRC_DATA) {
    f4 acc = f4{-x[0], -x[1], -x[2], -x[3]};
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (q < KS) {
        const int kk = 4 * q + g;
        acc = mfma4(ua[q], (jok && kk < a.k) ? t.vb[q] : 0.f, acc);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) G[r] = op_value<SRC>(acc[r], x[r], a.lam_s, a.kappa);
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) G[r] = x[r];
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (MASKED && !(jok && ((t.bits >> r) & 1u))) G[r] = 0.f;
}

template <int SRC>
__device__ __forceinline__ void load_ua(const GArgs& a, int64_t i0, int KS, float (&ua)[8]) {
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  const int64_t i = i0 + c < a.m ? i0 + c : a.m - 1;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int kk = 4 * q + g;
    float v = 0.f;
    if (SRC != SRC_DATA && q < KS) v = a.U[i * a.k + (kk < a.k ? kk : a.k - 1)];
    ua[q] = (SRC != SRC_DATA && q < KS && kk < a.k && i0 + c < a.m) ? v : 0.f;
  }
}

// X may be read 16 bytes at a time for strips that lie inside it.
__device__ __forceinline__ bool x_vec_ok(const GArgs& a, int64_t i0) {
  return ((reinterpret_cast<uintptr_t>(a.X) & 15) == 0) && ((a.m & 3) == 0) && (i0 + 16 <= a.m);
}

// Y[:, col0 + p] = Op W[:, col0 + p] (p < bw).  Wave = 16-row strip; the strip's
// column tiles are double-buffered (the loads of tile j0 + 16, X, V, W rows and
// mask, are issued before tile j0 is computed).
template <int SRC, bool MASKED>
__global__ __launch_bounds__(THREADS) void k_left(GArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int KS = (a.k + 3) >> 2;
  const int64_t nstrips = (a.m + 15) >> 4;
  const int64_t s_begin = (int64_t)blockIdx.x * a.strips_per_wg;
  int64_t s_end = s_begin + a.strips_per_wg;
  if (s_end > nstrips) s_end = nstrips;
  auto load_w = [&](int64_t j, bool jok, double (&w)[BP]) {
    const int64_t jc = jok ? j : a.n - 1;
#pragma unroll
    for (int p = 0; p < BP; ++p) w[p] = (p < a.bw) ? a.W[jc * a.ldw + a.col0 + p] : 0.0;
  };
  for (int64_t s = s_begin + wave; s < s_end; s += WAVES) {
    const int64_t i0 = s * 16;
    const bool vec = x_vec_ok(a, i0);
    float ua[8];
    load_ua<SRC>(a, i0, KS, ua);
    double acc[4][BP];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int p = 0; p < BP; ++p) acc[r][p] = 0.0;
    auto step = [&](const TileIn& t, const double (&w)[BP], int64_t j, bool jok) {
      float G[4];
      tile_op<SRC, MASKED>(a, t, i0, jok, ua, KS, G);
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int p = 0; p < BP; ++p) acc[r][p] = fma((double)G[r], jok ? w[p] : 0.0, acc[r][p]);
    };
    TileIn t0, t1;
    double w0[BP], w1[BP];
    tile_load<SRC, MASKED>(a, i0, c, c < a.n, vec, KS, t0);
    load_w(c, c < a.n, w0);
    for (int64_t j0 = 0; j0 < a.n; j0 += 32) {
      const int64_t ja = j0 + c, jb = j0 + 16 + c;
      const bool more = j0 + 16 < a.n;
      if (more) {
        tile_load<SRC, MASKED>(a, i0, jb, jb < a.n, vec, KS, t1);
        load_w(jb, jb < a.n, w1);
      }
      step(t0, w0, ja, ja < a.n);
      if (more) {
        const int64_t jn = j0 + 32 + c;
        if (j0 + 32 < a.n) {
          tile_load<SRC, MASKED>(a, i0, jn, jn < a.n, vec, KS, t0);
          load_w(jn, jn < a.n, w0);
        }
        step(t1, w1, jb, jb < a.n);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int p = 0; p < BP; ++p) {
        double v = acc[r][p];
        v += __shfl_xor(v, 1, 64);
        v += __shfl_xor(v, 2, 64);
        v += __shfl_xor(v, 4, 64);
        v += __shfl_xor(v, 8, 64);
        acc[r][p] = v;
      }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t i = i0 + 4 * g + r;
      double sel = 0.0;
#pragma unroll
      for (int p = 0; p < BP; ++p) sel = (p == c) ? acc[r][p] : sel;
      if (c < a.bw && i < a.m) a.Y[i * a.ldy + a.col0 + c] = sel;
    }
  }
}

// Y[:, col0 + p] = Op W[:, col0 + p] (p < bw) with W (and V, for the residual)
// staged in LDS once per workgroup, so the only global loads of the strip loop
// are X: each strip issues the X loads of LB column tiles at once (one latency
// per LB tiles instead of one per tile).  Used when W and V fit the LDS budget.
constexpr int LB = 8;
template <int SRC, bool MASKED>
__global__ __launch_bounds__(THREADS) void k_left_lds(GArgs a) {
  extern __shared__ double lds_left[];
  constexpr int LW = BP + 1;                              // padded row: 16 columns hit distinct banks
  double* sW = lds_left;                                  // [n][LW]
  float* sV = reinterpret_cast<float*>(sW + a.n * LW);    // [n][k] (residual only)
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c = lane & 15, g = lane >> 4;
  const int KS = (a.k + 3) >> 2;
  {
    const int64_t nw = a.n * BP;
    for (int64_t base = threadIdx.x; base < nw; base += 4 * THREADS) {
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t idx = base + u * THREADS;
        const int p = (int)(idx % BP);
        v[u] = (idx < nw && p < a.bw) ? a.W[(idx / BP) * a.ldw + a.col0 + p] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t idx = base + u * THREADS;
        if (idx < nw) sW[(idx / BP) * LW + idx % BP] = v[u];
      }
    }
    if (SRC != SRC_DATA) {
      const int64_t nv = a.n * a.k;
      for (int64_t base = threadIdx.x; base < nv; base += 4 * THREADS) {
        float v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = (base + u * THREADS < nv) ? a.V[base + u * THREADS] : 0.f;
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (base + u * THREADS < nv) sV[base + u * THREADS] = v[u];
      }
    }
  }
  __syncthreads();
  const int64_t nstrips = (a.m + 15) >> 4;
  const int64_t s_begin = (int64_t)blockIdx.x * a.strips_per_wg;
  int64_t s_end = s_begin + a.strips_per_wg;
  if (s_end > nstrips) s_end = nstrips;
  for (int64_t s = s_begin + wave; s < s_end; s += WAVES) {
    const int64_t i0 = s * 16;
    const bool vec = x_vec_ok(a, i0);
    float ua[8];
    load_ua<SRC>(a, i0, KS, ua);
    double acc[4][BP];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int p = 0; p < BP; ++p) acc[r][p] = 0.0;
    for (int64_t jb = 0; jb < a.n; jb += 16 * LB) {
      f4 xs[LB];
      uint32_t bits[LB];
#pragma unroll
      for (int t = 0; t < LB; ++t) {
        if (jb + 16 * t < a.n) {
          const int64_t j = jb + 16 * t + c;
          const int64_t jc = j < a.n ? j : a.n - 1;
          const float* col = a.X + jc * a.m;
          if (vec) {
            xs[t] = *reinterpret_cast<const f4*>(col + i0 + 4 * g);
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int64_t i = i0 + 4 * g + r;
              xs[t][r] = col[i < a.m ? i : a.m - 1];
            }
          }
          bits[t] = MASKED ? (a.mask[jc * a.mw + (i0 >> 5)] >> ((int)(i0 & 31) + 4 * g)) & 0xFu : 0xFu;
        }
      }
#pragma unroll
      for (int t = 0; t < LB; ++t) {
        if (jb + 16 * t < a.n) {
          const int64_t j = jb + 16 * t + c;
          const bool jok = j < a.n;
          const int64_t jc = jok ? j : a.n - 1;
          float G[4];
          float x[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) x[r] = (jok && i0 + 4 * g + r < a.m) ? xs[t][r] : 0.f;
          if (SRC != SRC_DATA) {
            f4 r4 = f4{-x[0], -x[1], -x[2], -x[3]};
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              if (q < KS) {
                const int kk = 4 * q + g;
                r4 = mfma4(ua[q], (jok && kk < a.k) ? sV[jc * a.k + kk] : 0.f, r4);
              }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) G[r] = op_value<SRC>(r4[r], x[r], a.lam_s, a.kappa);
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) G[r] = x[r];
          }
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (!jok || (MASKED && !((bits[t] >> r) & 1u))) G[r] = 0.f;
          double w[BP];
#pragma unroll
          for (int p = 0; p < BP; ++p) w[p] = sW[jc * LW + p];
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int p = 0; p < BP; ++p) acc[r][p] = fma((double)G[r], w[p], acc[r][p]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int p = 0; p < BP; ++p) {
        double v = acc[r][p];
        v += __shfl_xor(v, 1, 64);
        v += __shfl_xor(v, 2, 64);
        v += __shfl_xor(v, 4, 64);
        v += __shfl_xor(v, 8, 64);
        acc[r][p] = v;
      }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t i = i0 + 4 * g + r;
      double sel = 0.0;
#pragma unroll
      for (int p = 0; p < BP; ++p) sel = (p == c) ? acc[r][p] : sel;
      if (c < a.bw && i < a.m) a.Y[i * a.ldy + a.col0 + c] = sel;
    }
  }
}

// LDS bytes of k_left_lds for n columns and rank k (0 residual / 1 data).
size_t left_lds_bytes(int64_t n, int k, int src) {
  return (size_t)n * (BP + 1) * 8 + (src != SRC_DATA ? (size_t)n * k * 4 : 0);
}

// Per-row-group partials of Z[:, col0 + p] = Op^T Y[:, col0 + p] over one chunk of
// RJT column tiles (wave = every WAVES-th strip of the row group), with the
// chunk's V columns staged in LDS and each strip's Y rows brought in once per wave (lane l loads two of the strip's 16 x BP values into
// LDS; every lane then reads its rows from there instead of 32 scattered global
// loads).  The next strip's X tiles, Y values and U rows are loaded into
// registers while the current strip is computed.
template <int SRC, bool MASKED>
__global__ __launch_bounds__(THREADS) void k_right_lds(GArgs a) {
  __shared__ double sZ[RJT * 16 * BP];
  __shared__ float sV[RJT * 16 * 32];
  __shared__ double sY[WAVES][16 * BP];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c = lane & 15, g = lane >> 4;
  const int KS = (a.k + 3) >> 2;
  const int rg = blockIdx.x, ch = blockIdx.y;
  const int64_t j_begin = (int64_t)ch * RJT * 16;
  const int ncols = (int)((a.n - j_begin) < RJT * 16 ? (a.n - j_begin) : RJT * 16);
  if (SRC != SRC_DATA)
    for (int idx = threadIdx.x; idx < ncols * a.k; idx += THREADS) sV[idx] = a.V[j_begin * a.k + idx];
  __syncthreads();
  const int64_t nstrips = (a.m + 15) >> 4;
  const int64_t s_begin = (int64_t)rg * a.strips_per_wg;
  int64_t s_end = s_begin + a.strips_per_wg;
  if (s_end > nstrips) s_end = nstrips;
  double z[RJT][BP];
#pragma unroll
  for (int t = 0; t < RJT; ++t)
#pragma unroll
    for (int p = 0; p < BP; ++p) z[t][p] = 0.0;
  struct StripIn {
    float ua[8];
    double y2[2];  // Y[i0 + lane/4][col0 + 2 (lane%4) + {0, 1}]
    f4 x[RJT];
    uint32_t bits[RJT];
  };
  const int yrow = lane >> 2, yp = 2 * (lane & 3);
  auto load_strip = [&](int64_t s, StripIn& S) {
    const int64_t i0 = s * 16;
    const bool vec = x_vec_ok(a, i0);
    load_ua<SRC>(a, i0, KS, S.ua);
    const int64_t iy = (i0 + yrow < a.m) ? i0 + yrow : a.m - 1;
#pragma unroll
    for (int e = 0; e < 2; ++e) S.y2[e] = (yp + e < a.bw) ? a.Y[iy * a.ldy + a.col0 + yp + e] : 0.0;
#pragma unroll
    for (int t = 0; t < RJT; ++t) {
      if (t * 16 < ncols) {
        const int jl = t * 16 + c;
        const int64_t jc = j_begin + (jl < ncols ? jl : ncols - 1);
        const float* col = a.X + jc * a.m;
        if (vec) {
          S.x[t] = *reinterpret_cast<const f4*>(col + i0 + 4 * g);
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t i = i0 + 4 * g + r;
            S.x[t][r] = col[i < a.m ? i : a.m - 1];
          }
        }
        S.bits[t] = MASKED ? (a.mask[jc * a.mw + (i0 >> 5)] >> ((int)(i0 & 31) + 4 * g)) & 0xFu : 0xFu;
      }
    }
  };
  auto compute_strip = [&](int64_t s, const StripIn& S) {
    const int64_t i0 = s * 16;
    double* y = sY[wave];
    y[yrow * BP + yp] = (i0 + yrow < a.m) ? S.y2[0] : 0.0;
    y[yrow * BP + yp + 1] = (i0 + yrow < a.m) ? S.y2[1] : 0.0;
    // the wave's own LDS writes are visible to its later reads (in order within a wave)
#pragma unroll
    for (int t = 0; t < RJT; ++t) {
      if (t * 16 < ncols) {
        const int jl = t * 16 + c;
        const bool jok = jl < ncols;
        float x[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) x[r] = (jok && i0 + 4 * g + r < a.m) ? S.x[t][r] : 0.f;
        float G[4];
        if (SRC != SRC_DATA) {
          f4 r4 = f4{-x[0], -x[1], -x[2], -x[3]};
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            if (q < KS) {
              const int kk = 4 * q + g;
              r4 = mfma4(S.ua[q], (jok && kk < a.k) ? sV[jl * a.k + kk] : 0.f, r4);
            }
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) G[r] = op_value<SRC>(r4[r], x[r], a.lam_s, a.kappa);
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r) G[r] = x[r];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (!jok || (MASKED && !((S.bits[t] >> r) & 1u))) G[r] = 0.f;
#pragma unroll
        for (int p = 0; p < BP; ++p) {
          double v = z[t][p];
#pragma unroll
          for (int r = 0; r < 4; ++r) v = fma((double)G[r], y[(4 * g + r) * BP + p], v);
          z[t][p] = v;
        }
      }
    }
  };
  int64_t s = s_begin + wave;
  if (s < s_end) {
    StripIn A, B;
    load_strip(s, A);
    for (; s < s_end; s += 2 * WAVES) {
      const int64_t sb = s + WAVES;
      if (sb < s_end) load_strip(sb, B);
      compute_strip(s, A);
      if (sb < s_end) {
        if (sb + WAVES < s_end) load_strip(sb + WAVES, A);
        compute_strip(sb, B);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < RJT; ++t)
#pragma unroll
    for (int p = 0; p < BP; ++p) {
      double v = z[t][p];
      v += __shfl_xor(v, 16, 64);
      v += __shfl_xor(v, 32, 64);
      z[t][p] = v;
    }
  for (int w = 0; w < WAVES; ++w) {
    if (wave == w && g == 0) {
#pragma unroll
      for (int t = 0; t < RJT; ++t)
#pragma unroll
        for (int p = 0; p < BP; ++p) {
          const int idx = (t * 16 + c) * BP + p;
          sZ[idx] = (w == 0 ? 0.0 : sZ[idx]) + z[t][p];
        }
    }
    __syncthreads();
  }
  double* out = a.part + (int64_t)rg * a.n * BP;
  for (int idx = threadIdx.x; idx < ncols * BP; idx += THREADS)
    out[(j_begin + idx / BP) * BP + idx % BP] = sZ[idx];
}

// Z[:, col0 + p] = sum over row groups of the partials.  Block = RR_OUT outputs x
// RR_SUB row-group subsets (subset q sums groups q, q + RR_SUB, ...); the subsets
// are then added in a fixed order.
constexpr int RR_OUT = 32, RR_SUB = THREADS / RR_OUT;
__global__ __launch_bounds__(THREADS) void k_right_reduce(const double* part, int row_groups, int64_t n, double* Z,
                                                          int ldz, int col0, int bw) {
  __shared__ double sh[RR_SUB][RR_OUT];
  const int lo = threadIdx.x % RR_OUT, q = threadIdx.x / RR_OUT;
  const int64_t o = (int64_t)blockIdx.x * RR_OUT + lo;
  double s = 0.0;
  if (o < n * BP)
    for (int r = q; r < row_groups; r += RR_SUB) s += part[(int64_t)r * n * BP + o];
  sh[q][lo] = s;
  __syncthreads();
  if (q == 0 && o < n * BP) {
    double t = sh[0][lo];
    for (int u = 1; u < RR_SUB; ++u) t += sh[u][lo];
    const int p = (int)(o % BP);
    if (p < bw) Z[(o / BP) * ldz + col0 + p] = t;
  }
}

// Gram matrices of thin row sets, FP64.  mode 0: row i = [A_i, B_i - lam A_i]
// (A, B are FP32 rows of width k); mode 1: row i = D_i (FP64, width w).
struct GramArgs {
  int64_t rows;
  int32_t w, mode, k, ldd;
  float lam;
  const float* A;
  const float* B;
  const double* D;
  double* part;  // [blocks][w*w]
};

__global__ __launch_bounds__(THREADS) void k_gram(GramArgs a) {
  constexpr int TR = 32;
  __shared__ double tile[TR][64];
  const int w = a.w, ww = w * w;
  double acc[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = 0.0;
  for (int64_t r0 = (int64_t)blockIdx.x * TR; r0 < a.rows; r0 += (int64_t)gridDim.x * TR) {
    for (int idx = threadIdx.x; idx < TR * w; idx += THREADS) {
      const int rr = idx / w, cc = idx % w;
      const int64_t i = r0 + rr;
      double v = 0.0;
      if (i < a.rows) {
        if (a.mode == 0) {
          if (cc < a.k) v = a.A[i * a.k + cc];
          else v = (double)a.B[i * a.k + cc - a.k] - (double)a.lam * (double)a.A[i * a.k + cc - a.k];
        } else {
          v = a.D[i * a.ldd + cc];
        }
      }
      tile[rr][cc] = v;
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int idx = threadIdx.x + e * THREADS;
      if (idx < ww) {
        const int p = idx / w, q = idx % w;
        double s = acc[e];
        for (int rr = 0; rr < TR; ++rr) s = fma(tile[rr][p], tile[rr][q], s);
        acc[e] = s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int idx = threadIdx.x + e * THREADS;
    if (idx < ww) a.part[(int64_t)blockIdx.x * ww + idx] = acc[e];
  }
}

// out_i = in_i T  (in: FP64 rows of width win, ld ldi; T: win x wout FP64 in global;
// out: FP64 (ld ldo) or FP32 (ld ldo) rows of width wout).
__global__ void k_row_transform(const double* in, int ldi, int win, const double* T, int wout,
                                int64_t rows, double* out64, float* out32, int ldo) {
  const int64_t o = (int64_t)blockIdx.x * THREADS + threadIdx.x;
  if (o >= rows * wout) return;
  const int64_t i = o / wout;
  const int cc = (int)(o % wout);
  double s = 0.0;
  for (int t = 0; t < win; ++t) s = fma(in[i * ldi + t], T[t * wout + cc], s);
  if (out64) out64[i * ldo + cc] = s;
  else out32[i * ldo + cc] = (float)s;
}

// ----------------------------------------------------------------------------
// Host helpers.

struct Workspace {
  double* Wd;    // n x LMAX
  double* Yd;    // m x LMAX
  double* Y2;    // m x LMAX
  double* Zd;    // n x LMAX
  double* part;  // right-sweep partials
  double* gram;  // gram partials
  double* T;     // small transform (64 x 64)
  float* gU;     // m x k
  float* gV;     // n x k
  float* zU;     // zeros m x k
  float* zV;     // zeros n x k
  double* scal;  // 16 doubles
  // pinned host staging (the context's): [0, PIN_SMALL) Gram results and small
  // transforms, then n x LMAX doubles (sketches, Z^T Q), then n x 32 floats
  // (factor uploads); the certificate's power loop uses [0, 2 n x 32) on its own
  double* pin;
  int rg_left, spw_left, rg_right, spw_right, nch_right, gram_blocks;
  // fused Op^T Op W pass (n <= 256, k <= 16): W in FP32 (n x 16), per-workgroup
  // sums
  float* Wf;
  float* gpart;
  int rg_ga;
  // the power iteration's steps on the device (with the fused pass): two n x BLK
  // FP64 blocks, a second FP32 block (n x 16), the projected product (n x BLK),
  // V_1 and B_n (n x RMAX), V_1^T B_n, the top Ritz vector (n), and 64 doubles of
  // results and state
  double* pxd[2];
  float* Wf2;
  double* pzf;
  double* pv1;
  double* pbn;
  double* pvb;
  double* pvtop;
  double* pres;
};
constexpr size_t PIN_SMALL = 4096;

constexpr int LMAX = 48;

int64_t align_up(int64_t v) { return (v + 63) / 64 * 64; }

int get_workspace(rpca_ctx* c, Workspace* w, hipStream_t s);

hipError_t left_product(const rpca::CtxView& cv, const Workspace& w, const float* X, int src,
                        const float* U, const float* V, const double* W, int ldw, double* Y,
                        int ldy, int l, hipStream_t s) {
  GArgs a;
  memset(&a, 0, sizeof(a));
  a.X = X;
  a.mask = cv.mask;
  a.m = cv.m;
  a.n = cv.n;
  a.k = cv.k;
  a.mw = cv.mw;
  a.lam_s = (float)cv.lam_s;
  a.kappa = (float)cv.kappa;
  a.U = U;
  a.V = V;
  a.W = W;
  a.ldw = ldw;
  a.Y = Y;
  a.ldy = ldy;
  a.strips_per_wg = w.spw_left;
  for (int col0 = 0; col0 < l; col0 += BP) {
    a.col0 = col0;
    a.bw = std::min(BP, l - col0);
    const dim3 grid(w.rg_left);
    const size_t lb = left_lds_bytes(cv.n, cv.k, src);
    void* tok = nullptr;
    if (cv.ctx && rpca::prof_begin(cv.ctx, s, &tok) != hipSuccess) return hipErrorUnknown;
    if (src == SRC_PROX) {  // every entry observed (the caller checks)
      if (lb <= LEFT_LDS_MAX) hipLaunchKernelGGL((k_left_lds<SRC_PROX, false>), grid, dim3(THREADS), lb, s, a);
      else hipLaunchKernelGGL((k_left<SRC_PROX, false>), grid, dim3(THREADS), 0, s, a);
    } else if (lb <= LEFT_LDS_MAX) {
      if (src == SRC_RESID) {
        if (cv.mask) hipLaunchKernelGGL((k_left_lds<SRC_RESID, true>), grid, dim3(THREADS), lb, s, a);
        else hipLaunchKernelGGL((k_left_lds<SRC_RESID, false>), grid, dim3(THREADS), lb, s, a);
      } else {
        if (cv.mask) hipLaunchKernelGGL((k_left_lds<SRC_DATA, true>), grid, dim3(THREADS), lb, s, a);
        else hipLaunchKernelGGL((k_left_lds<SRC_DATA, false>), grid, dim3(THREADS), lb, s, a);
      }
    } else if (src == SRC_RESID) {
      if (cv.mask) hipLaunchKernelGGL((k_left<SRC_RESID, true>), grid, dim3(THREADS), 0, s, a);
      else hipLaunchKernelGGL((k_left<SRC_RESID, false>), grid, dim3(THREADS), 0, s, a);
    } else {
      if (cv.mask) hipLaunchKernelGGL((k_left<SRC_DATA, true>), grid, dim3(THREADS), 0, s, a);
      else hipLaunchKernelGGL((k_left<SRC_DATA, false>), grid, dim3(THREADS), 0, s, a);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (tok && rpca::prof_end(cv.ctx, RPCA_K_LEFT, s, tok) != hipSuccess) return hipErrorUnknown;
  }
  return hipSuccess;
}

hipError_t right_product(const rpca::CtxView& cv, const Workspace& w, const float* X, int src,
                         const float* U, const float* V, double* Y, int ldy, double* Z, int ldz,
                         int l, hipStream_t s) {
  GArgs a;
  memset(&a, 0, sizeof(a));
  a.X = X;
  a.mask = cv.mask;
  a.m = cv.m;
  a.n = cv.n;
  a.k = cv.k;
  a.mw = cv.mw;
  a.lam_s = (float)cv.lam_s;
  a.kappa = (float)cv.kappa;
  a.U = U;
  a.V = V;
  a.Y = Y;
  a.ldy = ldy;
  a.part = w.part;
  a.strips_per_wg = w.spw_right;
  a.nchunks = w.nch_right;
  a.row_groups = w.rg_right;
  for (int col0 = 0; col0 < l; col0 += BP) {
    a.col0 = col0;
    a.bw = std::min(BP, l - col0);
    const dim3 grid(w.rg_right, w.nch_right);
    void* tok = nullptr;
    if (cv.ctx && rpca::prof_begin(cv.ctx, s, &tok) != hipSuccess) return hipErrorUnknown;
    if (src == SRC_PROX) {  // every entry observed (the caller checks)
      hipLaunchKernelGGL((k_right_lds<SRC_PROX, false>), grid, dim3(THREADS), 0, s, a);
    } else if (src == SRC_RESID) {
      if (cv.mask) hipLaunchKernelGGL((k_right_lds<SRC_RESID, true>), grid, dim3(THREADS), 0, s, a);
      else hipLaunchKernelGGL((k_right_lds<SRC_RESID, false>), grid, dim3(THREADS), 0, s, a);
    } else {
      if (cv.mask) hipLaunchKernelGGL((k_right_lds<SRC_DATA, true>), grid, dim3(THREADS), 0, s, a);
      else hipLaunchKernelGGL((k_right_lds<SRC_DATA, false>), grid, dim3(THREADS), 0, s, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (tok && rpca::prof_end(cv.ctx, RPCA_K_RIGHT, s, tok) != hipSuccess) return hipErrorUnknown;
    const int64_t outs = cv.n * BP;
    hipLaunchKernelGGL(k_right_reduce, dim3((unsigned)((outs + RR_OUT - 1) / RR_OUT)), dim3(THREADS), 0, s,
                       (const double*)w.part, w.rg_right, cv.n, Z, ldz, col0, a.bw);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Growth column on the device (rank growth, Sec. 4.1).  part[b * k + j] = block b's
// share of U^T y (U: m x k FP32 row-major, y: m FP64), rows in a grid-stride order.
__global__ __launch_bounds__(THREADS) void k_uty(const float* __restrict__ U, const double* __restrict__ y,
                                                 int64_t m, int k, double* __restrict__ part) {
  __shared__ double red[WAVES][32];
  double acc[32];
#pragma unroll
  for (int j = 0; j < 32; ++j) acc[j] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * THREADS + threadIdx.x; i < m; i += (int64_t)gridDim.x * THREADS) {
    const double yi = y[i];
#pragma unroll
    for (int j = 0; j < 32; ++j)
      if (j < k) acc[j] += (double)U[i * k + j] * yi;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    double v = acc[j];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) red[w][j] = v;
  }
  __syncthreads();
  if (threadIdx.x < k) {
    double t = 0.0;
    for (int ww = 0; ww < WAVES; ++ww) t += red[ww][threadIdx.x];
    part[(int64_t)blockIdx.x * k + threadIdx.x] = t;
  }
}

// back = T_U (T_U^T Uty) (k values): one thread; T_U is k x r row-major
__global__ void k_growth_back(const double* __restrict__ Uty, const double* __restrict__ TU, int k, int r,
                              double* __restrict__ back) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double coef[32];
  for (int q = 0; q < r; ++q) {
    double c = 0.0;
    for (int j = 0; j < k; ++j) c += TU[j * r + q] * Uty[j];
    coef[q] = c;
  }
  for (int j = 0; j < k; ++j) {
    double b = 0.0;
    for (int q = 0; q < r; ++q) b += TU[j * r + q] * coef[q];
    back[j] = b;
  }
}

// y_i -= U_i . back (back null: y unchanged); part[b] = block b's share of ||y||^2
__global__ __launch_bounds__(THREADS) void k_growth_project(const float* __restrict__ U,
                                                            const double* __restrict__ back, int64_t m, int k,
                                                            double* __restrict__ y, double* __restrict__ part) {
  __shared__ double red[WAVES];
  double nn = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * THREADS + threadIdx.x; i < m; i += (int64_t)gridDim.x * THREADS) {
    double v = y[i];
    if (back) {
      double sacc = 0.0;
      for (int j = 0; j < k; ++j) sacc += (double)U[i * k + j] * back[j];
      v -= sacc;
      y[i] = v;
    }
    nn += v * v;
  }
  for (int o = 32; o > 0; o >>= 1) nn += __shfl_xor(nn, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nn;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < WAVES; ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

// From ||P_U^perp y_raw||^2 (nn) with D v = y_raw / lam_L: sigma, t = lam_L (sigma - 1)_+,
// u_col = sqrt(t) y / ||y||, v_col = -sqrt(t) v; res = {sigma, t}
__global__ __launch_bounds__(THREADS) void k_growth_cols(const double* __restrict__ y, const double* __restrict__ v,
                                                         const double* __restrict__ nn, int64_t m, int64_t n,
                                                         double lam_l, float* __restrict__ u_col,
                                                         float* __restrict__ v_col, double* __restrict__ res) {
  const double norm = sqrt(*nn);
  const double sigma = norm / lam_l;
  const double t = sigma > 1.0 ? lam_l * (sigma - 1.0) : 0.0;
  const double st = sqrt(t);
  const double su = norm > 0.0 ? st / norm : 0.0;
  const int64_t stride = (int64_t)gridDim.x * THREADS;
  for (int64_t i = (int64_t)blockIdx.x * THREADS + threadIdx.x; i < m; i += stride)
    u_col[i] = norm > 0.0 ? (float)(su * y[i]) : 0.f;  // y is not read without a Ritz vector
  for (int64_t j = (int64_t)blockIdx.x * THREADS + threadIdx.x; j < n; j += stride) v_col[j] = (float)(-st * v[j]);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    res[0] = sigma;
    res[1] = t;
  }
}

// Wf (n x 16 FP32) = columns [col0, col0 + bw) of the FP64 block W (ld ldw), zero beyond
__global__ void k_pack_w16(const double* W, int ldw, int col0, int bw, int64_t n, float* Wf) {
  const int64_t idx = (int64_t)blockIdx.x * THREADS + threadIdx.x;
  if (idx >= n * 16) return;
  const int64_t j = idx >> 4;
  const int p = (int)(idx & 15);
  Wf[idx] = p < bw ? (float)W[j * ldw + col0 + p] : 0.f;
}

// Z (n x b, ld ldz, FP64) = Op^T Op W for the FP32 block W in w.Wf (n x 16), one
// fused pass over X (the workspace has it when n <= 256 and k <= 16).
hipError_t gram_product(const rpca::CtxView& cv, const Workspace& w, const float* X, int src, const float* U,
                        const float* V, double* Z, int ldz, int b, hipStream_t s, int col0 = 0,
                        const float* Wsrc = nullptr, const double* skip = nullptr) {
  if (!w.gpart || src == SRC_PROX) return hipErrorInvalidValue;
  rpca::GramApplyArgs a;
  memset(&a, 0, sizeof(a));
  a.X = X;
  a.mask = cv.mask;
  a.m = cv.m;
  a.n = cv.n;
  a.k = cv.k;
  a.mw = cv.mw;
  a.lam_s = (float)cv.lam_s;
  a.kappa = (float)cv.kappa;
  a.U = U;
  a.V = V;
  a.W = Wsrc ? Wsrc : w.Wf;
  a.part = w.gpart;
  a.skip = skip;
  a.row_groups = w.rg_ga;
  a.xvec = ((reinterpret_cast<uintptr_t>(X) & 15) == 0 && cv.m % 4 == 0) ? 1 : 0;
  void* tok = nullptr;
  if (cv.ctx && rpca::prof_begin(cv.ctx, s, &tok) != hipSuccess) return hipErrorUnknown;
  hipError_t e = rpca::launch_gram_apply_pass(a, src == SRC_RESID, s);
  if (e != hipSuccess) return e;
  if (tok && rpca::prof_end(cv.ctx, RPCA_K_GRAM, s, tok) != hipSuccess) return hipErrorUnknown;
  return rpca::launch_gram_apply_sum(a, Z, ldz, col0, b, 1.0, s);
}

// Sum of the per-block Gram partials, one workgroup per entry e: out[e] = sum over
// b of part[b ww + e] (thread b takes partials b, b + THREADS, ...; then a fixed tree).
__global__ __launch_bounds__(THREADS) void k_gram_sum(const double* __restrict__ part, int blocks, int ww,
                                                      double* __restrict__ out) {
  __shared__ double red[WAVES];
  const int e = blockIdx.x;
  double v = 0.0;
  for (int b = threadIdx.x; b < blocks; b += THREADS) v += part[(size_t)b * ww + e];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < WAVES; ++w) t += red[w];
    out[e] = t;
  }
}

// Squared Frobenius norm of a projected thin block, FP64, per-block partials:
//   sum_i || (B_i - lam A_i) M1 - A_i M2 ||^2,   rows i < rows,
// with A, B FP32 rows of width k (U and its gradient, or V and its gradient) and
// M1, M2 k x r FP64 (row-major, in global memory).  B_i - lam A_i is the row of
// G V (or G^T U) the gradient sweep carries, formed in FP64 before the product, so
// a block that vanishes at a stationary point is summed entry by entry instead of
// as a difference of two large traces.
__global__ __launch_bounds__(THREADS) void k_proj_sq(int64_t rows, int k, int r, float lam, const float* A,
                                                     const float* B, const double* M1, const double* M2,
                                                     double* part) {
  __shared__ double sm[2 * 32 * 32];
  __shared__ double red[WAVES];
  for (int idx = threadIdx.x; idx < k * r; idx += THREADS) {
    sm[idx] = M1[idx];
    sm[k * r + idx] = M2[idx];
  }
  __syncthreads();
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * THREADS + threadIdx.x; i < rows; i += (int64_t)gridDim.x * THREADS) {
    double a[32], d[32];  // k <= 32; fully unrolled so both stay in registers
#pragma unroll
    for (int t = 0; t < 32; ++t) {
      a[t] = t < k ? (double)A[i * k + t] : 0.0;
      d[t] = t < k ? (double)B[i * k + t] - (double)lam * a[t] : 0.0;
    }
    for (int j = 0; j < r; ++j) {
      double y = 0.0;
#pragma unroll
      for (int t = 0; t < 32; ++t)
        if (t < k) y = fma(d[t], sm[t * r + j], fma(-a[t], sm[k * r + t * r + j], y));
      acc = fma(y, y, acc);
    }
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < WAVES; ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

// Gram of rows (synchronous; result on the host, w x w row-major).  The partials
// are summed on the device (into ws.T, free here: every user of T uploads it
// after the Gram it is built from), so only w x w values cross to the host.
int gram_host(const Workspace& ws, const GramArgs& ga_in, std::vector<double>& out, hipStream_t s) {
  GramArgs ga = ga_in;
  ga.part = ws.gram;
  const int blocks = ws.gram_blocks;
  hipLaunchKernelGGL(k_gram, dim3(blocks), dim3(THREADS), 0, s, ga);
  if (hipGetLastError() != hipSuccess) return RPCA_EHIP;
  const int ww = ga.w * ga.w;
  hipLaunchKernelGGL(k_gram_sum, dim3(ww), dim3(THREADS), 0, s, (const double*)ws.gram, blocks, ww, ws.T);
  if (hipGetLastError() != hipSuccess) return RPCA_EHIP;
  if (hipMemcpyAsync(ws.pin, ws.T, (size_t)ww * 8, hipMemcpyDeviceToHost, s) != hipSuccess) return RPCA_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return RPCA_EHIP;
  out.assign(ws.pin, ws.pin + ww);
  return RPCA_OK;
}

// The two projected-block norms of the certificate (synchronous):
//   T2 = || D^T U1 - V1 C^T ||^2 (n x r),  T3 = || D V1 - U1 C ||^2 (m x r),
// with D^T U1 = (G^T U) T_U / lam_L, D V1 = (G V) T_V / lam_L, U1 = U T_U,
// V1 = V T_V and C = U1^T D V1 (r x r).  G V and G^T U come from the gradient rows
// gU = G V + lam_L U, gV = G^T U + lam_L V of one sweep.
int proj_norms_host(const Workspace& ws, int64_t m, int64_t n, int k, int r, double lam_l, const float* U,
                    const float* V, const float* gU, const float* gV, const std::vector<double>& TU,
                    const std::vector<double>& TV, const std::vector<double>& C, double* T2, double* T3,
                    hipStream_t s) {
  *T2 = *T3 = 0.0;
  if (r == 0) return RPCA_OK;
  const size_t kr = (size_t)k * r;
  // pinned layout: [M1_2 | M2_2 | M1_3 | M2_3], each k x r
  double* h = ws.pin;
  for (int t = 0; t < k; ++t)
    for (int j = 0; j < r; ++j) {
      double vc = 0.0, uc = 0.0;  // (T_V C^T)[t][j], (T_U C)[t][j]
      for (int q = 0; q < r; ++q) {
        vc += TV[(size_t)t * r + q] * C[(size_t)j * r + q];
        uc += TU[(size_t)t * r + q] * C[(size_t)q * r + j];
      }
      h[t * r + j] = TU[(size_t)t * r + j] / lam_l;
      h[kr + t * r + j] = vc;
      h[2 * kr + t * r + j] = TV[(size_t)t * r + j] / lam_l;
      h[3 * kr + t * r + j] = uc;
    }
  double* dM = ws.T;           // 4 k r <= 4096 doubles (k <= 32)
  double* out = ws.gram;       // two sums, then the partials of each launch
  double* part = ws.gram + 64;
  const int blocks = ws.gram_blocks;
  if (hipMemcpyAsync(dM, h, 4 * kr * 8, hipMemcpyHostToDevice, s) != hipSuccess) return RPCA_EHIP;
  hipLaunchKernelGGL(k_proj_sq, dim3(blocks), dim3(THREADS), 0, s, n, k, r, (float)lam_l, V, gV,
                     (const double*)dM, (const double*)(dM + kr), part);
  if (hipGetLastError() != hipSuccess) return RPCA_EHIP;
  hipLaunchKernelGGL(k_gram_sum, dim3(1), dim3(THREADS), 0, s, (const double*)part, blocks, 1, out);
  if (hipGetLastError() != hipSuccess) return RPCA_EHIP;
  hipLaunchKernelGGL(k_proj_sq, dim3(blocks), dim3(THREADS), 0, s, m, k, r, (float)lam_l, U, gU,
                     (const double*)(dM + 2 * kr), (const double*)(dM + 3 * kr), part + blocks);
  if (hipGetLastError() != hipSuccess) return RPCA_EHIP;
  hipLaunchKernelGGL(k_gram_sum, dim3(1), dim3(THREADS), 0, s, (const double*)(part + blocks), blocks, 1,
                     out + 1);
  if (hipGetLastError() != hipSuccess) return RPCA_EHIP;
  // stream order: the upload from h has completed before this download writes h
  if (hipMemcpyAsync(h, out, 2 * 8, hipMemcpyDeviceToHost, s) != hipSuccess) return RPCA_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return RPCA_EHIP;
  *T2 = h[0];
  *T3 = h[1];
  return RPCA_OK;
}

// Orthonormalise the columns of an FP64 device matrix (rows x l, ld) in place:
// Cholesky QR, twice.  With Y^T Y = L L^T (columns in order), Q = Y L^{-T}; a
// column whose part outside the span of the previous ones has squared norm at
// most 1e-13 of the largest squared column norm is dropped (its Q column is zero).
int orthonormalize_dev(const Workspace& ws, double* Y, double* tmp, int64_t rows, int l, int ld,
                       hipStream_t s) {
  for (int pass = 0; pass < 2; ++pass) {
    GramArgs ga;
    memset(&ga, 0, sizeof(ga));
    ga.rows = rows;
    ga.w = l;
    ga.mode = 1;
    ga.D = Y;
    ga.ldd = ld;
    std::vector<double> G;
    int rc = gram_host(ws, ga, G, s);
    if (rc) return rc;
    std::vector<double> Lc((size_t)l * l, 0.0), T((size_t)l * l, 0.0), x(l);
    std::vector<char> keep(l, 0);
    double maxd = 0.0;
    for (int j = 0; j < l; ++j) maxd = std::max(maxd, G[(size_t)j * l + j]);
    for (int j = 0; j < l; ++j) {
      double d = G[(size_t)j * l + j];
      for (int t = 0; t < j; ++t) d -= Lc[(size_t)j * l + t] * Lc[(size_t)j * l + t];
      if (!(d > 1e-13 * maxd)) continue;  // dependent: column j of L stays zero
      keep[j] = 1;
      const double ljj = sqrt(d);
      Lc[(size_t)j * l + j] = ljj;
      for (int i = j + 1; i < l; ++i) {
        double v = G[(size_t)i * l + j];
        for (int t = 0; t < j; ++t) v -= Lc[(size_t)i * l + t] * Lc[(size_t)j * l + t];
        Lc[(size_t)i * l + j] = v / ljj;
      }
    }
    // T = L^{-T}: row c of T is column c of L^{-1} (forward substitution over kept rows)
    for (int c = 0; c < l; ++c) {
      if (!keep[c]) continue;
      std::fill(x.begin(), x.end(), 0.0);
      x[c] = 1.0 / Lc[(size_t)c * l + c];
      for (int i = c + 1; i < l; ++i) {
        if (!keep[i]) continue;
        double v = 0.0;
        for (int t = c; t < i; ++t) v -= Lc[(size_t)i * l + t] * x[t];
        x[i] = v / Lc[(size_t)i * l + i];
      }
      for (int i = 0; i < l; ++i) T[(size_t)c * l + i] = x[i];
    }
    memcpy(ws.pin, T.data(), T.size() * 8);
    if (hipMemcpyAsync(ws.T, ws.pin, T.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess) return RPCA_EHIP;
    const int64_t outs = rows * l;
    hipLaunchKernelGGL(k_row_transform, dim3((unsigned)((outs + THREADS - 1) / THREADS)), dim3(THREADS), 0, s,
                       (const double*)Y, ld, l, (const double*)ws.T, l, rows, tmp, (float*)nullptr, ld);
    if (hipGetLastError() != hipSuccess) return RPCA_EHIP;
    if (hipMemcpyAsync(Y, tmp, (size_t)rows * ld * 8, hipMemcpyDeviceToDevice, s) != hipSuccess) return RPCA_EHIP;
    // the pinned source of the T upload is rewritten by the next pass
    if (hipStreamSynchronize(s) != hipSuccess) return RPCA_EHIP;
  }
  return RPCA_OK;
}

// Counter-based normal deviates: SplitMix64 (Steele, Lea & Flood 2014) feeding
// Box-Muller.  Deviate number `idx` of stream `seed`.
uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

double normal_deviate(uint64_t seed, uint64_t idx) {
  const uint64_t a = splitmix64(seed * 0x100000001B3ull + 2 * idx);
  const uint64_t b = splitmix64(seed * 0x100000001B3ull + 2 * idx + 1);
  const double u1 = ((a >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  const double u2 = ((b >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

}  // namespace


namespace {

int get_workspace(rpca_ctx* c, Workspace* w, hipStream_t s) {
  const rpca::CtxView cv = rpca::ctx_view(c);
  const int64_t m = cv.m, n = cv.n, k = cv.k;
  const int64_t nstrips = (m + 15) / 16;
  // left sweep: ~1024 workgroups of 4 waves
  int64_t spw = std::max<int64_t>(4, ((nstrips + 1023) / 1024 + 3) / 4 * 4);
  w->spw_left = (int)spw;
  w->rg_left = (int)((nstrips + spw - 1) / spw);
  w->nch_right = (int)((n + RJT * 16 - 1) / (RJT * 16));
  int64_t target = std::max<int64_t>(1, 1024 / w->nch_right);
  int64_t spr = std::max<int64_t>(4, ((nstrips + target - 1) / target + 3) / 4 * 4);
  w->spw_right = (int)spr;
  w->rg_right = (int)((nstrips + spr - 1) / spr);
  w->gram_blocks = 256;
  {
    // fused Gram pass: one workgroup per compute unit, at least two strips per wave
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
    w->rg_ga = (int)std::max<int64_t>(1, std::min<int64_t>(cus, nstrips / 8));
  }
  const bool ga = rpca::gram_apply_fits(n, (int)k);
  const size_t sz_Wf = ga ? align_up(n * 16) * 4 : 0;
  const size_t sz_gpart = ga ? align_up((int64_t)w->rg_ga * n * 16) * 4 : 0;
  constexpr int BL = rpca_ritz::BLK, RM = rpca_ritz::RMAX;
  const size_t sz_pblk = ga ? align_up(n * BL) * 8 : 0, sz_prk = ga ? align_up(n * RM) * 8 : 0;
  const size_t sz_pdev = ga ? sz_pblk * 3 + sz_Wf + sz_prk * 2 + align_up(RM * RM) * 8 + align_up(n) * 8 + 64 * 8 : 0;
  size_t off = 0;
  const size_t sz_W = align_up(n * LMAX) * 8, sz_Y = align_up(m * LMAX) * 8;
  const size_t sz_part = align_up((int64_t)w->rg_right * n * BP) * 8;
  const size_t sz_gram = align_up((int64_t)w->gram_blocks * 64 * 64) * 8;
  const size_t sz_T = 64 * 64 * 8;
  const size_t sz_gU = align_up(m * k) * 4, sz_gV = align_up(n * k) * 4;
  const size_t total =
      sz_W * 2 + sz_Y * 2 + sz_part + sz_gram + sz_T + sz_gU * 2 + sz_gV * 2 + 256 + sz_Wf + sz_gpart + sz_pdev;
  int fresh = 0;
  char* base = (char*)rpca::ctx_workspace(c, total, &fresh);
  if (!base) return RPCA_ENOMEM;
  auto take = [&](size_t bytes) {
    char* p = base + off;
    off += bytes;
    return p;
  };
  w->Wd = (double*)take(sz_W);
  w->Zd = (double*)take(sz_W);
  w->Yd = (double*)take(sz_Y);
  w->Y2 = (double*)take(sz_Y);
  w->part = (double*)take(sz_part);
  w->gram = (double*)take(sz_gram);
  w->T = (double*)take(sz_T);
  w->gU = (float*)take(sz_gU);
  w->zU = (float*)take(sz_gU);
  w->gV = (float*)take(sz_gV);
  w->zV = (float*)take(sz_gV);
  w->scal = (double*)take(256);
  w->Wf = ga ? (float*)take(sz_Wf) : nullptr;
  w->gpart = ga ? (float*)take(sz_gpart) : nullptr;
  w->pxd[0] = ga ? (double*)take(sz_pblk) : nullptr;
  w->pxd[1] = ga ? (double*)take(sz_pblk) : nullptr;
  w->pzf = ga ? (double*)take(sz_pblk) : nullptr;
  w->Wf2 = ga ? (float*)take(sz_Wf) : nullptr;
  w->pv1 = ga ? (double*)take(sz_prk) : nullptr;
  w->pbn = ga ? (double*)take(sz_prk) : nullptr;
  w->pvb = ga ? (double*)take(align_up(RM * RM) * 8) : nullptr;
  w->pvtop = ga ? (double*)take(align_up(n) * 8) : nullptr;
  w->pres = ga ? (double*)take(64 * 8) : nullptr;
  w->pin = (double*)rpca::ctx_pinned(c, (PIN_SMALL + (size_t)n * 64) * sizeof(double));
  if (!w->pin) return RPCA_ENOMEM;
  if (fresh) {  // zero factors used for phi(0)
    if (hipMemsetAsync(w->zU, 0, sz_gU, s) != hipSuccess) return RPCA_EHIP;
    if (hipMemsetAsync(w->zV, 0, sz_gV, s) != hipSuccess) return RPCA_EHIP;
  }
  return RPCA_OK;
}

}  // namespace

namespace rpca {

// The certificate of (U, V).  quick_tol > 0 (the solver's own rounds): phi(0) is
// taken from the solve's cache when known, and when the terms that need no power
// iteration already put rel_gap above quick_tol the power iteration is skipped
// (T4 = 0 then, rel_gap is the lower bound it gives, certified = 0).
int certificate_impl(rpca_ctx* c, const float* X, const float* U, const float* V, rpca_cert* out,
                     double quick_tol, hipStream_t s, CertExtra* extra) {
  const rpca::CtxView cv = rpca::ctx_view(c);
  const int64_t m = cv.m, n = cv.n;
  const int k = cv.k;
  const double lam_l = cv.lam_l;
  Workspace ws;
  int rc = get_workspace(c, &ws, s);
  if (rc) return rc;
  memset(out, 0, sizeof(*out));
  // 1. phi(0) from a sweep at U = V = 0 (or the solve's cache), then one sweep at
  //    (U, V): G V, G^T U, phi(L), ||U||^2, ||V||^2, ||G||^2
  const bool cached = quick_tol > 0 && cv.phi0_X && *cv.phi0_X == (const void*)X && isfinite(*cv.phi0);
  if (!cached) {
    rc = rpca::ctx_objgrad_aux(c, X, ws.zU, ws.zV, ws.scal + 8, ws.scal + 9, ws.gU, ws.gV, s);
    if (rc) return rc;
  }
  rc = rpca::ctx_objgrad_aux(c, X, U, V, ws.scal, ws.scal + 1, ws.gU, ws.gV, s);
  if (rc) return rc;
  double scal[16];
  if (hipMemcpyAsync(ws.pin, ws.scal, sizeof(scal), hipMemcpyDeviceToHost, s) != hipSuccess) return RPCA_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return RPCA_EHIP;
  memcpy(scal, ws.pin, sizeof(scal));
  const double phiL = scal[1], g2 = scal[4];
  const double phi0 = cached ? *cv.phi0 : scal[9];
  if (cv.phi0_X) {
    *cv.phi0 = phi0;
    *cv.phi0_X = (const void*)X;
  }
  // 2. Gram matrices [U, G V] (m rows) and [V, G^T U] (n rows), 2k x 2k
  std::vector<double> GU, GV;
  GramArgs ga;
  memset(&ga, 0, sizeof(ga));
  ga.rows = m;
  ga.w = 2 * k;
  ga.mode = 0;
  ga.k = k;
  ga.lam = (float)lam_l;
  ga.A = U;
  ga.B = ws.gU;
  if ((rc = gram_host(ws, ga, GU, s))) return rc;
  ga.rows = n;
  ga.A = V;
  ga.B = ws.gV;
  if ((rc = gram_host(ws, ga, GV, s))) return rc;
  const int w2 = 2 * k;
  auto blk = [&](const std::vector<double>& G, int bi, int bj, std::vector<double>& o) {
    o.assign((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) o[(size_t)i * k + j] = G[(size_t)(bi * k + i) * w2 + bj * k + j];
  };
  std::vector<double> UtU, UtA, AtA, VtV, VtB, BtB;  // A = G V, B = G^T U
  blk(GU, 0, 0, UtU);
  blk(GU, 0, 1, UtA);
  blk(GU, 1, 1, AtA);
  blk(GV, 0, 0, VtV);
  blk(GV, 0, 1, VtB);
  blk(GV, 1, 1, BtB);
  // 3. factor SVD: U = Q_U R_U with R_U = Lam^{1/2} W^T (eigen of U^T U), same for V
  std::vector<double> eu(k), Wu((size_t)k * k), evv(k), Wv((size_t)k * k);
  rpca::la::sym_eig(UtU.data(), k, eu.data(), Wu.data());
  rpca::la::sym_eig(VtV.data(), k, evv.data(), Wv.data());
  std::vector<double> Ru((size_t)k * k), Rv((size_t)k * k), Pu((size_t)k * k, 0.0), Pv((size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      Ru[(size_t)i * k + j] = sqrt(std::max(eu[i], 0.0)) * Wu[(size_t)j * k + i];
      Rv[(size_t)i * k + j] = sqrt(std::max(evv[i], 0.0)) * Wv[(size_t)j * k + i];
    }
  // Pu = W_U Lam_U^{-1/2} (pseudo-inverse on tiny eigenvalues): Q_U = U Pu
  for (int j = 0; j < k; ++j) {
    const double su = (eu[j] > 1e-14 * std::max(eu[0], 0.0) && eu[j] > 0) ? 1.0 / sqrt(eu[j]) : 0.0;
    const double sv = (evv[j] > 1e-14 * std::max(evv[0], 0.0) && evv[j] > 0) ? 1.0 / sqrt(evv[j]) : 0.0;
    for (int i = 0; i < k; ++i) {
      Pu[(size_t)i * k + j] = Wu[(size_t)i * k + j] * su;
      Pv[(size_t)i * k + j] = Wv[(size_t)i * k + j] * sv;
    }
  }
  // SVD of Mk = R_U R_V^T via the eigen-decomposition of Mk^T Mk (k x k, FP64)
  std::vector<double> Mk((size_t)k * k), MtM((size_t)k * k), sig2(k), VR((size_t)k * k);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      double sacc = 0.0;
      for (int t = 0; t < k; ++t) sacc += Ru[(size_t)i * k + t] * Rv[(size_t)j * k + t];
      Mk[(size_t)i * k + j] = sacc;
    }
  rpca::la::matmul_tn(Mk.data(), Mk.data(), MtM.data(), k, k, k);
  rpca::la::sym_eig(MtM.data(), k, sig2.data(), VR.data());
  std::vector<double> sig(k);
  for (int i = 0; i < k; ++i) sig[i] = sqrt(std::max(sig2[i], 0.0));
  const double tau = 1e-6;  // FP32 factors: rank threshold relative to sigma_1
  int r = 0;
  for (int i = 0; i < k; ++i)
    if (sig[i] > tau * sig[0] && sig[0] > 0) ++r;
  // U_R = Mk V_R Sigma^{-1} (first r columns)
  std::vector<double> UR((size_t)k * std::max(r, 1), 0.0), VRr((size_t)k * std::max(r, 1), 0.0);
  for (int j = 0; j < r; ++j)
    for (int i = 0; i < k; ++i) {
      double sacc = 0.0;
      for (int t = 0; t < k; ++t) sacc += Mk[(size_t)i * k + t] * VR[(size_t)t * k + j];
      UR[(size_t)i * r + j] = sacc / sig[j];
      VRr[(size_t)i * r + j] = VR[(size_t)i * k + j];
    }
  // T_U = Pu U_R, T_V = Pv V_R  (U1 = U T_U, V1 = V T_V)
  std::vector<double> TU((size_t)k * std::max(r, 1), 0.0), TV((size_t)k * std::max(r, 1), 0.0);
  if (r) {
    rpca::la::matmul(Pu.data(), UR.data(), TU.data(), k, k, r);
    rpca::la::matmul(Pv.data(), VRr.data(), TV.data(), k, k, r);
  }
  // 4. cheap terms
  auto quad = [&](const std::vector<double>& Gm, const std::vector<double>& Ta,
                  const std::vector<double>& Tb, std::vector<double>& o) {  // o = Ta^T Gm Tb (r x r)
    std::vector<double> tmp((size_t)k * std::max(r, 1));
    rpca::la::matmul(Gm.data(), Tb.data(), tmp.data(), k, k, r);
    o.assign((size_t)r * r, 0.0);
    rpca::la::matmul_tn(Ta.data(), tmp.data(), o.data(), k, r, r);
  };
  std::vector<double> Cm, DV1n, DU1n;
  double T1 = 0, T2 = 0, T3 = 0, nC = 0, nDV1 = 0, nDtU1 = 0;
  if (r) {
    quad(UtA, TU, TV, Cm);  // U1^T (G V) T_V = lam_l * U1^T D V1
    for (int i = 0; i < r; ++i)
      for (int j = 0; j < r; ++j) {
        const double cij = Cm[(size_t)i * r + j] / lam_l;
        nC += cij * cij;
        const double e = (i == j ? 1.0 : 0.0) + cij;
        T1 += e * e;
      }
    quad(AtA, TV, TV, DV1n);  // T_V^T A^T A T_V
    quad(BtB, TU, TU, DU1n);  // T_U^T B^T B T_U
    for (int i = 0; i < r; ++i) {
      nDV1 += DV1n[(size_t)i * r + i] / (lam_l * lam_l);
      nDtU1 += DU1n[(size_t)i * r + i] / (lam_l * lam_l);
    }
    // T2, T3 entry by entry (a difference of the traces above cancels at a
    // stationary point, where both blocks vanish)
    std::vector<double> Cn((size_t)r * r);
    for (size_t e = 0; e < Cn.size(); ++e) Cn[e] = Cm[e] / lam_l;
    const int prc = proj_norms_host(ws, m, n, k, r, lam_l, U, V, ws.gU, ws.gV, TU, TV, Cn, &T2, &T3, s);
    if (prc) return prc;
  }
  const double nD2 = g2 / (lam_l * lam_l);
  const double normM2 = std::max(nD2 - nDtU1 - nDV1 + nC, 0.0);
  // Quick rejection: T4 >= 0, so the other terms alone bound rel_gap from below.
  if (quick_tol > 0) {
    double nuc = 0.0, normL2 = 0.0, trunc2 = 0.0;
    for (int i = 0; i < k; ++i) {
      nuc += sig[i];
      normL2 += sig[i] * sig[i];
      if (i >= r) trunc2 += sig[i] * sig[i];
    }
    const double E_lo = sqrt(std::max(T1 + T2 + T3, 0.0)) + sqrt(trunc2) / lam_l;
    const double F = lam_l * nuc + phiL;
    double* best = cv.best_F;
    if (F < *best) *best = F;
    const double Fb = std::min(std::min(F, phi0), *best);
    const double gap_lo = E_lo * (lam_l * sqrt(normL2) + Fb);
    const double rel_lo = F > 0 ? gap_lo / F : INFINITY;
    if (rel_lo > quick_tol) {
      out->T1 = T1;
      out->T2 = T2;
      out->T3 = T3;
      out->T4 = 0.0;
      out->E = E_lo;
      out->F = F;
      out->phi = phiL;
      out->phi0 = phi0;
      out->F_bound = Fb;
      out->normL = sqrt(normL2);
      out->gap = gap_lo;
      out->rel_gap = rel_lo;
      out->normM2 = normM2;
      for (int i = 0; i < k && i < 64; ++i) out->sigma[i] = sig[i];
      out->r = r;
      out->power_iters = 0;
      out->block = 0;
      out->certified = 0;
      return RPCA_OK;
    }
  }
  // 5. T4 by block power iteration on M^T M (host-side projections, n x b).  The
  //    block grows (8 -> 16 -> 32) while its smallest Ritz value is still above 1,
  //    so that every singular value above 1 is captured when there are at most 31.
  const int bmax = (int)std::min<int64_t>(32, std::max<int64_t>(1, n - r));
  int b = std::min(8, bmax);
  std::vector<double> Vh((size_t)n * k), Bh((size_t)n * k);
  {
    // through the pinned staging (n x LMAX doubles hold both n x k float blocks)
    const float* tmpV = reinterpret_cast<const float*>(ws.pin + PIN_SMALL);
    const float* tmpB = tmpV + (size_t)n * k;
    if (hipMemcpyAsync((void*)tmpV, V, (size_t)n * k * 4, hipMemcpyDeviceToHost, s) != hipSuccess) return RPCA_EHIP;
    if (hipMemcpyAsync((void*)tmpB, ws.gV, (size_t)n * k * 4, hipMemcpyDeviceToHost, s) != hipSuccess)
      return RPCA_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return RPCA_EHIP;
    for (size_t i = 0; i < (size_t)n * k; ++i) {
      Vh[i] = tmpV[i];
      Bh[i] = (double)tmpB[i] - lam_l * (double)tmpV[i];  // G^T U
    }
  }
  // V1 (n x r) and Bn = D^T U1 = (G^T U) T_U / lam_l (n x r)
  std::vector<double> V1((size_t)n * std::max(r, 1), 0.0), Bn((size_t)n * std::max(r, 1), 0.0);
  if (r) {
    rpca::la::matmul(Vh.data(), TV.data(), V1.data(), (int)n, k, r);
    rpca::la::matmul(Bh.data(), TU.data(), Bn.data(), (int)n, k, r);
    for (auto& x : Bn) x /= lam_l;
  }
  auto proj_v = [&](std::vector<double>& Xb, int bb) {  // Xb (n x bb) <- P_V^perp Xb
    if (!r) return;
    std::vector<double> coef((size_t)r * bb);
    rpca::la::matmul_tn(V1.data(), Xb.data(), coef.data(), (int)n, r, bb);
    for (int64_t i = 0; i < n; ++i)
      for (int p = 0; p < bb; ++p) {
        double sacc = 0.0;
        for (int t = 0; t < r; ++t) sacc += V1[(size_t)i * r + t] * coef[(size_t)t * bb + p];
        Xb[(size_t)i * bb + p] -= sacc;
      }
  };
  auto orth_host = [&](std::vector<double>& Xb, int bb) {  // modified Gram-Schmidt, twice
    for (int pass = 0; pass < 2; ++pass)
      for (int p = 0; p < bb; ++p) {
        for (int q = 0; q < p; ++q) {
          double d = 0.0;
          for (int64_t i = 0; i < n; ++i) d += Xb[(size_t)i * bb + p] * Xb[(size_t)i * bb + q];
          for (int64_t i = 0; i < n; ++i) Xb[(size_t)i * bb + p] -= d * Xb[(size_t)i * bb + q];
        }
        double nn = 0.0;
        for (int64_t i = 0; i < n; ++i) nn += Xb[(size_t)i * bb + p] * Xb[(size_t)i * bb + p];
        nn = sqrt(nn);
        for (int64_t i = 0; i < n; ++i) Xb[(size_t)i * bb + p] = nn > 0 ? Xb[(size_t)i * bb + p] / nn : 0.0;
      }
  };
  std::vector<double> Xb((size_t)n * b), Zb, ritz(b, 0.0);
  // pinned staging of the block copies (one in, one out per step); the stream is
  // synchronised every step, so a step never overwrites a copy still in flight
  double* pin = ws.pin;  // capacity PIN_SMALL + 64 n >= 2 n bmax
  for (int64_t i = 0; i < n * b; ++i) Xb[i] = normal_deviate(0xC0FFEEull, (uint64_t)i);
  int it_total = 0;
  const int max_it = 300;
  // The steps on the device (fused pass, a block of at most BLK columns): per step
  // the pass G^T G X, then k_block_ritz (the projection, Rayleigh-Ritz, the stop
  // test above, the next block, X w_0); the host reads 9 doubles per step.  Unless
  // kernel timing is on, the next step is queued before the host reads this one's
  // stop flag, its kernels doing nothing once the flag is set.  Fills ritz, the
  // next block Xbh and the top Ritz vector.
  constexpr int BL = rpca_ritz::BLK;
  const size_t o_blk = 32, o_w16 = o_blk + (size_t)n * BL, o_v1 = o_w16 + (size_t)n * 8,
               o_bn = o_v1 + (size_t)n * r, o_vb = o_bn + (size_t)n * r, o_end = o_vb + (size_t)r * r;
  const bool dev_ok = ws.pres != nullptr && r <= rpca_ritz::RMAX && n <= rpca_ritz::RT &&
                      o_end <= PIN_SMALL + (size_t)n * 64;
  auto power_dev = [&](std::vector<double>& Xbh, int bb, int* steps) -> int {
    struct Events {
      hipEvent_t e[2] = {nullptr, nullptr};
      ~Events() {
        for (hipEvent_t x : e)
          if (x) (void)hipEventDestroy(x);
      }
    } ev;
    for (int i = 0; i < 2; ++i)
      if (hipEventCreateWithFlags(&ev.e[i], hipEventDisableTiming) != hipSuccess) return RPCA_EHIP;
    // pinned layout (doubles): [0, 32) two result slots, then the block (n x BL),
    // its FP32 copy (n x 16 floats), V_1 and B_n (n x r), V_1^T B_n (r x r)
    double* blk = pin + o_blk;
    float* w16 = reinterpret_cast<float*>(pin + o_w16);
    for (int64_t i = 0; i < n; ++i)
      for (int c = 0; c < BL; ++c) blk[(size_t)i * BL + c] = c < bb ? Xbh[(size_t)i * bb + c] : 0.0;
    for (int64_t i = 0; i < n; ++i)
      for (int c = 0; c < 16; ++c) w16[(size_t)i * 16 + c] = c < bb ? (float)Xbh[(size_t)i * bb + c] : 0.f;
    if (hipMemcpyAsync(ws.pxd[0], blk, (size_t)n * BL * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(ws.Wf, w16, (size_t)n * 16 * 4, hipMemcpyHostToDevice, s) != hipSuccess)
      return RPCA_EHIP;
    if (r) {
      memcpy(pin + o_v1, V1.data(), (size_t)n * r * 8);
      memcpy(pin + o_bn, Bn.data(), (size_t)n * r * 8);
      rpca::la::matmul_tn(V1.data(), Bn.data(), pin + o_vb, (int)n, r, r);
      if (hipMemcpyAsync(ws.pv1, pin + o_v1, (size_t)n * r * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
          hipMemcpyAsync(ws.pbn, pin + o_bn, (size_t)n * r * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
          hipMemcpyAsync(ws.pvb, pin + o_vb, (size_t)r * r * 8, hipMemcpyHostToDevice, s) != hipSuccess)
        return RPCA_EHIP;
    }
    const bool ahead = !rpca::prof_enabled(cv.ctx);
    auto enqueue = [&](int p) -> int {
      const int cur = p & 1;
      const double* skip = (ahead && p > 0) ? ws.pres : nullptr;
      if (gram_product(cv, ws, X, SRC_RESID, U, V, ws.Zd, BL, bb, s, 0, cur ? ws.Wf2 : ws.Wf, skip) != hipSuccess)
        return RPCA_EHIP;
      rpca_ritz::RitzArgs ra;
      memset(&ra, 0, sizeof(ra));
      ra.X = ws.pxd[cur];
      ra.Z = ws.Zd;
      ra.n = n;
      ra.b = bb;
      ra.salt = 0xC0FFEEull + 977ull * (uint64_t)(p + 1);
      ra.Xn = ws.pxd[cur ^ 1];
      ra.Wfn = cur ? ws.Wf : ws.Wf2;
      ra.res = ws.pres;
      ra.skip = skip;
      ra.last = p + 1 >= max_it ? 1 : 0;
      ra.Zf = ws.pzf;
      ra.V1 = ws.pv1;
      ra.Bn = ws.pbn;
      ra.VB = ws.pvb;
      ra.r = r;
      ra.inv_lam2 = 1.0 / (lam_l * lam_l);
      ra.it = p;
      ra.conv_rel = 1e-6;
      ra.state = ws.pres + 32;
      ra.vtop = ws.pvtop;
      hipLaunchKernelGGL(rpca_ritz::k_block_ritz<rpca_ritz::RITZ_CERT>, dim3(1), dim3(rpca_ritz::RT), 0, s, ra);
      if (hipGetLastError() != hipSuccess) return RPCA_EHIP;
      if (hipMemcpyAsync(pin + 16 * (p & 1), ws.pres, 9 * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipEventRecord(ev.e[p & 1], s) != hipSuccess)
        return RPCA_EHIP;
      return RPCA_OK;
    };
    int rc2 = enqueue(0);
    if (rc2) return rc2;
    int p = 0;
    for (;; ++p) {
      if (ahead && p + 1 < max_it && (rc2 = enqueue(p + 1))) return rc2;
      if (hipEventSynchronize(ev.e[p & 1]) != hipSuccess) return RPCA_EHIP;
      if (pin[16 * (p & 1)] != 0.0 || p + 1 >= max_it) break;
      if (!ahead && (rc2 = enqueue(p + 1))) return rc2;
    }
    *steps = p + 1;
    const double* slot = pin + 16 * (p & 1);
    for (int q = 0; q < bb; ++q) ritz[q] = slot[1 + q];
    // the next block (a larger block starts from it) and the top Ritz vector
    if (hipMemcpyAsync(blk, ws.pxd[(p & 1) ^ 1], (size_t)n * BL * 8, hipMemcpyDeviceToHost, s) != hipSuccess)
      return RPCA_EHIP;
    double* vt = pin + o_w16;  // n doubles fit in the n x 16 floats
    if (extra && hipMemcpyAsync(vt, ws.pvtop, (size_t)n * 8, hipMemcpyDeviceToHost, s) != hipSuccess)
      return RPCA_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return RPCA_EHIP;
    for (int64_t i = 0; i < n; ++i)
      for (int c = 0; c < bb; ++c) Xbh[(size_t)i * bb + c] = blk[(size_t)i * BL + c];
    if (extra) extra->v.assign(vt, vt + n);
    return RPCA_OK;
  };
  for (;;) {
    proj_v(Xb, b);
    orth_host(Xb, b);
    std::vector<double> prev(b, -1.0);
    ritz.assign(b, 0.0);
    Zb.assign((size_t)n * b, 0.0);
    // blocks of at most 16 columns take the fused FP32 pass; its Ritz values settle
    // to about 1e-7 relative, so their convergence test is 1e-6 instead of 1e-8
    const bool fused = ws.gpart != nullptr && b <= 16;
    const double conv_rel = fused ? 1e-6 : 1e-8;
    if (fused && b <= BL && dev_ok) {
      int steps = 0;
      const int prc = power_dev(Xb, b, &steps);
      if (prc) return prc;
      it_total += steps;
    }
    for (int it = 0; it < max_it && !(fused && b <= BL && dev_ok); ++it) {
      ++it_total;
      if (fused) {
        // G^T G X in one pass over X: X as FP32 n x 16 (columns past b zero)
        float* wpin = reinterpret_cast<float*>(pin);
        for (int64_t i = 0; i < n; ++i)
          for (int p = 0; p < 16; ++p) wpin[(size_t)i * 16 + p] = p < b ? (float)Xb[(size_t)i * b + p] : 0.f;
        if (hipMemcpyAsync(ws.Wf, wpin, (size_t)n * 16 * 4, hipMemcpyHostToDevice, s) != hipSuccess) return RPCA_EHIP;
        if (gram_product(cv, ws, X, SRC_RESID, U, V, ws.Zd, b, b, s) != hipSuccess) return RPCA_EHIP;
      } else {
        memcpy(pin, Xb.data(), Xb.size() * 8);
        if (hipMemcpyAsync(ws.Wd, pin, Xb.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess) return RPCA_EHIP;
        if (left_product(cv, ws, X, SRC_RESID, U, V, ws.Wd, b, ws.Yd, b, b, s) != hipSuccess) return RPCA_EHIP;
        if (right_product(cv, ws, X, SRC_RESID, U, V, ws.Yd, b, ws.Zd, b, b, s) != hipSuccess) return RPCA_EHIP;
      }
      if (hipMemcpyAsync(pin + (size_t)n * bmax, ws.Zd, Zb.size() * 8, hipMemcpyDeviceToHost, s) != hipSuccess)
        return RPCA_EHIP;
      if (hipStreamSynchronize(s) != hipSuccess) return RPCA_EHIP;
      memcpy(Zb.data(), pin + (size_t)n * bmax, Zb.size() * 8);
      for (auto& z : Zb) z /= (lam_l * lam_l);
      if (r) {  // Z -= Bn (Bn^T X)
        std::vector<double> coef((size_t)r * b);
        rpca::la::matmul_tn(Bn.data(), Xb.data(), coef.data(), (int)n, r, b);
        for (int64_t i = 0; i < n; ++i)
          for (int p = 0; p < b; ++p) {
            double sacc = 0.0;
            for (int t = 0; t < r; ++t) sacc += Bn[(size_t)i * r + t] * coef[(size_t)t * b + p];
            Zb[(size_t)i * b + p] -= sacc;
          }
      }
      proj_v(Zb, b);
      // Rayleigh-Ritz on span(X): H = X^T Z
      std::vector<double> H((size_t)b * b), hw(b), HW((size_t)b * b);
      rpca::la::matmul_tn(Xb.data(), Zb.data(), H.data(), (int)n, b, b);
      for (int p = 0; p < b; ++p)
        for (int q = p + 1; q < b; ++q) {
          const double avg = 0.5 * (H[(size_t)p * b + q] + H[(size_t)q * b + p]);
          H[(size_t)p * b + q] = H[(size_t)q * b + p] = avg;
        }
      rpca::la::sym_eig(H.data(), b, hw.data(), HW.data());
      // convergence over the Ritz values that can matter for T4: those at or above
      // 0.9 (squared 0.81) and the leading one; lower ones contribute nothing unless
      // they rise by a tenth, and in a block they converge the slowest
      double dmax = 0.0;
      for (int p = 0; p < b; ++p) {
        ritz[p] = std::max(hw[p], 0.0);
        if (p == 0 || ritz[p] >= 0.81) dmax = std::max(dmax, fabs(ritz[p] - prev[p]));
      }
      const double d0 = fabs(ritz[0] - prev[0]);
      for (int p = 0; p < b; ++p) prev[p] = ritz[p];
      if (extra) {  // the top Ritz vector of this step: X w_0
        extra->v.assign((size_t)n, 0.0);
        for (int64_t i = 0; i < n; ++i) {
          double sacc = 0.0;
          for (int q = 0; q < b; ++q) sacc += Xb[(size_t)i * b + q] * HW[(size_t)q * b + 0];
          extra->v[(size_t)i] = sacc;
        }
      }
      Xb = Zb;
      orth_host(Xb, b);
      const bool all_conv = dmax <= conv_rel * std::max(ritz[0], 1e-300);
      const bool below_one = ritz[0] < 0.98 * 0.98 && d0 <= 1e-5 * ritz[0];
      // Largest singular value below 1 with high probability: the block's span holds
      // the power iterate of a Gaussian start in range(P_V^perp), whose Rayleigh
      // quotient after k products of M^T M is below (1 - eps) lambda_max with
      // probability at most 0.824 sqrt(N) (1 - eps)^(k - 1/2) (Kuczynski and
      // Wozniakowski 1992, power method with a random start).  With the top Ritz
      // value ritz[0] < 1, lambda_max > 1 would need eps >= 1 - ritz[0]; once that
      // probability is below 1e-9 (counting it products, one fewer than were made)
      // and ritz[0] has settled to 1e-3, T4 = 0 without converging the Ritz values.
      bool surely_below = false;
      if (it > 2 && ritz[0] < 1.0 && ritz[0] > 0.0 && d0 <= 1e-3 * ritz[0]) {
        const double log_p = log(0.824) + 0.5 * log((double)n) + ((double)it - 0.5) * log(ritz[0]);
        surely_below = log_p <= log(1e-9);
      }
      if (it > 2 && (all_conv || below_one || surely_below)) break;
    }
    if (sqrt(ritz[b - 1]) > 1.0 && b < bmax) {
      // grow the block, keeping the current subspace and adding fresh directions
      const int nb = std::min(2 * b, bmax);
      std::vector<double> Xn((size_t)n * nb);
      for (int64_t i = 0; i < n; ++i)
        for (int p = 0; p < nb; ++p)
          Xn[(size_t)i * nb + p] = p < b ? Xb[(size_t)i * b + p]
                                         : normal_deviate(0xC0FFEEull + nb, (uint64_t)(i * nb + p));
      Xb.swap(Xn);
      b = nb;
      continue;
    }
    break;
  }
  double T4 = 0.0, sum_t2 = 0.0;
  for (int p = 0; p < b; ++p) {
    const double th = sqrt(ritz[p]);
    if (p < 32) out->theta[p] = th;
    if (p < b - 1 || b == 1) {
      T4 += std::max(th - 1.0, 0.0) * std::max(th - 1.0, 0.0);
      sum_t2 += th * th;
    }
  }
  if (b > 1) {
    const double thb = sqrt(ritz[b - 1]);
    if (thb > 1.0) {
      // more than b-1 singular values may exceed 1: bound the rest by
      // (sigma - 1)_+ <= sigma (1 - 1/theta_b) for sigma <= theta_b
      const double tail = std::max(normM2 - sum_t2, 0.0);
      T4 += (1.0 - 1.0 / thb) * (1.0 - 1.0 / thb) * tail;
    } else {
      T4 += std::max(thb - 1.0, 0.0) * std::max(thb - 1.0, 0.0);
    }
  }
  const int it = it_total;
  // 6. gap bound (eq. Fbound)
  double nuc = 0.0, normL2 = 0.0, trunc2 = 0.0;
  for (int i = 0; i < k; ++i) {
    nuc += sig[i];
    normL2 += sig[i] * sig[i];
    if (i >= r) trunc2 += sig[i] * sig[i];
  }
  const double E = sqrt(std::max(T1 + T2 + T3 + T4, 0.0)) + sqrt(trunc2) / lam_l;
  const double F = lam_l * nuc + phiL;
  double* best = cv.best_F;
  if (F < *best) *best = F;
  const double Fb = std::min(std::min(F, phi0), *best);
  const double normL = sqrt(normL2);
  out->T1 = T1;
  out->T2 = T2;
  out->T3 = T3;
  out->T4 = T4;
  out->E = E;
  out->F = F;
  out->phi = phiL;
  out->phi0 = phi0;
  out->F_bound = Fb;
  out->normL = normL;
  out->gap = E * (lam_l * normL + Fb);
  out->rel_gap = F > 0 ? out->gap / F : (out->gap == 0 ? 0.0 : INFINITY);
  out->normM2 = normM2;
  for (int i = 0; i < k && i < 64; ++i) out->sigma[i] = sig[i];
  out->r = r;
  out->power_iters = it;
  out->block = b;
  out->certified = out->rel_gap <= 1e-3;
  if (extra) {
    extra->r = r;
    extra->TU = TU;
  }
  return RPCA_OK;
}

// Rank-growth direction (Sec. 4.1, read through the certificate's last block):
// the top Ritz vector v of M^T M from the certificate's power iteration, then
// u = P_U^perp D v / ||P_U^perp D v|| with sigma = ||P_U^perp D v|| (so u^T D v =
// sigma).  When sigma > 1 the column pair (sqrt(t) u, -sqrt(t) v) with t =
// lam_L (sigma - 1) lowers f by at least lam_L^2 (sigma - 1)^2 / 2 (phi's curvature
// along the unit-norm u v^T is at most 1); otherwise the columns are zero.
int growth_direction_impl(rpca_ctx* c, const float* X, const float* U, const float* V, float* u_col,
                          float* v_col, double* sigma_out, double* t_out, hipStream_t s, rpca_cert* cert_out) {
  const rpca::CtxView cv = rpca::ctx_view(c);
  const int64_t m = cv.m, n = cv.n;
  const int k = cv.k;
  const double lam_l = cv.lam_l;
  rpca_cert cert;
  CertExtra ex;
  int rc = certificate_impl(c, X, U, V, &cert, 0.0, s, &ex);
  if (rc < 0) return rc;
  if (cert_out) *cert_out = cert;
  Workspace ws;
  if ((rc = get_workspace(c, &ws, s))) return rc;
  // every early return below first waits for the copies that use this frame's
  // host vectors (ex.v, the transform)
  auto fail = [&]() {
    (void)hipStreamSynchronize(s);
    return RPCA_EHIP;
  };
  const unsigned gblocks = (unsigned)std::min<int64_t>(256, (m + THREADS - 1) / THREADS);
  const unsigned cblocks = (unsigned)std::min<int64_t>(1024, (std::max(m, n) + THREADS - 1) / THREADS);
  double* res = ws.scal + 20;  // {sigma, t}
  double* nnd = ws.scal + 22;  // ||P_U^perp y||^2
  const double* vdev = ws.Wd;
  if (!ex.v.empty()) {
    // y = G v (one left product, b = 1; D v = y / lam_L), then P_U^perp y with
    // U1 = U T_U and its norm, all on the device
    double* pin = ws.pin;  // the transform, then v (n doubles; capacity PIN_SMALL + 64 n)
    const int r = ex.r;
    memcpy(pin + PIN_SMALL, ex.v.data(), (size_t)n * 8);
    if (hipMemcpyAsync(ws.Wd, pin + PIN_SMALL, (size_t)n * 8, hipMemcpyHostToDevice, s) != hipSuccess)
      return fail();
    if (left_product(cv, ws, X, SRC_RESID, U, V, ws.Wd, 1, ws.Yd, 1, 1, s) != hipSuccess) return fail();
    const double* back = nullptr;
    if (r) {
      memcpy(pin, ex.TU.data(), (size_t)k * r * 8);
      double* TUd = ws.T;             // k x r
      double* Uty = ws.T + 64 * 32;   // k
      double* backd = Uty + 32;       // k
      if (hipMemcpyAsync(TUd, pin, (size_t)k * r * 8, hipMemcpyHostToDevice, s) != hipSuccess) return fail();
      hipLaunchKernelGGL(k_uty, dim3(gblocks), dim3(THREADS), 0, s, U, (const double*)ws.Yd, m, k, ws.gram);
      hipLaunchKernelGGL(k_gram_sum, dim3(k), dim3(THREADS), 0, s, (const double*)ws.gram, (int)gblocks, k, Uty);
      hipLaunchKernelGGL(k_growth_back, dim3(1), dim3(64), 0, s, (const double*)Uty, (const double*)TUd, k, r,
                         backd);
      if (hipGetLastError() != hipSuccess) return fail();
      back = backd;
    }
    hipLaunchKernelGGL(k_growth_project, dim3(gblocks), dim3(THREADS), 0, s, U, back, m, k, ws.Yd, ws.gram);
    hipLaunchKernelGGL(k_gram_sum, dim3(1), dim3(THREADS), 0, s, (const double*)ws.gram, (int)gblocks, 1, nnd);
    if (hipGetLastError() != hipSuccess) return fail();
  } else {
    // no Ritz vector (nothing to grow): zero columns
    if (hipMemsetAsync(nnd, 0, 8, s) != hipSuccess || hipMemsetAsync(ws.Wd, 0, (size_t)n * 8, s) != hipSuccess)
      return fail();
  }
  hipLaunchKernelGGL(k_growth_cols, dim3(cblocks), dim3(THREADS), 0, s, (const double*)ws.Yd, vdev,
                     (const double*)nnd, m, n, lam_l, u_col, v_col, res);
  if (hipGetLastError() != hipSuccess) return fail();
  if (hipMemcpyAsync(ws.pin, res, 2 * 8, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
    return fail();
  const double sigma = ws.pin[0], t = ws.pin[1];
  *sigma_out = sigma;
  *t_out = t;
  return RPCA_OK;
}

}  // namespace rpca

extern "C" int rpca_certificate(rpca_ctx* c, const float* X, const float* U, const float* V,
                                rpca_cert* out, void* stream) {
  if (!c || !X || !U || !V || !out) return RPCA_EINVAL;
  return rpca::certificate_impl(c, X, U, V, out, 0.0, (hipStream_t)stream, nullptr);
}

extern "C" int rpca_rank_direction(rpca_ctx* c, const float* X, const float* U, const float* V, float* u_col,
                                   float* v_col, double* sigma, double* t, void* stream) {
  if (!c || !X || !U || !V || !u_col || !v_col || !sigma || !t) return RPCA_EINVAL;
  return rpca::growth_direction_impl(c, X, U, V, u_col, v_col, sigma, t, (hipStream_t)stream);
}

extern "C" int rpca_init_rsvd(rpca_ctx* c, const float* X, const float* Omega_s, int32_t oversample,
                              int32_t power_steps, uint64_t seed, float* U, float* V, void* stream) {
  if (!c || !X || !U || !V) return RPCA_EINVAL;
  if (oversample < 0 || power_steps < 0 || power_steps > 16) return RPCA_EINVAL;
  const rpca::CtxView cv = rpca::ctx_view(c);
  const int64_t m = cv.m, n = cv.n;
  const int k = cv.k;
  const int l = (int)std::min<int64_t>(std::min<int64_t>(k + oversample, LMAX), std::min(m, n));
  if (l < k) return RPCA_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  Workspace ws;
  int rc = get_workspace(c, &ws, s);
  if (rc) return rc;
  // test matrix Omega_s (n x l) in FP64
  std::vector<double> Om((size_t)n * l);
  if (Omega_s) {
    std::vector<float> tmp((size_t)n * l);
    if (hipMemcpyAsync(tmp.data(), Omega_s, tmp.size() * 4, hipMemcpyDeviceToHost, s) != hipSuccess) return RPCA_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return RPCA_EHIP;
    for (size_t i = 0; i < tmp.size(); ++i) Om[i] = tmp[i];
  } else {
    for (size_t i = 0; i < Om.size(); ++i) Om[i] = normal_deviate(seed, i);
  }
  double* pinB = ws.pin + PIN_SMALL;  // n x l
  memcpy(pinB, Om.data(), Om.size() * 8);
  if (hipMemcpyAsync(ws.Wd, pinB, Om.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess) return RPCA_EHIP;
  if (ws.gpart) {
    // the same subspace, span A (A^T A)^q Omega, with the power steps on the n side:
    // W <- orth(A^T A W) in fused passes over X (16 columns each), then Y = A W
    double* Wcur = ws.Wd;
    double* Wnext = ws.Zd;
    for (int q = 0; q < power_steps; ++q) {
      for (int col0 = 0; col0 < l; col0 += 16) {
        const int bw = std::min(16, l - col0);
        hipLaunchKernelGGL(k_pack_w16, dim3((unsigned)((n * 16 + THREADS - 1) / THREADS)), dim3(THREADS), 0, s,
                           (const double*)Wcur, l, col0, bw, n, ws.Wf);
        if (hipGetLastError() != hipSuccess) return RPCA_EHIP;
        if (gram_product(cv, ws, X, SRC_DATA, nullptr, nullptr, Wnext, l, bw, s, col0) != hipSuccess)
          return RPCA_EHIP;
      }
      if ((rc = orthonormalize_dev(ws, Wnext, ws.Y2, n, l, l, s))) return rc;
      std::swap(Wcur, Wnext);
    }
    if (left_product(cv, ws, X, SRC_DATA, nullptr, nullptr, Wcur, l, ws.Yd, l, l, s) != hipSuccess) return RPCA_EHIP;
    if ((rc = orthonormalize_dev(ws, ws.Yd, ws.Y2, m, l, l, s))) return rc;
  } else {
    // Y = A Omega, Q = orth(Y), then q steps Q <- orth(A orth(A^T Q))
    if (left_product(cv, ws, X, SRC_DATA, nullptr, nullptr, ws.Wd, l, ws.Yd, l, l, s) != hipSuccess) return RPCA_EHIP;
    if ((rc = orthonormalize_dev(ws, ws.Yd, ws.Y2, m, l, l, s))) return rc;
    for (int q = 0; q < power_steps; ++q) {
      if (right_product(cv, ws, X, SRC_DATA, nullptr, nullptr, ws.Yd, l, ws.Zd, l, l, s) != hipSuccess)
        return RPCA_EHIP;
      if ((rc = orthonormalize_dev(ws, ws.Zd, ws.Wd, n, l, l, s))) return rc;
      if (left_product(cv, ws, X, SRC_DATA, nullptr, nullptr, ws.Zd, l, ws.Yd, l, l, s) != hipSuccess)
        return RPCA_EHIP;
      if ((rc = orthonormalize_dev(ws, ws.Yd, ws.Y2, m, l, l, s))) return rc;
    }
  }
  // B^T = A^T Q (n x l); B B^T = W Lam W^T
  if (right_product(cv, ws, X, SRC_DATA, nullptr, nullptr, ws.Yd, l, ws.Zd, l, l, s) != hipSuccess) return RPCA_EHIP;
  std::vector<double> Zb((size_t)n * l);
  if (hipMemcpyAsync(pinB, ws.Zd, Zb.size() * 8, hipMemcpyDeviceToHost, s) != hipSuccess) return RPCA_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return RPCA_EHIP;
  memcpy(Zb.data(), pinB, Zb.size() * 8);
  std::vector<double> BBt((size_t)l * l), lam(l), W((size_t)l * l);
  rpca::la::matmul_tn(Zb.data(), Zb.data(), BBt.data(), (int)n, l, l);
  rpca::la::sym_eig(BBt.data(), l, lam.data(), W.data());
  // U0 = Q W_k Sigma^{1/2}, V0 = B^T W_k Sigma^{-1/2}
  std::vector<double> TU((size_t)l * k, 0.0), TV((size_t)l * k, 0.0);
  for (int j = 0; j < k; ++j) {
    const double sg = sqrt(std::max(lam[j], 0.0));
    const double rs = sqrt(sg);
    const double irs = rs > 0 ? 1.0 / rs : 0.0;
    for (int i = 0; i < l; ++i) {
      TU[(size_t)i * k + j] = W[(size_t)i * l + j] * rs;
      TV[(size_t)i * k + j] = W[(size_t)i * l + j] * irs;
    }
  }
  memcpy(ws.pin, TU.data(), TU.size() * 8);
  if (hipMemcpyAsync(ws.T, ws.pin, TU.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess) return RPCA_EHIP;
  hipLaunchKernelGGL(k_row_transform, dim3((unsigned)((m * k + THREADS - 1) / THREADS)), dim3(THREADS), 0, s,
                     (const double*)ws.Yd, l, l, (const double*)ws.T, k, m, (double*)nullptr, U, k);
  if (hipGetLastError() != hipSuccess) return RPCA_EHIP;
  std::vector<float> V0((size_t)n * k);
  for (int64_t i = 0; i < n; ++i)
    for (int j = 0; j < k; ++j) {
      double sacc = 0.0;
      for (int t = 0; t < l; ++t) sacc += Zb[(size_t)i * l + t] * TV[(size_t)t * k + j];
      V0[(size_t)i * k + j] = (float)sacc;
    }
  float* pinC = reinterpret_cast<float*>(ws.pin + PIN_SMALL + (size_t)n * LMAX);  // n x k floats
  memcpy(pinC, V0.data(), V0.size() * 4);
  if (hipMemcpyAsync(V, pinC, V0.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess) return RPCA_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return RPCA_EHIP;
  return RPCA_OK;
}

// ----------------------------------------------------------------------------
// Convex baseline: accelerated proximal gradient on F(L) = lam_L ||L||_* + phi(L)
// (the solver class the paper compares against, Sec. 6.1), with the singular-value
// threshold computed by a randomized SVD of Z = Y - grad phi(Y) through the
// thin products (source SRC_PROX: Z is formed tile by tile from Y's factors and
// X, never stored).  Iterates are kept as balanced factors L = U V^T.

namespace {

// out (rows x k row-major) = [a P(:, 0:rp) | b Q(:, 0:rq) | 0]; P, Q rows x k row-major.
__global__ void k_pack_factors(const float* P, int rp, float a, const float* Q, int rq, float b, int64_t rows,
                               int k, float* out) {
  const int64_t o = (int64_t)blockIdx.x * THREADS + threadIdx.x;
  if (o >= rows * k) return;
  const int64_t i = o / k;
  const int cc = (int)(o % k);
  float v = 0.f;
  if (cc < rp) v = a * P[i * k + cc];
  else if (cc < rp + rq) v = b * Q[i * k + (cc - rp)];
  out[o] = v;
}

struct ProxState {
  rpca::CtxView cv;
  Workspace ws;
  const float* X;
  int oversample, power;
  uint64_t seed;
  int ell;                      // current sketch width
  std::vector<double> warm;     // n x rw right singular vectors of the last step
  int rw = 0;
  int truncated = 0;
  int draws = 0;
};

// One proximal step: L+ = SVT_{lam_L}(Z), Z = A B^T - grad phi(A B^T), into Uo, Vo
// (balanced factors, k columns, zero beyond the rank).  Returns F(L+) and its rank.
int prox_step(rpca_ctx* c, ProxState& P, const float* A, const float* B, float* Uo, float* Vo, int* rank_out,
              double* F_out, hipStream_t s) {
  const rpca::CtxView& cv = P.cv;
  const Workspace& ws = P.ws;
  const int64_t m = cv.m, n = cv.n;
  const int k = cv.k;
  const double lam_l = cv.lam_l;
  const int lcap = (int)std::min<int64_t>(LMAX, std::min(m, n));
  int rc;
  for (;;) {
    const int l = std::min(P.ell, lcap);
    // sketch: the last step's right singular vectors, then Gaussian columns
    std::vector<double> Om((size_t)n * l);
    const int rw = std::min(P.rw, l);
    ++P.draws;
    for (int64_t i = 0; i < n; ++i)
      for (int j = 0; j < l; ++j)
        Om[(size_t)i * l + j] = j < rw ? P.warm[(size_t)i * P.rw + j]
                                       : normal_deviate(P.seed + (uint64_t)P.draws, (uint64_t)(i * l + j));
    double* pinB = ws.pin + PIN_SMALL;  // n x l
    memcpy(pinB, Om.data(), Om.size() * 8);
    if (hipMemcpyAsync(ws.Wd, pinB, Om.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess) return RPCA_EHIP;
    if (left_product(cv, ws, P.X, SRC_PROX, A, B, ws.Wd, l, ws.Yd, l, l, s) != hipSuccess) return RPCA_EHIP;
    if ((rc = orthonormalize_dev(ws, ws.Yd, ws.Y2, m, l, l, s))) return rc;  // (syncs: Om may die)
    for (int q = 0; q < P.power; ++q) {
      if (right_product(cv, ws, P.X, SRC_PROX, A, B, ws.Yd, l, ws.Zd, l, l, s) != hipSuccess) return RPCA_EHIP;
      if ((rc = orthonormalize_dev(ws, ws.Zd, ws.Wd, n, l, l, s))) return rc;
      if (left_product(cv, ws, P.X, SRC_PROX, A, B, ws.Zd, l, ws.Yd, l, l, s) != hipSuccess) return RPCA_EHIP;
      if ((rc = orthonormalize_dev(ws, ws.Yd, ws.Y2, m, l, l, s))) return rc;
    }
    // Z^T Q (n x l) on the host; Z ~ Q W diag(sig) (Z^T Q W diag(1/sig))^T
    if (right_product(cv, ws, P.X, SRC_PROX, A, B, ws.Yd, l, ws.Zd, l, l, s) != hipSuccess) return RPCA_EHIP;
    std::vector<double> Zb((size_t)n * l);
    if (hipMemcpyAsync(pinB, ws.Zd, Zb.size() * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return RPCA_EHIP;
    memcpy(Zb.data(), pinB, Zb.size() * 8);
    std::vector<double> BBt((size_t)l * l), lam(l), W((size_t)l * l);
    rpca::la::matmul_tn(Zb.data(), Zb.data(), BBt.data(), (int)n, l, l);
    rpca::la::sym_eig(BBt.data(), l, lam.data(), W.data());
    int r = 0;
    while (r < l && sqrt(std::max(lam[r], 0.0)) > lam_l) ++r;
    if (r == l && l < lcap) {  // the sketch may miss values above the threshold: widen it
      P.ell = std::min(2 * l, lcap);
      continue;
    }
    if (r > k) {  // more singular values above lam_L than the factors hold
      r = k;
      P.truncated = 1;
    }
    // U+ = Q W_r diag(sqrt(sig - lam)), V+ = Z^T Q W_r diag(sqrt(sig - lam) / sig)
    std::vector<double> T((size_t)l * k, 0.0);
    std::vector<float> Vh((size_t)n * k, 0.f);
    std::vector<double> warm((size_t)n * std::max(r, 1), 0.0);
    double nuc = 0.0;
    for (int j = 0; j < r; ++j) {
      const double sig = sqrt(std::max(lam[j], 0.0));
      const double sh = sig - lam_l;
      nuc += sh;
      for (int t = 0; t < l; ++t) T[(size_t)t * k + j] = W[(size_t)t * l + j] * sqrt(sh);
      for (int64_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int t = 0; t < l; ++t) d += Zb[(size_t)i * l + t] * W[(size_t)t * l + j];
        warm[(size_t)i * std::max(r, 1) + j] = d / sig;
        Vh[(size_t)i * k + j] = (float)(d / sig * sqrt(sh));
      }
    }
    (void)nuc;
    memcpy(ws.pin, T.data(), T.size() * 8);
    if (hipMemcpyAsync(ws.T, ws.pin, T.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess) return RPCA_EHIP;
    hipLaunchKernelGGL(k_row_transform, dim3((unsigned)((m * k + THREADS - 1) / THREADS)), dim3(THREADS), 0, s,
                       (const double*)ws.Yd, l, l, (const double*)ws.T, k, m, (double*)nullptr, Uo, k);
    if (hipGetLastError() != hipSuccess) return RPCA_EHIP;
    float* pinC = reinterpret_cast<float*>(ws.pin + PIN_SMALL + (size_t)n * LMAX);  // n x k floats
    memcpy(pinC, Vh.data(), Vh.size() * 4);
    if (hipMemcpyAsync(Vo, pinC, Vh.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess) return RPCA_EHIP;
    // F(L+) = phi(L+) + lam_L ||L+||_* = f(U+, V+) for balanced factors
    if ((rc = rpca::ctx_objgrad_aux(c, P.X, Uo, Vo, ws.scal, ws.scal + 1, ws.gU, ws.gV, s))) return rc;
    double sc[2];
    if (hipMemcpyAsync(sc, ws.scal, sizeof(sc), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)  // T, Vh and sc are host frames of this call
      return RPCA_EHIP;
    *F_out = sc[0];
    *rank_out = r;
    P.warm.swap(warm);
    P.rw = r;
    P.ell = std::min(std::max(r + P.oversample, 8), lcap);
    return RPCA_OK;
  }
}

}  // namespace

namespace rpca {

int prox_solve_impl(rpca_ctx* c, const float* X, float* U, float* V, int32_t max_iter, double tol,
                    int32_t oversample, int32_t power, uint64_t seed, rpca_prox_info* info, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  ProxState P;
  P.cv = rpca::ctx_view(c);
  if (P.cv.mask) return RPCA_EINVAL;  // the proximal operator source assumes every entry observed
  const int64_t m = P.cv.m, n = P.cv.n;
  const int k = P.cv.k;
  int rc = get_workspace(c, &P.ws, s);
  if (rc) return rc;
  P.X = X;
  P.oversample = oversample;
  P.power = power;
  P.seed = seed;
  P.ell = (int)std::min<int64_t>(std::min<int64_t>(LMAX, std::min(m, n)), std::max(16, oversample + 8));
  // iterates: L (current), Lo (previous), Ln (new); A B^T = the extrapolated point
  float* buf = nullptr;
  const size_t fm = (size_t)m * k, fn = (size_t)n * k;
  if (hipMalloc(&buf, (fm + fn) * 4 * 4) != hipSuccess) return RPCA_ENOMEM;
  float *Uc = buf, *Vc = Uc + fm, *Uo = Vc + fn, *Vo = Uo + fm, *Un = Vo + fn, *Vn = Un + fm;
  float *A = Vn + fn, *B = A + fm;
  auto fail = [&](int e) {
    (void)hipStreamSynchronize(s);
    (void)hipFree(buf);
    return e;
  };
  if (hipMemsetAsync(buf, 0, (fm + fn) * 4 * 4, s) != hipSuccess) return fail(RPCA_EHIP);
  int rk = 0, ro = 0, restarts = 0, it = 0;
  // F(0) = phi(0)
  if ((rc = rpca::ctx_objgrad_aux(c, X, Uc, Vc, P.ws.scal, P.ws.scal + 1, P.ws.gU, P.ws.gV, s))) return fail(rc);
  double sc[2];
  if (hipMemcpyAsync(sc, P.ws.scal, sizeof(sc), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(RPCA_EHIP);
  double F = sc[0], rel = INFINITY, t = 1.0, beta = 0.0;
  auto pack = [&](float* out, int64_t rows, const float* Pm, int rp, float a, const float* Qm, int rq, float b) {
    hipLaunchKernelGGL(k_pack_factors, dim3((unsigned)((rows * k + THREADS - 1) / THREADS)), dim3(THREADS), 0, s,
                       Pm, rp, a, Qm, rq, b, rows, k, out);
    return hipGetLastError();
  };
  bool converged = false;
  for (it = 0; it < max_iter; ++it) {
    // extrapolated point Y = (1 + beta) L - beta Lo (plain L when the ranks do not fit)
    const bool mom = beta > 0.0 && rk + ro <= k;
    if (pack(A, m, Uc, rk, 1.f, Uo, mom ? ro : 0, 1.f) != hipSuccess ||
        pack(B, n, Vc, rk, (float)(mom ? 1.0 + beta : 1.0), Vo, mom ? ro : 0, (float)(-beta)) != hipSuccess)
      return fail(RPCA_EHIP);
    int rn = 0;
    double Fn = 0.0;
    if ((rc = prox_step(c, P, A, B, Un, Vn, &rn, &Fn, s))) return fail(rc);
    if (Fn > F && mom) {  // adaptive restart: drop the momentum, plain step from L
      ++restarts;
      t = 1.0;
      if (pack(A, m, Uc, rk, 1.f, Uo, 0, 1.f) != hipSuccess || pack(B, n, Vc, rk, 1.f, Vo, 0, 0.f) != hipSuccess)
        return fail(RPCA_EHIP);
      if ((rc = prox_step(c, P, A, B, Un, Vn, &rn, &Fn, s))) return fail(rc);
    }
    const double t_new = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
    beta = (t - 1.0) / t_new;
    t = t_new;
    rel = fabs(F - Fn) / std::max(fabs(Fn), 1e-300);
    F = Fn;
    // rotate: Lo <- L, L <- Ln
    std::swap(Uo, Uc);
    std::swap(Vo, Vc);
    std::swap(Uc, Un);
    std::swap(Vc, Vn);
    ro = rk;
    rk = rn;
    if (rel <= tol) {
      converged = true;
      ++it;
      break;
    }
  }
  if (hipMemcpyAsync(U, Uc, fm * 4, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(V, Vc, fn * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return fail(RPCA_EHIP);
  fail(RPCA_OK);  // synchronise and free the iterates
  if (info) {
    info->status = converged ? RPCA_OK : RPCA_ENOTCONV;
    info->iters = it;
    info->restarts = restarts;
    info->rank = rk;
    info->sketch = P.ell;
    info->truncated = P.truncated;
    info->F = F;
    info->rel_change = rel;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return converged ? RPCA_OK : RPCA_ENOTCONV;
}

}  // namespace rpca

extern "C" int rpca_prox_solve(rpca_ctx* c, const float* X, float* U, float* V, int32_t max_iter, double tol,
                               int32_t oversample, int32_t power_steps, uint64_t seed, rpca_prox_info* info,
                               void* stream) {
  if (!c || !X || !U || !V || max_iter < 1 || !(tol >= 0) || oversample < 0 || oversample > 32 ||
      power_steps < 0 || power_steps > 8)
    return RPCA_EINVAL;
  return rpca::prox_solve_impl(c, X, U, V, max_iter, tol, oversample, power_steps, seed, info, (hipStream_t)stream);
}
