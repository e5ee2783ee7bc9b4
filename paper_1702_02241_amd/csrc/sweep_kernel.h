// Fused Split-SPCP objective/gradient sweep for gfx950 (kernel template).
//
// One pass over X evaluates, tile by tile in registers,
//   R = U V^T - X                 (the residual inside the marginal phi, Sec. 5 eq. Thm5)
//   rho(R), G = Omega .* clip(R)  (Huber value and derivative, Sec. 1 eq. PhiDef, Sec. 3.2 eq. diff)
//   G^T U and G V                 (the two gradient products, chain rule on eq. smoothNC)
// so neither R nor G is ever written to memory.
//
// Work split.  The columns are cut into chunks of 16*TJ (grid.y); every wave
// owns a contiguous run of 16-row strips and, for each strip, walks all TJ
// column tiles of its chunk in a fully unrolled loop with no branches (padded
// columns compute zeros), so the compiler can issue the X loads of many tiles
// ahead.  Per 16x16 tile:
//   * R on MFMA with the accumulator seeded by -X.  In the MFMA output layout
//     (column j = lane%16, rows 4*(lane/16)+r) G is already the A operand of
//     G^T U with the K index running over rows: G^T U accumulates in registers
//     per tile across all strips of the wave and is combined over the
//     workgroup's waves once, at the end, in a fixed order.
//   * G V contracts over columns: G goes through a 16x17 per-wave LDS tile to
//     the transposed layout and into MFMA; the strip's G V accumulates in
//     registers across its tiles and is complete when the strip ends (one
//     chunk) or written as a per-chunk partial.
// FP32 mode uses v_mfma_f32_16x16x4_f32; BF16 mode rounds U, V and G to bf16 and
// uses v_mfma_f32_16x16x16_bf16 (FP32 accumulation, FP32 residual).  All
// cross-workgroup sums run in a fixed order: results are bitwise reproducible.
#pragma once

#include <math.h>

#include "rpca_internal.h"

namespace rpca_sweep {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

constexpr int WAVES = 4;
constexpr int NT = 64 * WAVES;
constexpr int LDT = 17;  // padded row of the per-wave transpose tile

__device__ __forceinline__ f4 mfma_f32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f4 mfma_bf16(s4 a, s4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// FP32 -> BF16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ short bf16_bits(float x) {
  const uint32_t u = __float_as_uint(x);
  return (short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ s4 pack_bf16(float a, float b, float c, float d) {
  return s4{bf16_bits(a), bf16_bits(b), bf16_bits(c), bf16_bits(d)};
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < WAVES; ++w) r += sh[w];
  return r;
}

// LDS: sVt[16 TJ][KMAX+1] (V_t of the chunk) | per-wave transpose tile [WAVES][16*LDT].
// At the end the G^T U combine buffer [16 TJ][KMAX] reuses the sVt space.
template <int KB, int TJ>
constexpr int lds_floats() {
  return 16 * TJ * (16 * KB + 1) + WAVES * 16 * LDT;
}

template <int KB, int TJ, bool MASKED, bool TRIAL, bool BF16>
__global__ __launch_bounds__(NT) void k_sweep(SweepArgs a) {
  constexpr int KMAX = 16 * KB;
  constexpr int KQ = 4 * KB;
  constexpr int LDV = KMAX + 1;
  constexpr int CW = 16 * TJ;
  __shared__ float lds[lds_floats<KB, TJ>()];
  __shared__ double sRed[WAVES];
  float* sVt = lds;
  float* sT = lds + CW * LDV;

  int cur = 0, outi = 0;
  float alpha = 0.f;
  if (TRIAL) {
    const SolverState* st = a.st;
    if (st->phase != PH_TRIAL) return;
    cur = st->cur;
    alpha = (float)st->alpha;
    outi = 1 - cur;
  }
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int ch = blockIdx.y;
  const int64_t m = a.m, n = a.n;
  const int k = a.k;
  const float lam_s = a.lam_s, lam_l = a.lam_l;
  const float* __restrict__ U = a.U[cur];
  const float* __restrict__ V = a.V[cur];
  const float* __restrict__ X = a.X;
  const float* __restrict__ dU = a.dU;
  float* myT = sT + w * 16 * LDT;

  const int64_t j_begin = (int64_t)ch * CW;
  const int ncols = (int)((n - j_begin) < CW ? (n - j_begin) : CW);

  // Stage the (trial) V rows of this chunk, zero padded.
  for (int idx = tid; idx < CW * KMAX; idx += NT) {
    const int jl = idx / KMAX, kk = idx % KMAX;
    float v = 0.f;
    if (jl < ncols && kk < k) {
      const int64_t o = (j_begin + jl) * k + kk;
      v = V[o];
      if (TRIAL) {
        v = fmaf(alpha, a.dV[o], v);
        if (blockIdx.x == 0) a.Vt[outi][o] = v;
      }
    }
    sVt[jl * LDV + kk] = v;
  }
  __syncthreads();

  f4 gv[TJ][KB];
#pragma unroll
  for (int t = 0; t < TJ; ++t)
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) gv[t][kb] = f4{0.f, 0.f, 0.f, 0.f};
  double f_acc = 0.0, uu_acc = 0.0, gud_acc = 0.0, gg_acc = 0.0;

  const int64_t nstrips = (m + 15) >> 4;
  const int64_t gw = (int64_t)blockIdx.x * WAVES + w;
  const int64_t s_begin = gw * a.strips_per_wave;
  int64_t s_end = s_begin + a.strips_per_wave;
  if (s_end > nstrips) s_end = nstrips;
  const bool vec = a.xvec != 0;

  for (int64_t s = s_begin; s < s_end; ++s) {
    const int64_t i0 = s * 16;
    const bool full = vec && (i0 + 16 <= m);
    // U_t operands of the strip.
    float ua[KQ];        // R:      A[i = c][kk = 4q + g]
    float ub[4][KB];     // G^T U:  B[row 4g + r][kk = 16 kb + c]
    float dub[4][KB];    // dU at the ub positions (trial)
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
      const int kk = 4 * q + g;
      const int64_t i = i0 + c;
      float v = 0.f;
      if (kk < k && i < m) {
        v = U[i * k + kk];
        if (TRIAL) v = fmaf(alpha, dU[i * k + kk], v);
      }
      ua[q] = v;
    }
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
            dv = dU[i * k + kk];
            v = fmaf(alpha, dv, v);
          }
        }
        ub[r][kb] = v;
        dub[r][kb] = dv;
      }
    s4 uab[KB], ubb[KB];
    if (BF16) {
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        // A[i = c][kk = 16 kb + 4 g + e] = ua[4 kb + e] of lanes with the same c
        float t4[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int kk = 16 * kb + 4 * g + e;
          const int64_t i = i0 + c;
          float v = 0.f;
          if (kk < k && i < m) {
            v = U[i * k + kk];
            if (TRIAL) v = fmaf(alpha, dU[i * k + kk], v);
          }
          t4[e] = v;
        }
        uab[kb] = pack_bf16(t4[0], t4[1], t4[2], t4[3]);
        ubb[kb] = pack_bf16(ub[0][kb], ub[1][kb], ub[2][kb], ub[3][kb]);
      }
    }
    f4 gu[KB];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) gu[kb] = f4{0.f, 0.f, 0.f, 0.f};
    float ftile = 0.f, gtile = 0.f;

#pragma unroll
    for (int t = 0; t < TJ; ++t) {
      const int jl = 16 * t + c;
      const bool jok = jl < ncols;
      const int64_t j = j_begin + jl;
      const float* xp = X + j * m + i0 + 4 * g;
      f4 xv;
      if (full) {
        xv = jok ? *reinterpret_cast<const f4*>(xp) : f4{0.f, 0.f, 0.f, 0.f};
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) xv[r] = (jok && i0 + 4 * g + r < m) ? xp[r] : 0.f;
      }
      uint32_t bits = 0xFu;
      if (MASKED) bits = jok ? (a.mask[j * a.mw + (i0 >> 5)] >> ((int)(i0 & 31) + 4 * g)) & 0xFu : 0u;
      f4 acc = -xv;
      if (!BF16) {
#pragma unroll
        for (int q = 0; q < KQ; ++q) acc = mfma_f32(ua[q], sVt[jl * LDV + 4 * q + g], acc);
      } else {
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          const float* vr = sVt + jl * LDV + 16 * kb + 4 * g;
          acc = mfma_bf16(uab[kb], pack_bf16(vr[0], vr[1], vr[2], vr[3]), acc);
        }
      }
      float G[4];
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
        myT[(4 * g + r) * LDT + c] = gr;
      }
      // G^T U for this tile (K = the strip's 16 rows)
      if (!BF16) {
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
#pragma unroll
          for (int r = 0; r < 4; ++r) gv[t][kb] = mfma_f32(G[r], ub[r][kb], gv[t][kb]);
      } else {
        const s4 gb = pack_bf16(G[0], G[1], G[2], G[3]);
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) gv[t][kb] = mfma_bf16(gb, ubb[kb], gv[t][kb]);
      }
      // G V for this tile (K = the tile's 16 columns) from the transposed G
      if (!BF16) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float gt = myT[c * LDT + 4 * q + g];
#pragma unroll
          for (int kb = 0; kb < KB; ++kb)
            gu[kb] = mfma_f32(gt, sVt[(16 * t + 4 * q + g) * LDV + 16 * kb + c], gu[kb]);
        }
      } else {
        const float* tr = myT + c * LDT + 4 * g;
        const s4 gtb = pack_bf16(tr[0], tr[1], tr[2], tr[3]);
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          const float* vc = sVt + (16 * t + 4 * g) * LDV + 16 * kb + c;
          gu[kb] = mfma_bf16(gtb, pack_bf16(vc[0], vc[LDV], vc[2 * LDV], vc[3 * LDV]), gu[kb]);
        }
      }
    }
    f_acc += (double)ftile;
    gg_acc += (double)gtile;
    // Finish the strip's rows: lane (g, c) holds G V for rows i0+4g+r, column 16 kb + c.
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t i = i0 + 4 * g + r;
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        const int kk = 16 * kb + c;
        if (kk < k && i < m) {
          const int64_t o = i * k + kk;
          if (a.nchunks == 1) {
            const float gval = fmaf(lam_l, ub[r][kb], gu[kb][r]);
            a.gU[outi][o] = gval;
            if (TRIAL) gud_acc += (double)gval * (double)dub[r][kb];
          } else {
            a.gupart[(int64_t)ch * m * k + o] = gu[kb][r];
          }
          if (ch == 0) {
            uu_acc += (double)ub[r][kb] * (double)ub[r][kb];
            if (TRIAL) a.Ut[outi][o] = ub[r][kb];
          }
        }
      }
    }
  }

  // Combine the waves' G^T U (fixed order) in the V staging space, write the partial.
  __syncthreads();
  float* sC = lds;
  for (int ww = 0; ww < WAVES; ++ww) {
    if (w == ww) {
#pragma unroll
      for (int t = 0; t < TJ; ++t)
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int idx = (16 * t + 4 * g + r) * KMAX + 16 * kb + c;
            sC[idx] = (ww == 0 ? 0.f : sC[idx]) + gv[t][kb][r];
          }
    }
    __syncthreads();
  }
  float* gvp = a.gvpart + (int64_t)blockIdx.x * n * k;
  for (int idx = tid; idx < ncols * k; idx += NT) {
    const int jl = idx / k, kk = idx - jl * k;
    gvp[(j_begin + jl) * k + kk] = sC[jl * KMAX + kk];
  }
  double* sp = a.spart + ((int64_t)blockIdx.x * a.nchunks + ch) * RPCA_NSCAL;
  const double v0 = block_sum(f_acc, sRed);
  const double v1 = block_sum(uu_acc, sRed);
  const double v2 = block_sum(gud_acc, sRed);
  const double v3 = block_sum(gg_acc, sRed);
  if (tid == 0) {
    sp[0] = v0;
    sp[1] = v1;
    sp[2] = v2;
    sp[3] = v3;
  }
}

// Tile counts instantiated per rank block count (a chunk uses the smallest
// count >= its 16-column tiles).
constexpr int TJ1[] = {1, 2, 3, 4, 5, 6, 8, 10, 13, 16};
constexpr int TJ2[] = {1, 2, 3, 4, 6, 8};

template <bool MASKED, bool TRIAL, bool BF16>
hipError_t launch_tj(const SweepArgs& sa, int kb, int tj, hipStream_t s) {
  const dim3 grid(sa.row_groups, sa.nchunks), block(NT);
#define RPCA_CASE(KBV, TJV)                                                           \
  if (kb == KBV && tj == TJV) {                                                       \
    hipLaunchKernelGGL((k_sweep<KBV, TJV, MASKED, TRIAL, BF16>), grid, block, 0, s, sa); \
    return hipGetLastError();                                                         \
  }
  RPCA_CASE(1, 1) RPCA_CASE(1, 2) RPCA_CASE(1, 3) RPCA_CASE(1, 4) RPCA_CASE(1, 5)
  RPCA_CASE(1, 6) RPCA_CASE(1, 8) RPCA_CASE(1, 10) RPCA_CASE(1, 13) RPCA_CASE(1, 16)
  RPCA_CASE(2, 1) RPCA_CASE(2, 2) RPCA_CASE(2, 3) RPCA_CASE(2, 4) RPCA_CASE(2, 6) RPCA_CASE(2, 8)
#undef RPCA_CASE
  return hipErrorInvalidValue;
}

}  // namespace rpca_sweep
