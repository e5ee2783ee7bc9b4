// Fused Split-SPCP objective/gradient sweep for gfx950 (kernel template).
//
// One pass over X evaluates, tile by tile in registers,
//   R = U V^T - X                 (the residual inside the marginal phi, Sec. 5 eq. Thm5)
//   rho(R), G = Omega .* clip(R)  (Huber value and derivative, Sec. 1 eq. PhiDef, Sec. 3.2 eq. diff)
//   G^T U and G V                 (the two gradient products, chain rule on eq. smoothNC)
// so neither R nor G is ever written to memory.
//
// Work split.  The columns are cut into chunks (grid.y) small enough for the
// LDS budget below; every wave owns a contiguous run of 16-row strips and, for
// each strip, walks the chunk's 16-column tiles in groups of four.  The X loads
// of the next group are issued before the current group is computed and pinned
// there with a scheduling barrier, so about eight tiles per wave are in flight
// while registers stay independent of the chunk width.  Per 16x16 tile:
//   * R on MFMA with the accumulator seeded by -X.  In the MFMA output layout
//     (column j = lane%16, rows 4*(lane/16)+r) G is already the A operand of
//     G^T U with the K index running over rows.  The tile's G^T U is added into
//     the wave's private LDS accumulator (one writer per address, so no
//     atomics); the waves' accumulators are summed in a fixed order at the end.
//   * G V contracts over columns: G goes through a 16x17 per-wave LDS tile to
//     the transposed layout and into MFMA; the strip's G V accumulates in
//     registers over the chunk and is complete when the strip ends (one chunk)
//     or written as a per-chunk partial.
// FP32 mode uses v_mfma_f32_16x16x4_f32; BF16 mode rounds U, V and G to bf16 and
// uses v_mfma_f32_16x16x16_bf16 (FP32 accumulation, FP32 residual).  Every
// cross-wave and cross-workgroup sum runs in a fixed order: bitwise reproducible.
#pragma once

#include <math.h>

#include <type_traits>

#include "rpca_internal.h"

namespace rpca_sweep {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

constexpr int WAVES = 4;
constexpr int NT = 64 * WAVES;
constexpr int LDT = 17;   // padded row of the per-wave transpose tile
constexpr int PF = 4;     // tiles per load group
constexpr int LDS_LIMIT_FLOATS = 16384;  // 64 KB per workgroup

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

// Dynamic LDS (floats): sVt[cwp][KMAX+1] | sGV[WAVES][cwp][k] | sT[WAVES][16*LDT]
__host__ __device__ constexpr int lds_floats(int kb, int k, int cwp) {
  return cwp * (16 * kb + 1) + WAVES * cwp * k + WAVES * 16 * LDT;
}

// Widest chunk (multiple of 16 columns) whose staging fits the LDS budget.
__host__ __device__ constexpr int max_chunk(int kb, int k) {
  return 16 * ((LDS_LIMIT_FLOATS - WAVES * 16 * LDT) / (16 * (16 * kb + 1 + WAVES * k)));
}

// One work item: the strips of workgroup row `rg` against column chunk `ch`.
template <int KB, bool MASKED, bool TRIAL, bool BF16>
__device__ __forceinline__ void sweep_item(const SweepArgs& a, const int rg, const int ch, float* lds,
                                           double* sRed) {
  constexpr int KMAX = 16 * KB;
  constexpr int KQ = 4 * KB;
  constexpr int LDV = KMAX + 1;

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
  const int64_t m = a.m, n = a.n;
  const int k = a.k;
  const float lam_s = a.lam_s, lam_l = a.lam_l;
  const float* __restrict__ U = a.U[cur];
  const float* __restrict__ V = a.V[cur];
  const float* __restrict__ X = a.X;
  const float* __restrict__ dU = a.dU;

  const int64_t j_begin = (int64_t)ch * a.chunk_w;
  const int ncols = (int)((n - j_begin) < a.chunk_w ? (n - j_begin) : a.chunk_w);
  const int ntiles = (ncols + 15) >> 4;
  const int cwp = ntiles * 16;
  float* sVt = lds;
  float* sGVall = lds + cwp * LDV;
  float* sGV = sGVall + w * cwp * k;
  float* myT = sGVall + WAVES * cwp * k + w * 16 * LDT;

  // Stage the (trial) V rows of this chunk (zero padded); clear the G^T U accumulators.
  for (int idx = tid; idx < cwp * KMAX; idx += NT) {
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
    sVt[jl * LDV + kk] = v;
  }
  for (int idx = tid; idx < WAVES * cwp * k; idx += NT) sGVall[idx] = 0.f;
  __syncthreads();

  double f_acc = 0.0, uu_acc = 0.0, gud_acc = 0.0, gg_acc = 0.0;
  const int64_t nstrips = (m + 15) >> 4;
  const int64_t gw = (int64_t)rg * WAVES + w;
  const int64_t s_begin = gw * a.strips_per_wave;
  int64_t s_end = s_begin + a.strips_per_wave;
  if (s_end > nstrips) s_end = nstrips;
  const bool vec = a.xvec != 0;
  const int64_t tile_stride = 16 * m;  // floats between the same lane's columns in consecutive tiles

  for (int64_t s = s_begin; s < s_end; ++s) {
    const int64_t i0 = s * 16;
    const bool full = vec && (i0 + 16 <= m);
    // U_t operands of the strip (clamped addresses + selects: no branches).
    const int64_t i_c = (i0 + c < m) ? i0 + c : m - 1;
    const bool row_c_ok = i0 + c < m;
    float ua[KQ];      // R:      A[i = c][kk = 4q + g]
    float ub[4][KB];   // G^T U:  B[row 4g + r][kk = 16 kb + c]
    float dub[4][KB];  // dU at the ub positions (trial)
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
      const int kk = 4 * q + g;
      const int kkc = kk < k ? kk : k - 1;
      float v = U[i_c * k + kkc];
      if (TRIAL) v = fmaf(alpha, dU[i_c * k + kkc], v);
      ua[q] = (kk < k && row_c_ok) ? v : 0.f;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t i = i0 + 4 * g + r;
      const int64_t ic = i < m ? i : m - 1;
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        const int kk = 16 * kb + c;
        const int kkc = kk < k ? kk : k - 1;
        const bool ok = kk < k && i < m;
        float v = U[ic * k + kkc], dv = 0.f;
        if (TRIAL) {
          dv = dU[ic * k + kkc];
          v = fmaf(alpha, dv, v);
        }
        ub[r][kb] = ok ? v : 0.f;
        dub[r][kb] = ok ? dv : 0.f;
      }
    }
    // BF16 A operand of R: lane (c, g) holds U_t[i0 + c][16 kb + 4 g + e], e = 0..3
    s4 uab[KB], ubb[KB];
    if (BF16) {
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        float t4[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int kk = 16 * kb + 4 * g + e;
          const int kkc = kk < k ? kk : k - 1;
          float v = U[i_c * k + kkc];
          if (TRIAL) v = fmaf(alpha, dU[i_c * k + kkc], v);
          t4[e] = (kk < k && row_c_ok) ? v : 0.f;
        }
        uab[kb] = pack_bf16(t4[0], t4[1], t4[2], t4[3]);
        ubb[kb] = pack_bf16(ub[0][kb], ub[1][kb], ub[2][kb], ub[3][kb]);
      }
    }
    f4 gu[KB];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) gu[kb] = f4{0.f, 0.f, 0.f, 0.f};
    float ftile = 0.f, gtile = 0.f;
    // lane's column base (column c of tile 0 of the chunk, rows i0 + 4g .. +3)
    const float* xbase = X + (j_begin + c) * m + i0 + 4 * g;

    auto strip = [&](auto full_tag) {
      constexpr bool FULL = decltype(full_tag)::value;
      auto load_group = [&](int t0, f4(&xr)[PF], uint32_t(&br)[PF]) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
          const int jl = 16 * (t0 + u) + c;
          // columns past the chunk re-read its last column (valid address; zeroed at use)
          const int64_t off = (jl < ncols) ? (int64_t)(t0 + u) * tile_stride
                                           : (int64_t)(ncols - 1 - c) * m;
          if (FULL) {
            xr[u] = *reinterpret_cast<const f4*>(xbase + off);
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int64_t i = i0 + 4 * g + r;
              const float xv_r = xbase[off + ((i < m) ? r : (m - 1 - i0 - 4 * g))];
              xr[u][r] = (i < m) ? xv_r : 0.f;
            }
          }
          if (MASKED) {
            const int64_t j = j_begin + ((jl < ncols) ? jl : ncols - 1);
            br[u] = (a.mask[j * a.mw + (i0 >> 5)] >> ((int)(i0 & 31) + 4 * g)) & 0xFu;
          }
        }
      };
      auto tile = [&](int t, f4 xraw, uint32_t braw) {
        const int jl = 16 * t + c;
        const bool jok = jl < ncols;
        const f4 xv = jok ? xraw : f4{0.f, 0.f, 0.f, 0.f};
        const uint32_t bits = MASKED ? (jok ? braw : 0u) : 0xFu;
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
        // G^T U of the tile (K = the strip's 16 rows) into the wave's LDS accumulator
        f4 gvt[KB];
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) gvt[kb] = f4{0.f, 0.f, 0.f, 0.f};
        if (!BF16) {
#pragma unroll
          for (int kb = 0; kb < KB; ++kb)
#pragma unroll
            for (int r = 0; r < 4; ++r) gvt[kb] = mfma_f32(G[r], ub[r][kb], gvt[kb]);
        } else {
          const s4 gb = pack_bf16(G[0], G[1], G[2], G[3]);
#pragma unroll
          for (int kb = 0; kb < KB; ++kb) gvt[kb] = mfma_bf16(gb, ubb[kb], gvt[kb]);
        }
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          const int kk = 16 * kb + c;
          if (kk < k) {
#pragma unroll
            for (int r = 0; r < 4; ++r) sGV[(16 * t + 4 * g + r) * k + kk] += gvt[kb][r];
          }
        }
        // G V of the tile (K = the tile's 16 columns) from the transposed G
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
      };
      f4 xa[PF], xb[PF];
      uint32_t ba[PF] = {}, bb[PF] = {};
      load_group(0, xa, ba);
      for (int t0 = 0; t0 < ntiles; t0 += 2 * PF) {
        // group t0 is in xa; issue group t0+PF into xb, compute xa; then the mirror.
        // The prefetches are unconditional (past the chunk they re-read its last
        // column): a conditional load would force a full vmcnt(0) wait at the join.
        load_group(t0 + PF, xb, bb);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < PF; ++u)
          if (t0 + u < ntiles) tile(t0 + u, xa[u], ba[u]);
        if (t0 + PF >= ntiles) break;
        load_group(t0 + 2 * PF, xa, ba);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < PF; ++u)
          if (t0 + PF + u < ntiles) tile(t0 + PF + u, xb[u], bb[u]);
      }
    };
    if (full) strip(std::true_type{});
    else strip(std::false_type{});

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

  // Sum the waves' G^T U accumulators in a fixed order and write the partial.
  __syncthreads();
  float* gvp = a.gvpart + (int64_t)rg * n * k;
  for (int idx = tid; idx < ncols * k; idx += NT) {
    float acc = 0.f;
#pragma unroll
    for (int ww = 0; ww < WAVES; ++ww) acc += sGVall[ww * cwp * k + idx];
    gvp[j_begin * k + idx] = acc;
  }
  double* sp = a.spart + ((int64_t)rg * a.nchunks + ch) * RPCA_NSCAL;
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

template <int KB, bool MASKED, bool TRIAL, bool BF16>
__global__ __launch_bounds__(NT) void k_sweep(SweepArgs a) {
  extern __shared__ float lds[];
  __shared__ double sRed[WAVES];
  sweep_item<KB, MASKED, TRIAL, BF16>(a, blockIdx.x, blockIdx.y, lds, sRed);
}

// Batched sweep: one persistent launch for every instance of a batch.  Each
// workgroup pulls (instance, workgroup row, chunk) items from a queue (a
// counter advanced by one atomic per item, re-armed by the reduction that
// follows) until the list is drained.  The list is sorted by decreasing cost,
// so the long items start first and the short ones fill the tail.
template <bool MASKED, bool TRIAL, bool BF16>
__global__ __launch_bounds__(NT) void k_sweep_batch(const SweepArgs* args, const SweepItem* items, int nitems,
                                                    unsigned* head) {
  extern __shared__ float lds[];
  __shared__ double sRed[WAVES];
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(head, 1u);
    __syncthreads();
    const int it = s_item;
    __syncthreads();
    if (it >= nitems) break;
    const SweepItem b = items[it];
    if (b.kb == 1)
      sweep_item<1, MASKED, TRIAL, BF16>(args[b.inst], b.rg, b.ch, lds, sRed);
    else
      sweep_item<2, MASKED, TRIAL, BF16>(args[b.inst], b.rg, b.ch, lds, sRed);
    __syncthreads();
  }
}

template <bool MASKED, bool TRIAL, bool BF16>
hipError_t launch_batch(const SweepArgs* args, const SweepItem* items, int nitems, unsigned* head, int grid,
                        int lds_floats_max, hipStream_t s) {
  if (lds_floats_max > LDS_LIMIT_FLOATS) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_sweep_batch<MASKED, TRIAL, BF16>), dim3(grid), dim3(NT), lds_floats_max * sizeof(float),
                     s, args, items, nitems, head);
  return hipGetLastError();
}

template <bool MASKED, bool TRIAL, bool BF16>
hipError_t launch_kb(const SweepArgs& sa, hipStream_t s) {
  const int kb = (sa.k + 15) / 16;
  const int cwp = (int)(((sa.n < sa.chunk_w ? sa.n : sa.chunk_w) + 15) / 16) * 16;
  const int lds = lds_floats(kb, sa.k, cwp);
  if (lds > LDS_LIMIT_FLOATS || sa.chunk_w > max_chunk(kb, sa.k)) return hipErrorInvalidValue;
  const dim3 grid(sa.row_groups, sa.nchunks), block(NT);
  if (kb == 1)
    hipLaunchKernelGGL((k_sweep<1, MASKED, TRIAL, BF16>), grid, block, lds * sizeof(float), s, sa);
  else if (kb == 2)
    hipLaunchKernelGGL((k_sweep<2, MASKED, TRIAL, BF16>), grid, block, lds * sizeof(float), s, sa);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace rpca_sweep
