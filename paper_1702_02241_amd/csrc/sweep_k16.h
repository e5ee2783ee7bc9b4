// Objective/gradient sweep for rank k <= 16 (included by sweep_kernel.h).
#pragma once

// ---------------------------------------------------------------------------
// Rank k <= 16: one 16-wide rank block.  Operand layouts in LDS are chosen so
// that every MFMA operand of a tile is one 16-byte LDS read per lane:
//
//   FP32 residual   B[K=g][N=c] at step q = V[col 16t+c][kk 4q+g]
//                   sVr[col][g][q]                    (row stride RS floats)
//   FP32 G V        B[K=g][N=c] at step q = V[col 16t+4q+g][kk c]
//                   sVg[t][g][c][q]                   (256 floats per tile)
//   FP32 transpose  lane (c, g) writes G[row 4g+r][col c] to T[row][c&3][c>>2]
//                   and reads T[row c][g][0..3] = G[row c][col 4q+g], q = 0..3
//   BF16 residual   v_mfma_f32_16x16x32_bf16, one per rank block kk in [8j, 8j+8):
//                   lane group g supplies (g = 0) hi(U) hi(V), (1) hi(U) lo(V),
//                   (2) lo(U) hi(V), (3) zeros, with hi = bf16(x), lo = bf16(x - hi):
//                   U V^T to about 2^-16 relative, so the residual keeps close to
//                   FP32 accuracy while the MFMA work stays a fraction of FP32's
//                   sVrb[col][j][g][8]  (bf16, holding -V: the tile product is X - U V^T)
//   BF16 G V        B[K=4g+e][N=c] = bf16 V[col 16t+4g+e][kk c]
//                   sVgb[t][g][c][e]    (bf16)
//   BF16 transpose  bf16 T[row][col] (row stride TSB), lane (c, g) reads the 4
//                   columns 4g..4g+3 of row c: the A operand of G V as it is
namespace k16 {
constexpr int RS = 20;   // row stride of sVr (floats): 16 used, 16-byte aligned rows
constexpr int TS = 20;   // row stride of a transpose tile (floats)
constexpr int NTB = 4;   // transpose tiles per wave (one group of tiles in flight)
constexpr int TSB = 24;  // row stride of a bf16 transpose tile (shorts), 8-byte aligned rows
__host__ __device__ constexpr int nsteps_bf16(int k) { return (k + 7) / 8; }
// floats of dynamic LDS for a chunk of cwp columns
__host__ __device__ constexpr int lds_start(int k, int cwp, bool bf16) {
  return bf16 ? cwp * nsteps_bf16(k) * 16 + cwp * 8 + WAVES * NTB * 16 * TS
              : cwp * RS + cwp * 16 + WAVES * NTB * 16 * TS;
}
__host__ __device__ constexpr int lds_floats(int k, int cwp) {
  // the larger of the two precisions' start layouts and the end reduction
  return (lds_start(k, cwp, false) > lds_start(k, cwp, true) ? lds_start(k, cwp, false)
                                                                : lds_start(k, cwp, true)) > WAVES * cwp * k
             ? (lds_start(k, cwp, false) > lds_start(k, cwp, true) ? lds_start(k, cwp, false)
                                                                    : lds_start(k, cwp, true))
             : WAVES * cwp * k;
}
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef uint32_t u4v __attribute__((ext_vector_type(4)));
typedef uint32_t u2v_ __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f4 mfma_bf16x32(u4v a, u4v b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}
// two floats to packed bf16 (round to nearest even, hardware conversion)
__device__ __forceinline__ uint32_t pk2(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f2v{a, b}, bf16x2));
}
__device__ __forceinline__ uint16_t bf16_bits(float x) {
  return __builtin_bit_cast(uint16_t, (__bf16)x);
}
__device__ __forceinline__ float bf16_val(uint16_t b) {
  return __builtin_bit_cast(float, (uint32_t)b << 16);
}
}  // namespace k16

template <int TMAX, bool MASKED, bool TRIAL, bool BF16, typename Args, bool ELASTIC>
__device__ __forceinline__ void sweep_item_k16(const Args& a, const int rg, const int ch, float* lds, double* sRed) {
  using namespace k16;
  constexpr int PF = TMAX >= 8 ? 4 : 2;
  constexpr int NG = (TMAX + PF - 1) / PF;
  // FP32: one group in flight ahead of the computed one (three groups measured slower:
  // the waves do not wait on these loads); BF16: three (its products leave the
  // registers for a deeper ring)
  constexpr int NBUF = BF16 ? (NG >= 4 ? 4 : 2) : 2;
  static_assert(NG % NBUF == 0, "group ring must line up with strips");
  constexpr int NS_MAX = 2;  // BF16 split steps for k <= 16

  int cur = 0, outi = 0;
  float alpha = 0.f;
  if (TRIAL) {
    const SolverState* st = a.st;
    if (st->phase != PH_TRIAL) return;
    cur = st->cur;
    alpha = (float)st->alpha;
    outi = 1 - cur;
  }
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c = lane & 15, g = lane >> 4;
  const int64_t m = a.m, n = a.n;
  const int k = a.k;
  const float lam_s = a.lam_s, lam_l = a.lam_l, kappa = a.kappa;
  const float* __restrict__ U = a.U[cur];
  const float* __restrict__ V = a.V[cur];
  const float* __restrict__ X = a.X;
  const float* __restrict__ dU = a.dU;
  const int ns = BF16 ? nsteps_bf16(k) : 0;

  const int64_t j_begin = (int64_t)ch * a.chunk_w;
  const int ncols = (int)((n - j_begin) < a.chunk_w ? (n - j_begin) : a.chunk_w);
  const int ntiles = (ncols + 15) >> 4;
  const int cwp = ntiles * 16;
  // start layout
  float* sVr = lds;                                      // FP32: [cwp][RS]
  float* sVg = lds + cwp * RS;                           // FP32: [ntiles][256]
  uint16_t* sVrb = reinterpret_cast<uint16_t*>(lds);     // BF16: [cwp][ns][4][8]
  uint16_t* sVgb = reinterpret_cast<uint16_t*>(lds + cwp * ns * 16);  // BF16: [ntiles][64][4]
  float* sT = lds + (BF16 ? cwp * ns * 16 + cwp * 8 : cwp * RS + cwp * 16);
  float* myT = sT + w * NTB * 16 * TS;

  f4 gva[TMAX];
#pragma unroll
  for (int t = 0; t < TMAX; ++t) gva[t] = f4{0.f, 0.f, 0.f, 0.f};

  double f_acc = 0.0, uu_acc = 0.0, gud_acc = 0.0, gg_acc = 0.0;
  const int64_t nstrips = (m + 15) >> 4;
  const int64_t R = a.row_groups;
  // workgroup rows split whole pairs of strips (a 128-byte line of a column holds two
  // strips' rows), so that the two halves of every line are read by the same
  // workgroup at about the same time
  const int64_t npairs = (nstrips + 1) >> 1;
  const int64_t s_lo = 2 * ((int64_t)rg * npairs / R);
  const int64_t s_hi_p = 2 * (((int64_t)rg + 1) * npairs / R);
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

  // per-strip U operands
  struct Ops {
    float ua[4];      // FP32 residual A: -U'[row c][4q+g]
    u4v uab[NS_MAX];  // BF16 residual A: 8 bf16 of U'[row c][8j ..]: hi (g 0, 1), lo (g 2), 0 (g 3)
    u2v_ ubb;         // BF16 G^T U B: bf16 of ub[0..3]
    float ub[4];      // G^T U B: U'[row 4g+r][c]
    float dub[4];     // dU at the ub positions (trial)
  };
  // the strip's U rows: uniform base pointer, 32-bit lane offsets (rows past m clamp to m - 1)
  auto load_ops = [&](int64_t s, Ops& o) {
    const int64_t i0 = s * 16;
    const bool full = i0 + 16 <= m;
    const float* __restrict__ Us = U + i0 * k;
    const float* __restrict__ dUs = dU + i0 * k;
    const int rows_in = full ? 16 : (int)(m - i0);
    const bool row_c_ok = c < rows_in;
    const int rc = row_c_ok ? c : rows_in - 1;
    if (!BF16) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int kk = 4 * q + g;
        const int kkc = kk < k ? kk : k - 1;
        const uint32_t off = (uint32_t)(rc * k + kkc);
        float v = Us[off];
        if (TRIAL) v = fmaf(alpha, dUs[off], v);
        o.ua[q] = (kk < k && row_c_ok) ? -v : 0.f;
      }
    } else {
#pragma unroll
      for (int j = 0; j < NS_MAX; ++j) {
        u4v w4 = {0u, 0u, 0u, 0u};
        if (j < ns) {
          float v[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int kk = 8 * j + e;  // uniform: the rank index test is scalar
            float x = 0.f;
            if (kk < k) {
              const uint32_t off = (uint32_t)(rc * k + kk);
              x = Us[off];
              if (TRIAL) x = fmaf(alpha, dUs[off], x);
            }
            v[e] = row_c_ok ? x : 0.f;
          }
#pragma unroll
          for (int h = 0; h < 4; ++h) {
            const uint32_t hi = pk2(v[2 * h], v[2 * h + 1]);
            const float h0 = __builtin_bit_cast(float, hi << 16), h1 = __builtin_bit_cast(float, hi & 0xFFFF0000u);
            const uint32_t lo = pk2(v[2 * h] - h0, v[2 * h + 1] - h1);
            w4[h] = g == 3 ? 0u : (g == 2 ? lo : hi);
          }
        }
        o.uab[j] = w4;
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int rr = 4 * g + r;
      const bool ok = c < k && rr < rows_in;
      const uint32_t off = (uint32_t)((rr < rows_in ? rr : rows_in - 1) * k + (c < k ? c : k - 1));
      float v = Us[off], dv = 0.f;
      if (TRIAL) {
        dv = dUs[off];
        v = fmaf(alpha, dv, v);
      }
      o.ub[r] = ok ? v : 0.f;
      o.dub[r] = ok ? dv : 0.f;
    }
    if (BF16) o.ubb = u2v_{pk2(o.ub[0], o.ub[1]), pk2(o.ub[2], o.ub[3])};
  };

  // X of the chunk through one buffer resource (its ncols columns; the pipelined path
  // needs them within 2^31 bytes): tile t of strip s at soffset 64 m t, lane offset
  // 4 (c m + 16 s + 4 g); columns past the chunk and dead prefetches read zero
  const __amdgpu_buffer_rsrc_t xrs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(X + j_begin * m), (short)0, (int)((int64_t)ncols * m * 4), BUF_DWORD3);
  const uint32_t lane_off = (uint32_t)(c * m * 4 + 16 * g);
  auto load_group = [&](int64_t s, int gi, f4(&xr)[PF], uint32_t(&br)[PF], bool live) {
    // the tile's column offset goes into the VGPR offset: the buffer range check covers
    // the VGPR and instruction offsets only, not the SGPR offset
    const uint32_t voff = live ? lane_off + (uint32_t)(s * 64) : 0xC0000000u;
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int t = gi * PF + u;
      if (t < TMAX) {
        xr[u] = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(xrs, voff + (uint32_t)(64 * t * m), 0, 0));
        if (MASKED && 16 * t < ncols) {
          const int jl = 16 * t + c;
          const int64_t i0 = s * 16;
          const uint32_t* __restrict__ mrow = a.mask + (j_begin + 16 * t) * a.mw + (i0 >> 5);
          const uint32_t moff = (uint32_t)(((jl < ncols) ? c : (ncols - 1 - 16 * t)) * a.mw);
          br[u] = (mrow[moff] >> ((int)(i0 & 31) + 4 * g)) & 0xFu;
        }
      }
    }
  };

  // Huber step on the negated residual of one tile: Gn = -G (4 entries)
  auto huber_tile = [&](const f4& acc, uint32_t bits, float (&Gn)[4], float& ftile, float& gtile) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float Rn = acc[r];
      float cl = __builtin_amdgcn_fmed3f(Rn, -lam_s, lam_s);
      if (MASKED && !((bits >> r) & 1u)) cl = 0.f;
      if (!ELASTIC) {
        // rho = c R - c^2 / 2 with c = clip(R): sum c R and c^2 separately
        ftile = fmaf(cl, (MASKED && !((bits >> r) & 1u)) ? 0.f : Rn, ftile);
        gtile = fmaf(cl, cl, gtile);
        Gn[r] = cl;
      } else {
        float gtmp = 0.f;
        Gn[r] = huber<true>(Rn, lam_s, kappa, MASKED ? ((bits >> r) & 1u) : 1u, ftile, gtmp);
        gtile += gtmp;
      }
    }
  };

  // One group of PF tiles [t0, t0 + PF) of the current strip: residual MFMAs for all of
  // them, then Huber + transpose, G^T U, G V.  Tiles at or past ntiles are skipped
  // (uniform branches).
  auto tile_group = [&](int gi, const Ops& o, f4(&xr)[PF], const uint32_t(&br)[PF], float& ftile, float& gtile,
                        f4& gu) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int t = gi * PF + u;
      if (t >= TMAX || t >= ntiles) continue;
      const int col = 16 * t + c;
      if (!BF16) {
        const f4 vr = *reinterpret_cast<const f4*>(sVr + col * RS + g * 4);
        xr[u] = mfma_f32(o.ua[0], vr[0], xr[u]);
        xr[u] = mfma_f32(o.ua[1], vr[1], xr[u]);
        xr[u] = mfma_f32(o.ua[2], vr[2], xr[u]);
        if (k > 12) xr[u] = mfma_f32(o.ua[3], vr[3], xr[u]);
      } else {
#pragma unroll
        for (int j = 0; j < NS_MAX; ++j) {
          if (j < ns) {
            const u4v vb = *reinterpret_cast<const u4v*>(sVrb + ((col * ns + j) * 4 + g) * 8);
            xr[u] = mfma_bf16x32(o.uab[j], vb, xr[u]);
          }
        }
      }
    }
    float G[PF][4];
    u2v_ Gp[PF];  // BF16: the tile's G rows 4g..4g+3 of column c, packed
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int t = gi * PF + u;
      if (t >= TMAX || t >= ntiles) continue;
      const int jl = 16 * t + c;
      const uint32_t bits = MASKED ? ((jl < ncols) ? br[u] : 0u) : 0xFu;
      huber_tile(xr[u], bits, G[u], ftile, gtile);
      if (!BF16) {
        float* tT = myT + u * 16 * TS;
#pragma unroll
        for (int r = 0; r < 4; ++r) tT[(4 * g + r) * TS + (c & 3) * 4 + (c >> 2)] = G[u][r];
      } else {
        Gp[u] = u2v_{pk2(G[u][0], G[u][1]), pk2(G[u][2], G[u][3])};
        uint16_t* tT = reinterpret_cast<uint16_t*>(myT + u * 16 * TS);
        tT[(4 * g + 0) * TSB + c] = (uint16_t)Gp[u][0];
        tT[(4 * g + 1) * TSB + c] = (uint16_t)(Gp[u][0] >> 16);
        tT[(4 * g + 2) * TSB + c] = (uint16_t)Gp[u][1];
        tT[(4 * g + 3) * TSB + c] = (uint16_t)(Gp[u][1] >> 16);
      }
    }
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int t = gi * PF + u;
      if (t >= TMAX || t >= ntiles) continue;
      if (!BF16) {
#pragma unroll
        for (int r = 0; r < 4; ++r) gva[t] = mfma_f32(G[u][r], o.ub[r], gva[t]);
      } else {
        gva[t] = mfma_bf16(__builtin_bit_cast(s4, Gp[u]), __builtin_bit_cast(s4, o.ubb), gva[t]);
      }
    }
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int t = gi * PF + u;
      if (t >= TMAX || t >= ntiles) continue;
      if (!BF16) {
        const float* tT = myT + u * 16 * TS;
        const f4 gt = *reinterpret_cast<const f4*>(tT + c * TS + g * 4);
        const f4 vg = *reinterpret_cast<const f4*>(sVg + t * 256 + g * 64 + c * 4);
#pragma unroll
        for (int q = 0; q < 4; ++q) gu = mfma_f32(gt[q], vg[q], gu);
      } else {
        const uint16_t* tT = reinterpret_cast<const uint16_t*>(myT + u * 16 * TS);
        const s4 gt = *reinterpret_cast<const s4*>(tT + c * TSB + 4 * g);
        const s4 vg = *reinterpret_cast<const s4*>(sVgb + (t * 64 + g * 16 + c) * 4);
        gu = mfma_bf16(gt, vg, gu);
      }
    }
  };

  auto strip_end = [&](int64_t s, const Ops& o, const f4& gu, float ftile, float gtile) {
    const int64_t i0 = s * 16;
    if (!ELASTIC) {
      f_acc += (double)ftile - 0.5 * (double)gtile;
    } else {
      f_acc += (double)ftile;
    }
    gg_acc += (double)gtile;
    float reg[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) reg[r] = o.ub[r];
    const float* __restrict__ pc = a.pc;
    if (pc) {
      // A M_U for the strip's rows: rows through the wave's first transpose tile
      const float* __restrict__ MU = pc + k * k;
#pragma unroll
      for (int r = 0; r < 4; ++r) myT[(4 * g + r) * TS + c] = o.ub[r];
#pragma unroll
      for (int r = 0; r < 4; ++r) reg[r] = 0.f;
      for (int t = 0; t < k; ++t) {
        const float mv = (c < k) ? MU[t * k + c] : 0.f;
#pragma unroll
        for (int r = 0; r < 4; ++r) reg[r] = fmaf(myT[(4 * g + r) * TS + t], mv, reg[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t i = i0 + 4 * g + r;
      if (c < k && i < m) {
        const int64_t oo = i * k + c;
        if (a.nchunks == 1) {
          const float gval = fmaf(lam_l, reg[r], -gu[r]);
          a.gU[outi][oo] = gval;
          if (TRIAL) gud_acc += (double)gval * (double)o.dub[r];
        } else {
          a.gupart[(int64_t)ch * m * k + oo] = -gu[r];
        }
        if (ch == 0) {
          uu_acc += (double)o.ub[r] * (double)reg[r];
          if (TRIAL) a.Ut[outi][oo] = o.ub[r];
        }
      }
    }
  };

  // the first strip's operands and X groups are requested before V' is staged, so
  // that their latency overlaps the staging
  constexpr int D = NBUF - 1;
  Ops ops, nops;
  f4 xbuf[NBUF][PF];
  uint32_t bbuf[NBUF][PF] = {};
  if (n_pipe > 0) {
    load_ops(s_first, ops);
#pragma unroll
    for (int d = 0; d < D; ++d) load_group(s_first, d, xbuf[d], bbuf[d], true);
  }

  // ---- stage V' (the trial point, or B W^T in preconditioned variables) ----
  // raw rows first (into the transpose area), then the operand layouts
  {
    float* raw = sT;  // [cwp][k] <= 4096 floats, inside the transpose area
    for (int idx = tid; idx < cwp * k; idx += NT) {
      const int jl = idx / k;
      float v = 0.f;
      if (jl < ncols) {
        const int64_t o = j_begin * k + idx;
        v = V[o];
        if (TRIAL) {
          v = fmaf(alpha, a.dV[o], v);
          if (rg == 0) a.Vt[outi][o] = v;
        }
      }
      raw[idx] = v;
    }
    __syncthreads();
    const float* __restrict__ pc = a.pc;
    if (pc) {
      // V' = B W^T row by row, in place (one row per thread; W = pc[0 .. k k))
      for (int jl = tid; jl < cwp; jl += NT) {
        float row[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) row[t] = t < k ? raw[jl * k + t] : 0.f;
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
          if (kk < k) {
            float v = 0.f;
#pragma unroll
            for (int t = 0; t < 16; ++t)
              if (t < k) v = fmaf(row[t], pc[kk * k + t], v);
            raw[jl * k + kk] = v;
          }
        }
      }
      __syncthreads();
    }
    auto vp = [&](int jl, int kk) -> float { return kk < k ? raw[jl * k + kk] : 0.f; };
    if (!BF16) {
      // residual operand: (col, g) -> V'[col][4q + g], q = 0..3
      for (int idx = tid; idx < cwp * 4; idx += NT) {
        const int jl = idx >> 2, gg = idx & 3;
        *reinterpret_cast<f4*>(sVr + jl * RS + gg * 4) = f4{vp(jl, gg), vp(jl, 4 + gg), vp(jl, 8 + gg), vp(jl, 12 + gg)};
      }
      // G V operand: (t, g, c) -> V'[16t + 4q + g][c], q = 0..3
      for (int idx = tid; idx < ntiles * 64; idx += NT) {
        const int t = idx >> 6, gg = (idx >> 4) & 3, cc = idx & 15;
        const int j0 = 16 * t + gg;
        *reinterpret_cast<f4*>(sVg + idx * 4) = f4{vp(j0, cc), vp(j0 + 4, cc), vp(j0 + 8, cc), vp(j0 + 12, cc)};
      }
    } else {
      // G V operand: (t, g, c) -> bf16 V'[16t + 4g + e][c], e = 0..3
      for (int idx = tid; idx < ntiles * 64; idx += NT) {
        const int t = idx >> 6, gg = (idx >> 4) & 3, cc = idx & 15;
        const int j0 = 16 * t + 4 * gg;
        *reinterpret_cast<u2v_*>(sVgb + idx * 4) =
            u2v_{pk2(vp(j0, cc), vp(j0 + 1, cc)), pk2(vp(j0 + 2, cc), vp(j0 + 3, cc))};
      }
      // residual operand: (col, j) -> 8 bf16 of -V'[col][8j .. 8j+7] for g = 0 (hi),
      // 1 (lo), 2 (hi), 3 (zeros)
      for (int idx = tid; idx < cwp * ns; idx += NT) {
        const int jl = idx / ns, j = idx - jl * ns;
        u4v hi4, lo4;
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const float v0 = -vp(jl, 8 * j + 2 * h), v1 = -vp(jl, 8 * j + 2 * h + 1);
          const uint32_t hi = pk2(v0, v1);
          const float h0 = __builtin_bit_cast(float, hi << 16), h1 = __builtin_bit_cast(float, hi & 0xFFFF0000u);
          hi4[h] = hi;
          lo4[h] = pk2(v0 - h0, v1 - h1);
        }
        u4v* dst = reinterpret_cast<u4v*>(sVrb + (size_t)idx * 32);
        dst[0] = hi4;
        dst[1] = lo4;
        dst[2] = hi4;
        dst[3] = u4v{0u, 0u, 0u, 0u};
      }
    }
    __syncthreads();
  }

  if (n_pipe > 0) {
    for (int64_t j = 0; j < n_pipe; ++j) {
      const int64_t s = s_first + WAVES * j;
      const bool more = j + 1 < n_pipe;
      const int64_t sn = more ? s + WAVES : s;
      f4 gu = f4{0.f, 0.f, 0.f, 0.f};
      float ftile = 0.f, gtile = 0.f;
#pragma unroll
      for (int gi = 0; gi < NG; ++gi) {
        const int ga = gi + D;
        if (ga < NG) {
          load_group(s, ga, xbuf[ga % NBUF], bbuf[ga % NBUF], true);
        } else {
          if (ga == NG) load_ops(sn, nops);
          load_group(sn, ga - NG, xbuf[ga % NBUF], bbuf[ga % NBUF], more);
        }
        __builtin_amdgcn_sched_barrier(0);
        tile_group(gi, ops, xbuf[gi % NBUF], bbuf[gi % NBUF], ftile, gtile, gu);
      }
      strip_end(s, ops, gu, ftile, gtile);
      ops = nops;
    }
  }
  // remaining strips (ragged last strip, or X without vector alignment): element loads
  for (int64_t j = n_pipe; j < n_all; ++j) {
    const int64_t s = s_first + WAVES * j;
    Ops ops;
    load_ops(s, ops);
    f4 gu = f4{0.f, 0.f, 0.f, 0.f};
    float ftile = 0.f, gtile = 0.f;
    const int64_t i0 = s * 16;
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
      f4 xr[PF];
      uint32_t br[PF] = {};
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int t = gi * PF + u;
        xr[u] = f4{0.f, 0.f, 0.f, 0.f};
        if (t < TMAX && t < ntiles) {
          const int jl = 16 * t + c;
          const int64_t jc = j_begin + (jl < ncols ? jl : ncols - 1);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t i = i0 + 4 * g + r;
            const float xv = X[jc * m + (i < m ? i : m - 1)];
            xr[u][r] = (i < m && jl < ncols) ? xv : 0.f;
          }
          if (MASKED) br[u] = (a.mask[jc * a.mw + (i0 >> 5)] >> ((int)(i0 & 31) + 4 * g)) & 0xFu;
        }
      }
      tile_group(gi, ops, xr, br, ftile, gtile, gu);
    }
    strip_end(s, ops, gu, ftile, gtile);
  }

  // ---- the waves' G^T U accumulators: through LDS (over the start layout), fixed order
  __syncthreads();
  float* sGV = lds + w * cwp * k;
#pragma unroll
  for (int t = 0; t < TMAX; ++t) {
    if (t < ntiles && c < k) {
#pragma unroll
      for (int r = 0; r < 4; ++r) sGV[(16 * t + 4 * g + r) * k + c] = -gva[t][r];
    }
  }
  __syncthreads();
  float* gvp = a.gvpart + (int64_t)rg * n * k;
  for (int idx = tid; idx < ncols * k; idx += NT) {
    float acc = 0.f;
#pragma unroll
    for (int ww = 0; ww < WAVES; ++ww) acc += lds[ww * cwp * k + idx];
    gvp[j_begin * k + idx] = acc;
  }
  double* sp = a.spart + ((int64_t)rg * a.nchunks + ch) * RPCA_NSCAL;
  double v4[4] = {f_acc, uu_acc, gud_acc, gg_acc};
  block_sum4(v4, sRed);
  if (tid == 0) {
    sp[0] = v4[0];
    sp[1] = v4[1];
    sp[2] = v4[2];
    sp[3] = v4[3];
  }
}
