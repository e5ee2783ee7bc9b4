// Fused Split-SPCP objective/gradient sweep for gfx950 (kernel template).
//
// One pass over X evaluates, tile by tile in registers,
//   R = U V^T - X                 (the residual inside the marginal phi, Sec. 5 eq. Thm5)
//   rho(R), G = Omega .* clip(R)  (Huber value and derivative, Sec. 1 eq. PhiDef, Sec. 3.2 eq. diff)
//   G^T U and G V                 (the two gradient products, chain rule on eq. smoothNC)
// so neither R nor G is ever written to memory.
//
// Work split.  The columns are cut into chunks (grid.y) of at most TMAX
// 16-column tiles that fit the LDS budget below; V of the chunk is staged in
// LDS.  Every wave owns every fourth 16-row strip of its workgroup's rows (the
// neighbouring waves read the other halves of the same cache lines) and walks the
// chunk's tiles of each strip in groups of PF.  While a group is computed the
// next one is in flight; the last group of a strip prefetches the next
// strip's operands and first group, so the load stream never drains between
// strips.  X is read with buffer loads: the tile's column base is scalar,
// the lane offset one VGPR, and columns past the chunk fall outside the
// resource's range and read as zero.  Per 16x16 tile:
//   * -R = X - U V^T on MFMA: the accumulator is seeded with X and the A
//     operand holds -U, so no per-entry negation is needed; the Huber step
//     then yields -G, and the products -G^T U and -G V are negated once, when
//     written.  In the MFMA output layout
//     (column j = lane%16, rows 4*(lane/16)+r) G is already the A operand of
//     G^T U with K running over rows, so the tile's G^T U goes straight into
//     that tile's accumulator, kept in (accumulation) registers across all
//     strips of the wave.  The waves' accumulators meet in LDS once, at the
//     end, and are summed in a fixed order.
//   * G V contracts over columns: G goes through a 16x17 per-wave LDS tile to
//     the transposed layout and into MFMA; the strip's G V accumulates in
//     registers over the chunk and is complete when the strip ends (one chunk)
//     or written as a per-chunk partial.
// FP32 mode uses v_mfma_f32_16x16x4f32.  Every cross-wave and cross-workgroup sum
// runs in a fixed order: bitwise reproducible.
//
// Rank k <= 16 (sweep_k16.h) follows this plan with operand layouts that make
// every MFMA operand one 16-byte LDS read, a single buffer resource per chunk,
// and two workgroups per CU; its BF16 mode forms the residual from a hi/lo
// split of U and V (three bf16 products, close to FP32 accuracy) and rounds G,
// U and V to bf16 for the two gradient products.  Rank 17..32 keeps the kernel
// below (BF16: U, V and G rounded to bf16 throughout).
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
constexpr int LDS_LIMIT_FLOATS = 16384;  // 64 KB per workgroup
constexpr int TMAX_KB1 = 16;  // most tiles per chunk (register accumulators), k <= 16
constexpr int TMAX_KB2 = 8;   // k in 17..32
constexpr uint32_t BUF_DWORD3 = 0x00020000;  // raw buffer resource word 3 on gfx9 (32-bit data format)

__device__ __forceinline__ f4 mfma_f32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f4 mfma_bf16(s4 a, s4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// FP32 -> BF16, round to nearest even, four at a time by the hardware
// conversion (v_cvt_pk_bf16_f32, two values per instruction).
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef uint32_t u2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ s4 pack_bf16(float a, float b, float c, float d) {
  const uint32_t lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(f2v{a, b}, bf16x2));
  const uint32_t hi = __builtin_bit_cast(uint32_t, __builtin_convertvector(f2v{c, d}, bf16x2));
  return __builtin_bit_cast(s4, u2v{lo, hi});
}

// Huber value and derivative at one entry of the negated residual Rn = -R (the
// tiles compute X - U V^T).  Returns Gn = clip(Rn, +-lam_s) = -G and adds
// rho(R) = G (R - G / 2) = Gn (Rn - Gn / 2) to f and Gn^2 to g2; an unobserved
// entry (observed = 0) contributes nothing.  ELASTIC (the elastic-net marginal,
// kappa = mu / (1 + mu)): the derivative continues with slope kappa beyond the
// threshold, Gn = c + kappa (Rn - c), and rho gains kappa (Rn - c)^2 / 2, c = clip(Rn).
template <bool ELASTIC>
__device__ __forceinline__ float huber(float Rn, float lam_s, float kappa, uint32_t observed, float& f,
                                       float& g2) {
  float c = __builtin_amdgcn_fmed3f(Rn, -lam_s, lam_s);
  float h = fmaf(-0.5f, c, Rn);
  float d = ELASTIC ? Rn - c : 0.f;
  if (!observed) {  // whatever X holds there (even a NaN) stays out of f and G
    c = 0.f;
    h = 0.f;
    d = 0.f;
  }
  f = fmaf(c, h, f);
  float gn = c;
  if (ELASTIC) {
    f = fmaf(0.5f * kappa * d, d, f);
    gn = fmaf(kappa, d, c);
  }
  g2 = fmaf(gn, gn, g2);
  return gn;
}

// Four block sums at once (sh: 4 * WAVES doubles); results in v on thread 0,
// each summed in a fixed order (the wave tree, then the waves in order).
__device__ __forceinline__ void block_sum4(double (&v)[4], double* sh) {
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v[e] += __shfl_xor(v[e], o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int e = 0; e < 4; ++e) sh[e * WAVES + (threadIdx.x >> 6)] = v[e];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      double r = 0.0;
      for (int w = 0; w < WAVES; ++w) r += sh[e * WAVES + w];
      v[e] = r;
    }
}

// Transpose tiles per wave: the tiles of a group use distinct ones so that their
// G -> G^T round trips through LDS overlap (k <= 16: all PF = 4 at once; k > 16,
// where LDS is scarcer, two at a time).
__host__ __device__ constexpr int ntb(int kb) { return kb == 1 ? 4 : 2; }

#include "sweep_k16.h"

// Dynamic LDS (floats).  k <= 16: see the k16 layouts.  k in 17..32:
// sVt[cwp][16 kb + 1] | sGV[WAVES][cwp][k] | sT[WAVES][ntb][16*LDT]
__host__ __device__ constexpr int lds_floats(int kb, int k, int cwp) {
  return kb == 1 ? k16::lds_floats(k, cwp) : cwp * (16 * kb + 1) + WAVES * cwp * k + WAVES * ntb(kb) * 16 * LDT;
}

// Widest chunk (multiple of 16 columns) that fits the LDS budget and the
// register accumulators.
__host__ __device__ constexpr int max_chunk_k16(int k, int cw) {
  return cw <= 16 ? 16 : (k16::lds_floats(k, cw) <= LDS_LIMIT_FLOATS ? cw : max_chunk_k16(k, cw - 16));
}
__host__ __device__ constexpr int max_chunk(int kb, int k) {
  return kb == 1 ? max_chunk_k16(k, 16 * TMAX_KB1) : 16 * ((LDS_LIMIT_FLOATS - WAVES * ntb(kb) * 16 * LDT) / (16 * (16 * kb + 1 + WAVES * k))) <
                 16 * (kb == 1 ? TMAX_KB1 : TMAX_KB2)
             ? 16 * ((LDS_LIMIT_FLOATS - WAVES * ntb(kb) * 16 * LDT) / (16 * (16 * kb + 1 + WAVES * k)))
             : 16 * (kb == 1 ? TMAX_KB1 : TMAX_KB2);
}

// Tile-count class of a chunk: the instantiated TMAX that covers ntiles.
__host__ __device__ constexpr int tmax_class(int kb, int ntiles) {
  return ntiles <= 4 ? 4 : (ntiles <= 8 || kb == 2) ? 8 : 16;
}

// Load pipeline of a wave: PF tiles per group, NG groups per strip, and a ring
// of NBUF group buffers (NG a multiple of NBUF, so the ring lines up at every
// strip start) of which NBUF - 1 are in flight while one is computed.  One
// workgroup per CU leaves the registers for a deep ring: up to 12 tiles (12 KB)
// per wave in flight is what covers HBM latency at this occupancy.
template <int TMAX>
struct Pipe {
  static constexpr int PF = TMAX >= 16 ? 4 : 2;
  static constexpr int NG = (TMAX + PF - 1) / PF;
  static constexpr int NBUF = NG >= 4 ? 4 : 2;
  static_assert(NG % NBUF == 0, "group ring must line up with strips");
};

template <int KB>
struct StripOps {
  float ua[4 * KB];   // R: A operand (layout per precision, see load_ops)
  float ub[4][KB];    // G^T U:  B[row 4g + r][kk = 16 kb + c]
  float dub[4][KB];   // dU at the ub positions (trial)
};

// Argument tables of the batched sweep are read through the constant address
// space: every field load is a scalar load the compiler may repeat at its use
// instead of holding some fifty fields live in registers across the item loop.
typedef __attribute__((address_space(4))) SweepArgs ConstSweepArgs;

// `Args` is SweepArgs (a kernel argument) or ConstSweepArgs (a batch table entry).
template <int KB, int TMAX, bool MASKED, bool TRIAL, bool BF16, typename Args, bool ELASTIC = false>
__device__ __forceinline__ void sweep_item_kb2(const Args& a, const int rg, const int ch, float* lds,
                                               double* sRed) {
  constexpr int KMAX = 16 * KB;
  constexpr int KQ = 4 * KB;
  constexpr int LDV = KMAX + 1;
  using P = Pipe<TMAX>;
  constexpr int PF = P::PF;
  constexpr int NG = P::NG;
  constexpr int NBUF = P::NBUF;

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
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: strip control stays scalar
  const int c = lane & 15, g = lane >> 4;
  const int64_t m = a.m, n = a.n;
  const int k = a.k;
  const float lam_s = a.lam_s, lam_l = a.lam_l, kappa = a.kappa;
  const float* __restrict__ U = a.U[cur];
  const float* __restrict__ V = a.V[cur];
  const float* __restrict__ X = a.X;
  const float* __restrict__ dU = a.dU;

  const int64_t j_begin = (int64_t)ch * a.chunk_w;
  const int ncols = (int)((n - j_begin) < a.chunk_w ? (n - j_begin) : a.chunk_w);
  const int ntiles = (ncols + 15) >> 4;  // <= TMAX (the launcher picks TMAX)
  const int cwp = ntiles * 16;
  float* sVt = lds;
  float* sGVall = lds + cwp * LDV;
  constexpr int NTB = ntb(KB);
  float* myT = sGVall + WAVES * cwp * k + w * NTB * 16 * LDT;  // transpose tile 0 of this wave

  // Preconditioned variables (the solver's A, B with U = A P_U, V = B P_V): the
  // product U V^T = A (B W^T)^T with W = P_U P_V, so the staged rows are B W^T
  // and everything else in the tile loop is unchanged.  pc = [W | M_U | M_V],
  // k x k each, row-major (M_U = P_U^2, M_V = P_V^2).
  const float* __restrict__ pc = a.pc;
  if (pc) {
    float* raw = sGVall;  // [cwp][k], free until the end of the item
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
    for (int idx = tid; idx < cwp * KMAX; idx += NT) {
      const int jl = idx / KMAX, kk = idx % KMAX;
      float v = 0.f;
      if (kk < k)
        for (int t = 0; t < k; ++t) v = fmaf(raw[jl * k + t], pc[kk * k + t], v);
      sVt[jl * LDV + kk] = v;
    }
  } else {
    // every thread's loads first (at most SLOTS each), then the LDS stores: the
    // loads are in flight together instead of one latency per element
    constexpr int SLOTS = (TMAX * 16 * KMAX + NT - 1) / NT;
    float vs[SLOTS];
#pragma unroll
    for (int u = 0; u < SLOTS; ++u) {
      const int idx = tid + u * NT;
      const int jl = idx / KMAX, kk = idx % KMAX;
      float v = 0.f;
      if (idx < cwp * KMAX && jl < ncols && kk < k) {
        const int64_t o = (j_begin + jl) * k + kk;
        v = V[o];
        if (TRIAL) v = fmaf(alpha, a.dV[o], v);
      }
      vs[u] = v;
    }
#pragma unroll
    for (int u = 0; u < SLOTS; ++u) {
      const int idx = tid + u * NT;
      if (idx < cwp * KMAX) {
        const int jl = idx / KMAX, kk = idx % KMAX;
        sVt[jl * LDV + kk] = vs[u];
        if (TRIAL && rg == 0 && jl < ncols && kk < k) a.Vt[outi][(j_begin + jl) * k + kk] = vs[u];
      }
    }
  }
  __syncthreads();

  f4 gva[TMAX][KB];
#pragma unroll
  for (int t = 0; t < TMAX; ++t)
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) gva[t][kb] = f4{0.f, 0.f, 0.f, 0.f};

  double f_acc = 0.0, uu_acc = 0.0, gud_acc = 0.0, gg_acc = 0.0;
  // Workgroup row rg of R owns the strips [rg S / R, (rg + 1) S / R) of the S
  // strips (as even a split as integers allow); wave w takes every WAVES-th of
  // them starting at w.  A 16-row strip reads half of each 128-byte line of a
  // column; the neighbouring wave reads the other half at about the same time,
  // so each line comes from HBM once.
  const int64_t nstrips = (m + 15) >> 4;
  const int64_t R = a.row_groups;
  const int64_t s_lo = (int64_t)rg * nstrips / R, s_hi = ((int64_t)rg + 1) * nstrips / R;
  const int64_t s_first = s_lo + w;
  int64_t n_all = 0;  // strips of this wave: s_first + WAVES * j, j < n_all
  if (s_first < s_hi) n_all = (s_hi - s_first + WAVES - 1) / WAVES;
  const bool vec = a.xvec != 0;
  // strips whose 16 rows are all inside X (a prefix of the wave's list) take the
  // pipelined vector path
  const int64_t full_lim = vec ? (m >> 4) : 0;
  int64_t n_pipe = 0;
  if (s_first < full_lim) {
    n_pipe = (full_lim - s_first + WAVES - 1) / WAVES;
    if (n_pipe > n_all) n_pipe = n_all;
  }
  const int64_t tile_stride = 16 * m;

  auto load_ops = [&](int64_t s, StripOps<KB>& o) {
    const int64_t i0 = s * 16;
    const int64_t i_c = (i0 + c < m) ? i0 + c : m - 1;
    const bool row_c_ok = i0 + c < m;
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
      // FP32: A[i = c][kk = 4q + g] per K-step q; BF16: lane holds kk = 16 kb + 4 g + e, q = 4 kb + e
      const int kk = BF16 ? 16 * (q >> 2) + 4 * g + (q & 3) : 4 * q + g;
      const int kkc = kk < k ? kk : k - 1;
      float v = U[i_c * k + kkc];
      if (TRIAL) v = fmaf(alpha, dU[i_c * k + kkc], v);
      o.ua[q] = (kk < k && row_c_ok) ? -v : 0.f;  // -U: the tile product is X - U V^T = -R
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
        o.ub[r][kb] = ok ? v : 0.f;
        o.dub[r][kb] = ok ? dv : 0.f;
      }
    }
  };

  // vector loads of tiles [gi*PF, gi*PF + PF) of strip s (rows inside X).  Buffer
  // loads: the tile's column base is scalar, the lane offset one VGPR, and
  // columns past the chunk fall outside the resource's range and read zero.
  const uint32_t lane_off = (uint32_t)(c * m * 4 + 16 * g);
  // live = false: a strip past the wave's last (the ring's tail) reads nothing.
  auto load_group = [&](int64_t s, int gi, f4(&xr)[PF], uint32_t(&br)[PF], bool live) {
    const uint32_t voff = lane_off + (uint32_t)(s * 64);
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int t = gi * PF + u;
      if (t < TMAX) {
        int valid = ncols - 16 * t;
        valid = (valid < 0 || !live) ? 0 : (valid > 16 ? 16 : valid);
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(X + (j_begin + 16 * t) * m), (short)0, (int)(valid * m * 4), BUF_DWORD3);
        xr[u] = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, 0, 0));
        if (MASKED) {
          const int jl = 16 * t + c;
          const int64_t j = j_begin + ((jl < ncols) ? jl : ncols - 1);
          const int64_t i0 = s * 16;
          br[u] = (a.mask[j * a.mw + (i0 >> 5)] >> ((int)(i0 & 31) + 4 * g)) & 0xFu;
        }
      }
    }
  };

  auto tile = [&](int t, const StripOps<KB>& o, f4 xraw, uint32_t braw, float& ftile, float& gtile,
                  f4(&gu)[KB]) {
    const int jl = 16 * t + c;
    const bool jok = jl < ncols;
    const f4 xv = jok ? xraw : f4{0.f, 0.f, 0.f, 0.f};
    const uint32_t bits = MASKED ? (jok ? braw : 0u) : 0xFu;
    f4 acc = xv;
    if (!BF16) {
#pragma unroll
      for (int q = 0; q < KQ; ++q)
        if (4 * q < k) acc = mfma_f32(o.ua[q], sVt[jl * LDV + 4 * q + g], acc);  // steps past k add zero
    } else {
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        const float* vr = sVt + jl * LDV + 16 * kb + 4 * g;
        const s4 ua4 = pack_bf16(o.ua[4 * kb + 0], o.ua[4 * kb + 1], o.ua[4 * kb + 2], o.ua[4 * kb + 3]);
        acc = mfma_bf16(ua4, pack_bf16(vr[0], vr[1], vr[2], vr[3]), acc);
      }
    }
    float G[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float gn = huber<ELASTIC>(acc[r], lam_s, kappa, MASKED ? ((bits >> r) & 1u) : 1u, ftile, gtile);
      G[r] = gn;
      myT[(4 * g + r) * LDT + c] = gn;
    }
    if (!BF16) {
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int r = 0; r < 4; ++r) gva[t][kb] = mfma_f32(G[r], o.ub[r][kb], gva[t][kb]);
    } else {
      const s4 gb = pack_bf16(G[0], G[1], G[2], G[3]);
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
        gva[t][kb] = mfma_bf16(gb, pack_bf16(o.ub[0][kb], o.ub[1][kb], o.ub[2][kb], o.ub[3][kb]), gva[t][kb]);
    }
    if (!BF16) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float gt = myT[c * LDT + 4 * q + g];
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) gu[kb] = mfma_f32(gt, sVt[(16 * t + 4 * q + g) * LDV + 16 * kb + c], gu[kb]);
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

  // A whole group of PF tiles (all inside the chunk), step by step across the
  // group so that the tiles' independent MFMA chains and LDS round trips
  // overlap: R for every tile, then per NTB tiles the Huber epilogue with its
  // transposes, the G^T U and the G V products.  Same arithmetic, same order per
  // accumulator as PF calls of `tile`.
  auto tile_group = [&](int gi, const StripOps<KB>& o, const f4(&xr)[PF], const uint32_t(&br)[PF],
                        float& ftile, float& gtile, f4(&gu)[KB]) {
    f4 acc[PF];  // columns past the chunk were read as zero by the buffer loads
#pragma unroll
    for (int u = 0; u < PF; ++u) acc[u] = xr[u];
    if (!BF16) {
#pragma unroll
      for (int q = 0; q < KQ; ++q) {
        if (4 * q >= k) continue;  // K-steps past k would add zero (k is uniform)
#pragma unroll
        for (int u = 0; u < PF; ++u)
          acc[u] = mfma_f32(o.ua[q], sVt[(16 * (gi * PF + u) + c) * LDV + 4 * q + g], acc[u]);
      }
    } else {
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        const s4 ua4 = pack_bf16(o.ua[4 * kb + 0], o.ua[4 * kb + 1], o.ua[4 * kb + 2], o.ua[4 * kb + 3]);
#pragma unroll
        for (int u = 0; u < PF; ++u) {
          const float* vr = sVt + (16 * (gi * PF + u) + c) * LDV + 16 * kb + 4 * g;
          acc[u] = mfma_bf16(ua4, pack_bf16(vr[0], vr[1], vr[2], vr[3]), acc[u]);
        }
      }
    }
    constexpr int NB = NTB < PF ? NTB : PF;  // tiles per transpose round (PF = 2 when TMAX = 4)
    static_assert(PF % NB == 0, "transpose rounds split the group evenly");
#pragma unroll
    for (int h = 0; h < PF; h += NB) {
      float G[NB][4];
#pragma unroll
      for (int v = 0; v < NB; ++v) {
        const int u = h + v;
        const int jl = 16 * (gi * PF + u) + c;
        const uint32_t bits = MASKED ? ((jl < ncols) ? br[u] : 0u) : 0xFu;
        float* tT = myT + v * 16 * LDT;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float gn = huber<ELASTIC>(acc[u][r], lam_s, kappa, MASKED ? ((bits >> r) & 1u) : 1u, ftile,
                                          gtile);
          G[v][r] = gn;
          tT[(4 * g + r) * LDT + c] = gn;
        }
      }
#pragma unroll
      for (int v = 0; v < NB; ++v) {
        const int t = gi * PF + h + v;
        const int ts = t < TMAX ? t : TMAX - 1;  // t < TMAX wherever a whole group is used
        if (!BF16) {
#pragma unroll
          for (int kb = 0; kb < KB; ++kb)
#pragma unroll
            for (int r = 0; r < 4; ++r) gva[ts][kb] = mfma_f32(G[v][r], o.ub[r][kb], gva[ts][kb]);
        } else {
          const s4 gb = pack_bf16(G[v][0], G[v][1], G[v][2], G[v][3]);
#pragma unroll
          for (int kb = 0; kb < KB; ++kb)
            gva[ts][kb] =
                mfma_bf16(gb, pack_bf16(o.ub[0][kb], o.ub[1][kb], o.ub[2][kb], o.ub[3][kb]), gva[ts][kb]);
        }
      }
#pragma unroll
      for (int v = 0; v < NB; ++v) {
        const int t = gi * PF + h + v;
        const float* tT = myT + v * 16 * LDT;
        if (!BF16) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float gt = tT[c * LDT + 4 * q + g];
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
              gu[kb] = mfma_f32(gt, sVt[(16 * t + 4 * q + g) * LDV + 16 * kb + c], gu[kb]);
          }
        } else {
          const float* tr = tT + c * LDT + 4 * g;
          const s4 gtb = pack_bf16(tr[0], tr[1], tr[2], tr[3]);
#pragma unroll
          for (int kb = 0; kb < KB; ++kb) {
            const float* vc = sVt + (16 * t + 4 * g) * LDV + 16 * kb + c;
            gu[kb] = mfma_bf16(gtb, pack_bf16(vc[0], vc[LDV], vc[2 * LDV], vc[3 * LDV]), gu[kb]);
          }
        }
      }
    }
  };

  auto strip_end = [&](int64_t s, const StripOps<KB>& o, const f4(&gu)[KB], float ftile, float gtile) {
    const int64_t i0 = s * 16;
    f_acc += (double)ftile;
    gg_acc += (double)gtile;
    // the regulariser's row term: U itself, or A M_U in preconditioned variables
    // (the strip's rows go through the wave's transpose tile, one 16-column block at a time)
    float reg[4][KB];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) reg[r][kb] = o.ub[r][kb];
    if (pc) {
      const float* __restrict__ MU = pc + k * k;
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) reg[r][kb] = 0.f;
#pragma unroll
      for (int kbi = 0; kbi < KB; ++kbi) {
#pragma unroll
        for (int r = 0; r < 4; ++r) myT[(4 * g + r) * LDT + c] = o.ub[r][kbi];
        for (int t = 0; t < 16 && 16 * kbi + t < k; ++t) {
#pragma unroll
          for (int kb = 0; kb < KB; ++kb) {
            const int kk = 16 * kb + c;
            const float mv = (kk < k) ? MU[(16 * kbi + t) * k + kk] : 0.f;
#pragma unroll
            for (int r = 0; r < 4; ++r) reg[r][kb] = fmaf(myT[(4 * g + r) * LDT + t], mv, reg[r][kb]);
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t i = i0 + 4 * g + r;
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        const int kk = 16 * kb + c;
        if (kk < k && i < m) {
          const int64_t oo = i * k + kk;
          if (a.nchunks == 1) {
            const float gval = fmaf(lam_l, reg[r][kb], -gu[kb][r]);  // gu holds -G V
            a.gU[outi][oo] = gval;
            if (TRIAL) gud_acc += (double)gval * (double)o.dub[r][kb];
          } else {
            a.gupart[(int64_t)ch * m * k + oo] = -gu[kb][r];
          }
          if (ch == 0) {
            uu_acc += (double)o.ub[r][kb] * (double)reg[r][kb];
            if (TRIAL) a.Ut[outi][oo] = o.ub[r][kb];
          }
        }
      }
    }
  };

  // ---- pipelined strips: while group gi is computed, the next NBUF - 1 groups (running on
  //      into the next strip, whose operands are requested with its first group) are in flight
  if (n_pipe > 0) {
    constexpr int D = NBUF - 1;
    StripOps<KB> ops, nops;
    load_ops(s_first, ops);
    f4 xbuf[NBUF][PF];
    uint32_t bbuf[NBUF][PF] = {};
#pragma unroll
    for (int d = 0; d < D; ++d) load_group(s_first, d, xbuf[d], bbuf[d], true);
    for (int64_t j = 0; j < n_pipe; ++j) {
      const int64_t s = s_first + WAVES * j;
      const bool more = j + 1 < n_pipe;
      const int64_t sn = more ? s + WAVES : s;
      f4 gu[KB];
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) gu[kb] = f4{0.f, 0.f, 0.f, 0.f};
      float ftile = 0.f, gtile = 0.f;
#pragma unroll
      for (int gi = 0; gi < NG; ++gi) {
        const int ga = gi + D;  // the group requested now
        if (ga < NG) {
          load_group(s, ga, xbuf[ga % NBUF], bbuf[ga % NBUF], true);
        } else {
          if (ga == NG) load_ops(sn, nops);
          load_group(sn, ga - NG, xbuf[ga % NBUF], bbuf[ga % NBUF], more);
        }
        __builtin_amdgcn_sched_barrier(0);
        const int cb = gi % NBUF;
        if ((gi + 1) * PF <= TMAX && (gi + 1) * PF <= ntiles) {
          tile_group(gi, ops, xbuf[cb], bbuf[cb], ftile, gtile, gu);
        } else {
#pragma unroll
          for (int u = 0; u < PF; ++u) {
            const int t = gi * PF + u;
            if (t < TMAX) {
              if (t < ntiles) tile(t, ops, xbuf[cb][u], bbuf[cb][u], ftile, gtile, gu);
            }
          }
        }
      }
      strip_end(s, ops, gu, ftile, gtile);
      ops = nops;
    }
  }
  // ---- remaining strips (ragged last strip, or X without vector alignment): scalar loads
  for (int64_t j = n_pipe; j < n_all; ++j) {
    const int64_t s = s_first + WAVES * j;
    StripOps<KB> ops;
    load_ops(s, ops);
    f4 gu[KB];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) gu[kb] = f4{0.f, 0.f, 0.f, 0.f};
    float ftile = 0.f, gtile = 0.f;
    const int64_t i0 = s * 16;
    const float* xbase = X + (j_begin + c) * m + i0 + 4 * g;
#pragma unroll
    for (int t = 0; t < TMAX; ++t) {
      if (t < ntiles) {
        const int jl = 16 * t + c;
        const int64_t off = (jl < ncols) ? (int64_t)t * tile_stride : (int64_t)(ncols - 1 - c) * m;
        f4 xr;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t i = i0 + 4 * g + r;
          const float xv_r = xbase[off + ((i < m) ? r : (m - 1 - i0 - 4 * g))];
          xr[r] = (i < m) ? xv_r : 0.f;
        }
        uint32_t br = 0;
        if (MASKED) {
          const int64_t j = j_begin + ((jl < ncols) ? jl : ncols - 1);
          br = (a.mask[j * a.mw + (i0 >> 5)] >> ((int)(i0 & 31) + 4 * g)) & 0xFu;
        }
        tile(t, ops, xr, br, ftile, gtile, gu);
      }
    }
    strip_end(s, ops, gu, ftile, gtile);
  }

  // ---- the waves' G^T U accumulators: through LDS, summed in a fixed order
  float* sGV = sGVall + w * cwp * k;
#pragma unroll
  for (int t = 0; t < TMAX; ++t) {
    if (t < ntiles) {
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        const int kk = 16 * kb + c;
        if (kk < k) {
#pragma unroll
          for (int r = 0; r < 4; ++r) sGV[(16 * t + 4 * g + r) * k + kk] = -gva[t][kb][r];  // -G^T U
        }
      }
    }
  }
  __syncthreads();
  float* gvp = a.gvpart + (int64_t)rg * n * k;
  for (int idx = tid; idx < ncols * k; idx += NT) {
    float acc = 0.f;
#pragma unroll
    for (int ww = 0; ww < WAVES; ++ww) acc += sGVall[ww * cwp * k + idx];
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


template <int KB, int TMAX, bool MASKED, bool TRIAL, bool BF16, typename Args, bool ELASTIC = false>
__device__ __forceinline__ void sweep_item(const Args& a, const int rg, const int ch, float* lds, double* sRed) {
  if constexpr (KB == 1)
    sweep_item_k16<TMAX, MASKED, TRIAL, BF16, Args, ELASTIC>(a, rg, ch, lds, sRed);
  else
    sweep_item_kb2<KB, TMAX, MASKED, TRIAL, BF16, Args, ELASTIC>(a, rg, ch, lds, sRed);
}

template <int KB, int TMAX, bool MASKED, bool TRIAL, bool BF16, bool ELASTIC>
// k <= 16: two waves per SIMD (the k16 layouts fit two workgroups' LDS per CU)
__global__ __launch_bounds__(NT, KB == 1 ? 2 : 1) void k_sweep(SweepArgs a) {
  extern __shared__ float lds[];
  __shared__ double sRed[4 * WAVES];
  sweep_item<KB, TMAX, MASKED, TRIAL, BF16, SweepArgs, ELASTIC>(a, blockIdx.x, blockIdx.y, lds, sRed);
}

// Batched sweep: one persistent launch per tile class (k block, tiles per
// chunk) for every instance of a batch in that class.  Each workgroup pulls
// (instance, workgroup row, chunk) items from the class's queue (a counter
// advanced by one atomic per item, re-armed by the reduction that follows)
// until the list is drained.  Lists are sorted by decreasing cost, so the long
// items start first and the short ones fill the tail.
template <int KB, int TMAX, bool MASKED, bool TRIAL, bool BF16>
__global__ __launch_bounds__(NT, KB == 1 ? 2 : 1) void k_sweep_batch(const SweepArgs* __restrict__ args,
                                                    const SweepItem* __restrict__ items, int nitems,
                                                    unsigned* head) {
  extern __shared__ float lds[];
  __shared__ double sRed[4 * WAVES];
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(head, 1u);
    __syncthreads();
    // the item index is uniform: keep it (and what it addresses) in scalar registers
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (it >= nitems) break;
    const int inst = __builtin_amdgcn_readfirstlane(items[it].inst);
    const int rg = __builtin_amdgcn_readfirstlane(items[it].rg);
    const int ch = __builtin_amdgcn_readfirstlane(items[it].ch);
    sweep_item<KB, TMAX, MASKED, TRIAL, BF16>(((const ConstSweepArgs*)args)[inst], rg, ch, lds,
                                              sRed);
    __syncthreads();
  }
}

template <bool MASKED, bool TRIAL, bool BF16>
hipError_t launch_batch(int kb, int tmax, const SweepArgs* args, const SweepItem* items, int nitems,
                        unsigned* head, int grid, int lds_floats_max, hipStream_t s) {
  if (lds_floats_max > LDS_LIMIT_FLOATS) return hipErrorInvalidValue;
  const size_t bytes = lds_floats_max * sizeof(float);
  if (kb == 1 && tmax == 4)
    hipLaunchKernelGGL((k_sweep_batch<1, 4, MASKED, TRIAL, BF16>), dim3(grid), dim3(NT), bytes, s, args, items, nitems, head);
  else if (kb == 1 && tmax == 8)
    hipLaunchKernelGGL((k_sweep_batch<1, 8, MASKED, TRIAL, BF16>), dim3(grid), dim3(NT), bytes, s, args, items, nitems, head);
  else if (kb == 1 && tmax == 16)
    hipLaunchKernelGGL((k_sweep_batch<1, 16, MASKED, TRIAL, BF16>), dim3(grid), dim3(NT), bytes, s, args, items, nitems, head);
  else if (kb == 2 && tmax == 4)
    hipLaunchKernelGGL((k_sweep_batch<2, 4, MASKED, TRIAL, BF16>), dim3(grid), dim3(NT), bytes, s, args, items, nitems, head);
  else if (kb == 2 && tmax == 8)
    hipLaunchKernelGGL((k_sweep_batch<2, 8, MASKED, TRIAL, BF16>), dim3(grid), dim3(NT), bytes, s, args, items, nitems, head);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// Resident workgroups of one class's batched sweep (per CU x CUs).
template <bool MASKED, bool TRIAL, bool BF16>
int batch_grid(int kb, int tmax, int lds_floats_max) {
  int per_cu = 0;
  const size_t bytes = lds_floats_max * sizeof(float);
  hipError_t e = hipErrorInvalidValue;
  if (kb == 1 && tmax == 4)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep_batch<1, 4, MASKED, TRIAL, BF16>, NT, bytes);
  else if (kb == 1 && tmax == 8)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep_batch<1, 8, MASKED, TRIAL, BF16>, NT, bytes);
  else if (kb == 1 && tmax == 16)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep_batch<1, 16, MASKED, TRIAL, BF16>, NT, bytes);
  else if (kb == 2 && tmax == 4)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep_batch<2, 4, MASKED, TRIAL, BF16>, NT, bytes);
  else if (kb == 2 && tmax == 8)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep_batch<2, 8, MASKED, TRIAL, BF16>, NT, bytes);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  return per_cu * cus;
}

template <bool MASKED, bool TRIAL, bool BF16, bool ELASTIC = false>
hipError_t launch_kb(const SweepArgs& sa, hipStream_t s) {
  const int kb = (sa.k + 15) / 16;
  const int cwp = (int)(((sa.n < sa.chunk_w ? sa.n : sa.chunk_w) + 15) / 16) * 16;
  const int lds = lds_floats(kb, sa.k, cwp);
  if (kb < 1 || kb > 2 || lds > LDS_LIMIT_FLOATS || sa.chunk_w > max_chunk(kb, sa.k)) return hipErrorInvalidValue;
  const int tm = tmax_class(kb, cwp / 16);
  const dim3 grid(sa.row_groups, sa.nchunks), block(NT);
  const size_t bytes = lds * sizeof(float);
  if (kb == 1) {
    if (tm == 4) hipLaunchKernelGGL((k_sweep<1, 4, MASKED, TRIAL, BF16, ELASTIC>), grid, block, bytes, s, sa);
    else if (tm == 8) hipLaunchKernelGGL((k_sweep<1, 8, MASKED, TRIAL, BF16, ELASTIC>), grid, block, bytes, s, sa);
    else hipLaunchKernelGGL((k_sweep<1, 16, MASKED, TRIAL, BF16, ELASTIC>), grid, block, bytes, s, sa);
  } else {
    if (tm == 4) hipLaunchKernelGGL((k_sweep<2, 4, MASKED, TRIAL, BF16, ELASTIC>), grid, block, bytes, s, sa);
    else hipLaunchKernelGGL((k_sweep<2, 8, MASKED, TRIAL, BF16, ELASTIC>), grid, block, bytes, s, sa);
  }
  return hipGetLastError();
}

}  // namespace rpca_sweep
