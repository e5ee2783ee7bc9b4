// The small dense work of a block power iteration step, on the device (one
// workgroup of RT threads), for blocks of at most BLK = 8 vectors.  Shared by
// Frank-Wolfe's linear minimisation (Sec. 6.2, Alg. 1: the top singular pair of
// G by block power iteration on G^T G) and the certificate's T4 (Sec. 3.4: the
// singular values of M = P_U^perp D P_V^perp above one by block power iteration
// on M^T M).
//
// Given the orthonormal block X (n x BLK, first b columns) and Z = Op^T Op X:
//   the certificate first forms Z = P_V^perp (G^T G X / lam_L^2 - B_n B_n^T X)
//     (B_n = D^T U_1, the U_1 part of D^T D; V_1 and B_n are n x r; the
//     coefficients B_n^T X and V_1^T (.) from one staged pass over the rows, with
//     V_1^T B_n given);
//   Rayleigh-Ritz: H = X^T Z, its eigenpairs (theta_p, w_p) by cyclic Jacobi
//     (parallel order: four disjoint rotations per round, one element of H and
//     of the eigenvector matrix per lane of one wave), sorted descending;
//   Frank-Wolfe's stop test: || Z w_0 - theta_0 X w_0 || <= ptol theta_0 (or the
//     last step, or theta_0 = 0), with v = X w_0 and the coefficients w_0
//     (y = G v = (G X) w_0); the certificate's: the change of the Ritz values
//     that can matter for T4 (the leading one and those at or above 0.81), the
//     leading one settling below 0.98^2, or the random-start bound of Kuczynski
//     and Wozniakowski (1992) putting lambda_max > 1 below probability 1e-9;
//   next block: orth(Z W) by Cholesky QR, the Gram of Z W taken as
//     W^T (Z^T Z) W.  One pass when Gershgorin puts the column-scaled Gram in
//     [0.5, 1.5] (Cholesky QR's loss of orthogonality grows with the square of
//     that condition number, so it stays at rounding level; near convergence
//     the columns of Z W are nearly orthogonal), else a second pass on the
//     result.  A Cholesky pivot that keeps less than 1e-12 of its diagonal
//     sends the block through modified Gram-Schmidt instead (twice per column,
//     a vanishing column replaced by hashed entries once, then zero).
// Rotating the block by W keeps the next H nearly diagonal, so its Jacobi
// settles in a sweep.  Every sum has a fixed order.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace rpca_ritz {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int BLK = 8;    // block vectors
constexpr int RT = 256;   // threads of k_block_ritz
constexpr int RMAX = 16;  // largest rank of V_1 and B_n (the certificate's r <= k <= 16 with the fused pass)
constexpr int PTR = 128;  // rows per tile of the certificate's projection passes

enum { RITZ_FW = 0, RITZ_CERT = 1 };

struct RitzArgs {
  const double* X;    // n x BLK block (orthonormal first b columns, zero padding)
  const double* Z;    // n x BLK product (first b columns used)
  int64_t n;
  int b;
  uint64_t salt;      // hashed replacement entries of a vanishing column
  double* Xn;         // n x BLK: the next block (not X)
  float* Xbn;         // n x BLK FP32 copy of it, or null
  float* Wfn;         // n x 16 FP32 copy of it (columns past BLK zero), or null
  double* res;        // results (see the modes); res[0] is the stop flag
  const double* skip; // null, or res[0] of the previous step
  // Frank-Wolfe: res = [stop, theta_0, residual]
  double ptol;
  int last;           // the last allowed step: stop
  float* v32;         // n: X w_0
  float* cw;          // BLK: w_0
  // certificate (n <= RT): res = [stop, ritz_0 .. ritz_7] (max(theta, 0), zero past b)
  double* Zf;         // n x BLK: the projected Z (written)
  const double* V1;   // n x r
  const double* Bn;   // n x r
  const double* VB;   // r x r: V_1^T B_n
  int r;
  double inv_lam2;    // 1 / lam_L^2
  int it;             // step number (the first step sees no previous Ritz values)
  double conv_rel;    // relative change of the relevant Ritz values that counts as converged
  double* state;      // BLK: the previous step's Ritz values (read, then rewritten)
  double* vtop;       // n: X w_0 (FP64)
};

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Deterministic start entries of a power-iteration block (SplitMix64 hash of
// the index, centred; Steele, Lea & Flood 2014).
__host__ __device__ inline double start_entry(uint64_t j) {
  uint64_t z = j + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}


__device__ __forceinline__ double block_sum1(double v, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < RT / 64; ++i) t += red[i];
  __syncthreads();
  return t;
}

// Row j of a row-major n x BLK FP64 matrix (64-byte aligned rows) in four
// 16-byte loads, all issued before any use.
__device__ __forceinline__ void load_row(const double* __restrict__ A, int64_t j, double (&x)[BLK]) {
  const double2* p = reinterpret_cast<const double2*>(A + j * BLK);
#pragma unroll
  for (int k = 0; k < BLK / 2; ++k) {
    const double2 v = p[k];
    x[2 * k] = v.x;
    x[2 * k + 1] = v.y;
  }
}

// 1 / sqrt(x) for finite x > 0: an FP32 estimate of the scaled mantissa and
// two Newton steps in FP64.
__device__ __forceinline__ double rsqrt_f64(double x) {
  int e;
  const double m = frexp(x, &e);  // x = m 2^e, m in [0.5, 1)
  const int e2 = e & ~1;          // even, so that 2^(-e2/2) is exact
  const double mm = ldexp(m, e - e2);
  double r = (double)__frsqrt_rn((float)mm);
  r = r * fma(-0.5 * mm, r * r, 1.5);
  r = r * fma(-0.5 * mm, r * r, 1.5);
  return ldexp(r, -(e2 / 2));
}

__device__ __forceinline__ float wave_sumf(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Jacobi rotation (FP32) that zeroes the off-diagonal of [[app, apq], [apq, aqq]]:
// c and t (s = t c) with J[p][p] = J[q][q] = c, J[q][p] = -s, J[p][q] = s, from
// the hardware reciprocal, square-root and reciprocal-square-root estimates.
// Lanes given the same entries return the same rotation.
__device__ __forceinline__ void jacobi_ct(float app, float aqq, float apq, float& c, float& t) {
  c = 1.f;
  t = 0.f;
  if (apq == 0.f) return;
  const float tau = (aqq - app) * __builtin_amdgcn_rcpf(2.f * apq), at = fabsf(tau);
  const float tt = at > 1e18f ? 0.5f * __builtin_amdgcn_rcpf(at)
                              : __builtin_amdgcn_rcpf(at + __builtin_amdgcn_sqrtf(fmaf(at, at, 1.f)));
  t = tau >= 0.f ? tt : -tt;
  c = __builtin_amdgcn_rsqf(fmaf(t, t, 1.f));
}

// Sums over the rows j < n, in tiles of RT rows staged in LDS (whole-row
// loads, every load of a tile in flight at once), each output over two row
// slices summed in order:
//   out1[a BLK + c] = sum_j A[j][a] B[j][c]   (a, c < b; A may be null: skipped)
//   out2[a BLK + c] = sum_j B[j][a] B[j][c]   (a <= c < b, mirrored)
// Entries past b are zero; columns past b of A and B are loaded but not used.
__device__ __forceinline__ void row_grams(const double* __restrict__ A, const double* __restrict__ B, int64_t n, int b,
                          double* out1, double* out2, double* red, double* sA, double* sB,
                          const double (&a0)[BLK], const double (&b0)[BLK]) {
  constexpr int NOP = 128, SL = RT / NOP;
  const int tid = threadIdx.x, o = tid % NOP, sl = tid / NOP;
  if (tid < BLK * BLK) {
    if (A) out1[tid] = 0.0;
    out2[tid] = 0.0;
  }
  int a = 0, c = 0;
  bool live;
  if (o < BLK * BLK) {
    a = o >> 3;
    c = o & 7;
    live = A != nullptr;
  } else {
    int r = o - BLK * BLK;  // -> (a, c), a <= c, row by row of the upper triangle
    live = r < BLK * (BLK + 1) / 2;
    while (live && r >= BLK - a) {
      r -= BLK - a;
      ++a;
    }
    c = a + r;
  }
  live = live && a < b && c < b;
  const double* sP = o < BLK * BLK ? sA : sB;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (int64_t r0 = 0; r0 < n; r0 += RT) {
    __syncthreads();  // the previous tile is consumed
    const int64_t j = r0 + tid;
    if (j < n) {
      double xa[BLK], xb[BLK];
      if (r0 == 0) {  // the caller's registers hold row tid
#pragma unroll
        for (int k = 0; k < BLK; ++k) {
          xa[k] = a0[k];
          xb[k] = b0[k];
        }
      } else {
        if (A) load_row(A, j, xa);
        load_row(B, j, xb);
      }
#pragma unroll
      for (int k = 0; k < BLK; ++k) {
        if (A) sA[tid * BLK + k] = k < b ? xa[k] : 0.0;
        sB[tid * BLK + k] = k < b ? xb[k] : 0.0;
      }
    }
    __syncthreads();
    const int rows = (int)(n - r0 < RT ? n - r0 : RT);
    if (live) {
      int r = sl;
      for (; r + 3 * SL < rows; r += 4 * SL) {
        s0 = fma(sP[r * BLK + a], sB[r * BLK + c], s0);
        s1 = fma(sP[(r + SL) * BLK + a], sB[(r + SL) * BLK + c], s1);
        s2 = fma(sP[(r + 2 * SL) * BLK + a], sB[(r + 2 * SL) * BLK + c], s2);
        s3 = fma(sP[(r + 3 * SL) * BLK + a], sB[(r + 3 * SL) * BLK + c], s3);
      }
      for (; r < rows; r += SL) s0 = fma(sP[r * BLK + a], sB[r * BLK + c], s0);
    }
  }
  red[sl * NOP + o] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (tid < NOP && live) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < SL; ++q) t += red[q * NOP + tid];
    if (o < BLK * BLK) out1[o] = t;
    else out2[a * BLK + c] = out2[c * BLK + a] = t;
  }
  __syncthreads();
}

// Partner of index i in round r of the round-robin pairing of eight indices:
// 7 meets r, the others meet (2r - i) mod 7.
__device__ __forceinline__ int jac_partner(int i, int r) {
  if (i == 7) return r;
  if (i == r) return 7;
  return (2 * r - i + 14) % 7;
}

// Upper Cholesky factor R (C = R^T R) of the symmetric b x b matrix C, one wave,
// lane i BLK + j holding C[i][j] (right-looking: after step q the lanes past q
// hold the Schur complement).  Returns R[i][j] for this lane (zero below the
// diagonal and past b) and 1 / R[j][j] in rinv_j; ok (the same on every lane)
// is false on a pivot that keeps less than 1e-12 of its diagonal (six digits of
// the column) or is not finite.
__device__ double chol_wave(double cij, int i, int j, int b, double& rinv_j, bool& ok) {
  double a = cij, r = 0.0;
  rinv_j = 0.0;
  ok = true;
  for (int q = 0; q < b; ++q) {
    const double d = __shfl(a, q * BLK + q, 64), cqq = __shfl(cij, q * BLK + q, 64);
    const double aqj = __shfl(a, q * BLK + j, 64), aqi = __shfl(a, q * BLK + i, 64);
    if (!(cqq > 0.0) || !(d > 1e-12 * cqq) || !isfinite(d)) {
      ok = false;
      return 0.0;
    }
    const double inv = rsqrt_f64(d);
    const double rqj = aqj * inv, rqi = aqi * inv;
    if (i == q && j >= q && j < b) r = rqj;
    if (j == q) rinv_j = inv;
    if (i > q && j > q) a = fma(-rqi, rqj, a);
  }
  return r;
}

// x <- x R^{-1} for one row (forward substitution over the b columns).
__device__ __forceinline__ void solve_row(double (&x)[BLK], const double* R, const double* rinv, int b) {
#pragma unroll
  for (int k = 0; k < BLK; ++k) {
    if (k < b) {
      double t = x[k];
#pragma unroll
      for (int p = 0; p < k; ++p) t = fma(-x[p], R[p * BLK + k], t);
      x[k] = t * rinv[k];
    } else {
      x[k] = 0.0;
    }
  }
}

__device__ __forceinline__ void store_block_row(int64_t j, const double (&x)[BLK], double* __restrict__ Xn,
                                                float* __restrict__ Xbn, float* __restrict__ Wfn) {
  double2* p = reinterpret_cast<double2*>(Xn + j * BLK);
#pragma unroll
  for (int k = 0; k < BLK / 2; ++k) p[k] = double2{x[2 * k], x[2 * k + 1]};
  const f4 lo = f4{(float)x[0], (float)x[1], (float)x[2], (float)x[3]};
  const f4 hi = f4{(float)x[4], (float)x[5], (float)x[6], (float)x[7]};
  if (Xbn) {
    f4* q = reinterpret_cast<f4*>(Xbn + j * BLK);
    q[0] = lo;
    q[1] = hi;
  }
  if (Wfn) {
    f4* w = reinterpret_cast<f4*>(Wfn + j * 16);
    w[0] = lo;
    w[1] = hi;
    w[2] = f4{0.f, 0.f, 0.f, 0.f};
    w[3] = f4{0.f, 0.f, 0.f, 0.f};
  }
}

// The certificate's projected product into a.Zf (and row tid of it into z0):
// Zf = S - B_n C_B - V_1 C_V with S = Z / lam_L^2, C_B = B_n^T X and
// C_V = V_1^T (S - B_n C_B) = V_1^T S - (V_1^T B_n) C_B.  One row per thread
// (n <= RT): the thread's rows of Z, B_n and V_1 are loaded at once (with X's,
// already in x0); C_B and V_1^T S are summed over the rows in tiles of PTR rows
// staged in LDS from those registers (two outputs per thread, rows in order);
// then each thread forms its own row of Zf.
__device__ __forceinline__ void cert_project(const RitzArgs& a, double* stage, const double (&x0)[BLK],
                                             double (&z0)[BLK]) {
  __shared__ double sCB[RMAX * BLK], sCV[RMAX * BLK];
  const int tid = threadIdx.x, b = a.b, r = a.r, rb = r * b;
  const int64_t n = a.n;
  const bool own = tid < n;
  double zr[BLK], bn[RMAX], v1[RMAX];
#pragma unroll
  for (int t = 0; t < RMAX; ++t) bn[t] = v1[t] = 0.0;
  if (own) {
    load_row(a.Z, tid, zr);
    if (r > 0) {
      const double* __restrict__ brow = a.Bn + (int64_t)tid * r;
      const double* __restrict__ vrow = a.V1 + (int64_t)tid * r;
#pragma unroll
      for (int t = 0; t < RMAX; ++t) {  // clamped columns: every load issued before any use
        const int tc = t < r ? t : r - 1;
        bn[t] = brow[tc];
        v1[t] = vrow[tc];
      }
    }
  }
  double* sX = stage;
  double* sZ = sX + PTR * BLK;
  double* sBn = sZ + PTR * BLK;
  double* sV = sBn + PTR * RMAX;
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  for (int64_t r0 = 0; r0 < n; r0 += PTR) {
    __syncthreads();  // the previous tile is consumed
    const int rows = (int)(n - r0 < PTR ? n - r0 : PTR);
    const int q = tid - (int)r0;
    if (own && q >= 0 && q < rows) {
#pragma unroll
      for (int c = 0; c < BLK; ++c) {
        sX[q * BLK + c] = c < b ? x0[c] : 0.0;
        sZ[q * BLK + c] = c < b ? zr[c] : 0.0;
      }
#pragma unroll
      for (int t = 0; t < RMAX; ++t)
        if (t < r) {
          sBn[q * r + t] = bn[t];
          sV[q * r + t] = v1[t];
        }
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int o = tid + h * RT;
      if (o < 2 * rb) {
        const bool isB = o < rb;
        const int oo = isB ? o : o - rb;
        const int t = oo / b, c = oo % b;
        const double* L = isB ? sBn : sV;
        const double* Rt = isB ? sX : sZ;
        // eight rows a step (all sixteen reads in flight), four partial sums
        double s4[4] = {0.0, 0.0, 0.0, 0.0};
        int qq = 0;
        for (; qq + 7 < rows; qq += 8) {
          double lv[8], rv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            lv[u] = L[(qq + u) * r + t];
            rv[u] = Rt[(qq + u) * BLK + c];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) s4[u & 3] = fma(lv[u], rv[u], s4[u & 3]);
        }
        for (; qq < rows; ++qq) s4[qq & 3] = fma(L[qq * r + t], Rt[qq * BLK + c], s4[qq & 3]);
        acc[h][0] += s4[0] + s4[1];
        acc[h][1] += s4[2] + s4[3];
      }
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int o = tid + h * RT;
    const double v = acc[h][0] + acc[h][1];
    if (o < rb) sCB[o] = v;
    else if (o < 2 * rb) sCV[o - rb] = v * a.inv_lam2;  // V_1^T S for now
  }
  __syncthreads();
  double cv = 0.0;
  if (tid < rb) {  // C_V = V_1^T S - (V_1^T B_n) C_B
    const int t = tid / b, c = tid % b;
    cv = sCV[tid];
    for (int u = 0; u < r; ++u) cv = fma(-a.VB[t * r + u], sCB[u * b + c], cv);
  }
  __syncthreads();
  if (tid < rb) sCV[tid] = cv;
  __syncthreads();
  if (own) {
    // column chains side by side: per t, the row's 2b coefficients read together
#pragma unroll
    for (int c = 0; c < BLK; ++c) z0[c] = c < b ? zr[c] * a.inv_lam2 : 0.0;
#pragma unroll
    for (int t = 0; t < RMAX; ++t) {
      if (t < r) {
        double cb[BLK], cvv[BLK];
#pragma unroll
        for (int c = 0; c < BLK; ++c) {
          const int cc = c < b ? c : 0;
          cb[c] = sCB[t * b + cc];
          cvv[c] = sCV[t * b + cc];
        }
#pragma unroll
        for (int c = 0; c < BLK; ++c)
          if (c < b) z0[c] = fma(-bn[t], cb[c], fma(-v1[t], cvv[c], z0[c]));
      }
    }
    double2* p = reinterpret_cast<double2*>(a.Zf + (int64_t)tid * BLK);
#pragma unroll
    for (int k = 0; k < BLK / 2; ++k) p[k] = double2{z0[2 * k], z0[2 * k + 1]};
  }
  __syncthreads();  // Zf complete
}

// The certificate's stop test (wave 0, lane i BLK + j; sth holds the Ritz
// values): see the header.  Writes res = [stop, ritz_0 .. ritz_7] and the state.
__device__ __forceinline__ void cert_stop(const RitzArgs& a, const double* sth) {
  const int tid = threadIdx.x, j = tid & 7, b = a.b;
  const double rj = j < b ? fmax(sth[j], 0.0) : 0.0;
  const double pj = a.it == 0 ? -1.0 : a.state[j];
  const double dj = fabs(rj - pj);
  double dmax = (j < b && (j == 0 || rj >= 0.81)) ? dj : 0.0;
  dmax = fmax(dmax, __shfl_xor(dmax, 1, 64));
  dmax = fmax(dmax, __shfl_xor(dmax, 2, 64));
  dmax = fmax(dmax, __shfl_xor(dmax, 4, 64));
  const double r0 = __shfl(rj, 0, 64), d0 = __shfl(dj, 0, 64);
  const bool all_conv = dmax <= a.conv_rel * fmax(r0, 1e-300);
  const bool below_one = r0 < 0.98 * 0.98 && d0 <= 1e-5 * r0;
  bool surely_below = false;
  if (a.it > 2 && r0 < 1.0 && r0 > 0.0 && d0 <= 1e-3 * r0) {
    const double log_p = log(0.824) + 0.5 * log((double)a.n) + ((double)a.it - 0.5) * log(r0);
    surely_below = log_p <= log(1e-9);
  }
  const bool stop = (a.it > 2 && (all_conv || below_one || surely_below)) || a.last != 0;
  if (tid < BLK) {  // after every lane's read of the state (the test above depends on all of them)
    a.state[j] = rj;
    a.res[1 + j] = rj;
  }
  if (tid == 0) a.res[0] = stop ? 1.0 : 0.0;
}

template <int MODE>
__global__ __launch_bounds__(RT) void k_block_ritz(RitzArgs a) {
  // a step queued ahead of the host's reading of the previous step's stop flag
  // does nothing once that flag is set (every thread reads it before thread 0
  // rewrites res[0])
  if (a.skip && *a.skip != 0.0) return;
  constexpr int STAGE = (2 * RT * BLK > PTR * (2 * BLK + 2 * RMAX)) ? 2 * RT * BLK : PTR * (2 * BLK + 2 * RMAX);
  __shared__ double stage[STAGE];
  __shared__ double red[RT];
  __shared__ double sH[BLK * BLK], sC0[BLK * BLK], sW[BLK * BLK], sT[BLK * BLK], sR[BLK * BLK], sRi[BLK], sth[BLK];
  __shared__ int sok, ssingle;
  const int tid = threadIdx.x;
  const int64_t n = a.n;
  const int b = a.b;
  const double* __restrict__ X = a.X;
  double* __restrict__ Xn = a.Xn;
  double* res = a.res;
  double* sA = stage;
  double* sB = stage + RT * BLK;

  // 1. H = X^T Z and Z^T Z (row tid of each kept in registers for step 3)
  double x0[BLK], z0[BLK];
  const double* Z = a.Z;
  if (tid < n) load_row(X, tid, x0);
  if (MODE == RITZ_CERT) {
    cert_project(a, stage, x0, z0);
    Z = a.Zf;
  } else if (tid < n) {
    load_row(Z, tid, z0);
  }
  row_grams(X, Z, n, b, sH, sC0, red, sA, sB, x0, z0);

  // 2. eigenpairs of H (one wave): cyclic Jacobi in FP32 on H scaled into FP32
  //    range (an approximate eigenbasis W: it rotates the next block), then in
  //    FP64 the Ritz values that are used: the top pair for Frank-Wolfe
  //    (Rayleigh quotient, one first-order correction of w_0 against the other
  //    Ritz vectors, normalisation, Rayleigh quotient), every Rayleigh quotient
  //    w_j^T H w_j / w_j^T w_j for the certificate
  double hsym = 0.0;
  int hexp = 0;
  if (tid < 64) {
    const int i = tid >> 3, j = tid & 7;
    hsym = (i < b && j < b) ? 0.5 * (sH[i * BLK + j] + sH[j * BLK + i]) : 0.0;
    double mx = fabs(hsym);
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    hexp = (mx > 0.0 && isfinite(mx)) ? ilogb(mx) : 0;
    float h = (float)ldexp(hsym, -hexp);
    float w = i == j ? 1.f : 0.f;
    // until the off-diagonal norm is below 1e-6 of the norm (about FP32 rounding)
    for (int sweep = 0; sweep < 16; ++sweep) {
      const float off = wave_sumf(i != j ? h * h : 0.f), dia = wave_sumf(i == j ? h * h : 0.f);
      if (!(off > 1e-12f * dia)) break;
      for (int r = 0; r < BLK - 1; ++r) {
        // this lane's two rotations (the pairs holding its row and column
        // indices), every exchange of the round issued at once
        const int pi = jac_partner(i, r), pj = jac_partner(j, r);
        const int ip = i < pi ? i : pi, iq = i < pi ? pi : i, jp = j < pj ? j : pj, jq = j < pj ? pj : j;
        const float aipp = __shfl(h, ip * BLK + ip, 64), aiqq = __shfl(h, iq * BLK + iq, 64);
        const float aipq = __shfl(h, ip * BLK + iq, 64);
        const float ajpp = __shfl(h, jp * BLK + jp, 64), ajqq = __shfl(h, jq * BLK + jq, 64);
        const float ajpq = __shfl(h, jp * BLK + jq, 64);
        const float h_ipj = __shfl(h, i * BLK + pj, 64), h_pij = __shfl(h, pi * BLK + j, 64);
        const float h_pipj = __shfl(h, pi * BLK + pj, 64), w_ipj = __shfl(w, i * BLK + pj, 64);
        float ci, ti, cj, tj;
        jacobi_ct(aipp, aiqq, aipq, ci, ti);
        jacobi_ct(ajpp, ajqq, ajpq, cj, tj);
        const float si = (i == ip ? -ti : ti) * ci, sj = (j == jp ? -tj : tj) * cj;
        h = ci * (cj * h + sj * h_ipj) + si * (cj * h_pij + sj * h_pipj);
        w = w * cj + w_ipj * sj;
      }
    }
    sT[tid] = (double)w;
    if (i == j) sth[i] = ldexp((double)h, hexp);
  }
  __syncthreads();
  if (tid < 64) {
    const int i = tid >> 3, j = tid & 7;
    // descending order of the b live eigenvalues (ties by index): rank of index j
    const double lj = sth[j];
    int rank = 0;
#pragma unroll
    for (int q = 0; q < BLK; ++q) {
      const double lq = sth[q];
      rank += (q < b && (lq > lj || (lq == lj && q < j))) ? 1 : 0;
    }
    int perm_i = 0;  // index whose rank is i (column i of the sorted W)
#pragma unroll
    for (int q = 0; q < BLK; ++q) perm_i = __shfl(rank, q, 64) == i && q < b ? q : perm_i;
    const int src = __shfl(perm_i, j * BLK, 64);  // index of rank j, from a lane with row j
    double wij = (i < b && j < b) ? sT[i * BLK + src] : 0.0;  // W[i][j], sorted
    const double thj = j < b ? sth[src] : 0.0;                // theta_j (FP32 accuracy)
    if (MODE == RITZ_FW) {
      // FP64: u = H w_0 (lane (i, .) gets u_i), m_j = w_j^T u, n0 = w_0^T w_0
      double u = hsym * __shfl(wij, j * BLK, 64);  // H[i][j] w_0[j]
      u += __shfl_xor(u, 1, 64);
      u += __shfl_xor(u, 2, 64);
      u += __shfl_xor(u, 4, 64);
      double m = wij * u;
      m += __shfl_xor(m, 8, 64);
      m += __shfl_xor(m, 16, 64);
      m += __shfl_xor(m, 32, 64);
      const double w0i = __shfl(wij, i * BLK, 64);
      double n0 = (j == 0) ? w0i * w0i : 0.0;
      n0 = wave_sum(n0);
      const double th0r = __shfl(m, 0, 64) / n0;  // Rayleigh quotient of w_0
      // w_0 += sum_j m_j / (theta_0 - theta_j) w_j over the well-separated j
      const double gap = th0r - thj;
      double coef = 0.0;
      if (j >= 1 && j < b && fabs(m) <= 0.1 * fabs(gap) * sqrt(n0)) coef = m / gap;
      double add = coef * wij;
      add += __shfl_xor(add, 1, 64);
      add += __shfl_xor(add, 2, 64);
      add += __shfl_xor(add, 4, 64);
      double w0n = i < b ? w0i + add : 0.0;  // lanes of row i: the corrected w_0[i]
      double nn = (j == 0) ? w0n * w0n : 0.0;
      nn = wave_sum(nn);
      w0n = nn > 0.0 ? w0n * rsqrt_f64(nn) : w0i;
      // theta_0 = w_0^T H w_0 with the corrected, unit w_0
      double u2 = hsym * __shfl(w0n, j * BLK, 64);
      u2 += __shfl_xor(u2, 1, 64);
      u2 += __shfl_xor(u2, 2, 64);
      u2 += __shfl_xor(u2, 4, 64);
      double th0 = (j == 0) ? w0n * u2 : 0.0;
      th0 = wave_sum(th0);
      if (j == 0) wij = w0n;
      sW[tid] = wij;
      if (i == 0) sR[j] = j == 0 ? th0 : thj;  // sorted eigenvalues, staged
    } else {
      // every Rayleigh quotient: u_ij = (H W)[i][j], theta_j = sum_i W[i][j] u_ij / sum_i W[i][j]^2
      double u = 0.0;
#pragma unroll
      for (int q = 0; q < BLK; ++q) u = fma(__shfl(hsym, i * BLK + q, 64), __shfl(wij, q * BLK + j, 64), u);
      double num = wij * u, den = wij * wij;
      num += __shfl_xor(num, 8, 64);
      num += __shfl_xor(num, 16, 64);
      num += __shfl_xor(num, 32, 64);
      den += __shfl_xor(den, 8, 64);
      den += __shfl_xor(den, 16, 64);
      den += __shfl_xor(den, 32, 64);
      sW[tid] = wij;
      if (i == 0) sR[j] = (j < b && den > 0.0) ? num / den : 0.0;
    }
  }
  __syncthreads();
  if (tid < 64) {  // sT = (Z^T Z) W
    const int i = tid >> 3, j = tid & 7;
    double t = 0.0;
#pragma unroll
    for (int l = 0; l < BLK; ++l) t = fma(sC0[i * BLK + l], sW[l * BLK + j], t);
    sT[tid] = t;
    if (i == 0) sth[j] = sR[j];
  }
  __syncthreads();
  if (tid < 64) {  // the Gram of Z W: W^T (Z^T Z) W (upper triangle, mirrored)
    const int i = tid >> 3, j = tid & 7;
    const int ii = i < j ? i : j, jj = i < j ? j : i;
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < BLK; ++k) t = fma(sW[k * BLK + ii], sT[k * BLK + jj], t);
    // Gershgorin on the column-scaled Gram: the largest off-diagonal row sum
    const double tii = __shfl(t, i * BLK + i, 64), tjj = __shfl(t, j * BLK + j, 64);
    double g = 0.0;
    if (i != j && i < b && j < b)
      g = (tii > 0.0 && tjj > 0.0 && isfinite(tii) && isfinite(tjj)) ? fabs(t) * rsqrt_f64(tii) * rsqrt_f64(tjj)
                                                                      : 2.0;
    g += __shfl_xor(g, 1, 64);
    g += __shfl_xor(g, 2, 64);
    g += __shfl_xor(g, 4, 64);
    g = fmax(g, __shfl_xor(g, 8, 64));
    g = fmax(g, __shfl_xor(g, 16, 64));
    g = fmax(g, __shfl_xor(g, 32, 64));
    bool ok;
    double rinv;
    const double r = chol_wave(t, i, j, b, rinv, ok);
    sR[tid] = r;
    if (i == 0) sRi[j] = rinv;
    if (tid == 0) {
      sok = ok ? 1 : 0;
      ssingle = g <= 0.5 ? 1 : 0;
    }
  }
  __syncthreads();
  const bool ok1 = sok != 0, single = ok1 && ssingle != 0;
  const double th0 = fmax(sth[0], 0.0);

  // 3. rows: Z W, the residual, v = X w_0; the next block after one
  //    factorisation (final when single)
  double rr = 0.0;
  for (int64_t j = tid; j < n; j += RT) {
    double zr[BLK], xr[BLK], y[BLK];
    if (j == tid) {
#pragma unroll
      for (int k = 0; k < BLK; ++k) {
        zr[k] = z0[k];
        xr[k] = x0[k];
      }
    } else {
      load_row(Z, j, zr);
      load_row(X, j, xr);
    }
    double xw = 0.0;
#pragma unroll
    for (int k = 0; k < BLK; ++k) y[k] = 0.0;
#pragma unroll
    for (int a = 0; a < BLK; ++a) {
      if (a < b) {
        xw = fma(xr[a], sW[a * BLK], xw);
#pragma unroll
        for (int k = 0; k < BLK; ++k) y[k] = fma(zr[a], sW[a * BLK + k], y[k]);
      }
    }
    const double e = y[0] - th0 * xw;
    rr = fma(e, e, rr);
    if (MODE == RITZ_FW) a.v32[j] = (float)xw;
    else a.vtop[j] = xw;
    if (ok1) solve_row(y, sR, sRi, b);
    if (single) {
      store_block_row(j, y, Xn, a.Xbn, a.Wfn);
    } else {
      double2* p = reinterpret_cast<double2*>(Xn + j * BLK);
#pragma unroll
      for (int k = 0; k < BLK / 2; ++k) p[k] = double2{y[2 * k], y[2 * k + 1]};
    }
  }
  rr = block_sum1(rr, red);
  if (MODE == RITZ_FW) {
    const double resid = th0 > 0.0 ? sqrt(rr) / th0 : 0.0;
    if (tid == 0) {
      const bool done = resid <= a.ptol || a.last != 0 || th0 == 0.0 || !isfinite(th0) || !isfinite(resid);
      res[0] = done ? 1.0 : 0.0;
      res[1] = th0;
      res[2] = resid;
    }
    if (tid < BLK) a.cw[tid] = (float)sW[tid * BLK];
  } else if (tid < 64) {
    cert_stop(a, sth);
  }
  if (single) return;
  __syncthreads();  // Xn complete

  // 4. second Cholesky QR pass, or Gram-Schmidt
  bool ok2 = false;
  if (ok1) {
    double y0[BLK];
    if (tid < n) load_row(Xn, tid, y0);
    row_grams(nullptr, Xn, n, b, nullptr, sH, red, sA, sB, y0, y0);
    if (tid < 64) {
      bool ok;
      double rinv;
      const double r = chol_wave(sH[tid], tid >> 3, tid & 7, b, rinv, ok);
      sR[tid] = r;
      if (tid < BLK) sRi[tid] = rinv;
      if (tid == 0) sok = ok ? 1 : 0;
    }
    __syncthreads();
    ok2 = sok != 0;
  }
  if (ok2) {
    for (int64_t j = tid; j < n; j += RT) {
      double x[BLK];
      load_row(Xn, j, x);
      solve_row(x, sR, sRi, b);
      store_block_row(j, x, Xn, a.Xbn, a.Wfn);
    }
    return;
  }
  // modified Gram-Schmidt on the columns of Xn, twice per column
  for (int q = 0; q < b; ++q) {
    for (int attempt = 0; attempt < 2; ++attempt) {
      double before = 0.0;
      for (int64_t j = tid; j < n; j += RT) before = fma(Xn[j * BLK + q], Xn[j * BLK + q], before);
      before = block_sum1(before, red);
      for (int pass = 0; pass < 2; ++pass)
        for (int p = 0; p < q; ++p) {
          double d = 0.0;
          for (int64_t j = tid; j < n; j += RT) d = fma(Xn[j * BLK + p], Xn[j * BLK + q], d);
          d = block_sum1(d, red);
          for (int64_t j = tid; j < n; j += RT) Xn[j * BLK + q] -= d * Xn[j * BLK + p];
          __syncthreads();
        }
      double nn = 0.0;
      for (int64_t j = tid; j < n; j += RT) nn = fma(Xn[j * BLK + q], Xn[j * BLK + q], nn);
      nn = block_sum1(nn, red);
      if (nn > 1e-20 * before && nn > 0.0) {
        const double inv = 1.0 / sqrt(nn);
        for (int64_t j = tid; j < n; j += RT) Xn[j * BLK + q] *= inv;
        __syncthreads();
        break;
      }
      for (int64_t j = tid; j < n; j += RT)
        Xn[j * BLK + q] = attempt == 0 ? start_entry(a.salt + (uint64_t)(j * BLK + q)) : 0.0;
      __syncthreads();
    }
  }
  for (int64_t j = tid; j < n; j += RT) {
    double x[BLK];
    load_row(Xn, j, x);
    store_block_row(j, x, Xn, a.Xbn, a.Wfn);
  }
}


}  // namespace rpca_ritz
