// Frank-Wolfe with the sparse part marginalised (Sec. 6.2, Alg. 1).  The
// iteration and its quantities are defined in rpca_fw.h.
//
// Every kernel here streams m x n FP32 matrices (L, X, G) from HBM with no
// reuse worth a matrix core, so the roofline is HBM bandwidth.  Layout follows
// X: column-major, column j contiguous, 16-byte vector accesses when m is a
// multiple of 4 and the buffers are 16-byte aligned.  Per iteration:
//   linear minimisation: block power iteration on G^T G with a block of BLK
//     vectors: Z = G^T G Xb in one fused pass over G when n <= 256, else
//     Y = G Xb (column chunks -> partial Y, fixed-order sum) and Z = G^T Y (row
//     chunks x a few columns -> FP64 partials, fixed-order sum); then
//     Rayleigh-Ritz, the stop test and the next orthonormal block in FP64 in one
//     workgroup; it stops when the top Ritz pair's residual is small, and the
//     Ritz-rotated block starts the next iteration;
//   bilinear pass (when the vertex is nonzero): u^T P_Omega(L) v and
//     sum_Omega u_i^2 v_j^2 with u = y / sigma, y = G v;
//   update pass: L <- a L + b y v^T, G = P_Omega(clip(L - X)), and FP64 sums of
//     phi(L), <G, L>, sum_Omega L^2 (per-block partials, fixed-order total).
// Every reduction has a fixed order, so results are reproducible run to run.

#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <new>
#include <vector>

#include "rpca.h"
#include "rpca_fw.h"
#include "rpca_internal.h"
#include "ritz_kernel.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int TH = 256;         // threads per block of the streaming kernels
constexpr int BLK = 8;          // vectors in the power-iteration block
constexpr int LEFT_COLS = 32;   // columns per block of Y = G Xb
constexpr int RIGHT_COLS = 4;   // columns per block of Z = G^T Y
constexpr int RIGHT_ITER = 4;   // row groups per thread in Z = G^T Y
constexpr int COL_ITER = 8;     // row groups per thread in the bilinear pass
constexpr int FIN_TH = 1024;    // threads of the single-block finishing kernels
constexpr int POWER_MAX = 100;  // power steps per iteration at most
constexpr double POWER_TOL = 1e-4;  // default bound on the top Ritz pair's relative residual

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block sums of Q values (fixed order); thread 0 gets them in out[].
template <int Q, int NT>
__device__ __forceinline__ void block_sums(double (&v)[Q], double* out) {
  __shared__ double red[Q][NT / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    v[q] = wave_sum(v[q]);
    if (lane == 0) red[q][w] = v[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      double s = 0.0;
      for (int i = 0; i < NT / 64; ++i) s += red[q][i];
      out[q] = s;
    }
  }
}

__device__ __forceinline__ f4 load4(const float* p) { return *reinterpret_cast<const f4*>(p); }
__device__ __forceinline__ void store4(float* p, f4 v) { *reinterpret_cast<f4*>(p) = v; }

// Observation bits of rows i .. i+VEC-1 of column j (all ones without a mask).
template <int VEC, bool MASK>
__device__ __forceinline__ unsigned obs_bits(const uint32_t* mask, int mw, int64_t j, int64_t i) {
  if (!MASK) return (1u << VEC) - 1u;
  return (mask[j * mw + (i >> 5)] >> (unsigned)(i & 31)) & ((1u << VEC) - 1u);
}

// L <- a L + b y_i v_j;  G = P_Omega(clip(L - X));  block partials of
// phi(L), <G, L>, sum_Omega L^2.  Block b covers rows (b % rb) * TH * VEC ... of
// column b / rb.
template <int VEC, bool MASK>
// a = st[1], b = st[2] from the step state; nothing once st[3] (done) is set.
__global__ __launch_bounds__(TH) void k_fw_update(float* __restrict__ L, const float* __restrict__ X,
                                                  const uint32_t* __restrict__ mask, int mw, int64_t m,
                                                  int64_t rb, const double* __restrict__ st,
                                                  const float* __restrict__ y, const float* __restrict__ v,
                                                  float lam_s, float* __restrict__ G, double* __restrict__ part) {
  if (st[3] != 0.0) return;
  const float a = (float)st[1], b = (float)st[2];
  const int64_t blk = blockIdx.x;
  const int64_t j = blk / rb;
  const int64_t i0 = (blk % rb) * (TH * VEC) + (int64_t)threadIdx.x * VEC;
  double s[3] = {0.0, 0.0, 0.0};
  if (i0 < m) {
    const float bv = b != 0.f ? b * v[j] : 0.f;
    const int64_t off = j * m + i0;
    float l[VEC], x[VEC], yy[VEC];
    if (VEC == 4) {
      const f4 lv = load4(L + off), xv = load4(X + off);
      const f4 yv = bv != 0.f ? load4(y + i0) : f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int c = 0; c < VEC; ++c) {
        l[c] = lv[c];
        x[c] = xv[c];
        yy[c] = yv[c];
      }
    } else {
      l[0] = L[off];
      x[0] = X[off];
      yy[0] = bv != 0.f ? y[i0] : 0.f;
    }
    const unsigned bits = obs_bits<VEC, MASK>(mask, mw, j, i0);
    float g[VEC];
#pragma unroll
    for (int c = 0; c < VEC; ++c) {
      l[c] = fmaf(bv, yy[c], a * l[c]);
      const float r = l[c] - x[c];
      const bool o = (bits >> c) & 1u;
      const float gc = fminf(fmaxf(r, -lam_s), lam_s);
      g[c] = o ? gc : 0.f;
      if (o) {
        s[0] += (double)(gc * (r - 0.5f * gc));
        s[1] += (double)gc * (double)l[c];
        s[2] += (double)l[c] * (double)l[c];
      }
    }
    if (VEC == 4) {
      store4(L + off, f4{l[0], l[1], l[2], l[3]});
      store4(G + off, f4{g[0], g[1], g[2], g[3]});
    } else {
      L[off] = l[0];
      G[off] = g[0];
    }
  }
  block_sums<3, TH>(s, part + blk * 3);
}

// Fixed-order total of Q-wide block partials into res[0..Q).
template <int Q>
__global__ __launch_bounds__(FIN_TH) void k_sum_parts(const double* __restrict__ part, int64_t nblocks,
                                                      double* __restrict__ res) {
  double s[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) s[q] = 0.0;
  for (int64_t b = threadIdx.x; b < nblocks; b += FIN_TH)
#pragma unroll
    for (int q = 0; q < Q; ++q) s[q] += part[b * Q + q];
  block_sums<Q, FIN_TH>(s, res);
}

// Partial Y over a chunk of LEFT_COLS columns: ypart[(cc m + i) BLK + q] =
// sum_{j in chunk cc} G_ij Xb[j BLK + q].
template <int VEC>
__global__ __launch_bounds__(TH) void k_fw_left(const float* __restrict__ G, const float* __restrict__ Xb, int64_t m,
                                                int64_t n, int64_t rb, float* __restrict__ ypart) {
  const int64_t blk = blockIdx.x;
  const int64_t cc = blk / rb;
  const int64_t i0 = (blk % rb) * (TH * VEC) + (int64_t)threadIdx.x * VEC;
  if (i0 >= m) return;
  const int64_t j0 = cc * LEFT_COLS;
  const int ncol = (int)(n - j0 < LEFT_COLS ? n - j0 : LEFT_COLS);
  float acc[VEC][BLK];
#pragma unroll
  for (int c = 0; c < VEC; ++c)
#pragma unroll
    for (int q = 0; q < BLK; ++q) acc[c][q] = 0.f;
#pragma unroll 8
  for (int t = 0; t < ncol; ++t) {
    const int64_t off = (j0 + t) * m + i0;
    float g[VEC];
    if (VEC == 4) {
      const f4 v = load4(G + off);
#pragma unroll
      for (int c = 0; c < VEC; ++c) g[c] = v[c];
    } else {
      g[0] = G[off];
    }
    const float* xr = Xb + (j0 + t) * BLK;
#pragma unroll
    for (int q = 0; q < BLK; ++q) {
      const float xq = xr[q];
#pragma unroll
      for (int c = 0; c < VEC; ++c) acc[c][q] = fmaf(g[c], xq, acc[c][q]);
    }
  }
  float* out = ypart + (cc * m + i0) * BLK;
#pragma unroll
  for (int c = 0; c < VEC; ++c)
#pragma unroll
    for (int q = 0; q < BLK; q += 4) store4(out + c * BLK + q, f4{acc[c][q], acc[c][q + 1], acc[c][q + 2], acc[c][q + 3]});
}

// Y[i BLK + q] = sum over column chunks of ypart (fixed order).
__global__ __launch_bounds__(TH) void k_fw_left_finish(const float* __restrict__ ypart, int64_t nchunks, int64_t mb,
                                                       float* __restrict__ Y) {
  const int64_t e = (int64_t)blockIdx.x * TH + threadIdx.x;
  if (e >= mb) return;
  float s = 0.f;
  for (int64_t c = 0; c < nchunks; ++c) s += ypart[c * mb + e];
  Y[e] = s;
}

// Partial Z over a chunk of rows and RIGHT_COLS columns: part[((rc_i n) + j) BLK + q]
// = sum_{i in chunk} G_ij Y[i BLK + q] (FP32 per thread, FP64 across the block).
template <int VEC>
__global__ __launch_bounds__(TH) void k_fw_right(const float* __restrict__ G, const float* __restrict__ Y, int64_t m,
                                                 int64_t n, int64_t ncb, double* __restrict__ part) {
  const int64_t blk = blockIdx.x;
  const int64_t rci = blk / ncb;
  const int64_t j0 = (blk % ncb) * RIGHT_COLS;
  const int64_t base = rci * (int64_t)(TH * VEC * RIGHT_ITER);
  float s[RIGHT_COLS][BLK];
#pragma unroll
  for (int c = 0; c < RIGHT_COLS; ++c)
#pragma unroll
    for (int q = 0; q < BLK; ++q) s[c][q] = 0.f;
#pragma unroll
  for (int it = 0; it < RIGHT_ITER; ++it) {
    const int64_t i0 = base + (int64_t)it * TH * VEC + (int64_t)threadIdx.x * VEC;
    if (i0 < m) {
      float y[VEC][BLK];
#pragma unroll
      for (int r = 0; r < VEC; ++r)
#pragma unroll
        for (int q = 0; q < BLK; q += 4) {
          const f4 v = load4(Y + (i0 + r) * BLK + q);
          y[r][q] = v[0];
          y[r][q + 1] = v[1];
          y[r][q + 2] = v[2];
          y[r][q + 3] = v[3];
        }
#pragma unroll
      for (int c = 0; c < RIGHT_COLS; ++c) {
        if (j0 + c < n) {
          float g[VEC];
          if (VEC == 4) {
            const f4 v = load4(G + (j0 + c) * m + i0);
#pragma unroll
            for (int r = 0; r < VEC; ++r) g[r] = v[r];
          } else {
            g[0] = G[(j0 + c) * m + i0];
          }
#pragma unroll
          for (int r = 0; r < VEC; ++r)
#pragma unroll
            for (int q = 0; q < BLK; ++q) s[c][q] = fmaf(g[r], y[r][q], s[c][q]);
        }
      }
    }
  }
  // block totals: FP32 within each wave, FP64 across the four waves
  __shared__ double red[RIGHT_COLS * BLK][TH / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < RIGHT_COLS; ++c)
#pragma unroll
    for (int q = 0; q < BLK; ++q) {
      float v = s[c][q];
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      if (lane == 0) red[c * BLK + q][w] = (double)v;
    }
  __syncthreads();
  if (threadIdx.x < RIGHT_COLS * BLK) {
    const int c = threadIdx.x / BLK, q = threadIdx.x % BLK;
    if (j0 + c < n) {
      double t = 0.0;
      for (int i = 0; i < TH / 64; ++i) t += red[threadIdx.x][i];
      part[(rci * n + j0 + c) * BLK + q] = t;
    }
  }
}

// Z[j BLK + q] = sum over row chunks of the partials (fixed order).
__global__ __launch_bounds__(TH) void k_fw_right_finish(const double* __restrict__ part, int64_t rc, int64_t nb,
                                                        double* __restrict__ Z) {
  const int64_t e = (int64_t)blockIdx.x * TH + threadIdx.x;
  if (e >= nb) return;
  double s = 0.0;
  for (int64_t r = 0; r < rc; ++r) s += part[r * nb + e];
  Z[e] = s;
}

// y_i = sum_q Y[i BLK + q] w_q  (G v for v = Xb w).
__global__ __launch_bounds__(TH) void k_fw_combine(const float* __restrict__ Y, const float* __restrict__ w,
                                                   int64_t m, float* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * TH + threadIdx.x;
  if (i >= m) return;
  float s = 0.f;
#pragma unroll
  for (int q = 0; q < BLK; ++q) s = fmaf(Y[i * BLK + q], w[q], s);
  y[i] = s;
}

// Bilinear pass over a chunk of rows of column j (observed entries only):
// part[0] = sum_i A_ij u_i, part[1] = sum_i u_i^2, u_i = ws w_i.
template <int VEC, bool MASK>
// u = w / sigma with sigma = sqrt(theta_0) (res[9]); nothing when sigma <= lam_L
// (no step: the sums are not used).
__global__ __launch_bounds__(TH) void k_fw_bilinear(const float* __restrict__ A, const float* __restrict__ w,
                                                    const double* __restrict__ res, double lam_l,
                                                    const uint32_t* __restrict__ mask, int mw, int64_t m, int64_t rc,
                                                    double* __restrict__ part) {
  const double sigma = sqrt(fmax(res[9], 0.0));
  if (!(sigma > lam_l)) return;
  const float ws = (float)(1.0 / sigma);
  const int64_t blk = blockIdx.x;
  const int64_t j = blk / rc;
  const int64_t base = (blk % rc) * (int64_t)(TH * VEC * COL_ITER);
  float s0 = 0.f, s1 = 0.f;
#pragma unroll
  for (int it = 0; it < COL_ITER; ++it) {
    const int64_t i0 = base + (int64_t)it * TH * VEC + (int64_t)threadIdx.x * VEC;
    if (i0 < m) {
      float av[VEC], wv[VEC];
      if (VEC == 4) {
        const f4 qa = load4(A + j * m + i0), qw = load4(w + i0);
#pragma unroll
        for (int c = 0; c < VEC; ++c) {
          av[c] = qa[c];
          wv[c] = qw[c];
        }
      } else {
        av[0] = A[j * m + i0];
        wv[0] = w[i0];
      }
      const unsigned bits = obs_bits<VEC, MASK>(mask, mw, j, i0);
#pragma unroll
      for (int c = 0; c < VEC; ++c) {
        if ((bits >> c) & 1u) {
          const float u = ws * wv[c];
          s0 = fmaf(av[c], u, s0);
          s1 = fmaf(u, u, s1);
        }
      }
    }
  }
  double s[2] = {(double)s0, (double)s1};
  block_sums<2, TH>(s, part + blk * 2);
}

// One block: res[2] = sum_j v_j p0_j, res[3] = sum_j v_j^2 p1_j over the
// bilinear partials.
__global__ __launch_bounds__(FIN_TH) void k_fw_bilinear_finish(const double* __restrict__ part, int64_t rc, int64_t n,
                                                               const float* __restrict__ v, double* __restrict__ res) {
  double s[2] = {0.0, 0.0};
  for (int64_t j = threadIdx.x; j < n; j += FIN_TH) {
    double p0 = 0.0, p1 = 0.0;
    for (int64_t r = 0; r < rc; ++r) {
      p0 += part[(j * rc + r) * 2];
      p1 += part[(j * rc + r) * 2 + 1];
    }
    const double vj = (double)v[j];
    s[0] += vj * p0;
    s[1] += vj * vj * p1;
  }
  block_sums<2, FIN_TH>(s, res + 2);
}

// The step of an iteration from its sums (one thread): res[4..6] = phi(L), <G, L>,
// sum_Omega L^2 (update pass), res[9] = theta_0 (sigma^2), res[2..3] = the
// bilinear sums; st = [t, a, b, done, F, gap, sigma, eta, step, nonfinite, t of this
// iteration, eta of the last applied step, phi].  With V = -B u v^T the gap and the
// exact line search need only these (Alg. 1); done when gap <= tol F or at the
// last iteration, else st[0..2] take the next t and the update's a, b.
__global__ void k_fw_step(const double* __restrict__ res, double* __restrict__ st, double lam_l, double tol,
                          int last) {
  if (threadIdx.x != 0) return;
  const double phi = res[4], gl = res[5], l2 = res[6], t = st[0];
  st[10] = t;
  st[12] = phi;
  if (!isfinite(phi) || !isfinite(gl) || !isfinite(l2)) {
    st[9] = 1.0;
    st[3] = 1.0;
    return;
  }
  const double F = phi + lam_l * t, B = phi / lam_l + t;
  const double sigma = sqrt(fmax(res[9], 0.0));
  const bool step = sigma > lam_l;
  double gap, eta = 0.0;
  if (step) {
    const double b1 = res[2], b2 = res[3];
    gap = gl + B * sigma + lam_l * (t - B);
    const double dd = B * B * b2 + 2.0 * B * b1 + l2;
    if (dd > 0.0) eta = (B * sigma + gl - lam_l * (B - t)) / dd;
  } else {
    gap = gl + lam_l * t;
    if (l2 > 0.0) eta = (gl + lam_l * t) / l2;
  }
  eta = fmin(fmax(eta, 0.0), 1.0);
  const bool done = gap <= tol * F || last != 0;
  st[4] = F;
  st[5] = gap;
  st[6] = sigma;
  st[7] = eta;
  st[8] = step ? 1.0 : 0.0;
  st[3] = done ? 1.0 : 0.0;
  if (!done) {
    st[1] = 1.0 - eta;
    st[2] = step ? -eta * B / sigma : 0.0;
    st[0] = (1.0 - eta) * t + eta * (step ? B : 0.0);
    st[11] = eta;
  }
}

// st = [t, a = 1, b = 0, not done, ...]: the first update pass forms G and the sums.
__global__ void k_fw_state_init(double* __restrict__ st, double t) {
  const int i = threadIdx.x;
  if (i < 16) st[i] = i == 0 ? t : (i == 1 ? 1.0 : 0.0);
}

using rpca_ritz::start_entry;
static_assert(rpca_ritz::BLK == BLK, "one block width");

}  // namespace

struct rpca_fw {
  int64_t m = 0, n = 0;
  double lam_s = 0, lam_l = 0;
  int mw = 0;
  int vec = 1;
  int b = BLK;                  // live block columns: min(BLK, n)
  uint32_t* mask = nullptr;
  float* G = nullptr;           // m x n
  float* ypart = nullptr;       // left-product chunks x m x BLK
  float* Y = nullptr;           // m x BLK
  float* y = nullptr;           // m: G v
  int cur = 0;                  // which of the two block copies is the current block
  double* Xd = nullptr;         // 2 x (n x BLK) FP64 blocks (orthonormal first b columns, zero padding)
  float* Xb = nullptr;          // 2 x (n x BLK) FP32 copies of them
  float* cw = nullptr;          // BLK: the top Ritz vector's coefficients (y = (G Xb) cw)
  float* v = nullptr;           // n: right singular vector
  double* part = nullptr;       // block partials
  double* Z = nullptr;          // n x BLK
  double* res = nullptr;        // small device results
  double* res_host = nullptr;   // pinned copy
  double* st = nullptr;         // 16 doubles: the iteration's step state (k_fw_step)
  double* st_host = nullptr;    // pinned copy of it
  hipEvent_t flag_ev[2] = {nullptr, nullptr};  // the power steps' stop-flag copies (two slots)
  double* zpin = nullptr;       // pinned staging of the start block (n x BLK doubles)
  float* xpin = nullptr;        // n x (BLK + 16) floats
  // fused G^T G Xb in one pass over G (n <= 256): the blocks as FP32 n x 16 and
  // the per-workgroup sums
  float* Wf = nullptr;          // 2 x (n x 16)
  float* gpart = nullptr;
  int rg_ga = 0;
  std::vector<double> Xh;       // the start block on the host (FP64)
  int64_t rb_upd = 0, nchunks_left = 0, rc_right = 0, rc_bil = 0;
  bool x_valid = false;
  // optional kernel timing (rpca_fw_profile_*): event pairs per kernel class
  bool prof_on = false;
  struct Pending {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> ev_free;
  int64_t launches[4] = {0, 0, 0, 0};
  double ms[4] = {0, 0, 0, 0};
};

namespace {

hipEvent_t fw_event(rpca_fw* h) {
  if (!h->ev_free.empty()) {
    hipEvent_t e = h->ev_free.back();
    h->ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

// Elapsed times of the recorded pairs (their stream has been synchronised).
void fw_collect(rpca_fw* h) {
  for (auto& p : h->pending) {
    float t = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
      h->launches[p.cls] += 1;
      h->ms[p.cls] += t;
    }
    h->ev_free.push_back(p.a);
    h->ev_free.push_back(p.b);
  }
  h->pending.clear();
}

// Launch with an event pair around it when timing is on.
template <typename Fn>
hipError_t fw_timed(rpca_fw* h, int cls, hipStream_t s, Fn&& launch) {
  if (!h->prof_on) {
    launch();
    return hipGetLastError();
  }
  hipEvent_t a = fw_event(h), b = fw_event(h);
  if (!a || !b || hipEventRecord(a, s) != hipSuccess) return hipErrorUnknown;
  launch();
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = hipEventRecord(b, s)) != hipSuccess) return e;
  h->pending.push_back({cls, a, b});
  if (h->pending.size() >= 4096) fw_collect(h);
  return hipSuccess;
}

void fw_free(rpca_fw* h) {
  fw_collect(h);
  for (hipEvent_t e : h->ev_free) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->flag_ev)
    if (e) (void)hipEventDestroy(e);
  for (void* p : {(void*)h->mask, (void*)h->G, (void*)h->ypart, (void*)h->Y, (void*)h->y, (void*)h->Xd, (void*)h->Xb,
                  (void*)h->cw, (void*)h->v, (void*)h->part, (void*)h->Z, (void*)h->res, (void*)h->Wf,
                  (void*)h->gpart, (void*)h->st})
    if (p) (void)hipFree(p);
  // a failed free must not stay pending: the caller's next error check would see it
  for (void* p : {(void*)h->res_host, (void*)h->zpin, (void*)h->xpin, (void*)h->st_host})
    if (p && hipHostFree(p) != hipSuccess) (void)hipGetLastError();
  delete h;
}

#define FWCHK(expr)                             \
  do {                                          \
    if ((expr) != hipSuccess) return RPCA_EHIP; \
  } while (0)

// L <- a L + b y v^T (a, b from the step state), G and the three sums into
// res[4..6] (host copy queued).
int fw_update(rpca_fw* h, const float* X, float* L, hipStream_t s) {
  const int64_t blocks = h->rb_upd * h->n;
  const float ls = (float)h->lam_s;
  FWCHK(fw_timed(h, RPCA_FW_K_UPDATE, s, [&] {
    if (h->vec == 4) {
      if (h->mask)
        hipLaunchKernelGGL((k_fw_update<4, true>), dim3((unsigned)blocks), dim3(TH), 0, s, L, X, h->mask, h->mw, h->m,
                           h->rb_upd, (const double*)h->st, h->y, h->v, ls, h->G, h->part);
      else
        hipLaunchKernelGGL((k_fw_update<4, false>), dim3((unsigned)blocks), dim3(TH), 0, s, L, X, h->mask, h->mw,
                           h->m, h->rb_upd, (const double*)h->st, h->y, h->v, ls, h->G, h->part);
    } else {
      if (h->mask)
        hipLaunchKernelGGL((k_fw_update<1, true>), dim3((unsigned)blocks), dim3(TH), 0, s, L, X, h->mask, h->mw, h->m,
                           h->rb_upd, (const double*)h->st, h->y, h->v, ls, h->G, h->part);
      else
        hipLaunchKernelGGL((k_fw_update<1, false>), dim3((unsigned)blocks), dim3(TH), 0, s, L, X, h->mask, h->mw,
                           h->m, h->rb_upd, (const double*)h->st, h->y, h->v, ls, h->G, h->part);
    }
  }));
  hipLaunchKernelGGL(k_sum_parts<3>, dim3(1), dim3(FIN_TH), 0, s, (const double*)h->part, blocks, h->res + 4);
  FWCHK(hipGetLastError());
  return RPCA_OK;
}

// Orthonormalise the first b columns of the n x BLK row-major block (modified
// Gram-Schmidt, twice); a column that vanishes is replaced by hashed entries
// (salt) and orthogonalised again, or left zero.
void orth_block(std::vector<double>& Xh, int64_t n, int b, uint64_t salt) {
  for (int q = 0; q < b; ++q) {
    for (int attempt = 0; attempt < 2; ++attempt) {
      double before = 0.0;
      for (int64_t j = 0; j < n; ++j) before += Xh[(size_t)j * BLK + q] * Xh[(size_t)j * BLK + q];
      for (int pass = 0; pass < 2; ++pass)
        for (int p = 0; p < q; ++p) {
          double d = 0.0;
          for (int64_t j = 0; j < n; ++j) d += Xh[(size_t)j * BLK + p] * Xh[(size_t)j * BLK + q];
          for (int64_t j = 0; j < n; ++j) Xh[(size_t)j * BLK + q] -= d * Xh[(size_t)j * BLK + p];
        }
      double nn = 0.0;
      for (int64_t j = 0; j < n; ++j) nn += Xh[(size_t)j * BLK + q] * Xh[(size_t)j * BLK + q];
      if (nn > 1e-20 * before && nn > 0.0) {
        const double inv = 1.0 / sqrt(nn);
        for (int64_t j = 0; j < n; ++j) Xh[(size_t)j * BLK + q] *= inv;
        break;
      }
      if (attempt == 0) {
        for (int64_t j = 0; j < n; ++j) Xh[(size_t)j * BLK + q] = start_entry(salt + (uint64_t)(j * BLK + q));
      } else {
        for (int64_t j = 0; j < n; ++j) Xh[(size_t)j * BLK + q] = 0.0;
      }
    }
  }
  for (int64_t j = 0; j < n; ++j)
    for (int q = b; q < BLK; ++q) Xh[(size_t)j * BLK + q] = 0.0;
}

double* xd_at(rpca_fw* h, int i) { return h->Xd + (size_t)i * h->n * BLK; }
float* xb_at(rpca_fw* h, int i) { return h->Xb + (size_t)i * h->n * BLK; }
float* wf_at(rpca_fw* h, int i) { return h->Wf ? h->Wf + (size_t)i * h->n * 16 : nullptr; }

// The start block (host, FP64) into the current device copies.  The pinned
// staging is written once per handle, before its first solve.
int upload_block(rpca_fw* h, hipStream_t s) {
  const size_t nb = h->Xh.size();
  memcpy(h->zpin, h->Xh.data(), nb * 8);
  FWCHK(hipMemcpyAsync(xd_at(h, h->cur), h->zpin, nb * 8, hipMemcpyHostToDevice, s));
  for (size_t e = 0; e < nb; ++e) h->xpin[e] = (float)h->Xh[e];
  FWCHK(hipMemcpyAsync(xb_at(h, h->cur), h->xpin, nb * 4, hipMemcpyHostToDevice, s));
  if (h->Wf) {  // the same block padded to 16 columns for the fused pass
    float* w16 = h->xpin + nb;
    for (int64_t j = 0; j < h->n; ++j)
      for (int c = 0; c < 16; ++c) w16[(size_t)j * 16 + c] = c < BLK ? h->xpin[(size_t)j * BLK + c] : 0.f;
    FWCHK(hipMemcpyAsync(wf_at(h, h->cur), w16, (size_t)h->n * 16 * 4, hipMemcpyHostToDevice, s));
  }
  return RPCA_OK;
}

// Y = G Xb (left product and its chunk sum)
hipError_t fw_left(rpca_fw* h, const float* Xb, hipStream_t s) {
  const int64_t m = h->m, n = h->n;
  const int64_t lblocks = h->rb_upd * h->nchunks_left;
  hipError_t e = fw_timed(h, RPCA_FW_K_LEFT, s, [&] {
    if (h->vec == 4)
      hipLaunchKernelGGL(k_fw_left<4>, dim3((unsigned)lblocks), dim3(TH), 0, s, (const float*)h->G, Xb, m, n,
                         h->rb_upd, h->ypart);
    else
      hipLaunchKernelGGL(k_fw_left<1>, dim3((unsigned)lblocks), dim3(TH), 0, s, (const float*)h->G, Xb, m, n,
                         h->rb_upd, h->ypart);
  });
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fw_left_finish, dim3((unsigned)((m * BLK + TH - 1) / TH)), dim3(TH), 0, s,
                     (const float*)h->ypart, h->nchunks_left, m * BLK, h->Y);
  return hipGetLastError();
}

// Linear minimisation: top singular triplet of G by block power iteration with
// Rayleigh-Ritz, every step on the device (k_block_ritz); the host reads back the
// stop flag, theta_0 and the residual (24 bytes) per step.  With the fused
// pass (and kernel timing off) the next step is queued before the host reads
// the current one's flag, its kernels doing nothing once the flag is set, so
// the device does not wait on the host between steps.  On return y = G v
// (device), v (device, unit), *sigma = ||G v||, and the other block copy holds
// the rotated, orthonormalised block (the next call's start).
constexpr int LMO_STOPPED = 100;  // the solve ended before this minimisation was needed

int fw_lmo(rpca_fw* h, double ptol, double* sigma, int* steps, hipStream_t s, const double* stop_when) {
  const int64_t m = h->m, n = h->n;
  const int b = h->b;
  const int64_t ncb = (n + RIGHT_COLS - 1) / RIGHT_COLS;
  const int64_t rblocks = h->rc_right * ncb;
  const int cur0 = h->cur;
  const bool ahead = h->gpart != nullptr && !h->prof_on;
  // step p: its block is copy cur0 ^ (p & 1), its flag slot p & 1
  auto enqueue_step = [&](int p) -> int {
    const int cur = cur0 ^ (p & 1), nxt = cur ^ 1;
    const double* skip = (ahead && p > 0) ? h->res + 8 : nullptr;
    if (h->gpart) {
      // Z = G^T G Xb in one pass over G (Y is formed once, at the end)
      rpca::GramApplyArgs ga;
      memset(&ga, 0, sizeof(ga));
      ga.X = h->G;
      ga.m = m;
      ga.n = n;
      ga.W = wf_at(h, cur);
      ga.part = h->gpart;
      ga.row_groups = h->rg_ga;
      ga.xvec = h->vec == 4 ? 1 : 0;
      ga.skip = skip;
      hipError_t ge = hipSuccess;
      FWCHK(fw_timed(h, RPCA_FW_K_RIGHT, s, [&] { ge = rpca::launch_gram_apply_pass(ga, false, s); }));
      FWCHK(ge);
      FWCHK(rpca::launch_gram_apply_sum(ga, h->Z, BLK, 0, b, 1.0, s));
    } else {
      FWCHK(fw_left(h, xb_at(h, cur), s));
      FWCHK(fw_timed(h, RPCA_FW_K_RIGHT, s, [&] {
        if (h->vec == 4)
          hipLaunchKernelGGL(k_fw_right<4>, dim3((unsigned)rblocks), dim3(TH), 0, s, (const float*)h->G,
                             (const float*)h->Y, m, n, ncb, h->part);
        else
          hipLaunchKernelGGL(k_fw_right<1>, dim3((unsigned)rblocks), dim3(TH), 0, s, (const float*)h->G,
                             (const float*)h->Y, m, n, ncb, h->part);
      }));
      hipLaunchKernelGGL(k_fw_right_finish, dim3((unsigned)((n * BLK + TH - 1) / TH)), dim3(TH), 0, s,
                         (const double*)h->part, h->rc_right, n * BLK, h->Z);
      FWCHK(hipGetLastError());
    }
    rpca_ritz::RitzArgs ra;
    memset(&ra, 0, sizeof(ra));
    ra.X = xd_at(h, cur);
    ra.Z = h->Z;
    ra.n = n;
    ra.b = b;
    ra.salt = 0x51ull * (uint64_t)(p + 1);
    ra.Xn = xd_at(h, nxt);
    ra.Xbn = xb_at(h, nxt);
    ra.Wfn = wf_at(h, nxt);
    ra.res = h->res + 8;
    ra.skip = skip;
    ra.ptol = ptol;
    ra.last = p + 1 == POWER_MAX ? 1 : 0;
    ra.v32 = h->v;
    ra.cw = h->cw;
    hipLaunchKernelGGL(rpca_ritz::k_block_ritz<rpca_ritz::RITZ_FW>, dim3(1), dim3(rpca_ritz::RT), 0, s, ra);
    FWCHK(hipGetLastError());
    double* slot = h->res_host + 8 + 4 * (p & 1);
    FWCHK(hipMemcpyAsync(slot, h->res + 8, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    FWCHK(hipEventRecord(h->flag_ev[p & 1], s));
    return RPCA_OK;
  };
  int rc = enqueue_step(0);
  if (rc) return rc;
  for (int p = 0;; ++p) {
    if (ahead && p + 1 < POWER_MAX && (rc = enqueue_step(p + 1))) return rc;
    FWCHK(hipEventSynchronize(h->flag_ev[p & 1]));
    // the previous iteration's step state (copied ahead of this minimisation) says done
    if (stop_when && *stop_when != 0.0) return LMO_STOPPED;
    const double* slot = h->res_host + 8 + 4 * (p & 1);
    ++*steps;
    // the kernel sets the flag at the last allowed step; the host stops there too
    if (slot[0] != 0.0 || p + 1 >= POWER_MAX) {
      const int cur = cur0 ^ (p & 1);
      // y = G v = (G Xb) w_0 for this step's block
      if (h->gpart) FWCHK(fw_left(h, xb_at(h, cur), s));
      hipLaunchKernelGGL(k_fw_combine, dim3((unsigned)((m + TH - 1) / TH)), dim3(TH), 0, s, (const float*)h->Y,
                         (const float*)h->cw, m, h->y);
      FWCHK(hipGetLastError());
      *sigma = sqrt(slot[1]);
      h->cur = cur ^ 1;
      return RPCA_OK;
    }
    if (!ahead && (rc = enqueue_step(p + 1))) return rc;
  }
}

// u^T P_Omega(L) v and sum_Omega u_i^2 v_j^2 with u = y / sigma into res[2..3]
// (sigma from the minimisation on the device; nothing without a step).
int fw_bilinear(rpca_fw* h, const float* L, hipStream_t s) {
  const int64_t cblocks = h->rc_bil * h->n;
  FWCHK(fw_timed(h, RPCA_FW_K_BILINEAR, s, [&] {
    if (h->vec == 4) {
      if (h->mask)
        hipLaunchKernelGGL((k_fw_bilinear<4, true>), dim3((unsigned)cblocks), dim3(TH), 0, s, L, (const float*)h->y,
                           (const double*)h->res, h->lam_l, (const uint32_t*)h->mask, h->mw, h->m, h->rc_bil,
                           h->part);
      else
        hipLaunchKernelGGL((k_fw_bilinear<4, false>), dim3((unsigned)cblocks), dim3(TH), 0, s, L, (const float*)h->y,
                           (const double*)h->res, h->lam_l, (const uint32_t*)h->mask, h->mw, h->m, h->rc_bil,
                           h->part);
    } else {
      if (h->mask)
        hipLaunchKernelGGL((k_fw_bilinear<1, true>), dim3((unsigned)cblocks), dim3(TH), 0, s, L, (const float*)h->y,
                           (const double*)h->res, h->lam_l, (const uint32_t*)h->mask, h->mw, h->m, h->rc_bil,
                           h->part);
      else
        hipLaunchKernelGGL((k_fw_bilinear<1, false>), dim3((unsigned)cblocks), dim3(TH), 0, s, L, (const float*)h->y,
                           (const double*)h->res, h->lam_l, (const uint32_t*)h->mask, h->mw, h->m, h->rc_bil,
                           h->part);
    }
  }));
  hipLaunchKernelGGL(k_fw_bilinear_finish, dim3(1), dim3(FIN_TH), 0, s, (const double*)h->part, h->rc_bil, h->n,
                     (const float*)h->v, h->res);
  FWCHK(hipGetLastError());
  return RPCA_OK;
}

}  // namespace

extern "C" {

int rpca_fw_create(int64_t m, int64_t n, double lam_s, double lam_l, const uint8_t* mask, rpca_fw** out) {
  if (!out) return RPCA_EINVAL;
  *out = nullptr;
  if (m < 1 || n < 1 || m > ((int64_t)1 << 31) || n > ((int64_t)1 << 24)) return RPCA_EINVAL;
  if (!(lam_s > 0) || !(lam_l > 0) || !isfinite(lam_s) || !isfinite(lam_l)) return RPCA_EINVAL;
  rpca_fw* h = new (std::nothrow) rpca_fw();
  if (!h) return RPCA_ENOMEM;
  h->m = m;
  h->n = n;
  h->lam_s = lam_s;
  h->lam_l = lam_l;
  h->b = (int)std::min<int64_t>(BLK, n);
  h->nchunks_left = (n + LEFT_COLS - 1) / LEFT_COLS;
  // partials sized for the scalar layout (the most blocks)
  const int64_t rb1 = (m + TH - 1) / TH;
  const int64_t rcr1 = (m + (int64_t)TH * RIGHT_ITER - 1) / ((int64_t)TH * RIGHT_ITER);
  const int64_t rcb1 = (m + (int64_t)TH * COL_ITER - 1) / ((int64_t)TH * COL_ITER);
  const int64_t parts = std::max(std::max(rb1 * n * 3, rcr1 * n * BLK), rcb1 * n * 2);
  bool ok = true;
  try {
    h->Xh.assign((size_t)n * BLK, 0.0);
  } catch (...) {
    ok = false;
  }
  ok = ok && hipMalloc(&h->G, (size_t)(m * n) * 4) == hipSuccess &&
       hipMalloc(&h->ypart, (size_t)(h->nchunks_left * m * BLK) * 4) == hipSuccess &&
       hipMalloc(&h->Y, (size_t)(m * BLK) * 4) == hipSuccess && hipMalloc(&h->y, (size_t)m * 4) == hipSuccess &&
       hipMalloc(&h->Xd, (size_t)(2 * n * BLK) * 8) == hipSuccess &&
       hipMalloc(&h->Xb, (size_t)(2 * n * BLK) * 4) == hipSuccess && hipMalloc(&h->cw, BLK * 4) == hipSuccess &&
       hipMalloc(&h->v, (size_t)n * 4) == hipSuccess &&
       hipMalloc(&h->part, (size_t)parts * 8) == hipSuccess && hipMalloc(&h->Z, (size_t)(n * BLK) * 8) == hipSuccess &&
       hipMalloc(&h->res, 16 * 8) == hipSuccess && hipHostMalloc(&h->res_host, 16 * 8, hipHostMallocDefault) == hipSuccess &&
       hipMalloc(&h->st, 16 * 8) == hipSuccess && hipHostMalloc(&h->st_host, 16 * 8, hipHostMallocDefault) == hipSuccess &&
       hipHostMalloc(&h->zpin, (size_t)(n * BLK) * 8, hipHostMallocDefault) == hipSuccess &&
       hipHostMalloc(&h->xpin, (size_t)(n * (BLK + 16)) * 4, hipHostMallocDefault) == hipSuccess;
  if (ok && (hipMemset(h->y, 0, (size_t)m * 4) != hipSuccess || hipMemset(h->v, 0, (size_t)n * 4) != hipSuccess))
    ok = false;
  for (int e = 0; e < 2 && ok; ++e) ok = hipEventCreateWithFlags(&h->flag_ev[e], hipEventDisableTiming) == hipSuccess;
  if (ok && rpca::gram_apply_fits(n, 0)) {
    // the fused power step: one workgroup per compute unit, two strips a wave at least
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
    h->rg_ga = (int)std::max<int64_t>(1, std::min<int64_t>(cus, ((m + 15) / 16) / 8));
    ok = hipMalloc(&h->Wf, (size_t)(2 * n * 16) * 4) == hipSuccess &&
         hipMalloc(&h->gpart, (size_t)h->rg_ga * n * 16 * 4) == hipSuccess;
  }
  if (ok && mask) {
    h->mw = (int)((m + 31) / 32);
    std::vector<uint32_t> bits((size_t)h->mw * (size_t)n, 0u);
    for (int64_t j = 0; j < n; ++j) {
      const uint8_t* col = mask + j * m;
      uint32_t* w = bits.data() + j * h->mw;
      for (int64_t i = 0; i < m; ++i)
        if (col[i]) w[i >> 5] |= 1u << (i & 31);
    }
    ok = hipMalloc(&h->mask, bits.size() * 4) == hipSuccess &&
         hipMemcpy(h->mask, bits.data(), bits.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
  }
  if (!ok) {
    fw_free(h);
    return RPCA_ENOMEM;
  }
  *out = h;
  return RPCA_OK;
}

void rpca_fw_destroy(rpca_fw* h) {
  if (h) fw_free(h);
}

int rpca_fw_profile_enable(rpca_fw* h, int32_t on) {
  if (!h) return RPCA_EINVAL;
  h->prof_on = on != 0;
  return RPCA_OK;
}

int rpca_fw_profile_read(rpca_fw* h, rpca_fw_profile* out, int32_t reset) {
  if (!h || !out) return RPCA_EINVAL;
  fw_collect(h);
  for (int i = 0; i < 4; ++i) {
    out->launches[i] = h->launches[i];
    out->ms[i] = h->ms[i];
    if (reset) {
      h->launches[i] = 0;
      h->ms[i] = 0.0;
    }
  }
  return RPCA_OK;
}

int rpca_fw_solve(rpca_fw* h, const float* X, float* L, double* t_io, int32_t max_iter, double tol,
                  double power_tol, rpca_fw_info* info, void* stream) {
  if (!h || !X || !L || !t_io) return RPCA_EINVAL;
  if (max_iter < 0 || !(tol >= 0) || !isfinite(*t_io) || *t_io < 0 || !(power_tol >= 0)) return RPCA_EINVAL;
  const double ptol = power_tol > 0 ? power_tol : POWER_TOL;
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = (hipStream_t)stream;
  const double lam_l = h->lam_l;
  // 16-byte vector accesses when every column start is 16-byte aligned
  const bool al = ((uintptr_t)X % 16 == 0) && ((uintptr_t)L % 16 == 0);
  h->vec = (h->m % 4 == 0 && al) ? 4 : 1;
  h->rb_upd = (h->m + TH * h->vec - 1) / (TH * h->vec);
  h->rc_right = (h->m + (int64_t)TH * h->vec * RIGHT_ITER - 1) / ((int64_t)TH * h->vec * RIGHT_ITER);
  h->rc_bil = (h->m + (int64_t)TH * h->vec * COL_ITER - 1) / ((int64_t)TH * h->vec * COL_ITER);
  int rc;
  if (!h->x_valid) {
    for (int64_t j = 0; j < h->n; ++j)
      for (int q = 0; q < BLK; ++q) h->Xh[(size_t)j * BLK + q] = start_entry((uint64_t)(j * BLK + q));
    orth_block(h->Xh, h->n, h->b, 0x9000ull);
    if ((rc = upload_block(h, s))) return rc;
    h->x_valid = true;
  }
  // G, phi, <G, L>, sum_Omega L^2 at the start (a = 1, b = 0)
  double t = *t_io;
  hipLaunchKernelGGL(k_fw_state_init, dim3(1), dim3(64), 0, s, h->st, t);
  FWCHK(hipGetLastError());
  if ((rc = fw_update(h, X, L, s))) return rc;
  rpca_fw_info fin;
  memset(&fin, 0, sizeof(fin));
  // Per iteration: the minimisation (the host waits on its steps), the bilinear
  // pass, the step (k_fw_step: gap, stop test, eta, the update's a and b) and the
  // update pass (nothing once done), with no other wait: the step state's copy
  // is read after the next minimisation's first wait, which ends that
  // minimisation when the state says done.
  for (int it = 0;; ++it) {
    double sigma = 0.0;
    rc = fw_lmo(h, ptol, &sigma, &fin.power_iters, s, it > 0 ? h->st_host + 3 : nullptr);
    if (rc != RPCA_OK && rc != LMO_STOPPED) return rc;
    if (it > 0) {
      const double* st = h->st_host;  // iteration it - 1
      if (st[9] != 0.0) {
        FWCHK(hipStreamSynchronize(s));
        *t_io = st[10];
        // the power block came from a nonfinite G: the next call starts cold
        h->x_valid = false;
        return RPCA_ENONFINITE;
      }
      fin.F = st[4];
      fin.phi = st[12];
      fin.gap = st[5];
      fin.sigma = st[6];
      fin.last_step = st[8] != 0.0;
      fin.iters = it - 1;
      fin.eta = st[11];
      t = st[0];
      if (st[3] != 0.0) break;
    }
    if (rc == LMO_STOPPED) break;
    if ((rc = fw_bilinear(h, L, s))) return rc;
    hipLaunchKernelGGL(k_fw_step, dim3(1), dim3(64), 0, s, (const double*)h->res, h->st, lam_l, tol,
                       it == max_iter ? 1 : 0);
    FWCHK(hipGetLastError());
    FWCHK(hipMemcpyAsync(h->st_host, h->st, 16 * sizeof(double), hipMemcpyDeviceToHost, s));
    if ((rc = fw_update(h, X, L, s))) return rc;  // L <- (1 - eta) L + eta V, V = -B u v^T
  }
  *t_io = t;
  // the warm-start block's upload from the pinned staging may still be in flight
  FWCHK(hipStreamSynchronize(s));
  fin.status = (fin.gap <= tol * fin.F) ? RPCA_OK : RPCA_ENOTCONV;
  fin.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = fin;
  return fin.status;
}

}  // extern "C"
