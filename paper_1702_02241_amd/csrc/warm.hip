// Learned warm start: window statistics, a 2-layer MLP (forward, backward,
// Adam) on FP32 MFMA, and the row pooling / upsampling that maps factors
// between full and low resolution.  The declarations and the definitions of
// every quantity are in rpca_warm.h.
//
// GEMM.  C = op(A) op(B) with op = identity or transpose, row-major storage,
// 64 x 64 output tiles per 256-thread workgroup (four waves of 32 x 32, each
// four 16x16 v_mfma_f32_16x16x4f32 accumulators), K staged through LDS in
// slices of 16.  Loads are coalesced along whichever index is contiguous in
// memory.  When the output has too few tiles to fill the chip (the 512-wide
// hidden layer against a K of 10^4 .. 10^5) K is split across workgroups
// and the partials are summed in a fixed order by a second kernel, so every
// result is bitwise reproducible.  The epilogue adds a bias, applies ReLU or
// gates by a previous activation (the ReLU derivative in the backward pass).

#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <vector>

#include "rpca.h"
#include "rpca_warm.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int GT = 256;
constexpr int BM = 64, BN = 64, BK = 16;
constexpr int LPAD = 4;
constexpr int KMAX_LOSS = 32;

__device__ __forceinline__ f4 mfma_f32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

struct GemmArgs {
  const float* A;
  const float* B;
  float* C;
  int64_t M, N, K;
  int64_t lda, ldb, ldc;
  int64_t kchunk;       // K range per split (multiple of BK)
  const float* bias;    // N values or null
  const float* gate;    // M x N (leading dimension ldg) or null: C = acc * (gate > 0)
  int64_t ldg;
  int32_t relu;
  float* part;          // [splits][M][N] partial products, or null (direct epilogue)
};

__device__ __forceinline__ float epilogue(const GemmArgs& a, int64_t i, int64_t j, float v) {
  if (a.bias) v += a.bias[j];
  if (a.relu) v = fmaxf(v, 0.f);
  if (a.gate && !(a.gate[i * a.ldg + j] > 0.f)) v = 0.f;
  return v;
}

template <bool TA, bool TB>
__global__ __launch_bounds__(GT) void k_gemm(GemmArgs a) {
  __shared__ float As[BK][BM + LPAD];  // As[kk][mm] = op(A)[m0 + mm][k0 + kk]
  __shared__ float Bs[BK][BN + LPAD];  // Bs[kk][nn] = op(B)[k0 + kk][n0 + nn]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
  const int64_t kbeg = (int64_t)blockIdx.z * a.kchunk;
  int64_t kend = kbeg + a.kchunk;
  if (kend > a.K) kend = a.K;
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
    for (int r = 0; r < (BM * BK) / GT; ++r) {
      const int idx = tid + GT * r;
      const int mm = TA ? (idx & (BM - 1)) : (idx >> 4);
      const int kk = TA ? (idx >> 6) : (idx & (BK - 1));
      const int64_t gm = m0 + mm, gk = k0 + kk;
      float v = 0.f;
      if (gm < a.M && gk < kend) v = TA ? a.A[gk * a.lda + gm] : a.A[gm * a.lda + gk];
      As[kk][mm] = v;
    }
#pragma unroll
    for (int r = 0; r < (BN * BK) / GT; ++r) {
      const int idx = tid + GT * r;
      const int nn = TB ? (idx >> 4) : (idx & (BN - 1));
      const int kk = TB ? (idx & (BK - 1)) : (idx >> 6);
      const int64_t gn = n0 + nn, gk = k0 + kk;
      float v = 0.f;
      if (gn < a.N && gk < kend) v = TB ? a.B[gn * a.ldb + gk] : a.B[gk * a.ldb + gn];
      Bs[kk][nn] = v;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      float av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) av[i] = As[ks + lk][wm * 32 + i * 16 + li];
#pragma unroll
      for (int j = 0; j < 2; ++j) bv[j] = Bs[ks + lk][wn * 32 + j * 16 + li];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma_f32(av[i], bv[j], acc[i][j]);
    }
    __syncthreads();
  }
  // lane holds rows 4*lk + r, column li of each 16x16 block
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gm = m0 + wm * 32 + i * 16 + 4 * lk + r;
        const int64_t gn = n0 + wn * 32 + j * 16 + li;
        if (gm < a.M && gn < a.N) {
          const float v = acc[i][j][r];
          if (a.part)
            a.part[(int64_t)blockIdx.z * a.M * a.N + gm * a.N + gn] = v;
          else
            a.C[gm * a.ldc + gn] = epilogue(a, gm, gn, v);
        }
      }
}

__global__ __launch_bounds__(GT) void k_splitk_reduce(GemmArgs a, int splits) {
  const int64_t mn = a.M * a.N;
  for (int64_t o = (int64_t)blockIdx.x * GT + threadIdx.x; o < mn; o += (int64_t)gridDim.x * GT) {
    float s = 0.f;
    for (int z = 0; z < splits; ++z) s += a.part[(int64_t)z * mn + o];
    const int64_t i = o / a.N, j = o % a.N;
    a.C[i * a.ldc + j] = epilogue(a, i, j, s);
  }
}

// out[j] = sum over rows of A (rows x cols, row-major), fixed order
__global__ __launch_bounds__(GT) void k_colsum(const float* A, int64_t rows, int64_t cols, float* out) {
  const int64_t j = (int64_t)blockIdx.x * GT + threadIdx.x;
  if (j >= cols) return;
  float s = 0.f;
  for (int64_t r = 0; r < rows; ++r) s += A[r * cols + j];
  out[j] = s;
}

// ---------------------------------------------------------------------------
// Loss on the factored target.  For batch element b with prediction (Uh, Vh)
// and target factors (TU, TV):
//   Guu = Uh^T Uh, Mtu = TU^T Uh, Gtu = TU^T TU  (k x k, over the mu rows)
//   Gvv = Vh^T Vh, Mtv = TV^T Vh, Gtv = TV^T TV  (k x k, over the nv rows)
//   ||Uh Vh^T - TU TV^T||^2 = <Guu, Gvv> - 2 <Mtu, Mtv> + <Gtu, Gtv>
//   d/dUh = 2 (Uh Gvv - TU Mtv),   d/dVh = 2 (Vh Guu - TV Mtu).
// k_loss_grams: one block per batch element, rows staged through LDS; the
// six matrices go to grams[b][6][k][k] (FP64).
__global__ __launch_bounds__(GT) void k_loss_grams(const float* y, const float* TU, const float* TV,
                                                   int mu, int nv, int k, int64_t d_out,
                                                   double* grams) {
  constexpr int ROWS = 64;
  __shared__ float sP[ROWS * KMAX_LOSS];
  __shared__ float sT[ROWS * KMAX_LOSS];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int kk2 = k * k;
  const float* yb = y + (int64_t)b * d_out;
  double* gb = grams + (int64_t)b * 6 * kk2;
  for (int side = 0; side < 2; ++side) {
    const int rows = side == 0 ? mu : nv;
    const float* P = side == 0 ? yb : yb + (int64_t)mu * k;
    const float* T = side == 0 ? TU + (int64_t)b * mu * k : TV + (int64_t)b * nv * k;
    double aPP[4] = {0, 0, 0, 0}, aTP[4] = {0, 0, 0, 0}, aTT[4] = {0, 0, 0, 0};
    for (int r0 = 0; r0 < rows; r0 += ROWS) {
      const int nr = rows - r0 < ROWS ? rows - r0 : ROWS;
      __syncthreads();
      for (int idx = tid; idx < nr * k; idx += GT) {
        sP[idx] = P[(int64_t)r0 * k + idx];
        sT[idx] = T[(int64_t)r0 * k + idx];
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int e = tid + GT * s;
        if (e < kk2) {
          const int p = e / k, q = e % k;
          double pp = 0, tp = 0, tt = 0;
          for (int i = 0; i < nr; ++i) {
            const double up = sP[i * k + p], uq = sP[i * k + q], tpv = sT[i * k + p], tq = sT[i * k + q];
            pp += up * uq;
            tp += tpv * uq;
            tt += tpv * tq;
          }
          aPP[s] += pp;
          aTP[s] += tp;
          aTT[s] += tt;
        }
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int e = tid + GT * s;
      if (e < kk2) {
        gb[(3 * side + 0) * kk2 + e] = aPP[s];
        gb[(3 * side + 1) * kk2 + e] = aTP[s];
        gb[(3 * side + 2) * kk2 + e] = aTT[s];
      }
    }
  }
}

// loss = (1/B) sum_b (<Guu,Gvv> - 2<Mtu,Mtv> + <Gtu,Gtv>)   (one block)
__global__ __launch_bounds__(GT) void k_loss_value(const double* grams, int batch, int k, double* loss) {
  __shared__ double sh[GT / 64];
  const int kk2 = k * k;
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < (int64_t)batch * kk2; e += GT) {
    const int b = (int)(e / kk2), o = (int)(e % kk2);
    const double* g = grams + (int64_t)b * 6 * kk2;
    acc += g[0 * kk2 + o] * g[3 * kk2 + o] - 2.0 * g[1 * kk2 + o] * g[4 * kk2 + o] +
           g[2 * kk2 + o] * g[5 * kk2 + o];
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < GT / 64; ++w) s += sh[w];
    *loss = s / batch;
  }
}

// dy[b][row*k + c]: rows < mu from the U side, the rest from the V side
__global__ __launch_bounds__(GT) void k_loss_dy(const float* y, const float* TU, const float* TV,
                                                const double* grams, int batch, int mu, int nv, int k,
                                                int64_t d_out, float* dy) {
  const int64_t total = (int64_t)batch * d_out;
  const int kk2 = k * k;
  const double sc = 2.0 / batch;
  for (int64_t e = (int64_t)blockIdx.x * GT + threadIdx.x; e < total; e += (int64_t)gridDim.x * GT) {
    const int b = (int)(e / d_out);
    const int64_t o = e % d_out;
    const bool uside = o < (int64_t)mu * k;
    const int64_t oo = uside ? o : o - (int64_t)mu * k;
    const int row = (int)(oo / k), c = (int)(oo % k);
    const double* g = grams + (int64_t)b * 6 * kk2;
    const double* Gpp = g + (uside ? 3 : 0) * kk2;  // U side uses Gvv, V side Guu
    const double* Mt = g + (uside ? 4 : 1) * kk2;   // U side uses Mtv, V side Mtu
    const float* P = y + (int64_t)b * d_out + (uside ? 0 : (int64_t)mu * k) + (int64_t)row * k;
    const float* T = (uside ? TU + (int64_t)b * mu * k : TV + (int64_t)b * nv * k) + (int64_t)row * k;
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += (double)P[j] * Gpp[j * k + c] - (double)T[j] * Mt[j * k + c];
    dy[e] = (float)(sc * s);
  }
}

__global__ __launch_bounds__(GT) void k_adam(float* p, const float* g, float* m1, float* m2, int64_t n,
                                             float lr, float b1, float b2, float eps, float bc1,
                                             float bc2) {
  for (int64_t i = (int64_t)blockIdx.x * GT + threadIdx.x; i < n; i += (int64_t)gridDim.x * GT) {
    const float gi = g[i];
    const float a = fmaf(b1, m1[i], (1.f - b1) * gi);
    const float v = fmaf(b2, m2[i], (1.f - b2) * gi * gi);
    m1[i] = a;
    m2[i] = v;
    const float mh = a / bc1, vh = v / bc2;
    p[i] -= lr * mh / (sqrtf(vh) + eps);
  }
}

// ---------------------------------------------------------------------------
// Window statistics.  Thread per pooled block: its pooled value per frame,
// accumulated over the frames in FP64 for the mean and the (population)
// standard deviation.  The per-frame means: one block per frame.
__global__ __launch_bounds__(GT) void k_feat_blocks(const float* X, int64_t W, int64_t H, int frames,
                                                    int f, const float* shift, const float* scale,
                                                    float* feat) {
  const int64_t wl = W / f, hl = H / f, mu = wl * hl, m = W * H;
  const int64_t p = (int64_t)blockIdx.x * GT + threadIdx.x;
  if (p >= mu) return;
  const int64_t by = p / wl, bx = p % wl;
  const double inv = 1.0 / ((double)f * f);
  double s1 = 0.0, s2 = 0.0;
  for (int t = 0; t < frames; ++t) {
    const float* col = X + (int64_t)t * m + (by * f) * W + bx * f;
    double v = 0.0;
    for (int dy = 0; dy < f; ++dy)
      for (int dx = 0; dx < f; ++dx) v += (double)col[dy * W + dx];
    v *= inv;
    s1 += v;
    s2 += v * v;
  }
  const double mean = s1 / frames;
  double var = s2 / frames - mean * mean;
  if (var < 0.0) var = 0.0;
  float a = (float)mean, b = (float)sqrt(var);
  if (shift) {
    a = (a - shift[p]) * scale[p];
    b = (b - shift[mu + p]) * scale[mu + p];
  }
  feat[p] = a;
  feat[mu + p] = b;
}

__global__ __launch_bounds__(GT) void k_feat_frames(const float* X, int64_t m, int64_t mu2,
                                                    const float* shift, const float* scale,
                                                    float* feat) {
  __shared__ double sh[GT / 64];
  const int t = blockIdx.x;
  const float* col = X + (int64_t)t * m;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += GT) s += (double)col[i];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < GT / 64; ++w) r += sh[w];
    float v = (float)(r / m);
    if (shift) v = (v - shift[mu2 + t]) * scale[mu2 + t];
    feat[mu2 + t] = v;
  }
}

__global__ __launch_bounds__(GT) void k_pool_rows(const float* A, int64_t W, int64_t H, int f, int c,
                                                  float* out) {
  const int64_t wl = W / f, mu = wl * (H / f);
  const int64_t e = (int64_t)blockIdx.x * GT + threadIdx.x;
  if (e >= mu * c) return;
  const int64_t p = e / c;
  const int cc = (int)(e % c);
  const int64_t by = p / wl, bx = p % wl;
  double s = 0.0;
  for (int dy = 0; dy < f; ++dy)
    for (int dx = 0; dx < f; ++dx) s += (double)A[((by * f + dy) * W + bx * f + dx) * c + cc];
  out[e] = (float)(s / ((double)f * f));
}

__global__ __launch_bounds__(GT) void k_upsample_rows(const float* A, int64_t W, int64_t H, int f, int c,
                                                      float* out) {
  const int64_t wl = W / f;
  const int64_t e = (int64_t)blockIdx.x * GT + threadIdx.x;
  if (e >= W * H * c) return;
  const int64_t i = e / c;
  const int cc = (int)(e % c);
  const int64_t y = i / W, x = i % W;
  out[e] = A[((y / f) * wl + x / f) * c + cc];
}

inline int grid_for(int64_t n, int cap = 4096) {
  int64_t g = (n + GT - 1) / GT;
  if (g < 1) g = 1;
  return (int)(g < cap ? g : cap);
}

uint64_t mix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// Standard normal deviate number idx of stream `seed` (SplitMix64 + Box-Muller).
double gauss(uint64_t seed, uint64_t idx) {
  const uint64_t a = mix64(seed ^ mix64(2 * idx)), b = mix64(seed ^ mix64(2 * idx + 1));
  const double u1 = ((a >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  const double u2 = ((b >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

}  // namespace

struct rpca_mlp {
  int d_in, d_h, mu, nv, k, max_batch;
  int64_t d_out;
  float* param[4];
  float* grad[4];
  float* mom1[4];
  float* mom2[4];
  int64_t count[4];
  float* h;       // max_batch x d_h: relu(x W1 + b1)
  float* y;       // max_batch x d_out
  float* dy;      // max_batch x d_out
  float* dz;      // max_batch x d_h
  float* part;    // split-K partials
  int64_t part_cap;
  double* grams;  // max_batch x 6 x k x k
  int step;
};

namespace {

// Launch C = op(A) op(B) with the epilogue in `e` (A, B, C, sizes filled by the caller).
hipError_t gemm(rpca_mlp* net, GemmArgs g, bool ta, bool tb, hipStream_t s) {
  const int64_t tm = (g.M + BM - 1) / BM, tn = (g.N + BN - 1) / BN;
  const int64_t tiles = tm * tn;
  const int64_t kslices = (g.K + BK - 1) / BK;
  int64_t splits = 1;
  if (tiles < 512 && kslices >= 8) {
    splits = (512 + tiles - 1) / tiles;
    if (splits > kslices / 4) splits = kslices / 4;
    const int64_t cap = net->part_cap / (g.M * g.N);
    if (splits > cap) splits = cap;
    if (splits < 1) splits = 1;
  }
  const int64_t per = (kslices + splits - 1) / splits;
  g.kchunk = per * BK;
  splits = (g.K + g.kchunk - 1) / g.kchunk;
  if (splits < 1) splits = 1;
  g.part = splits > 1 ? net->part : nullptr;
  if (tm > 65535 || splits > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)tn, (unsigned)tm, (unsigned)splits);
  if (!ta && !tb) hipLaunchKernelGGL((k_gemm<false, false>), grid, dim3(GT), 0, s, g);
  else if (ta && !tb) hipLaunchKernelGGL((k_gemm<true, false>), grid, dim3(GT), 0, s, g);
  else if (!ta && tb) hipLaunchKernelGGL((k_gemm<false, true>), grid, dim3(GT), 0, s, g);
  else hipLaunchKernelGGL((k_gemm<true, true>), grid, dim3(GT), 0, s, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || splits == 1) return e;
  hipLaunchKernelGGL(k_splitk_reduce, dim3(grid_for(g.M * g.N)), dim3(GT), 0, s, g, (int)splits);
  return hipGetLastError();
}

GemmArgs gemm_args(const float* A, int64_t lda, const float* B, int64_t ldb, float* C, int64_t ldc,
                   int64_t M, int64_t N, int64_t K) {
  GemmArgs g;
  memset(&g, 0, sizeof(g));
  g.A = A;
  g.B = B;
  g.C = C;
  g.M = M;
  g.N = N;
  g.K = K;
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  return g;
}

hipError_t forward_into(rpca_mlp* n, const float* x, int batch, float* y, hipStream_t s) {
  GemmArgs g1 = gemm_args(x, n->d_in, n->param[0], n->d_h, n->h, n->d_h, batch, n->d_h, n->d_in);
  g1.bias = n->param[1];
  g1.relu = 1;
  hipError_t e = gemm(n, g1, false, false, s);
  if (e != hipSuccess) return e;
  GemmArgs g2 = gemm_args(n->h, n->d_h, n->param[2], n->d_out, y, n->d_out, batch, n->d_out, n->d_h);
  g2.bias = n->param[3];
  return gemm(n, g2, false, false, s);
}

void free_net(rpca_mlp* n) {
  for (int t = 0; t < 4; ++t) {
    if (n->param[t]) (void)hipFree(n->param[t]);
    if (n->grad[t]) (void)hipFree(n->grad[t]);
    if (n->mom1[t]) (void)hipFree(n->mom1[t]);
    if (n->mom2[t]) (void)hipFree(n->mom2[t]);
  }
  if (n->h) (void)hipFree(n->h);
  if (n->y) (void)hipFree(n->y);
  if (n->dy) (void)hipFree(n->dy);
  if (n->dz) (void)hipFree(n->dz);
  if (n->part) (void)hipFree(n->part);
  if (n->grams) (void)hipFree(n->grams);
  delete n;
}

}  // namespace

extern "C" {

int rpca_mlp_create(int32_t d_in, int32_t d_h, int32_t mu, int32_t nv, int32_t k, int32_t max_batch,
                    uint64_t seed, rpca_mlp** out) {
  if (!out || d_in <= 0 || d_h <= 0 || mu <= 0 || nv <= 0 || k <= 0 || k > KMAX_LOSS ||
      max_batch < 1 || max_batch > 4096)
    return RPCA_EINVAL;
  *out = nullptr;
  rpca_mlp* n = new rpca_mlp;
  memset(n, 0, sizeof(*n));
  n->d_in = d_in;
  n->d_h = d_h;
  n->mu = mu;
  n->nv = nv;
  n->k = k;
  n->max_batch = max_batch;
  n->d_out = (int64_t)(mu + nv) * k;
  n->count[0] = (int64_t)d_in * d_h;
  n->count[1] = d_h;
  n->count[2] = (int64_t)d_h * n->d_out;
  n->count[3] = n->d_out;
  n->part_cap = (int64_t)64 * max_batch * (d_h > 512 ? d_h : 512);
  bool ok = true;
  for (int t = 0; t < 4 && ok; ++t) {
    const size_t bytes = (size_t)n->count[t] * 4;
    ok = hipMalloc(&n->param[t], bytes) == hipSuccess && hipMalloc(&n->grad[t], bytes) == hipSuccess &&
         hipMalloc(&n->mom1[t], bytes) == hipSuccess && hipMalloc(&n->mom2[t], bytes) == hipSuccess &&
         hipMemset(n->mom1[t], 0, bytes) == hipSuccess && hipMemset(n->mom2[t], 0, bytes) == hipSuccess &&
         hipMemset(n->grad[t], 0, bytes) == hipSuccess;
  }
  ok = ok && hipMalloc(&n->h, (size_t)max_batch * d_h * 4) == hipSuccess &&
       hipMalloc(&n->dz, (size_t)max_batch * d_h * 4) == hipSuccess &&
       hipMalloc(&n->y, (size_t)max_batch * n->d_out * 4) == hipSuccess &&
       hipMalloc(&n->dy, (size_t)max_batch * n->d_out * 4) == hipSuccess &&
       hipMalloc(&n->part, (size_t)n->part_cap * 4) == hipSuccess &&
       hipMalloc(&n->grams, (size_t)max_batch * 6 * k * k * 8) == hipSuccess;
  if (!ok) {
    free_net(n);
    return RPCA_ENOMEM;
  }
  // He initialisation of the weights, zero biases
  const int64_t fan[2] = {d_in, d_h};
  for (int l = 0; l < 2; ++l) {
    const int t = 2 * l;
    std::vector<float> w((size_t)n->count[t]);
    const double sd = sqrt(2.0 / (double)fan[l]);
    const uint64_t s = mix64(seed + 0x51ED2701ull * (l + 1));
    for (int64_t i = 0; i < n->count[t]; ++i) w[i] = (float)(sd * gauss(s, (uint64_t)i));
    std::vector<float> z((size_t)n->count[t + 1], 0.f);
    if (hipMemcpy(n->param[t], w.data(), w.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(n->param[t + 1], z.data(), z.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
      free_net(n);
      return RPCA_EHIP;
    }
  }
  *out = n;
  return RPCA_OK;
}

int rpca_mlp_param(rpca_mlp* n, int32_t which, float** ptr, int64_t* count) {
  if (!n || which < 0 || which > 3 || !ptr) return RPCA_EINVAL;
  *ptr = n->param[which];
  if (count) *count = n->count[which];
  return RPCA_OK;
}

int rpca_mlp_grad(rpca_mlp* n, int32_t which, float** ptr, int64_t* count) {
  if (!n || which < 0 || which > 3 || !ptr) return RPCA_EINVAL;
  *ptr = n->grad[which];
  if (count) *count = n->count[which];
  return RPCA_OK;
}

int rpca_mlp_forward(rpca_mlp* n, const float* x, int32_t batch, float* y, void* stream) {
  if (!n || !x || !y || batch < 1 || batch > n->max_batch) return RPCA_EINVAL;
  return forward_into(n, x, batch, y, (hipStream_t)stream) == hipSuccess ? RPCA_OK : RPCA_EHIP;
}

int rpca_mlp_loss_grad(rpca_mlp* n, const float* x, const float* TU, const float* TV, int32_t batch,
                       double* loss, void* stream) {
  if (!n || !x || !TU || !TV || !loss || batch < 1 || batch > n->max_batch) return RPCA_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (forward_into(n, x, batch, n->y, s) != hipSuccess) return RPCA_EHIP;
  hipLaunchKernelGGL(k_loss_grams, dim3(batch), dim3(GT), 0, s, n->y, TU, TV, n->mu, n->nv, n->k, n->d_out,
                     n->grams);
  hipLaunchKernelGGL(k_loss_value, dim3(1), dim3(GT), 0, s, n->grams, batch, n->k, loss);
  hipLaunchKernelGGL(k_loss_dy, dim3(grid_for((int64_t)batch * n->d_out)), dim3(GT), 0, s, n->y, TU, TV,
                     n->grams, batch, n->mu, n->nv, n->k, n->d_out, n->dy);
  if (hipGetLastError() != hipSuccess) return RPCA_EHIP;
  // dW2 = h^T dy, db2 = colsum(dy)
  GemmArgs a = gemm_args(n->h, n->d_h, n->dy, n->d_out, n->grad[2], n->d_out, n->d_h, n->d_out, batch);
  if (gemm(n, a, true, false, s) != hipSuccess) return RPCA_EHIP;
  hipLaunchKernelGGL(k_colsum, dim3(grid_for(n->d_out, 1 << 30)), dim3(GT), 0, s, n->dy, (int64_t)batch,
                     n->d_out, n->grad[3]);
  // dz = (dy W2^T) .* (h > 0)
  GemmArgs b = gemm_args(n->dy, n->d_out, n->param[2], n->d_out, n->dz, n->d_h, batch, n->d_h, n->d_out);
  b.gate = n->h;
  b.ldg = n->d_h;
  if (gemm(n, b, false, true, s) != hipSuccess) return RPCA_EHIP;
  // dW1 = x^T dz, db1 = colsum(dz)
  GemmArgs c = gemm_args(x, n->d_in, n->dz, n->d_h, n->grad[0], n->d_h, n->d_in, n->d_h, batch);
  if (gemm(n, c, true, false, s) != hipSuccess) return RPCA_EHIP;
  hipLaunchKernelGGL(k_colsum, dim3(grid_for(n->d_h, 1 << 30)), dim3(GT), 0, s, n->dz, (int64_t)batch,
                     (int64_t)n->d_h, n->grad[1]);
  return hipGetLastError() == hipSuccess ? RPCA_OK : RPCA_EHIP;
}

int rpca_mlp_adam_step(rpca_mlp* n, float lr, float beta1, float beta2, float eps, void* stream) {
  if (!n || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return RPCA_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  n->step += 1;
  const float bc1 = (float)(1.0 - pow((double)beta1, n->step));
  const float bc2 = (float)(1.0 - pow((double)beta2, n->step));
  for (int t = 0; t < 4; ++t)
    hipLaunchKernelGGL(k_adam, dim3(grid_for(n->count[t])), dim3(GT), 0, s, n->param[t], n->grad[t],
                       n->mom1[t], n->mom2[t], n->count[t], lr, beta1, beta2, eps, bc1, bc2);
  return hipGetLastError() == hipSuccess ? RPCA_OK : RPCA_EHIP;
}

int rpca_mlp_train_step(rpca_mlp* n, const float* x, const float* TU, const float* TV, int32_t batch,
                        float lr, double* loss, void* stream) {
  const int rc = rpca_mlp_loss_grad(n, x, TU, TV, batch, loss, stream);
  if (rc != RPCA_OK) return rc;
  return rpca_mlp_adam_step(n, lr, 0.9f, 0.999f, 1e-8f, stream);
}

void rpca_mlp_destroy(rpca_mlp* n) {
  if (n) free_net(n);
}

int rpca_window_features(const float* X, int64_t W, int64_t H, int32_t frames, int32_t f,
                         const float* shift, const float* scale, float* feat, void* stream) {
  if (!X || !feat || W <= 0 || H <= 0 || frames <= 0 || f <= 0 || W % f || H % f ||
      (!shift) != (!scale))
    return RPCA_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int64_t mu = (W / f) * (H / f);
  hipLaunchKernelGGL(k_feat_blocks, dim3(grid_for(mu, 1 << 30)), dim3(GT), 0, s, X, W, H, frames, f, shift,
                     scale, feat);
  hipLaunchKernelGGL(k_feat_frames, dim3(frames), dim3(GT), 0, s, X, W * H, 2 * mu, shift, scale, feat);
  return hipGetLastError() == hipSuccess ? RPCA_OK : RPCA_EHIP;
}

int rpca_pool_rows(const float* A, int64_t W, int64_t H, int32_t f, int32_t c, float* out, void* stream) {
  if (!A || !out || W <= 0 || H <= 0 || f <= 0 || c <= 0 || W % f || H % f) return RPCA_EINVAL;
  const int64_t n = (W / f) * (H / f) * c;
  hipLaunchKernelGGL(k_pool_rows, dim3(grid_for(n, 1 << 30)), dim3(GT), 0, (hipStream_t)stream, A, W, H, f,
                     c, out);
  return hipGetLastError() == hipSuccess ? RPCA_OK : RPCA_EHIP;
}

int rpca_upsample_rows(const float* A, int64_t W, int64_t H, int32_t f, int32_t c, float* out, void* stream) {
  if (!A || !out || W <= 0 || H <= 0 || f <= 0 || c <= 0 || W % f || H % f) return RPCA_EINVAL;
  const int64_t n = W * H * c;
  hipLaunchKernelGGL(k_upsample_rows, dim3(grid_for(n, 1 << 30)), dim3(GT), 0, (hipStream_t)stream, A, W, H,
                     f, c, out);
  return hipGetLastError() == hipSuccess ? RPCA_OK : RPCA_EHIP;
}

}  // extern "C"
