// Preconditioned variables for the L-BFGS solve.
//
// In the factored objective f(U, V) = phi(U V^T) + lam_L/2 (||U||^2 + ||V||^2)
// (eq. smoothNC) the curvature along U scales with V^T V and along V with
// U^T U: the leading factor directions see a curvature of sigma_1 + lam_L,
// a dying component of L only about lam_L.  With sigma_1 / lam_L in the
// hundreds, L-BFGS from the scalar initial matrix needs many iterations
// for the small components, which are exactly the ones the certificate of
// Sec. 3.4 weighs most (through 1/sigma_r).  The solver therefore works in
//   A = U P_U^{-1},  B = V P_V^{-1},
//   P_U = (V^T V + lam_L I)^{-1/2},  P_V = (U^T U + lam_L I)^{-1/2},
// fixed over a cycle of iterations and refreshed from the current (U, V)
// between cycles (the scaling of "scaled gradient descent" for low-rank
// factorisations, Tong, Ma & Chi 2021, used here as a change of variables).
// The objective and its minimisers are unchanged; in the new variables
//   U V^T = A W B^T,  W = P_U P_V,
//   grad_A = G (B W^T) + lam_L A M_U,  grad_B = G^T A W + lam_L B M_V,
//   M_U = P_U^2,  M_V = P_V^2,
// which the sweep and the finishing reduction evaluate from pc = [W | M_U |
// M_V | P_U | P_V | P_U^{-1} | P_V^{-1}] (k x k each, FP32, device).
#include <math.h>
#include <string.h>

#include <vector>

#include "ctx.h"
#include "smalllinalg.h"

namespace {

constexpr int TH = 256;

// Per-block partial Gram matrices of the rows of an FP32 row-major matrix
// (rows x k, k <= 32), FP64: part[blockIdx][k*k].
__global__ __launch_bounds__(TH) void k_gram_rows(const float* A, int64_t rows, int k, double* part) {
  constexpr int TR = 64;
  __shared__ float tile[TR * 32];
  const int kk2 = k * k;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t r0 = (int64_t)blockIdx.x * TR; r0 < rows; r0 += (int64_t)gridDim.x * TR) {
    const int nr = (int)((rows - r0) < TR ? (rows - r0) : TR);
    __syncthreads();
    for (int idx = threadIdx.x; idx < nr * k; idx += TH) tile[idx] = A[r0 * k + idx];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = threadIdx.x + e * TH;
      if (idx < kk2) {
        const int p = idx / k, q = idx % k;
        double sacc = 0.0;
        for (int rr = 0; rr < nr; ++rr) sacc = fma((double)tile[rr * k + p], (double)tile[rr * k + q], sacc);
        acc[e] += sacc;
      }
    }
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int idx = threadIdx.x + e * TH;
    if (idx < kk2) part[(int64_t)blockIdx.x * kk2 + idx] = acc[e];
  }
}

// In place, row by row: A_i <- A_i T  (A: rows x k FP32 row-major; T: k x k FP32 row-major).
__global__ __launch_bounds__(TH) void k_rows_times(float* A, int64_t rows, int k, const float* T) {
  // the whole tile is written: the unrolled products below touch rows t >= k
  // (times a zero row entry), which must not meet stale LDS contents
  __shared__ float sT[32 * 32];
  for (int idx = threadIdx.x; idx < 32 * 32; idx += TH) sT[idx] = idx < k * k ? T[idx] : 0.f;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * TH + threadIdx.x;
  if (i >= rows) return;
  float a[32];
#pragma unroll
  for (int t = 0; t < 32; ++t) a[t] = t < k ? A[i * k + t] : 0.f;
  for (int c = 0; c < k; ++c) {
    float s = 0.f;
#pragma unroll
    for (int t = 0; t < 32; ++t) s = fmaf(a[t], sT[t * k + c], s);
    A[i * k + c] = s;
  }
}

// out[e] = sum over the blocks of part[b kk2 + e], one workgroup per entry
// (thread-strided, then the wave tree and the waves in order: a fixed order).
__global__ __launch_bounds__(TH) void k_gram_rows_sum(const double* part, int blocks, int kk2, double* out) {
  __shared__ double red[TH / 64];
  const int e = blockIdx.x;
  double v = 0.0;
  for (int b = threadIdx.x; b < blocks; b += TH) v += part[(int64_t)b * kk2 + e];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < TH / 64; ++w) t += red[w];
    out[e] = t;
  }
}

// Gram of the rows of A (k x k, on the host).  The block partials are summed on
// the device (into the slot after the largest partial set) and the k x k result
// comes back through the context's pinned staging.
int gram(rpca_ctx* c, const float* A, int64_t rows, std::vector<double>& out, hipStream_t s) {
  const int k = c->k;
  const int kk2 = k * k;
  int64_t blocks = (rows + 63) / 64;
  if (blocks > rpca::PC_GRAM_BLOCKS) blocks = rpca::PC_GRAM_BLOCKS;
  hipLaunchKernelGGL(k_gram_rows, dim3((unsigned)blocks), dim3(TH), 0, s, A, rows, k, c->pc_gram);
  if (hipGetLastError() != hipSuccess) return RPCA_EHIP;
  double* sum = c->pc_gram + (size_t)rpca::PC_GRAM_BLOCKS * kk2;
  hipLaunchKernelGGL(k_gram_rows_sum, dim3((unsigned)kk2), dim3(TH), 0, s, (const double*)c->pc_gram, (int)blocks,
                     kk2, sum);
  if (hipGetLastError() != hipSuccess) return RPCA_EHIP;
  double* pin = (double*)rpca::ctx_pinned(c, (size_t)kk2 * sizeof(double));
  if (!pin) return RPCA_ENOMEM;
  if (hipMemcpyAsync(pin, sum, (size_t)kk2 * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return RPCA_EHIP;
  out.assign(pin, pin + kk2);
  return RPCA_OK;
}

// (G + lam I)^{power} for a symmetric PSD G (k x k), power = +-1/2.
void sym_power(const std::vector<double>& G, int k, double lam, double power, std::vector<double>& out) {
  std::vector<double> M(G), w(k), Q((size_t)k * k);
  for (int i = 0; i < k; ++i) M[(size_t)i * k + i] += lam;
  rpca::la::sym_eig(M.data(), k, w.data(), Q.data());
  out.assign((size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      double s = 0.0;
      for (int t = 0; t < k; ++t) s += Q[(size_t)i * k + t] * pow(std::max(w[t], 1e-300), power) * Q[(size_t)j * k + t];
      out[(size_t)i * k + j] = s;
    }
}

int rows_times(rpca_ctx* c, float* A, int64_t rows, const float* T, hipStream_t s) {
  hipLaunchKernelGGL(k_rows_times, dim3((unsigned)((rows + TH - 1) / TH)), dim3(TH), 0, s, A, rows, c->k, T);
  return hipGetLastError() == hipSuccess ? RPCA_OK : RPCA_EHIP;
}

}  // namespace

namespace rpca {

// x[cur] in preconditioned variables -> plain (U, V), in place.
int precond_to_plain(rpca_ctx* c, int cur, hipStream_t s) {
  if (!c->pc_on) return RPCA_OK;
  const int k = c->k;
  const int64_t kk2 = (int64_t)k * k;
  int rc;
  if ((rc = rows_times(c, c->x[cur], c->m, c->pc_dev + 3 * kk2, s))) return rc;               // U = A P_U
  if ((rc = rows_times(c, c->x[cur] + c->m * k, c->n, c->pc_dev + 4 * kk2, s))) return rc;     // V = B P_V
  c->pc_on = false;
  return RPCA_OK;
}

// New preconditioner from the current point; x[cur] ends in the new variables.
int precond_refresh(rpca_ctx* c, int cur, hipStream_t s) {
  int rc;
  if ((rc = precond_to_plain(c, cur, s))) return rc;
  const int k = c->k;
  const int64_t kk2 = (int64_t)k * k;
  float* U = c->x[cur];
  float* V = c->x[cur] + c->m * k;
  std::vector<double> UtU, VtV, PU, PV, PUi, PVi;
  if ((rc = gram(c, U, c->m, UtU, s)) || (rc = gram(c, V, c->n, VtV, s))) return rc;
  sym_power(VtV, k, c->lam_l, -0.5, PU);
  sym_power(VtV, k, c->lam_l, 0.5, PUi);
  sym_power(UtU, k, c->lam_l, -0.5, PV);
  sym_power(UtU, k, c->lam_l, 0.5, PVi);
  std::vector<float> h((size_t)7 * kk2);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      double w = 0.0, mu = 0.0, mv = 0.0;
      for (int t = 0; t < k; ++t) {
        w += PU[(size_t)i * k + t] * PV[(size_t)t * k + j];
        mu += PU[(size_t)i * k + t] * PU[(size_t)t * k + j];
        mv += PV[(size_t)i * k + t] * PV[(size_t)t * k + j];
      }
      const size_t o = (size_t)i * k + j;
      h[o] = (float)w;
      h[kk2 + o] = (float)mu;
      h[2 * kk2 + o] = (float)mv;
      h[3 * kk2 + o] = (float)PU[o];
      h[4 * kk2 + o] = (float)PV[o];
      h[5 * kk2 + o] = (float)PUi[o];
      h[6 * kk2 + o] = (float)PVi[o];
    }
  float* pin = (float*)rpca::ctx_pinned(c, h.size() * 4);
  if (!pin) return RPCA_ENOMEM;
  memcpy(pin, h.data(), h.size() * 4);
  if (hipMemcpyAsync(c->pc_dev, pin, h.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess) return RPCA_EHIP;
  if ((rc = rows_times(c, U, c->m, c->pc_dev + 5 * kk2, s))) return rc;   // A = U P_U^{-1}
  if ((rc = rows_times(c, V, c->n, c->pc_dev + 6 * kk2, s))) return rc;   // B = V P_V^{-1}
  // the pinned staging is reused by the next copy through it
  if (hipStreamSynchronize(s) != hipSuccess) return RPCA_EHIP;
  c->pc_on = true;
  return RPCA_OK;
}

}  // namespace rpca
