// Autotuner of the sweep decomposition.  For every (k bucket, n bucket) of
// the table it builds a probe instance (m_probe rows, the bucket's largest
// k and n, seeded synthetic X and factors generated on the device), times
// rpca_objgrad with HIP events for each candidate (waves the strips are
// spread over x divisor of the widest chunk) and keeps the fastest.
#include <math.h>

#include "rpca_internal.h"

namespace {

__device__ __forceinline__ float hash_uniform(uint64_t seed, uint64_t i) {
  uint64_t x = seed + 0x9E3779B97F4A7C15ull * (i + 1);
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  x ^= x >> 31;
  return (float)((double)(x >> 11) * (1.0 / 9007199254740992.0)) * 2.f - 1.f;  // [-1, 1)
}

__global__ void k_fill(float* p, int64_t n, uint64_t seed, float scale) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = scale * hash_uniform(seed, (uint64_t)i);
}

const int K_REP[rpca::TUNE_KB] = {8, 16, 24, 32};
const int64_t N_REP[rpca::TUNE_NB] = {64, 128, 256, 512, 1024};
const int WAVE_CAND[] = {1024, 2048, 4096};
const int DIV_CAND[] = {1, 2};

}  // namespace

extern "C" {

int rpca_autotune(int64_t m_probe, int32_t reps, void* stream) {
  // the probes reach k = 32, which needs at least 32 rows
  if (m_probe < 32 || m_probe > (int64_t)1 << 24 || reps < 1 || reps > 10000) return RPCA_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int64_t nmax = N_REP[rpca::TUNE_NB - 1];
  const int kmax = K_REP[rpca::TUNE_KB - 1];
  float *X = nullptr, *U = nullptr, *V = nullptr, *gU = nullptr, *gV = nullptr;
  double* f = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = RPCA_OK;
  if (hipMalloc(&X, (size_t)m_probe * nmax * 4) != hipSuccess || hipMalloc(&U, (size_t)m_probe * kmax * 4) != hipSuccess ||
      hipMalloc(&V, (size_t)nmax * kmax * 4) != hipSuccess || hipMalloc(&gU, (size_t)m_probe * kmax * 4) != hipSuccess ||
      hipMalloc(&gV, (size_t)nmax * kmax * 4) != hipSuccess || hipMalloc(&f, 8) != hipSuccess) {
    rc = RPCA_ENOMEM;
  } else if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    rc = RPCA_EHIP;
  }
  if (rc == RPCA_OK) {
    hipLaunchKernelGGL(k_fill, dim3(1024), dim3(256), 0, s, X, m_probe * nmax, 11ull, 1.0f);
    hipLaunchKernelGGL(k_fill, dim3(1024), dim3(256), 0, s, U, m_probe * kmax, 12ull, 0.3f);
    hipLaunchKernelGGL(k_fill, dim3(64), dim3(256), 0, s, V, nmax * kmax, 13ull, 0.3f);
    if (hipGetLastError() != hipSuccess) rc = RPCA_EHIP;
  }
  for (int kb = 0; kb < rpca::TUNE_KB && rc == RPCA_OK; ++kb) {
    for (int nb = 0; nb < rpca::TUNE_NB && rc == RPCA_OK; ++nb) {
      const int k = K_REP[kb];
      const int64_t n = N_REP[nb];
      float best = INFINITY;
      rpca::SweepTune best_t{1024, 1};
      for (int w : WAVE_CAND) {
        for (int d : DIV_CAND) {
          rpca::tune_set(kb, nb, rpca::SweepTune{w, d});
          rpca_ctx* c = nullptr;
          if ((rc = rpca_create(m_probe, n, k, 0.1, 1.0, nullptr, &c)) != RPCA_OK) break;
          for (int r = 0; r < 2 && rc == RPCA_OK; ++r) rc = rpca_objgrad(c, X, U, V, f, gU, gV, s);
          if (rc == RPCA_OK && hipEventRecord(e0, s) != hipSuccess) rc = RPCA_EHIP;
          for (int r = 0; r < reps && rc == RPCA_OK; ++r) rc = rpca_objgrad(c, X, U, V, f, gU, gV, s);
          float ms = INFINITY;
          if (rc == RPCA_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            rc = RPCA_EHIP;
          rpca_destroy(c);
          if (rc != RPCA_OK) break;
          if (ms < best) {
            best = ms;
            best_t = rpca::SweepTune{w, d};
          }
        }
        if (rc != RPCA_OK) break;
      }
      rpca::tune_set(kb, nb, best_t);
    }
  }
  if (X) (void)hipFree(X);
  if (U) (void)hipFree(U);
  if (V) (void)hipFree(V);
  if (gU) (void)hipFree(gU);
  if (gV) (void)hipFree(gV);
  if (f) (void)hipFree(f);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return rc;
}

int rpca_tune_get(int32_t k, int64_t n, int32_t* target_waves, int32_t* chunk_div) {
  if (k < 1 || k > 32 || n < 1 || !target_waves || !chunk_div) return RPCA_EINVAL;
  const rpca::SweepTune t = rpca::tune_get(k, n);
  *target_waves = t.target_waves;
  *chunk_div = t.chunk_div;
  return RPCA_OK;
}

int rpca_tune_set(int32_t k, int64_t n, int32_t target_waves, int32_t chunk_div) {
  if (k < 1 || k > 32 || n < 1 || target_waves < 64 || target_waves > (1 << 20) || chunk_div < 1 || chunk_div > 16)
    return RPCA_EINVAL;
  rpca::tune_set(rpca::tune_k_bucket(k), rpca::tune_n_bucket(n), rpca::SweepTune{target_waves, chunk_div});
  return RPCA_OK;
}

}  // extern "C"
