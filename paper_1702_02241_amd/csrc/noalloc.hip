// Objective/gradient without any allocation: rpca_objgrad_noalloc runs the
// same fused sweep and finishing reduction as rpca_objgrad, with every partial
// sum in one library-owned device array instead of a context's workspace.
//
// The array below lives in the device code object, so each GPU the library runs
// on holds its own copy until the process ends.  Its name is only a host-side
// stand-in: host code resolves the device address once per device with
// hipGetSymbolAddress and passes that address to the kernels.
#include <math.h>
#include <string.h>

#include <mutex>

#include "rpca_internal.h"

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)RPCA_NOALLOC_SCRATCH_MB << 20;
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex g_mu;
void* g_addr[MAX_DEVICES] = {nullptr};

// Device address of this GPU's copy of the array (resolved on first use).
hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_addr[dev] = p;
  }
  *out = g_addr[dev];
  return hipSuccess;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Scratch layout of one call (byte offsets; every region 256-byte aligned).
struct Layout {
  size_t counters, spart, fpart, level2, gvpart, gupart, total;
};

Layout layout_for(int64_t m, int64_t n, int k, int row_groups, int nchunks, int sweep_wgs, int segs) {
  Layout L;
  size_t o = 0;
  L.counters = o;
  o += align256(16 * sizeof(unsigned));
  L.spart = o;
  o += align256((size_t)sweep_wgs * RPCA_NSCAL * sizeof(double));
  L.fpart = o;
  o += align256(((size_t)rpca::finish_blocks(m, n, k, nchunks, nullptr) * 3 + 16) * sizeof(double));
  L.level2 = o;
  o += align256((size_t)segs * n * k * sizeof(double));
  L.gvpart = o;
  o += align256((size_t)row_groups * n * k * sizeof(float));
  L.gupart = o;
  if (nchunks > 1) o += align256((size_t)nchunks * m * k * sizeof(float));
  L.total = o;
  return L;
}

}  // namespace

extern "C" int rpca_objgrad_noalloc(int64_t m, int64_t n, int32_t k, double lam_s, double lam_l,
                                    const uint32_t* mask_bits, const float* X, const float* U, const float* V,
                                    double* f, float* gU, float* gV, void* stream) {
  // the same argument rules as rpca_create + rpca_objgrad
  if (m < 1 || n < 1 || k < 1 || k > 32 || k > m || k > n) return RPCA_EINVAL;
  if (!(lam_s > 0) || !(lam_l > 0) || !isfinite(lam_s) || !isfinite(lam_l)) return RPCA_EINVAL;
  if (m > (int64_t)1 << 31 || n > (int64_t)1 << 24) return RPCA_EINVAL;
  if (!X || !U || !V || !f || !gU || !gV) return RPCA_EINVAL;
  // the decomposition rpca_create would choose for this instance
  int row_groups = 0, spw = 0, chunk_w = 0, nchunks = 0;
  const int sweep_wgs = rpca::sweep_blocks_for(m, n, k, &row_groups, &spw, &chunk_w, &nchunks, 0);
  const int rps = 16;
  const int segs = (row_groups + rps - 1) / rps;
  const Layout L = layout_for(m, n, k, row_groups, nchunks, sweep_wgs, segs);
  if (L.total > SCRATCH_BYTES) return RPCA_ETOOBIG;

  void* base = nullptr;
  if (scratch_address(&base) != hipSuccess) return RPCA_EHIP;
  unsigned char* b = static_cast<unsigned char*>(base);

  SweepArgs sa;
  memset(&sa, 0, sizeof(sa));
  sa.X = X;
  sa.mask = mask_bits;
  sa.m = m;
  sa.n = n;
  sa.k = k;
  sa.mw = mask_bits ? (int)((m + 31) / 32) : 0;
  sa.lam_s = (float)lam_s;
  sa.lam_l = (float)lam_l;
  sa.kappa = 0.f;
  sa.xvec = (m % 4 == 0) && (((uintptr_t)X & 15u) == 0) && m < ((int64_t)1 << 26);
  sa.U[0] = sa.U[1] = U;
  sa.V[0] = sa.V[1] = V;
  sa.gU[0] = sa.gU[1] = gU;
  sa.gupart = nchunks > 1 ? reinterpret_cast<float*>(b + L.gupart) : nullptr;
  sa.gvpart = reinterpret_cast<float*>(b + L.gvpart);
  sa.spart = reinterpret_cast<double*>(b + L.spart);
  sa.strips_per_wave = spw;
  sa.chunk_w = chunk_w;
  sa.nchunks = nchunks;
  sa.row_groups = row_groups;

  FinishArgs fa;
  memset(&fa, 0, sizeof(fa));
  fa.m = m;
  fa.n = n;
  fa.k = k;
  fa.lam_l = (float)lam_l;
  fa.U[0] = fa.U[1] = U;
  fa.V[0] = fa.V[1] = V;
  fa.gU[0] = fa.gU[1] = gU;
  fa.gV[0] = fa.gV[1] = gV;
  fa.gupart = sa.gupart;
  fa.gvpart = sa.gvpart;
  fa.spart = sa.spart;
  fa.level2 = reinterpret_cast<double*>(b + L.level2);
  fa.fpart = reinterpret_cast<double*>(b + L.fpart);
  // the finishing reduction's first kernel zeroes this counter before the
  // second one counts on it
  fa.counter = reinterpret_cast<unsigned*>(b + L.counters);
  fa.f_out = f;
  fa.segs = segs;
  fa.rows_per_seg = rps;
  fa.nchunks = nchunks;
  fa.row_groups = row_groups;
  fa.sweep_wgs = sweep_wgs;
  if (rpca::launch_objgrad(sa, fa, false, false, (hipStream_t)stream) != hipSuccess) return RPCA_EHIP;
  return RPCA_OK;
}
