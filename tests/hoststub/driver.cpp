// Drives the library's host code against the HIP stand-in (hip_stub.cpp) under
// a sanitizer: batched objective/gradient and solves of uneven instances (the
// batch's 16 worker threads run the rSVD start, the preconditioner refreshes,
// restarts and certificates), certificates and rSVD starts on single contexts
// from 16 threads at once, the allocation-free entry point, and a sweep of
// injected HIP failures over a batched solve (every error path must return
// without leaving a queued copy behind or a device allocation held).
//
// Exit status 0 when the stand-in reported no problem and every check held;
// the sanitizers report on their own (and end the process with an error).
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <thread>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "rpca.h"
#include "rpca_batch.h"

// Controls of the stand-in; absent when the driver is linked with the real HIP
// runtime (then the batched and single-context paths run on the GPU with
// AddressSanitizer on the host side, and the failure sweep is skipped).
extern "C" {
__attribute__((weak)) void stub_fail_at(int64_t n);
__attribute__((weak)) int64_t stub_calls();
__attribute__((weak)) int64_t stub_problems();
__attribute__((weak)) int64_t stub_pending();
__attribute__((weak)) int64_t stub_live_allocations();
__attribute__((weak)) void stub_drain_all();
}
bool have_stub() { return &stub_problems != nullptr; }
int64_t pending() { return have_stub() ? stub_pending() : 0; }


namespace {

int g_fail = 0;
#define CHECK(cond, ...)                      \
  do {                                        \
    if (!(cond)) {                            \
      fprintf(stderr, "CHECK failed: " __VA_ARGS__); \
      fprintf(stderr, "\n");                  \
      ++g_fail;                               \
    }                                         \
  } while (0)

float* dev_floats(size_t n, unsigned seed) {
  void* p = nullptr;
  if (hipMalloc(&p, n * 4) != 0) return nullptr;
  std::vector<float> h(n);
  unsigned s = seed * 2654435761u + 1;
  for (auto& v : h) {
    s = s * 1664525u + 1013904223u;
    v = (float)((s >> 8) * (1.0 / 16777216.0) - 0.5);
  }
  hipMemcpy(p, h.data(), n * 4, hipMemcpyHostToDevice);
  return static_cast<float*>(p);
}

struct Instances {
  std::vector<int64_t> m, n;
  std::vector<int32_t> k;
  std::vector<double> ls, ll;
  std::vector<float*> X, U, V, gU, gV;
  std::vector<double*> f;
  explicit Instances(int count) {
    for (int i = 0; i < count; ++i) {
      m.push_back(96 + 37 * ((i * 7) % 23));
      n.push_back(24 + 9 * ((i * 5) % 11));
      k.push_back(i % 4 == 3 ? 20 : 4 + i % 9);  // both sweep forms (k <= 16, k > 16)
      ls.push_back(0.05);
      ll.push_back(1.0);
      X.push_back(dev_floats((size_t)m[i] * n[i], 3 * i + 1));
      U.push_back(dev_floats((size_t)m[i] * k[i], 3 * i + 2));
      V.push_back(dev_floats((size_t)n[i] * k[i], 3 * i + 3));
      gU.push_back(dev_floats((size_t)m[i] * k[i], 0));
      gV.push_back(dev_floats((size_t)n[i] * k[i], 0));
      void* p = nullptr;
      hipMalloc(&p, 8);
      f.push_back(static_cast<double*>(p));
    }
  }
  ~Instances() {
    for (auto* v : {&X, &U, &V, &gU, &gV})
      for (float* p : *v) hipFree(p);
    for (double* p : f) hipFree(p);
  }
  int count() const { return (int)m.size(); }
};

rpca_opts solve_opts(int precision, int precond) {
  rpca_opts o;
  rpca_default_opts(&o);
  o.init = RPCA_INIT_RSVD;
  o.certify = 1;
  o.precision = precision;
  o.precond = precond;
  return o;
}

// One batched solve on a fresh batch; returns the solve's status (or the
// creation's error).
int batch_solve(const Instances& in, const rpca_opts& o, int graphs) {
  rpca_batch* b = nullptr;
  int rc = rpca_batch_create(in.count(), in.m.data(), in.n.data(), in.k.data(), in.ls.data(), in.ll.data(), &b);
  if (rc != RPCA_OK) return rc;
  rpca_batch_set_graphs(b, graphs);
  std::vector<rpca_info> info(in.count());
  rc = rpca_batch_solve(b, in.X.data(), in.U.data(), in.V.data(), &o, info.data(), nullptr);
  rpca_batch_destroy(b);
  return rc;
}

void batch_paths(const Instances& in) {
  rpca_batch* b = nullptr;
  CHECK(rpca_batch_create(in.count(), in.m.data(), in.n.data(), in.k.data(), in.ls.data(), in.ll.data(), &b) ==
            RPCA_OK,
        "batch create");
  for (int prec : {RPCA_PREC_FP32, RPCA_PREC_BF16})
    CHECK(rpca_batch_objgrad(b, in.X.data(), in.U.data(), in.V.data(), in.f.data(), in.gU.data(), in.gV.data(),
                             prec, nullptr) == RPCA_OK,
          "batch objgrad precision %d", prec);
  rpca_batch_destroy(b);
  struct Case {
    int precision, precond, graphs;
  } cases[] = {{RPCA_PREC_FP32, 1, 1}, {RPCA_PREC_FP32, 1, 0}, {RPCA_PREC_BF16_POLISH, 1, 1}, {RPCA_PREC_FP32, 0, 0}};
  for (const Case& c : cases) {
    const int rc = batch_solve(in, solve_opts(c.precision, c.precond), c.graphs);
    CHECK(rc >= 0, "batch solve precision %d precond %d graphs %d: %d", c.precision, c.precond, c.graphs, rc);
    CHECK(pending() == 0, "queued work left after a batch solve");
  }
}

// Certificates, rSVD starts and evaluations on single contexts, 16 threads at once.
void context_paths(const Instances& in) {
  std::vector<std::thread> th;
  std::vector<int> bad(16, 0);
  for (int t = 0; t < 16; ++t)
    th.emplace_back([&, t] {
      const int i = t % in.count();
      rpca_ctx* c = nullptr;
      if (rpca_create(in.m[i], in.n[i], in.k[i], in.ls[i], in.ll[i], nullptr, &c) != RPCA_OK) {
        bad[t] = 1;
        return;
      }
      if (rpca_objgrad(c, in.X[i], in.U[i], in.V[i], in.f[i], in.gU[i], in.gV[i], nullptr) != RPCA_OK) bad[t] |= 2;
      if (rpca_init_rsvd(c, in.X[i], nullptr, 10, 2, 7 + t, in.gU[i], in.gV[i], nullptr) != RPCA_OK) bad[t] |= 4;
      rpca_cert cert;
      if (rpca_certificate(c, in.X[i], in.U[i], in.V[i], &cert, nullptr) < 0) bad[t] |= 8;
      rpca_destroy(c);
    });
  for (auto& x : th) x.join();
  for (int t = 0; t < 16; ++t) CHECK(bad[t] == 0, "context thread %d: flags %d", t, bad[t]);
  CHECK(pending() == 0, "queued work left after the context threads");
}

void noalloc_path(const Instances& in) {
  for (int i = 0; i < 2; ++i)
    CHECK(rpca_objgrad_noalloc(in.m[i], in.n[i], in.k[i], in.ls[i], in.ll[i], nullptr, in.X[i], in.U[i], in.V[i],
                               in.f[i], in.gU[i], in.gV[i], nullptr) == RPCA_OK,
          "noalloc %d", i);
  if (have_stub()) stub_drain_all();
  else hipDeviceSynchronize();
}

// Fail the n-th HIP call of a batched solve, for n spread over the whole solve.
void failure_sweep(const Instances& in, int points) {
  const rpca_opts o = solve_opts(RPCA_PREC_FP32, 1);
  const int64_t live0 = stub_live_allocations();
  stub_fail_at(-1);
  CHECK(batch_solve(in, o, 1) >= 0, "reference solve of the failure sweep");
  const int64_t calls = stub_calls();
  int failed = 0;
  for (int p = 0; p < points; ++p) {
    const int64_t at = 1 + (calls - 1) * p / (points > 1 ? points - 1 : 1);
    stub_fail_at(at);
    const int rc = batch_solve(in, o, p % 2);
    failed += rc < 0;
    stub_fail_at(-1);
    CHECK(stub_pending() == 0, "call %lld failed: queued work left after the batch was destroyed", (long long)at);
    CHECK(stub_live_allocations() == live0, "call %lld failed: %lld allocations leaked", (long long)at,
          (long long)(stub_live_allocations() - live0));
  }
  printf("failure sweep: %d points over %lld calls, %d solves returned an error\n", points, (long long)calls, failed);
}

// Planted mistakes in the driver's own code (not the library's), each of which
// the harness must report: a host vector freed while its copy is queued, a
// pinned destination read before the wait, a host source rewritten while its
// copy is queued, a read on one stream of what another stream has yet to
// write, and two threads writing one variable.
int canary(const char* which) {
  void* d = nullptr;
  hipMalloc(&d, 64 * sizeof(float));
  hipStream_t s1 = nullptr, s2 = nullptr;
  hipStreamCreateWithFlags(&s1, hipStreamNonBlocking);
  hipStreamCreateWithFlags(&s2, hipStreamNonBlocking);
  if (!strcmp(which, "freed-source")) {
    {
      std::vector<float> h(64, 1.0f);
      hipMemcpyAsync(d, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice, s1);
    }
    hipStreamSynchronize(s1);
  } else if (!strcmp(which, "early-read")) {
    float* h = nullptr;
    hipHostMalloc((void**)&h, 64 * sizeof(float), 0);
    hipMemcpyAsync(h, d, 64 * sizeof(float), hipMemcpyDeviceToHost, s1);
    volatile float x = h[3];
    (void)x;
    hipStreamSynchronize(s1);
  } else if (!strcmp(which, "rewritten-source")) {
    std::vector<float> h(64, 1.0f);
    hipMemcpyAsync(d, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice, s1);
    h[5] = 2.0f;
    hipStreamSynchronize(s1);
  } else if (!strcmp(which, "cross-stream")) {
    void* d2 = nullptr;
    hipMalloc(&d2, 64 * sizeof(float));
    std::vector<float> h(64, 1.0f);
    hipMemcpyAsync(d, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice, s1);
    hipMemcpyAsync(d2, d, 64 * sizeof(float), hipMemcpyDeviceToDevice, s2);
    hipStreamSynchronize(s2);
    hipStreamSynchronize(s1);
  } else if (!strcmp(which, "race")) {
    int shared = 0;
    std::thread a([&] { for (int i = 0; i < 1000; ++i) shared = shared + 1; });
    std::thread b([&] { for (int i = 0; i < 1000; ++i) shared = shared + 1; });
    a.join();
    b.join();
  } else {
    return 2;
  }
  return stub_problems() ? 1 : 0;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc > 2 && !strcmp(argv[1], "--canary")) return have_stub() ? canary(argv[2]) : 2;
  const int points = argc > 1 ? atoi(argv[1]) : 120;
  {
    Instances in(24);
    batch_paths(in);
    printf("batch paths done\n");
    fflush(stdout);
    context_paths(in);
    printf("context paths done\n");
    fflush(stdout);
    noalloc_path(in);
    if (have_stub() && points > 0) failure_sweep(in, points);
  }
  const int64_t problems = have_stub() ? stub_problems() : 0;
  printf("stand-in problems %lld, failed checks %d, allocations left %lld\n", (long long)problems, g_fail,
         (long long)(have_stub() ? stub_live_allocations() : -1));
  return (problems || g_fail) ? 1 : 0;
}
