// Host-only stand-in for the HIP runtime, so that the library's host code (the
// batch's worker threads, the certificate, the preconditioner, the solver's
// host loop) can run under AddressSanitizer and ThreadSanitizer on a machine
// without a GPU.  Test infrastructure: linked only into the sanitizer driver.
//
// Model
//  - Device memory is host memory (allocated here, zero-filled, tracked).
//  - Kernels do not run.  Their launches are queued like copies.  The one
//    exception is the batch's phase gather, which reports every instance done,
//    so that every solver loop ends after one group of slots.
//  - Asynchronous copies and memsets are queued on their stream and executed
//    only when something waits for them: a stream or event synchronisation, a
//    synchronous copy, or a free (hipFree and hipHostFree wait for the whole
//    device, as HIP's do).  That is the latest moment the runtime may still
//    touch the host buffers, so
//      * a buffer freed or gone out of scope before the wait is reported by
//        AddressSanitizer in the queued copy (heap-use-after-free,
//        stack-use-after-return);
//      * a host source rewritten while its copy is queued is reported here (a
//        checksum taken at the call and at the copy differ);
//      * a destination read before the wait is reported by AddressSanitizer
//        (the range stays poisoned until the copy lands);
//      * a copy between pointers of the wrong kind, or past the end of a
//        device allocation, is reported here.
//  - hipStreamWaitEvent orders a stream after the event's point on another
//    stream; nothing else orders streams, so a missing dependency shows up as a
//    read of a poisoned range.
//  - One mutex orders every call, so ThreadSanitizer sees the hand-offs between
//    threads as synchronisation and reports races in the library's own code.
//  - stub_fail_at(n) makes the n-th call from then on return an error (a
//    launch sets the pending error instead), to drive the library's error paths.
#include <execinfo.h>
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#if defined(__has_feature)
#if __has_feature(address_sanitizer)
#include <sanitizer/asan_interface.h>
#define STUB_POISON(p, n) __asan_poison_memory_region((p), (n))
#define STUB_UNPOISON(p, n) __asan_unpoison_memory_region((p), (n))
#endif
#endif
#ifndef STUB_POISON
#define STUB_POISON(p, n) ((void)0)
#define STUB_UNPOISON(p, n) ((void)0)
#endif

struct ihipStream_t;
struct ihipEvent_t;
struct ihipGraph;
struct hipGraphExec;

namespace {

enum OpKind { OP_COPY, OP_SET, OP_WAIT, OP_KERNEL };

struct Stream;

struct Op {
  OpKind kind;
  void* dst = nullptr;
  const void* src = nullptr;
  size_t n = 0;
  int value = 0;
  bool check = false;  // host source: compare its checksum at the copy
  uint64_t sum = 0;
  Stream* ws = nullptr;  // OP_WAIT: drain ws up to wseq first
  uint64_t wseq = 0;
  bool host_dst = false;  // destination is host memory (poisoned while queued)
  uint64_t id = 0;        // issue order over all streams
  int gather_count = 0;  // OP_KERNEL of the phase gather
  int* gather_out = nullptr;
  void* where[12];
  int depth = 0;
};

struct Graph {
  std::vector<Op> ops;
};

struct Stream {
  std::vector<Op> q;  // queued, in order; q[i] has sequence number base + i + 1
  uint64_t base = 0;  // operations executed
  Graph* cap = nullptr;
  bool destroyed = false;
  uint64_t enqueued() const { return base + q.size(); }
};

struct Event {
  Stream* s = nullptr;
  uint64_t seq = 0;
};

// Global state, built on first use: the library's registration calls run from
// static constructors, possibly before this file's own.
struct Globals {
  std::recursive_mutex mu;
  std::map<uintptr_t, size_t> dev, pinned;  // base -> bytes
  std::map<const void*, std::string> kernels;  // host stub -> device name
  std::map<const void*, size_t> vars;          // __device__ variable shadows
  std::vector<Stream*> streams;
  Stream null_stream;
  int64_t calls = 0, fail_at = -1, problems = 0;
  uint64_t next_id = 0;
};
Globals& G() {
  static Globals* g = new Globals;
  return *g;
}
#define g_mu G().mu
#define g_dev G().dev
#define g_pinned G().pinned
#define g_kernels G().kernels
#define g_vars G().vars
#define g_streams G().streams
#define g_null G().null_stream
#define g_calls G().calls
#define g_fail_at G().fail_at
#define g_problems G().problems
#define g_next_id G().next_id
thread_local hipError_t t_last = hipSuccess;
thread_local dim3 t_grid, t_block;
thread_local size_t t_shmem = 0;
thread_local hipStream_t t_cfg_stream = nullptr;

Stream* S(hipStream_t s) { return s ? reinterpret_cast<Stream*>(s) : &g_null; }

void problem(const char* what, const Op* op) {
  ++g_problems;
  fprintf(stderr, "hip_stub: %s\n", what);
  if (op && op->depth) {
    fprintf(stderr, "  queued at:\n");
    backtrace_symbols_fd(const_cast<void**>(op->where), op->depth, 2);
  }
  fprintf(stderr, "  detected at:\n");
  void* bt[16];
  backtrace_symbols_fd(bt, backtrace(bt, 16), 2);
  if (getenv("HIP_STUB_ABORT")) abort();
}

// Injected failure: true for the n-th counted call after stub_fail_at(n).
bool fail_now() {
  ++g_calls;
  if (g_fail_at >= 0 && g_calls == g_fail_at) {
    g_fail_at = -1;
    return true;
  }
  return false;
}

const std::map<uintptr_t, size_t>::value_type* find(const std::map<uintptr_t, size_t>& m, const void* p) {
  const uintptr_t a = reinterpret_cast<uintptr_t>(p);
  auto it = m.upper_bound(a);
  if (it == m.begin()) return nullptr;
  --it;
  return (a < it->first + it->second) ? &*it : nullptr;
}

bool is_dev(const void* p) { return find(g_dev, p) != nullptr; }

uint64_t checksum(const void* p, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  return h;
}

// Kind and bounds of one side of a copy: device pointers must stay inside
// their allocation, host pointers must not be device memory.
bool side_ok(const void* p, size_t n, bool device, const char* side) {
  if (!n) return true;
  const auto* d = find(g_dev, p);
  if (device) {
    if (!d) {
      char msg[160];
      snprintf(msg, sizeof msg, "%s %p is not device memory", side, p);
      problem(msg, nullptr);
      return false;
    }
    if (reinterpret_cast<uintptr_t>(p) + n > d->first + d->second) {
      char msg[160];
      snprintf(msg, sizeof msg, "%s %p + %zu runs past its device allocation", side, p, n);
      problem(msg, nullptr);
      return false;
    }
  } else if (d) {
    char msg[160];
    snprintf(msg, sizeof msg, "%s %p is device memory in a host position", side, p);
    problem(msg, nullptr);
    return false;
  }
  return true;
}

bool kind_ok(void* dst, const void* src, size_t n, hipMemcpyKind kind) {
  switch (kind) {
    case hipMemcpyHostToDevice: return side_ok(dst, n, true, "destination") && side_ok(src, n, false, "source");
    case hipMemcpyDeviceToHost: return side_ok(dst, n, false, "destination") && side_ok(src, n, true, "source");
    case hipMemcpyDeviceToDevice: return side_ok(dst, n, true, "destination") && side_ok(src, n, true, "source");
    case hipMemcpyHostToHost: return side_ok(dst, n, false, "destination") && side_ok(src, n, false, "source");
    default: return true;
  }
}

void run(Stream* s, Op& op);

// Execute s's queued operations up to sequence number upto.
void drain(Stream* s, uint64_t upto) {
  while (s->base < upto && !s->q.empty()) {
    Op op = s->q.front();
    s->q.erase(s->q.begin());
    run(s, op);
    ++s->base;
  }
}

void drain_all() {
  bool more = true;
  while (more) {
    more = false;
    for (Stream* s : g_streams)
      if (!s->q.empty()) {
        drain(s, s->enqueued());
        more = true;
      }
    if (!g_null.q.empty()) {
      drain(&g_null, g_null.enqueued());
      more = true;
    }
  }
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return na && nb && x < y + nb && y < x + na;
}

// Queued copies and memsets whose destination overlaps [p, p + n).
template <typename F>
void for_pending_dst(const void* p, size_t n, F f) {
  auto visit = [&](Stream* s) {
    for (Op& q : s->q)
      if ((q.kind == OP_COPY || q.kind == OP_SET) && overlap(q.dst, q.n, p, n)) f(q);
  };
  for (Stream* s : g_streams) visit(s);
  visit(&g_null);
}

// Run a copy or memset.  A range it reads that an operation issued earlier (on
// another stream: this stream's earlier ones have run) has yet to write is a
// missing dependency.  Host ranges that later operations will write stay
// poisoned for the library's code; this operation reads and writes around them.
void run_transfer(Op& op) {
  std::vector<std::pair<char*, size_t>> later;
  bool raced = false;
  auto note = [&](const void* p, size_t n) {
    for_pending_dst(p, n, [&](Op& q) {
      if (q.id < op.id) {
        if (p == op.src) raced = true;
        return;
      }
      if (!q.host_dst) return;
      const uintptr_t lo = std::max(reinterpret_cast<uintptr_t>(q.dst), reinterpret_cast<uintptr_t>(p));
      const uintptr_t hi = std::min(reinterpret_cast<uintptr_t>(q.dst) + q.n, reinterpret_cast<uintptr_t>(p) + n);
      later.push_back({reinterpret_cast<char*>(lo), hi - lo});
    });
  };
  if (op.kind == OP_COPY) note(op.src, op.n);
  note(op.dst, op.n);
  if (raced)
    problem("a queued copy reads a range that an operation issued earlier on another stream has not written "
            "yet (no event orders them)",
            &op);
  for (auto& r : later) STUB_UNPOISON(r.first, r.second);
  STUB_UNPOISON(op.dst, op.n);
  if (op.kind == OP_COPY) {
    if (op.check && checksum(op.src, op.n) != op.sum)
      problem("host source of a queued copy changed before the copy ran", &op);
    memmove(op.dst, op.src, op.n);
  } else {
    memset(op.dst, op.value, op.n);
  }
  for (auto& r : later) STUB_POISON(r.first, r.second);
}

void run(Stream*, Op& op) {
  switch (op.kind) {
    case OP_COPY:
    case OP_SET:
      run_transfer(op);
      break;
    case OP_WAIT:
      drain(op.ws, op.wseq);
      break;
    case OP_KERNEL:
      for (int i = 0; i < op.gather_count; ++i) op.gather_out[i] = 3;  // every instance done
      break;
  }
}

void enqueue(Stream* s, Op op) {
  op.depth = backtrace(op.where, 12);
  if (s->cap) {
    s->cap->ops.push_back(op);
    return;
  }
  op.id = ++g_next_id;
  if (op.host_dst) STUB_POISON(op.dst, op.n);
  s->q.push_back(op);
}

hipError_t copy_async(void* dst, const void* src, size_t n, hipMemcpyKind kind, hipStream_t stream) {
  if (fail_now()) return hipErrorInvalidValue;
  if (!kind_ok(dst, src, n, kind)) return hipErrorInvalidValue;
  if (!n) return hipSuccess;
  Op op{OP_COPY};
  op.dst = dst;
  op.src = src;
  op.n = n;
  op.host_dst = kind == hipMemcpyDeviceToHost || kind == hipMemcpyHostToHost;
  if (kind == hipMemcpyHostToDevice || kind == hipMemcpyHostToHost) {
    // a source that an earlier queued copy has yet to write has no value to check
    bool produced = false;
    for_pending_dst(src, n, [&](Op&) { produced = true; });
    op.check = !produced;
    if (op.check) op.sum = checksum(src, n);
  }
  enqueue(S(stream), op);
  return hipSuccess;
}

}  // namespace

extern "C" {

// ---- test controls ----
void stub_fail_at(int64_t n) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  g_calls = 0;
  g_fail_at = n;
}
int64_t stub_calls() {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  return g_calls;
}
int64_t stub_problems() {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  return g_problems;
}
// Queued operations on all streams (0 once everything has been waited for).
int64_t stub_pending() {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  int64_t p = (int64_t)g_null.q.size();
  for (Stream* s : g_streams) p += (int64_t)s->q.size();
  return p;
}
// Device allocations still held.
int64_t stub_live_allocations() {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  return (int64_t)(g_dev.size() + g_pinned.size());
}
void stub_drain_all() {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  drain_all();
}

// ---- registration (what hipcc's host pass emits) ----
void** __hipRegisterFatBinary(const void*) {
  static void* handle = nullptr;
  return &handle;
}
void __hipUnregisterFatBinary(void**) {}
void __hipRegisterFunction(void**, const void* hostFunction, char*, const char* deviceName, unsigned int,
                           uint3*, uint3*, dim3*, dim3*, int*) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  g_kernels[hostFunction] = deviceName ? deviceName : "";
}
void __hipRegisterVar(void**, void* var, char*, char*, int, size_t size, int, int) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  g_vars[var] = size;
}
hipError_t __hipPushCallConfiguration(dim3 grid, dim3 block, size_t shmem, hipStream_t stream) {
  t_grid = grid;
  t_block = block;
  t_shmem = shmem;
  t_cfg_stream = stream;
  return hipSuccess;
}
hipError_t __hipPopCallConfiguration(dim3* grid, dim3* block, size_t* shmem, hipStream_t* stream) {
  *grid = t_grid;
  *block = t_block;
  *shmem = t_shmem;
  *stream = t_cfg_stream;
  return hipSuccess;
}

hipError_t hipLaunchKernel(const void* f, dim3 grid, dim3 block, void** args, size_t, hipStream_t stream) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  if (fail_now()) {
    t_last = hipErrorLaunchFailure;
    return hipErrorLaunchFailure;
  }
  auto it = g_kernels.find(f);
  if (it == g_kernels.end()) {
    problem("launch of an unregistered kernel", nullptr);
    return hipErrorInvalidDeviceFunction;
  }
  if (grid.x == 0 || grid.y == 0 || grid.z == 0 || block.x == 0 || block.x * block.y * block.z > 1024) {
    problem(("launch shape out of range: " + it->second).c_str(), nullptr);
    t_last = hipErrorInvalidConfiguration;
    return hipErrorInvalidConfiguration;
  }
  Op op{OP_KERNEL};
  if (it->second.find("k_gather_phase") != std::string::npos) {
    op.gather_count = *static_cast<int*>(args[1]);
    op.gather_out = *static_cast<int**>(args[2]);
    if (!side_ok(op.gather_out, (size_t)op.gather_count * sizeof(int), true, "phase output")) return hipErrorInvalidValue;
  }
  enqueue(S(stream), op);
  return hipSuccess;
}

hipError_t hipGetLastError(void) {
  const hipError_t e = t_last;
  t_last = hipSuccess;
  return e;
}
hipError_t hipPeekAtLastError(void) { return t_last; }
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "hipSuccess" : "hip_stub error"; }
const char* hipGetErrorName(hipError_t e) { return hipGetErrorString(e); }

hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDeviceCount(int* n) {
  *n = 1;
  return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int) {
  *v = a == hipDeviceAttributeMultiprocessorCount ? 256 : 0;
  return hipSuccess;
}
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, const void*, int, size_t) {
  *n = 2;
  return hipSuccess;
}
hipError_t hipDeviceSynchronize(void) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  drain_all();
  return hipSuccess;
}

// ---- memory ----
hipError_t hipMalloc(void** p, size_t n) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  if (fail_now()) return hipErrorOutOfMemory;
  *p = nullptr;
  if (!n) return hipSuccess;
  void* q = nullptr;
  if (posix_memalign(&q, 256, n)) return hipErrorOutOfMemory;
  memset(q, 0, n);
  g_dev[reinterpret_cast<uintptr_t>(q)] = n;
  *p = q;
  return hipSuccess;
}
hipError_t hipFree(void* p) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  drain_all();
  if (!p) return hipSuccess;
  auto it = g_dev.find(reinterpret_cast<uintptr_t>(p));
  if (it == g_dev.end()) {
    problem("hipFree of a pointer that is not a device allocation", nullptr);
    return hipErrorInvalidValue;
  }
  g_dev.erase(it);
  free(p);
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned int) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  if (fail_now()) return hipErrorOutOfMemory;
  void* q = nullptr;
  if (posix_memalign(&q, 256, n ? n : 1)) return hipErrorOutOfMemory;
  memset(q, 0, n ? n : 1);
  g_pinned[reinterpret_cast<uintptr_t>(q)] = n ? n : 1;
  *p = q;
  return hipSuccess;
}
hipError_t hipHostFree(void* p) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  drain_all();
  if (!p) return hipSuccess;
  auto it = g_pinned.find(reinterpret_cast<uintptr_t>(p));
  if (it == g_pinned.end()) {
    problem("hipHostFree of a pointer that is not a pinned allocation", nullptr);
    return hipErrorInvalidValue;
  }
  g_pinned.erase(it);
  free(p);
  return hipSuccess;
}
hipError_t hipGetSymbolAddress(void** p, const void* symbol) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  auto it = g_vars.find(symbol);
  if (it == g_vars.end()) return hipErrorInvalidSymbol;
  // the host shadow of the variable stands in for its device copy
  g_dev[reinterpret_cast<uintptr_t>(symbol)] = it->second;
  *p = const_cast<void*>(symbol);
  return hipSuccess;
}

hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind kind, hipStream_t s) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  return copy_async(dst, src, n, kind, s);
}
hipError_t hipMemcpy2DAsync(void* dst, size_t dpitch, const void* src, size_t spitch, size_t width, size_t height,
                            hipMemcpyKind kind, hipStream_t s) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  if (fail_now()) return hipErrorInvalidValue;
  for (size_t r = 0; r < height; ++r) {
    const hipError_t e = copy_async(static_cast<char*>(dst) + r * dpitch,
                                    static_cast<const char*>(src) + r * spitch, width, kind, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind kind) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  if (fail_now()) return hipErrorInvalidValue;
  drain(&g_null, g_null.enqueued());
  if (!kind_ok(dst, src, n, kind)) return hipErrorInvalidValue;
  memmove(dst, src, n);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* dst, int value, size_t n, hipStream_t s) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  if (fail_now()) return hipErrorInvalidValue;
  if (!side_ok(dst, n, true, "memset destination")) return hipErrorInvalidValue;
  if (!n) return hipSuccess;
  Op op{OP_SET};
  op.dst = dst;
  op.n = n;
  op.value = value;
  enqueue(S(s), op);
  return hipSuccess;
}
hipError_t hipMemset(void* dst, int value, size_t n) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  if (fail_now()) return hipErrorInvalidValue;
  drain(&g_null, g_null.enqueued());
  if (!side_ok(dst, n, true, "memset destination")) return hipErrorInvalidValue;
  memset(dst, value, n);
  return hipSuccess;
}

// ---- streams and events ----
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  if (fail_now()) return hipErrorOutOfMemory;
  Stream* st = new Stream;
  g_streams.push_back(st);
  *s = reinterpret_cast<hipStream_t>(st);
  return hipSuccess;
}
hipError_t hipStreamCreate(hipStream_t* s) { return hipStreamCreateWithFlags(s, 0); }
hipError_t hipStreamDestroy(hipStream_t s) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  if (!s) return hipErrorInvalidHandle;
  Stream* st = S(s);
  drain(st, st->enqueued());
  st->destroyed = true;  // kept: waits queued elsewhere may still name it
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  if (fail_now()) return hipErrorLaunchFailure;  // the queued work stays queued
  Stream* st = S(s);
  if (st->destroyed) problem("synchronisation of a destroyed stream", nullptr);
  drain(st, st->enqueued());
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  if (fail_now()) return hipErrorOutOfMemory;
  *e = reinterpret_cast<hipEvent_t>(new Event);
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) { return hipEventCreateWithFlags(e, 0); }
hipError_t hipEventDestroy(hipEvent_t e) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  delete reinterpret_cast<Event*>(e);
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  if (fail_now()) return hipErrorInvalidHandle;
  Event* ev = reinterpret_cast<Event*>(e);
  Stream* st = S(s);
  if (st->cap) {
    problem("event recorded during capture", nullptr);
    return hipErrorInvalidValue;
  }
  ev->s = st;
  ev->seq = st->enqueued();
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  if (fail_now()) return hipErrorLaunchFailure;
  Event* ev = reinterpret_cast<Event*>(e);
  if (ev->s) drain(ev->s, ev->seq);
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.0f;
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  if (fail_now()) return hipErrorInvalidHandle;
  Event* ev = reinterpret_cast<Event*>(e);
  if (!ev->s) return hipSuccess;  // never recorded: nothing to wait for
  Op op{OP_WAIT};
  op.ws = ev->s;
  op.wseq = ev->seq;
  enqueue(S(s), op);
  return hipSuccess;
}

// ---- graphs: a captured list of operations, replayed on launch ----
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  if (fail_now()) return hipErrorInvalidValue;
  Stream* st = S(s);
  if (st->cap) return hipErrorIllegalState;
  st->cap = new Graph;
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  Stream* st = S(s);
  if (!st->cap) return hipErrorIllegalState;
  *g = reinterpret_cast<hipGraph_t>(st->cap);
  st->cap = nullptr;
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  if (fail_now()) return hipErrorInvalidValue;
  *x = reinterpret_cast<hipGraphExec_t>(new Graph(*reinterpret_cast<Graph*>(g)));
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  delete reinterpret_cast<Graph*>(g);
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  delete reinterpret_cast<Graph*>(x);
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
  std::lock_guard<std::recursive_mutex> l(g_mu);
  if (fail_now()) return hipErrorLaunchFailure;
  for (const Op& op : reinterpret_cast<Graph*>(x)->ops) enqueue(S(s), op);
  return hipSuccess;
}

}  // extern "C"
