// Batched solver: many independent Split-SPCP instances of uneven shape
// solved together.  Every step of an L-BFGS slot covers the whole batch:
//   direction  (blocks of all instances in one grid, then one block per instance)
//   sweep      (one persistent kernel per tile class, each pulling (instance,
//               row group, chunk) items from its queue; decreasing cost first)
//   finish     (two batched reductions with the line-search step per instance)
//   update     (batched history pass, then one block per instance)
// Per-instance solver states live in device memory and every kernel skips the
// instances that are not in its phase, so converged instances cost nothing but
// the phase test.  A group of slots is captured once in a hipGraph and
// replayed until every instance reports done.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <numeric>
#include <thread>
#include <vector>

#include "../../include/rpca_batch.h"
#include "rpca_internal.h"

namespace {

// Host worker threads (and streams) of the per-instance phases of a batched solve
// (at most; fewer when the host has fewer hardware threads).  Measured on the
// 64-instance batch: 4 workers 686 ms, 8 573 ms, 16 540 ms per solve.
constexpr int BATCH_WORKERS = 16;

// RPCA_BATCH_WORKERS (1..16) in the environment overrides the host's count.
int worker_count() {
  static const int w = [] {
    if (const char* e = getenv("RPCA_BATCH_WORKERS")) {
      const int v = atoi(e);
      if (v >= 1 && v <= BATCH_WORKERS) return v;
    }
    const unsigned hw = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min((unsigned)BATCH_WORKERS, hw ? hw : 1u));
  }();
  return w;
}

// Sweep waves per compute unit that a batch's decomposition aims at (per tile
// class), and the fewest strips a wave of a batched sweep is given.
constexpr int BATCH_WAVES_PER_CU = 16;
constexpr int BATCH_MIN_STRIPS = 4;

__global__ void k_gather_phase(SolverState* const* st, int count, int* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = st[i]->phase;
}

template <typename T>
bool dalloc(T** p, size_t count) {
  void* q = nullptr;
  if (hipMalloc(&q, (count ? count : 1) * sizeof(T)) != hipSuccess) return false;
  *p = static_cast<T*>(q);
  return true;
}

void dfree(void* p) {
  if (p) (void)hipFree(p);
}

}  // namespace

struct rpca_batch {
  int count = 0;
  std::vector<rpca_ctx*> ctx;
  std::vector<int> waves;  // sweep wave target per instance
  bool masked = false;
  // decomposition (fixed by the shapes): sweep items grouped by tile class
  struct SweepClass {
    int kb, tmax;
    int begin, count;  // range in d_items
    int lds;           // dynamic LDS floats (largest instance of the class)
    int grid[2];       // persistent workgroups, FP32 / BF16
  };
  std::vector<SweepClass> classes;
  int nitems = 0, lds_max = 0;
  int tot_fin1 = 0, tot_fin2 = 0, tot_lb = 0;
  std::vector<int> off_fin1, off_fin2, off_lb;
  SweepItem* d_items = nullptr;
  int* d_off_fin1 = nullptr;
  int* d_off_fin2 = nullptr;
  int* d_off_lb = nullptr;
  unsigned* d_head = nullptr;
  // argument tables (rewritten by every call: they carry the X pointers)
  SweepArgs* d_sa_loop = nullptr;
  SweepArgs* d_sa_eval = nullptr;
  FinishArgs* d_fa_loop = nullptr;
  FinishArgs* d_fa_eval = nullptr;
  LbfgsArgs* d_lu = nullptr;
  LbfgsArgs* d_ld = nullptr;
  SolverState** d_states = nullptr;
  int* d_phase = nullptr;
  int* h_phase = nullptr;  // pinned
  // the batch runs on its own stream, ordered after / before the caller's by events
  hipStream_t stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // per-instance host-driven phases (rSVD start, certificates: each with its own
  // host synchronisations) run on worker threads, one stream each, ordered
  // after / before the batch stream by events
  hipStream_t aux[BATCH_WORKERS] = {};
  hipEvent_t ev_aux[BATCH_WORKERS] = {};
  // captured slot groups, keyed by (bf16, mem, slots)
  struct Graph {
    bool bf16;
    int mem, slots;
    hipGraphExec_t exec;
  };
  std::vector<Graph> graphs;
  int sweep_grid[2] = {0, 0};  // persistent grid for FP32 / BF16
  bool use_graphs = true;
};

namespace {

void destroy_batch(rpca_batch* b) {
  for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.exec);
  for (rpca_ctx* c : b->ctx)
    if (c) rpca_destroy(c);
  dfree(b->d_items);
  dfree(b->d_off_fin1);
  dfree(b->d_off_fin2);
  dfree(b->d_off_lb);
  dfree(b->d_head);
  dfree(b->d_sa_loop);
  dfree(b->d_sa_eval);
  dfree(b->d_fa_loop);
  dfree(b->d_fa_eval);
  dfree(b->d_lu);
  dfree(b->d_ld);
  dfree(b->d_states);
  dfree(b->d_phase);
  rpca::host_free(b->h_phase);
  for (int t = 0; t < BATCH_WORKERS; ++t) {
    if (b->ev_aux[t]) (void)hipEventDestroy(b->ev_aux[t]);
    if (b->aux[t]) (void)hipStreamDestroy(b->aux[t]);
  }
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

// Upload the argument tables (synchronous: the host vectors are the caller's temporaries).
hipError_t upload_tables(rpca_batch* b, const std::vector<SweepArgs>& sl, const std::vector<SweepArgs>& se,
                         const std::vector<FinishArgs>& fl, const std::vector<FinishArgs>& fe,
                         const std::vector<LbfgsArgs>& lu, const std::vector<LbfgsArgs>& ld) {
  const int n = b->count;
  hipStream_t s = b->stream;
  // a failed call leaves the earlier copies in flight from the caller's vectors:
  // wait for them before returning
  auto fail = [&](hipError_t e) {
    (void)hipStreamSynchronize(s);
    return e;
  };
  hipError_t e;
  if ((e = hipMemcpyAsync(b->d_sa_loop, sl.data(), n * sizeof(SweepArgs), hipMemcpyHostToDevice, s))) return fail(e);
  if ((e = hipMemcpyAsync(b->d_sa_eval, se.data(), n * sizeof(SweepArgs), hipMemcpyHostToDevice, s))) return fail(e);
  if ((e = hipMemcpyAsync(b->d_fa_loop, fl.data(), n * sizeof(FinishArgs), hipMemcpyHostToDevice, s))) return fail(e);
  if ((e = hipMemcpyAsync(b->d_fa_eval, fe.data(), n * sizeof(FinishArgs), hipMemcpyHostToDevice, s))) return fail(e);
  if ((e = hipMemcpyAsync(b->d_lu, lu.data(), n * sizeof(LbfgsArgs), hipMemcpyHostToDevice, s))) return fail(e);
  if ((e = hipMemcpyAsync(b->d_ld, ld.data(), n * sizeof(LbfgsArgs), hipMemcpyHostToDevice, s))) return fail(e);
  return hipStreamSynchronize(s);
}

// One batched objective/gradient pass (plain: at x[0] into st->f and g[0]; trial:
// solver slot): one persistent sweep per tile class, then the batched reductions.
hipError_t batched_objgrad(rpca_batch* b, bool trial, bool bf16) {
  hipStream_t s = b->stream;
  const SweepArgs* args = trial ? b->d_sa_loop : b->d_sa_eval;
  for (size_t c = 0; c < b->classes.size(); ++c) {
    const auto& cl = b->classes[c];
    const hipError_t e = rpca::launch_sweep_batch(cl.kb, cl.tmax, args, b->d_items + cl.begin, cl.count,
                                                  b->d_head + c, cl.grid[bf16 ? 1 : 0], cl.lds, b->masked, trial,
                                                  bf16, s);
    if (e != hipSuccess) return e;
  }
  return rpca::launch_finish_batch(trial ? b->d_fa_loop : b->d_fa_eval, b->d_off_fin1, b->tot_fin1,
                                   b->d_off_fin2, b->tot_fin2, b->count, b->d_head, (int)b->classes.size(), trial,
                                   s);
}

// One batched solver slot; the direction pass's own finish (states entering
// PH_DIRECTION only) runs in the first slot of a group.
hipError_t batched_slot(rpca_batch* b, int mem, bool bf16, bool first) {
  hipStream_t s = b->stream;
  hipError_t e = rpca::launch_lbfgs_direction_batch(b->d_ld, b->d_off_lb, b->count, b->tot_lb, mem, s, first);
  if (e != hipSuccess) return e;
  if ((e = batched_objgrad(b, true, bf16)) != hipSuccess) return e;
  return rpca::launch_lbfgs_update_batch(b->d_lu, b->d_off_lb, b->count, b->tot_lb, mem, s);
}

// The captured group of `slots` solver slots (built on first use).
hipError_t slot_graph(rpca_batch* b, int mem, bool bf16, int slots, hipGraphExec_t* out) {
  for (auto& g : b->graphs)
    if (g.bf16 == bf16 && g.mem == mem && g.slots == slots) {
      *out = g.exec;
      return hipSuccess;
    }
  hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t le = hipSuccess;
  for (int q = 0; q < slots && le == hipSuccess; ++q) le = batched_slot(b, mem, bf16, q == 0);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(b->stream, &graph);
  if (le != hipSuccess || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return le != hipSuccess ? le : e;
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return e;
  b->graphs.push_back({bf16, mem, slots, exec});
  *out = exec;
  return hipSuccess;
}

// Run slot groups until every instance is done.
int batched_run(rpca_batch* b, const rpca_opts& o, bool bf16, bool use_graph) {
  const int slots = o.slots_per_sync > 0 ? o.slots_per_sync : 16;
  hipGraphExec_t exec = nullptr;
  if (use_graph && slot_graph(b, o.mem, bf16, slots, &exec) != hipSuccess) return RPCA_EHIP;
  const int nb = (b->count + 255) / 256;
  for (int guard = 0; guard < 1000000; ++guard) {
    if (use_graph) {
      if (hipGraphLaunch(exec, b->stream) != hipSuccess) return RPCA_EHIP;
    } else {
      for (int q = 0; q < slots; ++q)
        if (batched_slot(b, o.mem, bf16, q == 0) != hipSuccess) return RPCA_EHIP;
    }
    hipLaunchKernelGGL(k_gather_phase, dim3(nb), dim3(256), 0, b->stream, b->d_states, b->count, b->d_phase);
    if (hipMemcpyAsync(b->h_phase, b->d_phase, b->count * sizeof(int), hipMemcpyDeviceToHost, b->stream) !=
            hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess)
      return RPCA_EHIP;
    bool all = true;
    for (int i = 0; i < b->count && all; ++i) all = b->h_phase[i] == PH_DONE;
    if (all) return RPCA_OK;
  }
  return RPCA_OK;
}


// Run fn(i, stream) for every instance i with sel[i] on the worker threads
// (instance i on worker i % worker_count(), in increasing i), each worker on its
// own stream ordered after the batch stream; the batch stream is then ordered
// after every worker's work.  Returns the first error.
template <typename Fn>
int on_workers(rpca_batch* b, const std::vector<char>& sel, Fn fn) {
  if (hipEventRecord(b->ev_in, b->stream) != hipSuccess) return RPCA_EHIP;
  const int nw = worker_count();
  int rc[BATCH_WORKERS] = {};
  auto work = [&](int t) {
    if (hipStreamWaitEvent(b->aux[t], b->ev_in, 0) != hipSuccess) {
      rc[t] = RPCA_EHIP;
      return;
    }
    for (int i = t; i < b->count; i += nw) {
      if (!sel[i]) continue;
      const int r = fn(i, b->aux[t]);
      if (r < 0) {
        rc[t] = r;
        return;
      }
    }
    if (hipEventRecord(b->ev_aux[t], b->aux[t]) != hipSuccess) rc[t] = RPCA_EHIP;
  };
  std::vector<std::thread> th;
  for (int t = 1; t < nw; ++t) th.emplace_back(work, t);
  work(0);
  for (auto& x : th) x.join();
  for (int t = 0; t < nw; ++t)
    if (rc[t]) return rc[t];
  for (int t = 0; t < nw; ++t)
    if (hipStreamWaitEvent(b->stream, b->ev_aux[t], 0) != hipSuccess) return RPCA_EHIP;
  return RPCA_OK;
}

// Solver cycles over the instances in `start` (the others stay done): each
// restarts from its plain iterate with its own gradient tolerance and
// iteration limit; in preconditioned variables it runs cycles of
// o.precond_cycle iterations, each with a fresh preconditioner and an empty
// memory, while it keeps stopping at a cycle's cap below its limit.  Ends
// with every instance's x[cur] plain and its host state current.
int batch_cycles(rpca_batch* b, const float* const* X, const rpca_opts& o, bool bf16,
                 const std::vector<double>& gtol, double ftol, const std::vector<int>& limit,
                 const std::vector<char>& start) {
  hipStream_t s = b->stream;
  const int n = b->count;
  std::vector<rpca::InstanceArgs> ia(n);
  int rc;
  for (int cyc = 0;; ++cyc) {
    std::vector<char> active(n, 0);
    int nact = 0;
    for (int i = 0; i < n; ++i) {
      const SolverState* h = rpca::ctx_state_host(b->ctx[i]);
      if (cyc == 0) active[i] = start[i];
      else active[i] = o.precond && h->stop == STOP_MAXITER && h->iter < limit[i];
      nact += active[i];
    }
    if (!nact) break;
    // fresh preconditioners and restarted states (host-synchronising steps) on the workers
    if ((rc = on_workers(b, active, [&](int i, hipStream_t ws) -> int {
           rpca_ctx* c = b->ctx[i];
           const SolverState* h = rpca::ctx_state_host(c);
           int cap = limit[i];
           int r;
           if (o.precond) {
             if ((r = rpca::precond_refresh(c, h->cur, ws))) return r;
             cap = (limit[i] - h->iter > o.precond_cycle) ? h->iter + o.precond_cycle : limit[i];
           }
           return rpca::restart_state(c, gtol[i], ftol, cap, o.precond != 0, ws);
         })))
      return rc;
    // argument tables at each instance's current iterate and variables
    std::vector<SweepArgs> sl(n), se(n);
    std::vector<FinishArgs> fl(n), fe(n);
    std::vector<LbfgsArgs> lu(n), ld(n);
    for (int i = 0; i < n; ++i) {
      rpca::instance_args(b->ctx[i], X[i], rpca::ctx_state_host(b->ctx[i])->cur, &ia[i]);
      sl[i] = ia[i].sa_loop;
      se[i] = ia[i].sa_eval;
      fl[i] = ia[i].fa_loop;
      fe[i] = ia[i].fa_eval;
      if (!active[i]) fe[i].f_out = nullptr;  // a finished instance keeps its f
      lu[i] = ia[i].lu;
      ld[i] = ia[i].ld;
    }
    if (upload_tables(b, sl, se, fl, fe, lu, ld) != hipSuccess) return RPCA_EHIP;
    if (batched_objgrad(b, false, bf16) != hipSuccess) return RPCA_EHIP;
    if ((rc = batched_run(b, o, bf16, b->use_graphs))) return rc;
    for (int i = 0; i < n; ++i)
      if (hipMemcpyAsync(ia[i].state_host, ia[i].state_dev, sizeof(SolverState), hipMemcpyDeviceToHost, s) !=
          hipSuccess)
        return RPCA_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return RPCA_EHIP;
  }
  for (int i = 0; i < n; ++i) {
    rpca_ctx* c = b->ctx[i];
    if ((rc = rpca::precond_to_plain(c, rpca::ctx_state_host(c)->cur, s))) return rc;
  }
  return RPCA_OK;
}
}  // namespace

extern "C" {

int rpca_batch_create(int32_t count, const int64_t* m, const int64_t* n, const int32_t* k, const double* lam_s,
                      const double* lam_l, rpca_batch** out) {
  if (!out) return RPCA_EINVAL;
  *out = nullptr;
  if (count < 1 || count > 65536 || !m || !n || !k || !lam_s || !lam_l) return RPCA_EINVAL;
  for (int i = 0; i < count; ++i)
    if (m[i] < 1 || n[i] < 1 || k[i] < 1 || k[i] > 32 || k[i] > m[i] || k[i] > n[i] || !(lam_s[i] > 0) ||
        !(lam_l[i] > 0) || !isfinite(lam_s[i]) || !isfinite(lam_l[i]))
      return RPCA_EINVAL;
  rpca_batch* b = new rpca_batch;
  b->count = count;
  b->ctx.assign(count, nullptr);
  b->waves.assign(count, 0);
  // The tile classes' persistent sweeps run one after another, so each class
  // shares one chip's worth of waves (BATCH_WAVES_PER_CU per CU) over its
  // instances in proportion to their work: the queue holds a few items per
  // resident workgroup for balance, and no wave gets fewer than BATCH_MIN_STRIPS
  // strips (each item carries the staging of a V chunk and a partial G^T U
  // write, which short items cannot amortise).
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  std::vector<double> icost(count);
  std::vector<int> icls(count);
  std::vector<double> class_cost(64 * 3, 0.0);
  for (int i = 0; i < count; ++i) {
    const int kb = (k[i] + 15) / 16;
    int rg0, spw0, cw0, nch0;
    rpca::sweep_blocks_for(m[i], n[i], k[i], &rg0, &spw0, &cw0, &nch0, 1024);
    const int tm = rpca::sweep_tmax_class(kb, (int)((std::min<int64_t>(n[i], cw0) + 15) / 16));
    icls[i] = kb * 64 + tm;
    icost[i] = (double)m[i] * (double)n[i] * (1.0 + 0.6 * (kb - 1));
    class_cost[icls[i]] += icost[i];
  }
  for (int i = 0; i < count; ++i) {
    const int64_t nstrips = (m[i] + 15) / 16;
    // the tuned entry of the instance's (k, n) bucket scales its share and its cap: an
    // entry that spreads one sweep over more waves than the default 1024 gives the
    // instance more waves here too, with proportionally fewer strips each
    const double tuned = rpca::tune_get(k[i], n[i]).target_waves / 1024.0;
    const int64_t cap = std::max<int64_t>(4, (int64_t)(tuned * (double)nstrips) / BATCH_MIN_STRIPS);
    const int64_t share = llround(BATCH_WAVES_PER_CU * (double)cus * tuned * icost[i] / class_cost[icls[i]]);
    b->waves[i] = (int)std::max<int64_t>(4, std::min<int64_t>(share, cap));
    const int rc = rpca::create_ctx(m[i], n[i], k[i], lam_s[i], lam_l[i], nullptr, b->waves[i], &b->ctx[i]);
    if (rc != RPCA_OK) {
      destroy_batch(b);
      return rc;
    }
  }
  // decomposition: sweep items (sorted by decreasing cost) and block offsets
  std::vector<rpca::InstanceArgs> ia(count);
  std::vector<SweepItem> items;
  std::vector<double> cost;
  b->off_fin1.assign(count + 1, 0);
  b->off_fin2.assign(count + 1, 0);
  b->off_lb.assign(count + 1, 0);
  for (int i = 0; i < count; ++i) {
    rpca::instance_args(b->ctx[i], nullptr, 0, &ia[i]);
    const int kb = (k[i] + 15) / 16;
    const int64_t nstrips = (m[i] + 15) / 16;
    const int tmax = rpca::sweep_tmax_class(kb, (int)((std::min<int64_t>(n[i], ia[i].chunk_w) + 15) / 16));
    for (int rg = 0; rg < ia[i].row_groups; ++rg)
      for (int ch = 0; ch < ia[i].nchunks; ++ch) {
        items.push_back({i, rg, ch, kb, tmax});
        const int64_t s0 = (int64_t)rg * nstrips / ia[i].row_groups;
        const int64_t s1 = ((int64_t)rg + 1) * nstrips / ia[i].row_groups;
        const int64_t c0 = (int64_t)ch * ia[i].chunk_w;
        const int64_t cols = std::min<int64_t>(ia[i].chunk_w, n[i] - c0);
        cost.push_back((double)std::max<int64_t>(s1 - s0, 0) * (double)cols * (1.0 + 0.6 * (kb - 1)));
      }
    b->off_fin1[i + 1] = b->off_fin1[i] + ia[i].fin1_blocks;
    b->off_fin2[i + 1] = b->off_fin2[i] + ia[i].fin2_blocks;
    b->off_lb[i + 1] = b->off_lb[i] + ia[i].lb_blocks;
  }
  // group by tile class, then decreasing cost within a class
  auto cls = [](const SweepItem& it) { return it.kb * 64 + it.tmax; };
  std::vector<int> ord(items.size());
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
    if (cls(items[x]) != cls(items[y])) return cls(items[x]) < cls(items[y]);
    return cost[x] > cost[y];
  });
  std::vector<SweepItem> sorted(items.size());
  for (size_t j = 0; j < ord.size(); ++j) sorted[j] = items[ord[j]];
  for (size_t j = 0; j < sorted.size(); ++j) {
    if (b->classes.empty() || b->classes.back().kb != sorted[j].kb || b->classes.back().tmax != sorted[j].tmax)
      b->classes.push_back({sorted[j].kb, sorted[j].tmax, (int)j, 0, 0, {0, 0}});
    auto& cl = b->classes.back();
    cl.count += 1;
    const int i = sorted[j].inst;
    const int cwp = (int)((std::min<int64_t>(n[i], ia[i].chunk_w) + 15) / 16) * 16;
    cl.lds = std::max(cl.lds, rpca::sweep_lds_floats(sorted[j].kb, k[i], cwp));
  }
  b->nitems = (int)sorted.size();
  b->tot_fin1 = b->off_fin1[count];
  b->tot_fin2 = b->off_fin2[count];
  b->tot_lb = b->off_lb[count];
  std::vector<SolverState*> states(count);
  for (int i = 0; i < count; ++i) states[i] = ia[i].state_dev;
  bool ok = dalloc(&b->d_items, sorted.size()) && dalloc(&b->d_off_fin1, count + 1) &&
            dalloc(&b->d_off_fin2, count + 1) && dalloc(&b->d_off_lb, count + 1) && dalloc(&b->d_head, b->classes.size()) &&
            dalloc(&b->d_sa_loop, count) && dalloc(&b->d_sa_eval, count) && dalloc(&b->d_fa_loop, count) &&
            dalloc(&b->d_fa_eval, count) && dalloc(&b->d_lu, count) && dalloc(&b->d_ld, count) &&
            dalloc(&b->d_states, count) && dalloc(&b->d_phase, count) &&
            hipHostMalloc((void**)&b->h_phase, count * sizeof(int), 0) == hipSuccess;
  if (!ok) {
    destroy_batch(b);
    return RPCA_ENOMEM;
  }
  ok = hipMemcpy(b->d_items, sorted.data(), sorted.size() * sizeof(SweepItem), hipMemcpyHostToDevice) ==
           hipSuccess &&
       hipMemcpy(b->d_off_fin1, b->off_fin1.data(), (count + 1) * sizeof(int), hipMemcpyHostToDevice) ==
           hipSuccess &&
       hipMemcpy(b->d_off_fin2, b->off_fin2.data(), (count + 1) * sizeof(int), hipMemcpyHostToDevice) ==
           hipSuccess &&
       hipMemcpy(b->d_off_lb, b->off_lb.data(), (count + 1) * sizeof(int), hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(b->d_states, states.data(), count * sizeof(SolverState*), hipMemcpyHostToDevice) ==
           hipSuccess &&
       hipMemset(b->d_head, 0, b->classes.size() * sizeof(unsigned)) == hipSuccess &&
       hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) == hipSuccess &&
       hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) == hipSuccess &&
       hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) == hipSuccess;
  for (int t = 0; t < BATCH_WORKERS && ok; ++t)
    ok = hipStreamCreateWithFlags(&b->aux[t], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&b->ev_aux[t], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    destroy_batch(b);
    return RPCA_EHIP;
  }
  for (auto& cl : b->classes) {
    cl.grid[0] = std::min(cl.count, rpca::sweep_batch_grid(cl.kb, cl.tmax, cl.lds, false, true, false));
    cl.grid[1] = std::min(cl.count, rpca::sweep_batch_grid(cl.kb, cl.tmax, cl.lds, false, true, true));
    b->sweep_grid[0] += cl.grid[0];
    b->sweep_grid[1] += cl.grid[1];
    b->lds_max = std::max(b->lds_max, cl.lds);
  }
  *out = b;
  return RPCA_OK;
}

int rpca_batch_objgrad(rpca_batch* b, const float* const* X, const float* const* U, const float* const* V,
                       double* const* f, float* const* gU, float* const* gV, int32_t precision, void* stream) {
  if (!b || !X || !U || !V || !f || !gU || !gV) return RPCA_EINVAL;
  if (precision != RPCA_PREC_FP32 && precision != RPCA_PREC_BF16) return RPCA_EINVAL;
  for (int i = 0; i < b->count; ++i)
    if (!X[i] || !U[i] || !V[i] || !f[i] || !gU[i] || !gV[i]) return RPCA_EINVAL;
  hipStream_t cs = (hipStream_t)stream;
  if (hipEventRecord(b->ev_in, cs) != hipSuccess || hipStreamWaitEvent(b->stream, b->ev_in, 0) != hipSuccess)
    return RPCA_EHIP;
  // plain evaluations at the caller's points: point the eval tables at them
  std::vector<rpca::InstanceArgs> ia(b->count);
  std::vector<SweepArgs> se(b->count);
  std::vector<FinishArgs> fe(b->count);
  for (int i = 0; i < b->count; ++i) {
    rpca::instance_args(b->ctx[i], X[i], 0, &ia[i]);
    SweepArgs& sa = ia[i].sa_eval;
    FinishArgs& fa = ia[i].fa_eval;
    sa.U[0] = sa.U[1] = U[i];
    sa.V[0] = sa.V[1] = V[i];
    sa.gU[0] = sa.gU[1] = gU[i];
    fa.U[0] = fa.U[1] = U[i];
    fa.V[0] = fa.V[1] = V[i];
    fa.gU[0] = fa.gU[1] = gU[i];
    fa.gV[0] = fa.gV[1] = gV[i];
    fa.f_out = f[i];
    se[i] = sa;
    fe[i] = fa;
  }
  if (hipMemcpyAsync(b->d_sa_eval, se.data(), b->count * sizeof(SweepArgs), hipMemcpyHostToDevice, b->stream) !=
          hipSuccess ||
      hipMemcpyAsync(b->d_fa_eval, fe.data(), b->count * sizeof(FinishArgs), hipMemcpyHostToDevice,
                     b->stream) != hipSuccess ||
      hipStreamSynchronize(b->stream) != hipSuccess) {
    (void)hipStreamSynchronize(b->stream);  // se, fe are read until the copies end
    return RPCA_EHIP;
  }
  if (batched_objgrad(b, false, precision == RPCA_PREC_BF16) != hipSuccess) return RPCA_EHIP;
  if (hipEventRecord(b->ev_out, b->stream) != hipSuccess || hipStreamWaitEvent(cs, b->ev_out, 0) != hipSuccess)
    return RPCA_EHIP;
  return RPCA_OK;
}

int rpca_batch_solve(rpca_batch* b, const float* const* X, float* const* U, float* const* V,
                     const rpca_opts* opts, rpca_info* info, void* stream) {
  if (!b || !X || !U || !V) return RPCA_EINVAL;
  for (int i = 0; i < b->count; ++i)
    if (!X[i] || !U[i] || !V[i]) return RPCA_EINVAL;
  rpca_opts o;
  if (opts) o = *opts;
  else rpca_default_opts(&o);
  if (!rpca::valid_opts(o)) return RPCA_EINVAL;
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t cs = (hipStream_t)stream;
  hipStream_t s = b->stream;
  if (hipEventRecord(b->ev_in, cs) != hipSuccess || hipStreamWaitEvent(s, b->ev_in, 0) != hipSuccess)
    return RPCA_EHIP;
  rpca::SolvePhase phases[2];
  const int nph = rpca::solve_phases(o, phases);
  const int n = b->count;
  int rc;
  std::vector<char> all(n, 1);
  if ((rc = on_workers(b, all, [&](int i, hipStream_t ws) -> int {
         return rpca::solve_setup(b->ctx[i], X[i], U[i], V[i], o, phases[0].gtol, ws);
       })))
    return rc;
  std::vector<int> iters_bf16(n, 0), limit(n, o.max_iter);
  std::vector<char> open(n, 1);
  bool final_bf16 = phases[0].bf16;
  for (int ph = 0; ph < nph; ++ph) {
    std::vector<double> gt(n, phases[ph].gtol);
    if ((rc = batch_cycles(b, X, o, phases[ph].bf16, gt, o.ftol, limit, open))) return rc;
    for (int i = 0; i < n; ++i) {
      const SolverState* h = rpca::ctx_state_host(b->ctx[i]);
      if (ph == 0 && phases[0].bf16) iters_bf16[i] = h->iter;
      if (h->stop == STOP_NONFINITE || h->stop == STOP_MAXITER) open[i] = 0;
    }
    final_bf16 = phases[ph].bf16;
  }
  // Certification rounds, batched: every instance still open takes a
  // certificate (on the workers); those not certified yet continue together
  // for one round.
  std::vector<int> rounds(n, 0), certified(n, 0);
  std::vector<double> gap(n, NAN), gtol(n, phases[nph - 1].gtol);
  double round_ftol = o.ftol;
  int round_budget = 0;
  {
    double g0 = 1.0;
    round_budget = rpca::round_tolerances(o, &g0, &round_ftol);
  }
  open.assign(n, 1);
  for (;;) {
    std::vector<char> again(n, 0);
    if ((rc = on_workers(b, open, [&](int i, hipStream_t ws) -> int {
           rpca_ctx* c = b->ctx[i];
           int r = rpca::copy_out(c, U[i], V[i], ws);
           if (r) return r;
           const int stop = rpca::ctx_state_host(c)->stop;
           if (!o.certify || stop == STOP_NONFINITE) return RPCA_OK;
           rpca_cert cert;
           r = rpca::certificate_impl(c, X[i], U[i], V[i], &cert, o.cert_tol, ws);
           if (r < 0) return r;
           ++rounds[i];
           gap[i] = cert.rel_gap;
           certified[i] = gap[i] <= o.cert_tol;
           if (certified[i] || stop == STOP_MAXITER || rounds[i] >= rpca::CERT_ROUNDS) return RPCA_OK;
           double ft;
           rpca::round_tolerances(o, &gtol[i], &ft);
           const int it = rpca::ctx_state_host(c)->iter;
           limit[i] = (round_budget > 0 && o.max_iter - it > round_budget) ? it + round_budget : o.max_iter;
           again[i] = 1;
           return RPCA_OK;
         })))
      return rc;
    open = again;
    int nagain = 0;
    for (int i = 0; i < n; ++i) nagain += again[i];
    if (!nagain) break;
    if ((rc = batch_cycles(b, X, o, final_bf16, gtol, round_ftol, limit, again))) return rc;
    for (int i = 0; i < n; ++i)
      if (again[i]) rpca::end_round(b->ctx[i], o);
  }
  if (hipStreamSynchronize(s) != hipSuccess) return RPCA_EHIP;
  int worst = RPCA_OK;
  for (int i = 0; i < n; ++i) {
    rc = rpca::finish_status(b->ctx[i], o, certified[i], gap[i], rounds[i], iters_bf16[i], t0,
                             info ? &info[i] : nullptr);
    if (rc > worst) worst = rc;
  }
  if (hipEventRecord(b->ev_out, s) != hipSuccess || hipStreamWaitEvent(cs, b->ev_out, 0) != hipSuccess)
    return RPCA_EHIP;
  return worst;
}

int rpca_batch_set_graphs(rpca_batch* b, int32_t on) {
  if (!b) return RPCA_EINVAL;
  b->use_graphs = on != 0;
  return RPCA_OK;
}

int rpca_batch_info(rpca_batch* b, rpca_batch_layout* out) {
  if (!b || !out) return RPCA_EINVAL;
  out->count = b->count;
  out->sweep_items = b->nitems;
  out->sweep_grid_fp32 = b->sweep_grid[0];
  out->sweep_grid_bf16 = b->sweep_grid[1];
  out->lds_bytes = b->lds_max * 4;
  out->graphs = (int32_t)b->graphs.size();
  out->sweep_classes = (int32_t)b->classes.size();
  return RPCA_OK;
}

int rpca_batch_instance_waves(rpca_batch* b, int32_t i, int32_t* waves) {
  if (!b || !waves || i < 0 || i >= b->count) return RPCA_EINVAL;
  *waves = b->waves[i];
  return RPCA_OK;
}

void rpca_batch_destroy(rpca_batch* b) {
  if (b) destroy_batch(b);
}

}  // extern "C"
