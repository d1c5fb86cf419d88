// fock_apply_batched: all cells of a plan in one launch, replayed from a
// captured hipGraph while the caller passes the same buffers. Three forms: one
// persistent kernel over all cells (0), each cell's own fused kernel on a
// forked stream (1), or those kernels one after another (2); the tuner
// measures all three.
//
// Per call: one complex64 shadow per orbital array (and per distinct target
// array), a reset of the sub-queue counters (a one-thread kernel, no memset
// node), and the persistent kernel over per-XCD sub-queues of (cell, target)
// entries ordered by decreasing cost. With a tuning cache, the first call
// measures the number of persistent workgroups per CU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "../../include/fockmi.h"
#include "plan.hpp"

using namespace fockmi;

namespace fockmi {

extern thread_local std::string g_last_error;

void BatchState::reset_graph() {
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  exec = nullptr;
  graph = nullptr;
  ready = false;
}

void BatchState::release() {
  reset_graph();
  for (int i = 0; i < kMaxBatchCells; ++i) {
    shadow_u[i].release();
    shadow_x[i].release();
    comp[i].release();
  }
  accs.release();
  queue.release();
  counters.release();
  if (cap) (void)hipStreamDestroy(cap);
  cap = nullptr;
  for (int i = 0; i < kMaxBatchCells; ++i) {
    if (side[i]) (void)hipStreamDestroy(side[i]);
    if (join[i]) (void)hipEventDestroy(join[i]);
    side[i] = nullptr;
    join[i] = nullptr;
  }
  if (fork) (void)hipEventDestroy(fork);
  fork = nullptr;
  key.clear();
}

// cost of one target of a cell: pairs x nominal flops of one pair
static double item_cost(const Cell& c) {
  const double nr = (double)c.nr;
  return (double)c.nk * c.nb * (10.0 * nr * std::log2(nr) + 16.0 * nr);
}

fock_status Plan::run_batched(const void* const* u, const void* const* phi, const int* nphi, void* const* vphi,
                              hipStream_t st) {
  const int nc = (int)cells.size();
  BatchState& B = bstate;
  // the cells in decreasing cost
  std::vector<int> by_cost(nc);
  std::iota(by_cost.begin(), by_cost.end(), 0);
  std::stable_sort(by_cost.begin(), by_cost.end(),
                   [&](int x, int y) { return item_cost(cells[x]) * cells[x].nk > item_cost(cells[y]) * cells[y].nk; });
  // form 1: every cell's fused kernel (its grid form, one workgroup per target)
  // on its own stream, so that the cells' last rounds may overlap; form 2: the
  // same kernels one after another on the caller's stream, costliest first
  auto launch_cells = [&](hipStream_t q, bool forked) -> fock_status {
    hipError_t ee;
    if (forked && (ee = hipEventRecord(B.fork, q)) != hipSuccess) return hip_fail(ee, "fork");
    for (int ci : by_cost) {
      FusedArgs a = B.args.cells[ci];
      a.xcd_map = 1;
      hipStream_t cs = forked ? B.side[ci] : q;
      if (forked && (ee = hipStreamWaitEvent(cs, B.fork, 0)) != hipSuccess) return hip_fail(ee, "fork");
      if ((ee = launch_fused_apply(a.n, a, cs, 0)) != hipSuccess) return hip_fail(ee, "cell kernel");
      if (forked && (ee = hipEventRecord(B.join[ci], cs)) != hipSuccess) return hip_fail(ee, "join");
    }
    for (int ci = 0; forked && ci < nc; ++ci)
      if ((ee = hipStreamWaitEvent(q, B.join[ci], 0)) != hipSuccess) return hip_fail(ee, "join");
    return FOCK_OK;
  };
  std::vector<const void*> key;
  for (int ci = 0; ci < nc; ++ci) {
    key.push_back(u[ci]);
    key.push_back(phi[ci]);
    key.push_back(vphi[ci]);
    key.push_back((const void*)(intptr_t)nphi[ci]);
  }
  hipError_t e;
  fock_status s;
  if (!(B.ready && key == B.key)) {
    B.reset_graph();
    B.key = key;
    // buffers (allocated before any capture; their addresses are baked into the graph)
    int nmax = 0;
    size_t acc_slots_needed = 0;
    std::vector<int> order(nc);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return item_cost(cells[x]) > item_cost(cells[y]); });
    // entries (cell, target, second target or -1): a 16^3 entry carries two
    // targets of its cell. Every cell's entries are split into kBatchQueues
    // contiguous shares, one per sub-queue, cells in decreasing cost order.
    std::vector<std::vector<int>> sub(kBatchQueues);
    for (int ci : order) {
      Cell& c = cells[ci];
      nmax = std::max(nmax, c.geom.n1);
      const int ntg = c.nk * nphi[ci];
      const int per = c.geom.n1 == 16 ? 2 : 1;
      std::vector<int> ent;
      for (int it = 0; it < ntg; it += per) {
        ent.push_back(ci);
        ent.push_back(it);
        ent.push_back(per == 2 && it + 1 < ntg ? it + 1 : -1);
      }
      const int ne = (int)ent.size() / 3;
      for (int x = 0; x < kBatchQueues; ++x) {
        const int b = (int)((long)ne * x / kBatchQueues), e2 = (int)((long)ne * (x + 1) / kBatchQueues);
        sub[x].insert(sub[x].end(), ent.begin() + 3 * b, ent.begin() + 3 * e2);
      }
    }
    std::vector<int> q;
    int qoff[kBatchQueues], qlen[kBatchQueues];
    for (int x = 0; x < kBatchQueues; ++x) {
      qoff[x] = (int)q.size() / 3;
      qlen[x] = (int)sub[x].size() / 3;
      q.insert(q.end(), sub[x].begin(), sub[x].end());
    }
    B.entries = (int)q.size() / 3;
    B.nthreads = batched_threads(nmax);
    const std::string tkey = [&] {
      std::string k = arch_name() + "/fp32/batched";
      for (int ci = 0; ci < nc; ++ci) k += "/" + key_for(cells[ci], cells[ci].fwd(), nphi[ci], "cell");
      return k;
    }();
    int mult = 1;
    bool measure = false;
    {
      TuneEntry te;
      if (tune.get(tkey, &te)) {
        mult = std::max(1, (int)te.fields["wg_per_cu"]);
        B.form = te.fields.count("form") ? (int)te.fields["form"] : kDefaultBatchForm;
      } else {
        measure = tuning;
      }
    }
    B.nwg = num_cus * mult;
    for (int ci = 0; ci < nc; ++ci) {
      Cell& c = cells[ci];
      if (c.geom.n1 == 32) acc_slots_needed = (size_t)B.nwg;
      const size_t nu = (size_t)c.nk * c.nb * c.nr, nx = (size_t)c.nk * nphi[ci] * c.nr;
      if ((s = B.shadow_u[ci].ensure(nu * sizeof(c64), workspace_cap, "batched shadow (u)")) != FOCK_OK) return s;
      if (phi[ci] != u[ci] &&
          (s = B.shadow_x[ci].ensure(nx * sizeof(c64), workspace_cap, "batched shadow (phi)")) != FOCK_OK)
        return s;
      if ((s = B.comp[ci].ensure(nx * sizeof(c64), workspace_cap, "batched compensation")) != FOCK_OK) return s;
    }
    if (acc_slots_needed &&
        (s = B.accs.ensure(fused_acc_scratch_elems(32, (int)acc_slots_needed) * sizeof(c64), workspace_cap,
                           "batched FP32 sums")) != FOCK_OK)
      return s;
    if ((s = B.queue.ensure(q.size() * sizeof(int), 0, "batched queue")) != FOCK_OK) return s;
    if ((s = B.counters.ensure(kBatchQueues * sizeof(int), 0, "batched counters")) != FOCK_OK) return s;
    if ((e = hipMemcpy(B.queue.ptr, q.data(), q.size() * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "upload queue");
    BatchArgs& A = B.args;
    A = BatchArgs{};
    for (int ci = 0; ci < nc; ++ci) {
      Cell& c = cells[ci];
      FusedArgs& a = A.cells[ci];
      a.P = a.M = (const c64*)B.shadow_u[ci].ptr;
      a.X = phi[ci] == u[ci] ? a.P : (const c64*)B.shadow_x[ci].ptr;
      a.Kt = (const float*)c.Kt.ptr;
      a.qidx = (const int*)c.qidx.ptr;
      a.out = (c128*)vphi[ci];
      a.comp = (c64*)B.comp[ci].ptr;
      a.accs = (c64*)B.accs.ptr;
      a.nk = c.nk;
      a.nx = nphi[ci];
      a.nb = c.nb;
      a.item0 = 0;
      a.nitems = c.nk * nphi[ci];
      a.scale = -1.0 / c.nk;
      a.accumulate = 0;
      a.xcd_map = 0;
      a.n = c.geom.n1;
    }
    A.queue = (const int*)B.queue.ptr;
    A.counters = (int*)B.counters.ptr;
    for (int x = 0; x < kBatchQueues; ++x) {
      A.qoff[x] = qoff[x];
      A.qlen[x] = qlen[x];
    }
    if (!B.cap && (e = hipStreamCreateWithFlags(&B.cap, hipStreamNonBlocking)) != hipSuccess)
      return hip_fail(e, "capture stream");
    // streams (default priority) and events of the forked form
    if (!B.fork && (e = hipEventCreateWithFlags(&B.fork, hipEventDisableTiming)) != hipSuccess)
      return hip_fail(e, "fork event");
    for (int ci = 0; ci < nc; ++ci) {
      if (!B.side[ci] && (e = hipStreamCreateWithFlags(&B.side[ci], hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "cell stream");
      if (!B.join[ci] && (e = hipEventCreateWithFlags(&B.join[ci], hipEventDisableTiming)) != hipSuccess)
        return hip_fail(e, "join event");
    }
    B.ready = true;
    if (measure) {
      // persistent workgroups per CU: each candidate runs the whole batch on
      // this call's data (every run writes the same result)
      for (int cid = 0; cid < nc; ++cid) {
        Cell& c = cells[cid];
        const long nu = (long)c.nk * c.nb * c.nr, nx = (long)c.nk * nphi[cid] * c.nr;
        if ((e = launch_to_c64((c64*)B.shadow_u[cid].ptr, (const c128*)u[cid], nu, st)) != hipSuccess)
          return hip_fail(e, "batched shadow");
        if (phi[cid] != u[cid] &&
            (e = launch_to_c64((c64*)B.shadow_x[cid].ptr, (const c128*)phi[cid], nx, st)) != hipSuccess)
          return hip_fail(e, "batched shadow");
      }
      hipEvent_t e0, e1;
      if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e, "tuning event");
      if ((e = hipEventCreate(&e1)) != hipSuccess) return hip_fail(e, "tuning event");
      double best = 1e300;
      int bm = 1, bf = 0;
      // persistent with 1 or 2 workgroups per CU (m = 1, 2), the forked cells (m = 0),
      // the cells in sequence (m = -1)
      for (int m : {1, 2, 0, -1}) {
        (void)hipEventRecord(e0, st);
        if (m > 0) {
          if ((e = launch_fused_batched(B.args, B.nthreads, num_cus * m, st)) != hipSuccess)
            return hip_fail(e, "persistent kernel");
        } else if ((s = launch_cells(st, m == 0)) != FOCK_OK) {
          return s;
        }
        (void)hipEventRecord(e1, st);
        if ((e = hipEventSynchronize(e1)) != hipSuccess) return hip_fail(e, "tuning sync");
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) {
          best = ms;
          bm = m > 0 ? m : bm;
          bf = m > 0 ? 0 : (m == 0 ? 1 : 2);
        }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      B.form = bf;
      TuneEntry te;
      te.fields["wg_per_cu"] = bm;
      te.fields["form"] = bf;
      te.fields["ms"] = best;
      tune.put(tkey, te);
      save_tune();
      B.nwg = num_cus * bm;
    }
  }

  auto enqueue = [&](hipStream_t q) -> fock_status {
    hipError_t ee;
    for (int ci = 0; ci < nc; ++ci) {
      Cell& c = cells[ci];
      const long nu = (long)c.nk * c.nb * c.nr, nx = (long)c.nk * nphi[ci] * c.nr;
      if ((ee = launch_to_c64((c64*)B.shadow_u[ci].ptr, (const c128*)u[ci], nu, q)) != hipSuccess)
        return hip_fail(ee, "batched shadow");
      if (phi[ci] != u[ci] &&
          (ee = launch_to_c64((c64*)B.shadow_x[ci].ptr, (const c128*)phi[ci], nx, q)) != hipSuccess)
        return hip_fail(ee, "batched shadow");
    }
    if (B.form == 1 || B.form == 2) return launch_cells(q, B.form == 1);
    if ((ee = launch_fused_batched(B.args, B.nthreads, B.nwg, q)) != hipSuccess)
      return hip_fail(ee, "persistent kernel");
    return FOCK_OK;
  };

  if (!use_graph) {
    if ((e = prof_begin(st)) != hipSuccess) return hip_fail(e, "profile event");
    if ((s = enqueue(st)) != FOCK_OK) return s;
    if ((e = prof_end(st)) != hipSuccess) return hip_fail(e, "profile event");
    return FOCK_OK;
  }
  if (!B.exec) {
    // the capture stream waits for the caller's prior work through the graph
    // launch itself; capture only records
    if ((e = hipStreamBeginCapture(B.cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return hip_fail(e, "begin capture");
    s = enqueue(B.cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(B.cap, &g);
    if (s != FOCK_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    B.graph = g;
    if ((e = hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0)) != hipSuccess) {
      B.exec = nullptr;
      return hip_fail(e, "instantiate graph");
    }
  }
  if ((e = prof_begin(st)) != hipSuccess) return hip_fail(e, "profile event");
  if ((e = hipGraphLaunch(B.exec, st)) != hipSuccess) return hip_fail(e, "graph launch");
  if ((e = prof_end(st)) != hipSuccess) return hip_fail(e, "profile event");
  return FOCK_OK;
}

}  // namespace fockmi

extern "C" fock_status fock_apply_batched(fockmi_plan plan, const void* const* u_occ, const void* const* phi,
                                          const int* nphi, void* const* vphi, void* stream) {
  g_last_error.clear();
  if (!plan) return fail(FOCK_ERR_ARG, "plan is NULL");
  Plan* p = reinterpret_cast<Plan*>(plan);
  fock_status s = p->check_ready(0);
  if (s != FOCK_OK) return s;
  if (!u_occ || !phi || !nphi || !vphi) return fail(FOCK_ERR_ARG, "NULL pointer array");
  const int nc = (int)p->cells.size();
  for (int ci = 0; ci < nc; ++ci) {
    const Cell& c = p->cells[ci];
    if (!u_occ[ci] || !phi[ci] || !vphi[ci]) return fail(FOCK_ERR_ARG, "cell %d: NULL device pointer", ci);
    if (!aligned16(u_occ[ci]) || !aligned16(phi[ci]) || !aligned16(vphi[ci]))
      return fail(FOCK_ERR_ARG, "cell %d: device pointers must be 16-byte aligned", ci);
    if (nphi[ci] < 1) return fail(FOCK_ERR_ARG, "cell %d: nphi must be >= 1", ci);
    const size_t bu = (size_t)c.nk * c.nb * c.nr * sizeof(c128), bp = (size_t)c.nk * nphi[ci] * c.nr * sizeof(c128);
    if (overlap(vphi[ci], bp, u_occ[ci], bu) || overlap(vphi[ci], bp, phi[ci], bp))
      return fail(FOCK_ERR_ARG, "cell %d: vphi overlaps an input array", ci);
  }
  int nmax = 0;
  bool any_ds = false;
  for (const Cell& c : p->cells) {
    nmax = std::max(nmax, c.geom.n1);
    any_ds = any_ds || c.ds || c.f32plain;
  }
  if (p->prec != FOCK_FP32_COMP || nc > kMaxBatchCells || batched_threads(nmax) == 0 || any_ds) {
    // the plain FP64 path, plans with a 32^3 cell, down-sampled cells and cells that are not
    // cubic run the cells one after another
    for (int ci = 0; ci < nc; ++ci) {
      if ((s = p->apply_op(p->cells[ci], (const c128*)u_occ[ci], (const c128*)phi[ci], nphi[ci], (c128*)vphi[ci],
                           (hipStream_t)stream)) != FOCK_OK)
        return s;
    }
    return FOCK_OK;
  }
  return p->run_batched(u_occ, phi, nphi, vphi, (hipStream_t)stream);
}
