// Serving pool: many episodes at once, each on a library handle and a HIP
// stream of its own, advanced unit by unit (one step, one replayed step, one
// adjoint step, the loss or one projection per tick) so that their kernels
// overlap on the device; admission by HBM footprint with idle-handle reuse.
// In-flight work is bounded (two units per episode, and optionally a number
// of grid cells over all episodes) so that the concurrent working sets stay
// small, and released episode buffers are kept for reuse, so a steady stream
// of episodes allocates nothing.  Built only on the library's own entry points (sim_step, sim_step_replay,
// sim_step_adjoint, sim_project, sim_loss_box, the solve-mode and warm-start
// controls), so every episode computes exactly what those calls compute.
#include "neuralfluid.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

namespace {

constexpr int kMaxPoolSlots = 64;
constexpr int kRing = 2;   // units of one episode in flight at once

struct PoolHandle {
  sim_desc desc;
  sim_handle h = nullptr;
  size_t bytes = 0;
  bool busy = false;
  uint64_t last_use = 0;
};

// A learned iteration budget per descriptor (grid, geometry, solver settings).
struct BudgetEntry {
  sim_desc desc;
  int budget;
};

enum Phase { kForward, kLoss, kReplay, kAdjoint, kProject, kFinished };

struct Episode {
  bool active = false;
  int kind = 0, T = 0, K = 1, np = 0, nc = 0;
  PoolHandle* ph = nullptr;
  std::vector<double> theta, ctrl;
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  size_t F = 0, C = 0;
  // device buffers (one allocation)
  void* mem = nullptr;
  size_t bytes = 0;
  float *a = nullptr, *b = nullptr, *ckpt = nullptr, *states = nullptr, *P = nullptr, *g = nullptr,
        *gprev = nullptr;
  double *J = nullptr, *g_theta = nullptr, *g_ctrl = nullptr;
  sim_stats* dstats = nullptr;   // device-mode reports, one per solve
  int nsolves = 0;               // reports written so far
  // progress
  Phase phase = kForward;
  int n = 0, s = 0, e = 0;       // step, segment [s, e)
  bool host_checked = false;     // solves wait for their convergence state (budget learning)
  int most_iters = 0;
  sim_stats worst{};
  int status = SIM_OK;           // first failure, else first warning
  bool enqueued = false;
  // units enqueued and not yet seen complete: ring of events, oldest first
  int inflight = 0, ring_head = 0;
  uint64_t ring_seq[2] = {0, 0};
};

// Sections of an episode's device buffer, 256-byte aligned.
struct Layout {
  size_t off_a, off_b, off_ckpt, off_states, off_P, off_g, off_gprev, off_J, off_gth, off_gct, off_stats, total;
};

size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t faces_of(const sim_desc& d) {
  const size_t nx = d.n[0], ny = d.n[1], nz = d.n[2];
  return (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1);
}
size_t cells_of(const sim_desc& d) { return (size_t)d.n[0] * d.n[1] * d.n[2]; }

int solves_of(int kind, int T) { return kind == SIM_EP_PROJECT ? 1 : (kind == SIM_EP_FORWARD ? T : 2 * T); }

Layout layout_of(const sim_episode& ep) {
  const size_t F = faces_of(ep.desc) * 4, C = cells_of(ep.desc) * 4;
  const int T = ep.steps, K = ep.every;
  const bool adj = ep.kind == SIM_EP_FORWARD_ADJOINT;
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t at = o;
    o += up256(b);
    return at;
  };
  L.off_a = take(F);
  L.off_b = take(F);
  L.off_ckpt = take(adj ? (size_t)((T + K - 1) / K) * F : 0);
  L.off_states = take(adj ? (size_t)(K + 1) * F : 0);
  L.off_P = take(adj ? (size_t)T * C : 0);
  L.off_g = take(adj ? F : 0);
  L.off_gprev = take(adj ? F : 0);
  L.off_J = take(adj ? 8 : 0);
  L.off_gth = take(adj ? (size_t)T * ep.desc.n_params * 8 : 0);
  L.off_gct = take(adj ? (size_t)T * ep.desc.n_ctrl * 8 : 0);
  L.off_stats = take((size_t)solves_of(ep.kind, T) * sizeof(sim_stats));
  L.total = o;
  return L;
}

bool same_desc(const sim_desc& x, const sim_desc& y) { return std::memcmp(&x, &y, sizeof(sim_desc)) == 0; }

// A released episode buffer kept for reuse (its episode's stream has drained).
struct CachedBuffer {
  void* mem;
  size_t bytes;
};

}  // namespace

struct sim_pool {
  int device = 0;
  size_t budget = 0, used = 0;   // used: handles, live episode buffers and cached buffers
  int max_active = 0;
  int64_t inflight_cells = 0;    // bound on the grid cells of the units in flight (0: none)
  uint64_t clock = 0, seq = 0;
  int rr = 0;                    // round-robin start of the next tick
  std::vector<PoolHandle*> handles;
  std::vector<BudgetEntry> budgets;
  std::vector<CachedBuffer> cache;
  Episode slots[kMaxPoolSlots];
  hipStream_t streams[kMaxPoolSlots] = {};
  hipEvent_t done[kMaxPoolSlots] = {};
  hipEvent_t ring[kMaxPoolSlots][kRing] = {};
};

namespace {

int learned_budget(const sim_pool* p, const sim_desc& d) {
  for (const BudgetEntry& b : p->budgets)
    if (same_desc(b.desc, d)) return b.budget;
  return 0;
}

BudgetEntry* budget_entry(sim_pool* p, const sim_desc& d) {
  for (BudgetEntry& b : p->budgets)
    if (same_desc(b.desc, d)) return &b;
  return nullptr;
}

void free_handle(sim_pool* p, PoolHandle* ph) {
  (void)sim_destroy(ph->h);
  p->used -= ph->bytes;
  p->handles.erase(std::find(p->handles.begin(), p->handles.end(), ph));
  delete ph;
}

// The smallest cached buffer that holds `bytes` and is at most twice that,
// taken out of the cache (it stays counted in `used`); nullptr if none.
void* take_cached(sim_pool* p, size_t bytes, size_t* got) {
  int best = -1;
  for (int i = 0; i < (int)p->cache.size(); ++i) {
    const size_t b = p->cache[i].bytes;
    if (b >= bytes && b <= 2 * bytes && (best < 0 || b < p->cache[best].bytes)) best = i;
  }
  if (best < 0) return nullptr;
  void* m = p->cache[best].mem;
  *got = p->cache[best].bytes;
  p->cache.erase(p->cache.begin() + best);
  return m;
}

// Free the largest cached buffer; false when the cache is empty.
bool drop_cached(sim_pool* p) {
  if (p->cache.empty()) return false;
  auto it = std::max_element(p->cache.begin(), p->cache.end(),
                             [](const CachedBuffer& x, const CachedBuffer& y) { return x.bytes < y.bytes; });
  (void)hipFree(it->mem);
  p->used -= it->bytes;
  p->cache.erase(it);
  return true;
}

// Retire the units of slot q that have completed (oldest first).
void retire(sim_pool* p, int q) {
  Episode& E = p->slots[q];
  while (E.inflight > 0) {
    const hipError_t e = hipEventQuery(p->ring[q][E.ring_head]);
    if (e == hipErrorNotReady) break;
    if (e != hipSuccess) {
      (void)hipGetLastError();
      if (E.status >= 0) E.status = SIM_EHIP;
    }
    E.ring_head = (E.ring_head + 1) % kRing;
    --E.inflight;
  }
}

// Fold one solver report into the episode's summary.
void fold(Episode& E, const sim_stats& st) {
  E.worst.iters = std::max(E.worst.iters, st.iters);
  E.worst.converged = E.worst.converged && st.converged;
  E.worst.nonfinite = E.worst.nonfinite || st.nonfinite;
  E.worst.rel_res = std::max(E.worst.rel_res, st.rel_res);
  E.worst.true_rel_res = std::max(E.worst.true_rel_res, st.true_rel_res);
}

void note(Episode& E, int r) {
  if (r < 0) {
    if (E.status >= 0) E.status = r;
    E.phase = kFinished;
  } else if (r > 0 && E.status == SIM_OK) {
    E.status = r;
  }
}

// The stats pointer of the next solve: a host struct when host-checked (read
// at once), else the next device report.
sim_stats* stats_slot(Episode& E, sim_stats& host) {
  if (E.host_checked) return &host;
  return E.dstats + E.nsolves;
}

void after_solve(Episode& E, const sim_stats& host) {
  if (E.host_checked) {
    fold(E, host);
    E.most_iters = std::max(E.most_iters, host.iters);
  }
  ++E.nsolves;
}

// One unit of episode E on its stream.
void unit(sim_pool* p, int slot) {
  Episode& E = p->slots[slot];
  hipStream_t st = p->streams[slot];
  sim_handle h = E.ph->h;
  const size_t F = E.F, C = E.C;
  auto th = [&](int n) { return E.np ? E.theta.data() + (size_t)n * E.np : nullptr; };
  auto ct = [&](int n) { return E.nc ? E.ctrl.data() + (size_t)n * E.nc : nullptr; };
  sim_stats host{};
  switch (E.phase) {
    case kProject: {
      const int r = sim_project(h, E.a, th(0), ct(0), E.b, nullptr, stats_slot(E, host), st);
      after_solve(E, host);
      note(E, r);
      E.phase = kFinished;
      break;
    }
    case kForward: {
      const bool adj = E.kind == SIM_EP_FORWARD_ADJOINT;
      const int n = E.n;
      const int r = sim_step(h, E.a, th(n), ct(n), E.b, adj ? E.P + (size_t)n * C : nullptr, stats_slot(E, host), st);
      after_solve(E, host);
      note(E, r);
      if (E.phase == kFinished) break;
      std::swap(E.a, E.b);
      if (adj && (n + 1) % E.K == 0 && n + 1 < E.T &&
          hipMemcpyAsync(E.ckpt + (size_t)((n + 1) / E.K) * F, E.a, F * 4, hipMemcpyDeviceToDevice, st) != hipSuccess)
        note(E, SIM_EHIP);
      if (E.phase == kFinished) break;
      if (++E.n == E.T) E.phase = adj ? kLoss : kFinished;
      break;
    }
    case kLoss: {
      note(E, sim_loss_box(h, E.a, E.lo, E.hi, E.J, E.g, st));
      if (E.phase == kFinished) break;
      note(E, sim_set_warm_start(h, SIM_WARM_ADJOINT));
      E.s = ((E.T - 1) / E.K) * E.K;
      E.e = std::min(E.s + E.K, E.T);
      E.n = E.s;
      if (E.phase != kFinished) E.phase = kReplay;
      break;
    }
    case kReplay: {
      const int n = E.n;
      if (n == E.s && hipMemcpyAsync(E.states, E.ckpt + (size_t)(E.s / E.K) * F, F * 4, hipMemcpyDeviceToDevice,
                                     st) != hipSuccess) {
        note(E, SIM_EHIP);
        break;
      }
      note(E, sim_step_replay(h, E.states + (size_t)(n - E.s) * F, th(n), ct(n), E.P + (size_t)n * C,
                              E.states + (size_t)(n - E.s + 1) * F, st));
      if (E.phase == kFinished) break;
      if (++E.n == E.e) {
        E.n = E.e - 1;
        E.phase = kAdjoint;
      }
      break;
    }
    case kAdjoint: {
      const int n = E.n;
      const int r = sim_step_adjoint(h, E.states + (size_t)(n - E.s) * F, E.P + (size_t)n * C, th(n), ct(n), E.g,
                                     E.gprev, E.np ? E.g_theta + (size_t)n * E.np : nullptr,
                                     E.nc ? E.g_ctrl + (size_t)n * E.nc : nullptr, stats_slot(E, host), st);
      after_solve(E, host);
      note(E, r);
      if (E.phase == kFinished) break;
      std::swap(E.g, E.gprev);
      if (--E.n < E.s) {
        if (E.s == 0) {
          note(E, sim_set_warm_start(h, 0));
          E.phase = kFinished;
        } else {
          E.s -= E.K;
          E.e = E.s + E.K;
          E.n = E.s;
          E.phase = kReplay;
        }
      }
      break;
    }
    case kFinished:
      break;
  }
  if (E.phase == kFinished && !E.enqueued) {
    if (hipEventRecord(p->done[slot], st) != hipSuccess && E.status >= 0) E.status = SIM_EHIP;
    E.enqueued = true;
    // a host-checked episode sets its descriptor's budget, or raises it
    if (E.host_checked && E.status >= 0 && E.most_iters > 0) {
      const int b = std::min(8 * (int)std::ceil((1.5 * E.most_iters + 2.0) / 8.0), E.ph->desc.max_iter);
      BudgetEntry* be = budget_entry(p, E.ph->desc);
      if (be)
        be->budget = std::max(be->budget, b);
      else
        p->budgets.push_back(BudgetEntry{E.ph->desc, b});
    }
  }
}

}  // namespace

extern "C" {

int32_t sim_pool_create(size_t budget_bytes, int32_t max_active, int64_t inflight_cells, sim_pool_handle* out) {
  if (!out || budget_bytes == 0 || max_active < 1 || max_active > kMaxPoolSlots || inflight_cells < 0)
    return SIM_EINVAL;
  sim_pool* p = new (std::nothrow) sim_pool();
  if (!p) return SIM_ENOMEM;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return SIM_EHIP;
  }
  p->budget = budget_bytes;
  p->max_active = max_active;
  p->inflight_cells = inflight_cells;
  for (int q = 0; q < max_active; ++q) {
    // default priority; non-blocking with respect to the null stream
    if (hipStreamCreateWithFlags(&p->streams[q], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p->done[q], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ring[q][0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ring[q][1], hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      (void)sim_pool_destroy(p);
      return SIM_EHIP;
    }
  }
  *out = p;
  return SIM_OK;
}

int32_t sim_pool_destroy(sim_pool_handle p) {
  if (!p) return SIM_EINVAL;
  (void)hipSetDevice(p->device);
  for (int q = 0; q < p->max_active; ++q) {
    if (p->streams[q]) (void)hipStreamSynchronize(p->streams[q]);
    Episode& E = p->slots[q];
    if (E.mem) (void)hipFree(E.mem);
    E = Episode();
  }
  for (const CachedBuffer& c : p->cache) (void)hipFree(c.mem);
  p->cache.clear();
  while (!p->handles.empty()) {
    PoolHandle* ph = p->handles.back();
    (void)sim_destroy(ph->h);
    delete ph;
    p->handles.pop_back();
  }
  for (int q = 0; q < p->max_active; ++q) {
    if (p->done[q]) (void)hipEventDestroy(p->done[q]);
    for (int k = 0; k < kRing; ++k)
      if (p->ring[q][k]) (void)hipEventDestroy(p->ring[q][k]);
    if (p->streams[q]) (void)hipStreamDestroy(p->streams[q]);
  }
  delete p;
  return SIM_OK;
}

int32_t sim_pool_admit(sim_pool_handle p, const sim_episode* ep, const float* u0, int32_t* slot) {
  if (!p || !ep || !u0 || !slot) return SIM_EINVAL;
  if (ep->kind < SIM_EP_FORWARD || ep->kind > SIM_EP_PROJECT) return SIM_EINVAL;
  const int T = ep->kind == SIM_EP_PROJECT ? 1 : ep->steps;
  if (T < 1 || (ep->kind == SIM_EP_PROJECT && ep->steps != 1)) return SIM_EINVAL;
  if (ep->kind == SIM_EP_FORWARD_ADJOINT && ep->every < 1) return SIM_EINVAL;
  if (ep->flags != 0 && ep->flags != SIM_EP_HOST_CHECKED) return SIM_EINVAL;
  if ((ep->desc.n_params > 0 && !ep->theta) || (ep->desc.n_ctrl > 0 && !ep->ctrl)) return SIM_EINVAL;
  size_t hb = 0;
  int v = sim_footprint(&ep->desc, &hb);
  if (v != SIM_OK) return v;
  (void)hipSetDevice(p->device);
  int q = 0;
  while (q < p->max_active && p->slots[q].active) ++q;
  if (q == p->max_active) return SIM_EBUSY;
  sim_episode norm = *ep;
  norm.steps = T;
  if (ep->kind != SIM_EP_FORWARD_ADJOINT) norm.every = 1;
  const Layout L = layout_of(norm);
  // a matching idle handle, else room for a new one (idle handles freed
  // least recently used first)
  PoolHandle* ph = nullptr;
  for (PoolHandle* c : p->handles)
    if (!c->busy && same_desc(c->desc, ep->desc)) {
      ph = c;
      break;
    }
  // the episode's buffer: a released one of about its size, else a new one;
  // room is made by freeing cached buffers, then idle handles (least
  // recently used first).  A released buffer is reused without any
  // allocation, and hipFree (which waits for the device) runs only when the
  // budget forces it.
  size_t got = 0;
  void* mem = take_cached(p, L.total, &got);
  const size_t need = (mem ? 0 : L.total) + (ph ? 0 : hb);
  while (p->used + need > p->budget) {
    if (drop_cached(p)) continue;
    PoolHandle* lru = nullptr;
    for (PoolHandle* c : p->handles)
      if (!c->busy && c != ph && (!lru || c->last_use < lru->last_use)) lru = c;
    if (!lru) {
      if (mem) p->cache.push_back(CachedBuffer{mem, got});
      return SIM_EBUSY;
    }
    free_handle(p, lru);
  }
  if (!mem) {
    if (hipMalloc(&mem, L.total) != hipSuccess) {
      (void)hipGetLastError();
      return SIM_ENOMEM;
    }
    got = L.total;
    p->used += got;
  }
  // from here a failure returns the buffer to the cache
  if (!ph) {
    ph = new (std::nothrow) PoolHandle();
    if (!ph) {
      p->cache.push_back(CachedBuffer{mem, got});
      return SIM_ENOMEM;
    }
    ph->desc = ep->desc;
    ph->bytes = hb;
    v = sim_create(&ep->desc, &ph->h);
    if (v != SIM_OK) {
      delete ph;
      p->cache.push_back(CachedBuffer{mem, got});
      return v;
    }
    p->handles.push_back(ph);
    p->used += hb;
  }
  const int budget = (ep->flags & SIM_EP_HOST_CHECKED) ? 0 : learned_budget(p, ep->desc);
  v = sim_set_solve_mode(ph->h, budget > 0 ? SIM_SOLVE_DEVICE : SIM_SOLVE_HOST, budget);
  if (v == SIM_OK) v = sim_set_warm_start(ph->h, 0);
  if (v != SIM_OK) {
    p->cache.push_back(CachedBuffer{mem, got});
    return v;
  }
  Episode& E = p->slots[q];
  E = Episode();
  E.active = true;
  E.kind = ep->kind;
  E.T = T;
  E.K = norm.every;
  E.np = ep->desc.n_params;
  E.nc = ep->desc.n_ctrl;
  E.ph = ph;
  E.theta.assign(ep->theta ? ep->theta : nullptr, ep->theta ? ep->theta + (size_t)T * E.np : nullptr);
  E.ctrl.assign(ep->ctrl ? ep->ctrl : nullptr, ep->ctrl ? ep->ctrl + (size_t)T * E.nc : nullptr);
  for (int a = 0; a < 3; ++a) {
    E.lo[a] = ep->box_lo[a];
    E.hi[a] = ep->box_hi[a];
  }
  E.F = faces_of(ep->desc);
  E.C = cells_of(ep->desc);
  E.mem = mem;
  E.bytes = got;
  char* m = (char*)mem;
  E.a = (float*)(m + L.off_a);
  E.b = (float*)(m + L.off_b);
  E.ckpt = (float*)(m + L.off_ckpt);
  E.states = (float*)(m + L.off_states);
  E.P = (float*)(m + L.off_P);
  E.g = (float*)(m + L.off_g);
  E.gprev = (float*)(m + L.off_gprev);
  E.J = (double*)(m + L.off_J);
  E.g_theta = (double*)(m + L.off_gth);
  E.g_ctrl = (double*)(m + L.off_gct);
  E.dstats = (sim_stats*)(m + L.off_stats);
  E.host_checked = budget == 0;
  E.worst.converged = 1;
  E.phase = ep->kind == SIM_EP_PROJECT ? kProject : kForward;
  ph->busy = true;
  hipStream_t st = p->streams[q];
  bool ok = hipMemcpyAsync(E.a, u0, E.F * 4, hipMemcpyDeviceToDevice, st) == hipSuccess;
  if (ep->kind == SIM_EP_FORWARD_ADJOINT) {
    ok = ok && hipMemcpyAsync(E.ckpt, u0, E.F * 4, hipMemcpyDeviceToDevice, st) == hipSuccess;
    // the per-step partials are accumulated (+=) by the adjoint
    const size_t gb = (size_t)T * (E.np + E.nc) * 8;
    if (gb) ok = ok && hipMemsetAsync(E.g_theta, 0, (size_t)T * E.np * 8, st) == hipSuccess &&
                 hipMemsetAsync(E.g_ctrl, 0, (size_t)T * E.nc * 8, st) == hipSuccess;
  }
  if (!ok) {
    (void)hipGetLastError();
    E.status = SIM_EHIP;
    E.phase = kFinished;
    (void)hipEventRecord(p->done[q], st);
    E.enqueued = true;
  }
  *slot = q;
  return SIM_OK;
}

int32_t sim_pool_tick(sim_pool_handle p, int32_t* pending) {
  if (!p) return SIM_EINVAL;
  (void)hipSetDevice(p->device);
  const int m = p->max_active;
  int64_t cells = 0;
  for (int q = 0; q < m; ++q) {
    Episode& E = p->slots[q];
    if (!E.active) continue;
    retire(p, q);
    cells += (int64_t)E.inflight * (int64_t)E.C;
  }
  int left = 0;
  bool enqueued_any = false;
  for (int i = 0; i < m; ++i) {
    const int q = (p->rr + i) % m;
    Episode& E = p->slots[q];
    if (!E.active || E.enqueued) continue;
    // at most kRing units of an episode, and (when bounded) inflight_cells
    // grid cells of all episodes, in flight; one unit may always run
    const bool over = p->inflight_cells > 0 && cells > 0 && cells + (int64_t)E.C > p->inflight_cells;
    if (E.inflight >= kRing || over) {
      ++left;
      continue;
    }
    unit(p, q);
    const int k = (E.ring_head + E.inflight) % kRing;
    if (hipEventRecord(p->ring[q][k], p->streams[q]) == hipSuccess) {
      E.ring_seq[k] = ++p->seq;
      ++E.inflight;
      cells += (int64_t)E.C;
    } else {
      (void)hipGetLastError();
      if (E.status >= 0) E.status = SIM_EHIP;
    }
    enqueued_any = true;
    if (!E.enqueued) ++left;
  }
  p->rr = (p->rr + 1) % m;
  if (!enqueued_any) {
    // nothing could be enqueued: wait for the oldest unit in flight
    int oldest = -1;
    for (int q = 0; q < m; ++q) {
      const Episode& E = p->slots[q];
      if (E.active && E.inflight > 0 &&
          (oldest < 0 || E.ring_seq[E.ring_head] < p->slots[oldest].ring_seq[p->slots[oldest].ring_head]))
        oldest = q;
    }
    if (oldest >= 0) {
      if (hipEventSynchronize(p->ring[oldest][p->slots[oldest].ring_head]) != hipSuccess) (void)hipGetLastError();
      retire(p, oldest);
    }
  }
  if (pending) *pending = left;
  return SIM_OK;
}

int32_t sim_pool_poll(sim_pool_handle p, int32_t slot, int32_t* done) {
  if (!p || !done || slot < 0 || slot >= p->max_active || !p->slots[slot].active) return SIM_EINVAL;
  const Episode& E = p->slots[slot];
  *done = 0;
  if (!E.enqueued) return SIM_OK;
  const hipError_t e = hipEventQuery(p->done[slot]);
  if (e == hipSuccess) *done = 1;
  else if (e != hipErrorNotReady) return SIM_EHIP;
  return SIM_OK;
}

int32_t sim_pool_result(sim_pool_handle p, int32_t slot, float* u_out, float* g_u0, double* g_theta, double* g_ctrl,
                        double* J, sim_stats* worst) {
  if (!p || slot < 0 || slot >= p->max_active || !p->slots[slot].active) return SIM_EINVAL;
  Episode& E = p->slots[slot];
  if (!E.enqueued) return SIM_EINVAL;   // work still to be enqueued: tick first
  (void)hipSetDevice(p->device);
  hipStream_t st = p->streams[slot];
  bool ok = true;
  const bool adj = E.kind == SIM_EP_FORWARD_ADJOINT;
  if (E.status >= 0) {
    // u_T is in a (forward episodes) or the projection's output in b
    const float* u = E.kind == SIM_EP_PROJECT ? E.b : E.a;
    if (u_out) ok = ok && hipMemcpyAsync(u_out, u, E.F * 4, hipMemcpyDeviceToDevice, st) == hipSuccess;
    if (adj && g_u0) ok = ok && hipMemcpyAsync(g_u0, E.g, E.F * 4, hipMemcpyDeviceToDevice, st) == hipSuccess;
    if (adj && g_theta && E.np)
      ok = ok && hipMemcpyAsync(g_theta, E.g_theta, (size_t)E.T * E.np * 8, hipMemcpyDeviceToDevice, st) == hipSuccess;
    if (adj && g_ctrl && E.nc)
      ok = ok && hipMemcpyAsync(g_ctrl, E.g_ctrl, (size_t)E.T * E.nc * 8, hipMemcpyDeviceToDevice, st) == hipSuccess;
  }
  std::vector<sim_stats> rep(!E.host_checked ? E.nsolves : 0);
  if (!rep.empty())
    ok = ok && hipMemcpyAsync(rep.data(), E.dstats, rep.size() * sizeof(sim_stats), hipMemcpyDeviceToHost, st) ==
                   hipSuccess;
  double Jh = 0.0;
  if (adj && J && E.status >= 0) ok = ok && hipMemcpyAsync(&Jh, E.J, 8, hipMemcpyDeviceToHost, st) == hipSuccess;
  ok = ok && hipStreamSynchronize(st) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    if (E.status >= 0) E.status = SIM_EHIP;
  }
  bool missed = false;
  for (const sim_stats& s : rep) {
    fold(E, s);
    if (E.status == SIM_OK && !(s.converged && !s.nonfinite)) E.status = s.nonfinite ? SIM_WNONFINITE : SIM_WNOCONV;
    missed = missed || (!s.converged && !s.nonfinite);
  }
  if (missed) {
    // the device-mode budget was too small for this descriptor: double it
    BudgetEntry* be = budget_entry(p, E.ph->desc);
    if (be) be->budget = std::min(2 * be->budget, E.ph->desc.max_iter);
  }
  if (J) *J = Jh;
  if (worst) *worst = E.worst;
  const int status = E.status;
  // the stream has drained: the buffer is kept for the next episode
  p->cache.push_back(CachedBuffer{E.mem, E.bytes});
  E.ph->busy = false;
  E.ph->last_use = ++p->clock;
  E = Episode();
  return status;
}

}  // extern "C"
