// Serving loop: continuous batching of likelihood requests from many
// concurrent samplers on one GPU.
//
// Requests queue in arrival order.  A scheduler thread admits them while
// slots are free: a request is admissible when its model is resident, or can
// be made resident within the HBM budget after evicting idle models in LRU
// order.  Admitted requests for the same (model, precision) that are waiting
// together are merged into one group (rows are independent and every row's
// reduction order is fixed, so merging never changes a result bit).  With
// sharing on (fgl_serve_set_sharing), the groups of other waiting models
// whose likelihood kernel is the same compiled variant join it: one launch
// of each of the three kernels then serves models of different sizes, each
// workgroup finding its model in a descriptor table.  Each slot owns a HIP
// stream, so the launches of different slots overlap on the device;
// completion is signalled by a host function enqueued behind the launch, and
// the scheduler admits the next request as soon as a slot frees.  A queued
// request can be cancelled, and with a wait limit set a request still queued
// after that long is completed with FGL_ETIMEDOUT.
#include "fgl_host.h"

#include <algorithm>
#include <cmath>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <list>
#include <thread>

namespace fgl {

using Clock = std::chrono::steady_clock;

struct Req {
  uint64_t ticket = 0;
  Model* m = nullptr;
  const double* theta = nullptr;
  int B = 0;
  double* out = nullptr;
  int prec = 0;
  Clock::time_point t0;
  int status = FGL_OK;
  std::string err;
  bool done = false;
  double latency_us = 0.0;
};

struct Server;

struct Slot {
  Server* srv = nullptr;
  hipStream_t s = nullptr;
  bool busy = false;
  std::atomic<bool> finished{false};  // set by the stream callback
  std::vector<Req*> reqs;      // in launch order; outputs are laid out in this order
  int ngroups = 0;             // (model, precision) groups in the launch
  int rows = 0;
  size_t cap = 0;              // doubles of theta the staging buffers hold
  int ocap = 0;                // rows of output they hold
  double* d_theta = nullptr;
  double* d_out = nullptr;
  double* h_theta = nullptr;   // pinned
  double* h_out = nullptr;     // pinned
  GroupDesc* d_desc = nullptr; // descriptor table of a shared launch
  GroupDesc* h_desc = nullptr; // pinned
};

struct Server {
  size_t budget = 0;
  int max_inflight = 1;
  int merge_rows = 16384;
  int share = 1;                    // models per launch (1: no sharing)
  int share_rows = 65536;           // rows per shared launch
  uint64_t n_launches = 0, n_shared = 0, n_shared_groups = 0;
  std::mutex mu;
  std::condition_variable cv_done;  // completions (drain), with mu
  // Scheduler wake-up.  Kept apart from `mu` because the stream callback
  // takes it, and HIP calls made under `mu` may wait for that callback.
  std::mutex sig_mu;
  std::condition_variable sig_cv;
  bool signal = false;
  std::deque<Req*> pending;
  std::unordered_map<uint64_t, Req*> tickets;
  std::vector<Slot*> slots;
  std::thread th;
  bool stop = false;
  uint64_t next_ticket = 1;
  uint64_t clock = 0;
  std::list<Model*> lru;            // models this server keeps resident
  size_t used = 0;
  uint64_t fail_ticket = 0;         // host-forced failure (tests)
  int inflight = 0;
  bool held = false;                // fgl_serve_hold: queue, admit nothing
  double max_wait_us = 0.0;         // fgl_serve_set_timeout (0: none)
};

static std::mutex g_servers_mu;
static std::vector<Server*> g_servers;

static void wake(Server* srv) {
  {
    std::lock_guard<std::mutex> lk(srv->sig_mu);
    srv->signal = true;
  }
  srv->sig_cv.notify_all();
}

// Stream callback behind every launch: no HIP calls, no `mu`.
static void on_done(void* p) {
  Slot* sl = static_cast<Slot*>(p);
  sl->finished.store(true);
  wake(sl->srv);
}

static void finish(Server* srv, Req* r, int status, const std::string& err) {
  r->status = status;
  r->err = err;
  r->done = true;
  r->latency_us = std::chrono::duration<double, std::micro>(Clock::now() - r->t0).count();
  r->m->served.fetch_sub(1);
  (void)srv;
}

static size_t bytes_of(Model* m) { return resident_bytes(m); }

// Make room for `m` within the budget; true when it is (or now can be)
// resident.  Called with srv->mu held.
static bool admit_model(Server* srv, Model* m) {
  auto it = std::find(srv->lru.begin(), srv->lru.end(), m);
  if (it != srv->lru.end() && m->resident) {
    srv->lru.splice(srv->lru.end(), srv->lru, it);   // most recent
    return true;
  }
  if (it != srv->lru.end()) {                        // evicted by someone else
    srv->used -= bytes_of(m);
    srv->lru.erase(it);
  }
  const size_t need = bytes_of(m);
  if (srv->budget) {
    auto cand = srv->lru.begin();
    while (srv->used + need > srv->budget && cand != srv->lru.end()) {
      Model* old = *cand;
      if (old->served.load() == 0 && old->inflight.load() == 0 && old->mu.try_lock()) {
        evict(old);
        old->mu.unlock();
        srv->used -= bytes_of(old);
        cand = srv->lru.erase(cand);
      } else {
        ++cand;
      }
    }
    if (srv->used + need > srv->budget) return false;
  }
  srv->lru.push_back(m);
  srv->used += need;
  return true;
}

// Staging for `nth` doubles of parameters and `rows` outputs.
static int grow_slot(Slot* sl, size_t nth, int rows) {
  if (nth <= sl->cap && rows <= sl->ocap) return FGL_OK;
  const size_t cap = std::max(nth, sl->cap);
  const int ocap = std::max(rows, sl->ocap);
  if (sl->d_theta) (void)hipFree(sl->d_theta);
  if (sl->d_out) (void)hipFree(sl->d_out);
  if (sl->h_theta) (void)hipHostFree(sl->h_theta);
  if (sl->h_out) (void)hipHostFree(sl->h_out);
  sl->d_theta = sl->d_out = sl->h_theta = sl->h_out = nullptr;
  sl->cap = 0;
  sl->ocap = 0;
  hipError_t e;
  const size_t tb = cap * 8, ob = (size_t)ocap * 8;
  if ((e = hipMalloc(reinterpret_cast<void**>(&sl->d_theta), tb)) != hipSuccess ||
      (e = hipMalloc(reinterpret_cast<void**>(&sl->d_out), ob)) != hipSuccess ||
      (e = hipHostMalloc(reinterpret_cast<void**>(&sl->h_theta), tb, hipHostMallocDefault)) != hipSuccess ||
      (e = hipHostMalloc(reinterpret_cast<void**>(&sl->h_out), ob, hipHostMallocDefault)) != hipSuccess)
    return hip_err(e, "serving staging buffers");
  sl->cap = cap;
  sl->ocap = ocap;
  return FGL_OK;
}

// Launch the requests of sl->reqs (same model and precision) on the slot's
// stream.  Called with srv->mu held and the slot idle.
static int launch_slot(Server* srv, Slot* sl) {
  Model* m = sl->reqs.front()->m;
  const int prec = sl->reqs.front()->prec;
  int rows = 0;
  for (Req* r : sl->reqs) rows += r->B;
  TraceRange tr("serve launch: %zu requests, %d rows, prec=%d", sl->reqs.size(), rows, prec);
  std::lock_guard<std::mutex> mlk(m->mu);
  hipError_t e = hipSetDevice(m->dev);
  if (e != hipSuccess) return hip_err(e, "hipSetDevice");
  int rc = make_resident(m);
  if (rc != FGL_OK) return rc;
  if ((rc = grow_slot(sl, (size_t)rows * m->P, rows)) != FGL_OK) return rc;
  size_t off = 0;
  for (Req* r : sl->reqs) {
    std::memcpy(sl->h_theta + off, r->theta, (size_t)r->B * m->P * 8);
    off += (size_t)r->B * m->P;
  }
  const Kind k = kind_of(prec, m->dm);
  WorkBuf& wb = m->work[sl->s];
  wb.stream_synced_free = true;     // the slot's stream is idle here
  const Tile tile = tile_for(m, k, rows);
  if ((rc = ensure_work(m, wb, rows, n_groups(m->dm, tile), false)) != FGL_OK) return rc;
  if ((e = hipMemcpyAsync(sl->d_theta, sl->h_theta, (size_t)rows * m->P * 8,
                          hipMemcpyHostToDevice, sl->s)) != hipSuccess)
    return hip_err(e, "copy theta");
  if ((rc = enqueue(m, k, tile, wb, sl->d_theta, rows, sl->d_out, sl->s)) != FGL_OK) return rc;
  if ((e = hipMemcpyAsync(sl->h_out, sl->d_out, (size_t)rows * 8, hipMemcpyDeviceToHost,
                          sl->s)) != hipSuccess)
    return hip_err(e, "copy out");
  sl->rows = rows;
  sl->ngroups = 1;
  sl->finished = false;
  if ((e = hipLaunchHostFunc(sl->s, on_done, sl)) != hipSuccess)
    return hip_err(e, "hipLaunchHostFunc");
  m->last_use = ++srv->clock;
  ++srv->n_launches;
  return FGL_OK;
}

// One launch of each kernel for the groups in sl->reqs (consecutive runs of
// requests of one model; all in precision `prec`, all with likelihood
// variant `variant`).  Called with srv->mu held and the slot idle.
static int launch_slot_shared(Server* srv, Slot* sl, int prec) {
  TraceRange tr("serve shared launch: %zu requests, prec=%d", sl->reqs.size(), prec);
  // the groups, in order
  struct G {
    Model* m;
    int rows;
    size_t th_off, out_off;
  };
  std::vector<G> groups;
  size_t nth = 0;
  int rows = 0;
  for (Req* r : sl->reqs) {
    if (groups.empty() || groups.back().m != r->m) groups.push_back(G{r->m, 0, nth, (size_t)rows});
    groups.back().rows += r->B;
    nth += (size_t)r->B * r->m->P;
    rows += r->B;
  }
  if ((int)groups.size() > kMaxGroups) return set_err(FGL_EINVAL, "too many groups in a launch");
  // models locked in address order (only this thread locks several)
  std::vector<Model*> order;
  for (const G& g : groups) order.push_back(g.m);
  std::sort(order.begin(), order.end());
  std::vector<std::unique_lock<std::mutex>> locks;
  for (Model* m : order) locks.emplace_back(m->mu);
  hipError_t e = hipSetDevice(groups.front().m->dev);
  if (e != hipSuccess) return hip_err(e, "hipSetDevice");
  int rc = grow_slot(sl, nth, rows);
  if (rc != FGL_OK) return rc;
  if (!sl->d_desc) {
    if ((e = hipMalloc(reinterpret_cast<void**>(&sl->d_desc), kMaxGroups * sizeof(GroupDesc))) != hipSuccess ||
        (e = hipHostMalloc(reinterpret_cast<void**>(&sl->h_desc), kMaxGroups * sizeof(GroupDesc),
                           hipHostMallocDefault)) != hipSuccess)
      return hip_err(e, "serving descriptor table");
  }
  size_t off = 0;
  for (Req* r : sl->reqs) {
    std::memcpy(sl->h_theta + off, r->theta, (size_t)r->B * r->m->P * 8);
    off += (size_t)r->B * r->m->P;
  }
  Kind k0 = kMixed;
  Tile t0{};
  for (size_t j = 0; j < groups.size(); ++j) {
    Model* m = groups[j].m;
    if ((rc = make_resident(m)) != FGL_OK) return rc;
    const Kind k = kind_of(prec, m->dm);
    const Tile tile = tile_for(m, k, groups[j].rows);
    WorkBuf& wb = m->work[sl->s];
    wb.stream_synced_free = true;   // the slot's stream is idle here
    if ((rc = ensure_work(m, wb, groups[j].rows, n_groups(m->dm, tile), false)) != FGL_OK) return rc;
    if (j == 0) {
      k0 = k;
      t0 = tile;
    }
    GroupDesc& d = sl->h_desc[j];
    d = GroupDesc{};
    d.m = m->dm;
    d.w = wb.w;
    d.fc = tile.fc;
    d.G = tile.group;
    d.ngroups = n_groups(m->dm, tile);
    d.theta = sl->d_theta + groups[j].th_off;
    d.out = sl->d_out + groups[j].out_off;
    d.nFT = (double)m->dm.F * (double)m->dm.T;
    d.chi0 = chi0_of(k, m->dm);
  }
  int grid[3], lds = 0;
  plan_groups(k0, t0, sl->h_desc, (int)groups.size(), grid, &lds);
  if ((e = hipMemcpyAsync(sl->d_desc, sl->h_desc, groups.size() * sizeof(GroupDesc),
                          hipMemcpyHostToDevice, sl->s)) != hipSuccess)
    return hip_err(e, "copy descriptors");
  if ((e = hipMemcpyAsync(sl->d_theta, sl->h_theta, nth * 8, hipMemcpyHostToDevice, sl->s)) != hipSuccess)
    return hip_err(e, "copy theta");
  if ((e = launch_groups(k0, groups.front().m->dm, t0, sl->d_desc, (int)groups.size(), grid, lds,
                         sl->s)) != hipSuccess)
    return hip_err(e, "shared launch");
  if ((e = hipMemcpyAsync(sl->h_out, sl->d_out, (size_t)rows * 8, hipMemcpyDeviceToHost,
                          sl->s)) != hipSuccess)
    return hip_err(e, "copy out");
  sl->rows = rows;
  sl->ngroups = (int)groups.size();
  sl->finished = false;
  if ((e = hipLaunchHostFunc(sl->s, on_done, sl)) != hipSuccess)
    return hip_err(e, "hipLaunchHostFunc");
  for (const G& g : groups) g.m->last_use = ++srv->clock;
  ++srv->n_launches;
  ++srv->n_shared;
  srv->n_shared_groups += groups.size();
  return FGL_OK;
}

// The compiled likelihood variant a group of `rows` rows of model m in
// precision prec would launch (0: not shareable).  Reads the model's tile
// table, so it takes the model's lock.
static uint64_t group_variant(Model* m, int prec, int rows) {
  std::lock_guard<std::mutex> lk(m->mu);
  const Kind k = kind_of(prec, m->dm);
  return variant_of(k, m->dm, tile_for(m, k, rows));
}

static void complete_slot(Server* srv, Slot* sl) {
  // the callback that marked the slot finished ran behind the launch; the
  // stream may still report the callback itself as pending
  hipError_t e = hipStreamQuery(sl->s);
  if (e == hipErrorNotReady) e = hipSuccess;
  const int status = (e == hipSuccess) ? FGL_OK : FGL_EDEVICE;
  std::string err = status == FGL_OK ? "" : hipGetErrorString(e);
  size_t off = 0;
  for (Req* r : sl->reqs) {
    if (status == FGL_OK) std::memcpy(r->out, sl->h_out + off, (size_t)r->B * 8);
    off += r->B;
    finish(srv, r, status, err);
  }
  sl->reqs.clear();
  sl->busy = false;
  sl->finished = false;
  --srv->inflight;
  srv->cv_done.notify_all();
}

// Queued requests older than the wait limit: completed with FGL_ETIMEDOUT.
// Returns the earliest deadline of those still queued (max() if none).
static Clock::time_point expire(Server* srv) {
  Clock::time_point next = Clock::time_point::max();
  if (srv->max_wait_us <= 0.0) return next;
  const auto limit = std::chrono::duration_cast<Clock::duration>(
      std::chrono::duration<double, std::micro>(srv->max_wait_us));
  const Clock::time_point now = Clock::now();
  bool any = false;
  for (auto it = srv->pending.begin(); it != srv->pending.end();) {
    Req* r = *it;
    if (now - r->t0 >= limit) {
      it = srv->pending.erase(it);
      finish(srv, r, FGL_ETIMEDOUT, "queued longer than the server's wait limit");
      any = true;
    } else {
      next = std::min(next, r->t0 + limit);
      ++it;
    }
  }
  if (any) srv->cv_done.notify_all();
  return next;
}

static void scheduler(Server* srv) {
  std::unique_lock<std::mutex> lk(srv->mu);
  while (true) {
    // completions
    for (Slot* sl : srv->slots)
      if (sl->busy && sl->finished) complete_slot(srv, sl);
    if (srv->stop && srv->inflight == 0) break;
    expire(srv);
    // admissions, in arrival order, while slots are free
    bool progressed = true;
    while (progressed && !srv->pending.empty() && !srv->stop && !srv->held) {
      progressed = false;
      Slot* free_slot = nullptr;
      for (Slot* sl : srv->slots)
        if (!sl->busy) {
          free_slot = sl;
          break;
        }
      if (!free_slot) break;
      for (auto it = srv->pending.begin(); it != srv->pending.end(); ++it) {
        Req* r = *it;
        if (r->ticket == srv->fail_ticket) {       // host-forced failure
          srv->pending.erase(it);
          finish(srv, r, FGL_EDEVICE, "forced failure (FGL_SERVE_FAIL_TICKET)");
          srv->cv_done.notify_all();
          progressed = true;
          break;
        }
        if (!admit_model(srv, r->m)) continue;
        // merge every waiting request of the same model and precision
        free_slot->reqs.clear();
        int rows = 0;
        for (auto jt = srv->pending.begin(); jt != srv->pending.end();) {
          Req* q = *jt;
          if (q->m == r->m && q->prec == r->prec && q->ticket != srv->fail_ticket &&
              (free_slot->reqs.empty() || rows + q->B <= srv->merge_rows)) {
            free_slot->reqs.push_back(q);
            rows += q->B;
            jt = srv->pending.erase(jt);
          } else {
            ++jt;
          }
        }
        // sharing: the groups of other waiting models of the same variant
        uint64_t var = 0;
        if (srv->share > 1) var = group_variant(r->m, r->prec, rows);
        int ngroups = 1;
        if (var != 0) {
          for (auto it2 = srv->pending.begin();
               it2 != srv->pending.end() && ngroups < srv->share && rows < srv->share_rows;) {
            Req* q = *it2;
            bool taken = false;
            if (q->m != r->m && q->prec == r->prec && q->ticket != srv->fail_ticket &&
                std::none_of(free_slot->reqs.begin(), free_slot->reqs.end(),
                             [&](Req* x) { return x->m == q->m; })) {
              // q's group: every waiting request of its model and precision
              std::vector<Req*> grp;
              int grows = 0;
              for (Req* x : srv->pending)
                if (x->m == q->m && x->prec == q->prec && x->ticket != srv->fail_ticket &&
                    (grp.empty() || grows + x->B <= srv->merge_rows)) {
                  grp.push_back(x);
                  grows += x->B;
                }
              // same variant first, then room in the budget
              if (rows + grows <= srv->share_rows && group_variant(q->m, q->prec, grows) == var &&
                  admit_model(srv, q->m)) {
                for (Req* x : grp) {
                  free_slot->reqs.push_back(x);
                  srv->pending.erase(std::find(srv->pending.begin(), srv->pending.end(), x));
                }
                rows += grows;
                ++ngroups;
                taken = true;
              }
            }
            it2 = taken ? srv->pending.begin() : std::next(it2);
          }
        }
        free_slot->busy = true;
        ++srv->inflight;
        const int rc = var != 0 && ngroups > 1 ? launch_slot_shared(srv, free_slot, r->prec)
                                               : launch_slot(srv, free_slot);
        if (rc != FGL_OK) {
          const std::string err = last_error();
          (void)hipStreamSynchronize(free_slot->s);
          for (Req* q : free_slot->reqs) finish(srv, q, rc, err);
          free_slot->reqs.clear();
          free_slot->busy = false;
          --srv->inflight;
          srv->cv_done.notify_all();
        }
        progressed = true;
        break;
      }
    }
    bool any_finished = false;
    for (Slot* sl : srv->slots) any_finished = any_finished || (sl->busy && sl->finished);
    if (!any_finished) {
      const Clock::time_point deadline = expire(srv);
      lk.unlock();
      {
        std::unique_lock<std::mutex> sg(srv->sig_mu);
        if (deadline == Clock::time_point::max()) {
          srv->sig_cv.wait(sg, [&] { return srv->signal; });
        } else {
          // the wake-up is timed on the system clock (a timed wait every
          // thread tool understands); expiry itself is judged on the
          // steady clock, so a clock step only wakes the loop early or late
          const auto sys = std::chrono::system_clock::now() +
                           std::chrono::duration_cast<std::chrono::system_clock::duration>(
                               deadline - Clock::now());
          srv->sig_cv.wait_until(sg, sys, [&] { return srv->signal; });
        }
        srv->signal = false;
      }
      lk.lock();
    }
  }
}

void serve_forget_model(Model* m) {
  std::lock_guard<std::mutex> g(g_servers_mu);
  for (Server* srv : g_servers) {
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = std::find(srv->lru.begin(), srv->lru.end(), m);
    if (it != srv->lru.end()) {
      srv->used -= bytes_of(m);
      srv->lru.erase(it);
    }
  }
}

}  // namespace fgl

using namespace fgl;

extern "C" {

int fgl_serve_create(size_t hbm_budget_bytes, int max_inflight, fgl_server** out) {
  if (!out) return set_err(FGL_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_inflight < 1 || max_inflight > 64)
    return set_err(FGL_EINVAL, "max_inflight=%d outside 1..64", max_inflight);
  Server* srv = new (std::nothrow) Server();
  if (!srv) return set_err(FGL_ENOMEM, "host allocation");
  srv->budget = hbm_budget_bytes;
  if (const char* mb = std::getenv("FGL_HBM_BUDGET_MB"))
    if (hbm_budget_bytes == 0) srv->budget = (size_t)(std::max(0.0, std::atof(mb)) * 1048576.0);
  srv->max_inflight = max_inflight;
  if (const char* f = std::getenv("FGL_SERVE_FAIL_TICKET")) srv->fail_ticket = std::strtoull(f, nullptr, 10);
  if (const char* mr = std::getenv("FGL_SERVE_MERGE_ROWS")) srv->merge_rows = std::max(1, std::atoi(mr));
  if (const char* sh = std::getenv("FGL_SERVE_SHARE"))
    srv->share = std::min(kMaxGroups, std::max(1, std::atoi(sh)));
  for (int i = 0; i < max_inflight; ++i) {
    Slot* sl = new Slot();
    sl->srv = srv;
    hipError_t e = hipStreamCreateWithFlags(&sl->s, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete sl;
      for (Slot* x : srv->slots) {
        (void)hipStreamDestroy(x->s);
        delete x;
      }
      delete srv;
      return hip_err(e, "hipStreamCreate");
    }
    srv->slots.push_back(sl);
  }
  srv->th = std::thread(scheduler, srv);
  {
    std::lock_guard<std::mutex> g(g_servers_mu);
    g_servers.push_back(srv);
  }
  *out = reinterpret_cast<fgl_server*>(srv);
  return FGL_OK;
}

int fgl_serve_submit(fgl_server* sh, fgl_model* mh, const double* theta, int B,
                     double* out_logL, int prec, uint64_t* ticket) {
  Server* srv = reinterpret_cast<Server*>(sh);
  Model* m = reinterpret_cast<Model*>(mh);
  if (!srv || !m || !ticket) return set_err(FGL_EINVAL, "server, model and ticket must be non-NULL");
  if (B < 1 || B > kMaxRows) return set_err(FGL_EINVAL, "B=%d outside 1..2^26", B);
  if (!theta || !out_logL) return set_err(FGL_EINVAL, "theta and out must be non-NULL");
  if (prec != FGL_PREC_MIXED && prec != FGL_PREC_FP32 && prec != FGL_PREC_FP64)
    return set_err(FGL_EINVAL, "unknown precision %d", prec);
  if (m->dying.load()) return set_err(FGL_EBUSY, "model is being destroyed");
  if (srv->budget && bytes_of(m) > srv->budget)
    return set_err(FGL_EAGAIN, "model needs %zu bytes, budget is %zu", bytes_of(m), srv->budget);
  Req* r = new (std::nothrow) Req();
  if (!r) return set_err(FGL_ENOMEM, "host allocation");
  r->m = m;
  r->theta = theta;
  r->B = B;
  r->out = out_logL;
  r->prec = prec;
  r->t0 = Clock::now();
  m->served.fetch_add(1);
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) {
      m->served.fetch_sub(1);
      delete r;
      return set_err(FGL_EINVAL, "server is shutting down");
    }
    r->ticket = srv->next_ticket++;
    srv->tickets[r->ticket] = r;
    srv->pending.push_back(r);
  }
  wake(srv);
  *ticket = r->ticket;
  return FGL_OK;
}

int fgl_serve_set_sharing(fgl_server* sh, int max_models_per_launch) {
  Server* srv = reinterpret_cast<Server*>(sh);
  if (!srv) return set_err(FGL_EINVAL, "server is NULL");
  if (max_models_per_launch < 1 || max_models_per_launch > kMaxGroups)
    return set_err(FGL_EINVAL, "max_models_per_launch=%d outside 1..%d", max_models_per_launch,
                   kMaxGroups);
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->share = max_models_per_launch;
  return FGL_OK;
}

int fgl_serve_stats(fgl_server* sh, uint64_t* launches, uint64_t* shared_launches,
                    uint64_t* shared_groups) {
  Server* srv = reinterpret_cast<Server*>(sh);
  if (!srv) return set_err(FGL_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(srv->mu);
  if (launches) *launches = srv->n_launches;
  if (shared_launches) *shared_launches = srv->n_shared;
  if (shared_groups) *shared_groups = srv->n_shared_groups;
  return FGL_OK;
}

int fgl_serve_poll(fgl_server* sh, uint64_t ticket, int* done, double* latency_us) {
  Server* srv = reinterpret_cast<Server*>(sh);
  if (!srv || !done) return set_err(FGL_EINVAL, "server and done must be non-NULL");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->tickets.find(ticket);
  if (it == srv->tickets.end()) return set_err(FGL_EINVAL, "unknown or retired ticket %llu",
                                               (unsigned long long)ticket);
  Req* r = it->second;
  if (!r->done) {
    *done = 0;
    return FGL_OK;
  }
  *done = 1;
  if (latency_us) *latency_us = r->latency_us;
  const int st = r->status;
  if (st != FGL_OK) set_err(st, "%s", r->err.c_str());
  srv->tickets.erase(it);
  delete r;
  return st;
}

int fgl_serve_cancel(fgl_server* sh, uint64_t ticket) {
  Server* srv = reinterpret_cast<Server*>(sh);
  if (!srv) return set_err(FGL_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->tickets.find(ticket);
  if (it == srv->tickets.end()) return set_err(FGL_EINVAL, "unknown or retired ticket %llu",
                                               (unsigned long long)ticket);
  Req* r = it->second;
  auto q = std::find(srv->pending.begin(), srv->pending.end(), r);
  if (q == srv->pending.end())
    return set_err(FGL_EBUSY, "ticket %llu is already launched or complete",
                   (unsigned long long)ticket);
  srv->pending.erase(q);
  finish(srv, r, FGL_ECANCELED, "cancelled by the caller");
  srv->cv_done.notify_all();
  return FGL_OK;
}

int fgl_serve_set_timeout(fgl_server* sh, double max_wait_us) {
  Server* srv = reinterpret_cast<Server*>(sh);
  if (!srv) return set_err(FGL_EINVAL, "server is NULL");
  if (!(max_wait_us >= 0.0) || !std::isfinite(max_wait_us))
    return set_err(FGL_EINVAL, "max_wait_us must be finite and >= 0");
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->max_wait_us = max_wait_us;
  }
  wake(srv);
  return FGL_OK;
}

int fgl_serve_drain(fgl_server* sh) {
  Server* srv = reinterpret_cast<Server*>(sh);
  if (!srv) return set_err(FGL_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(srv->mu);
  srv->cv_done.wait(lk, [&] {
    return srv->inflight == 0 && (srv->pending.empty() || srv->held);
  });
  if (!srv->pending.empty())
    return set_err(FGL_EAGAIN, "the server is held with %zu requests queued", srv->pending.size());
  return FGL_OK;
}

int fgl_serve_hold(fgl_server* sh, int hold) {
  Server* srv = reinterpret_cast<Server*>(sh);
  if (!srv) return set_err(FGL_EINVAL, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->held = hold != 0;
    srv->cv_done.notify_all();     // a drain waiting on queued work returns
  }
  if (!hold) wake(srv);
  return FGL_OK;
}

int fgl_serve_destroy(fgl_server* sh) {
  Server* srv = reinterpret_cast<Server*>(sh);
  if (!srv) return set_err(FGL_EINVAL, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (!srv->pending.empty() || srv->inflight != 0)
      return set_err(FGL_EBUSY, "%zu requests pending, %d launches in flight",
                     srv->pending.size(), srv->inflight);
    srv->stop = true;
  }
  wake(srv);
  srv->th.join();
  {
    std::lock_guard<std::mutex> g(g_servers_mu);
    g_servers.erase(std::find(g_servers.begin(), g_servers.end(), srv));
  }
  for (Slot* sl : srv->slots) {
    drop_stream_work(sl->s);
    if (sl->d_theta) (void)hipFree(sl->d_theta);
    if (sl->d_out) (void)hipFree(sl->d_out);
    if (sl->h_theta) (void)hipHostFree(sl->h_theta);
    if (sl->h_out) (void)hipHostFree(sl->h_out);
    if (sl->d_desc) (void)hipFree(sl->d_desc);
    if (sl->h_desc) (void)hipHostFree(sl->h_desc);
    (void)hipStreamDestroy(sl->s);
    delete sl;
  }
  for (auto& kv : srv->tickets) delete kv.second;
  delete srv;
  return FGL_OK;
}

}  // extern "C"
