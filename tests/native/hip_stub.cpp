// A CPU stand-in for the part of the HIP runtime that the library's host
// code calls (fgl_host.cpp, fgl_serve.cpp, fgl_plan.cpp), so that this code
// can be built with g++ under AddressSanitizer or ThreadSanitizer and run
// with no GPU.  Test infrastructure only.
//
// The model of the runtime:
//  * device and pinned memory are host heap blocks; the allocator tracks
//    them, so a free of an unknown pointer is reported as an error;
//  * a stream is a worker thread that runs its operations in order; a host
//    function runs on that thread, as the runtime runs it on a thread of its
//    own; the legacy default stream (NULL) is one more such stream;
//  * an event records a steady-clock reading in stream order;
//  * stream capture records the operations enqueued on the capturing stream
//    instead of running them, and a graph launch enqueues them again (the
//    same pointers and sizes, as a replayed graph reuses its node arguments);
//  * one device, 0, reported as gfx950.
// The operations a stream runs are C++ closures; the stand-ins of the kernel
// launchers (launch_stub.cpp) enqueue theirs through stub_enqueue below.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

#include "hip_stub.h"

struct ihipGraph {
  std::vector<std::function<void()>> ops;
};

struct hipGraphExec {
  std::vector<std::function<void()>> ops;
};

struct ihipStream_t {
  std::mutex mu;
  std::condition_variable work_cv, idle_cv;
  std::deque<std::function<void()>> q;
  bool busy = false;
  bool stop = false;
  ihipGraph* capture = nullptr;        // non-NULL while capturing
  std::thread::id capture_thread;
  std::thread th;

  void run() {
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      work_cv.wait(lk, [&] { return stop || !q.empty(); });
      if (q.empty()) return;           // stop requested and drained
      std::function<void()> op = std::move(q.front());
      q.pop_front();
      busy = true;
      lk.unlock();
      op();
      lk.lock();
      busy = false;
      if (q.empty()) idle_cv.notify_all();
    }
  }
  void push(std::function<void()> op) {
    std::lock_guard<std::mutex> lk(mu);
    q.push_back(std::move(op));
    work_cv.notify_one();
  }
  void drain() {
    std::unique_lock<std::mutex> lk(mu);
    idle_cv.wait(lk, [&] { return q.empty() && !busy; });
  }
};

struct ihipEvent_t {
  std::mutex mu;
  std::condition_variable cv;
  int pending = 0;
  double t = 0.0;   // seconds
};

namespace {

std::mutex g_mu;                       // streams and allocations
std::set<ihipStream_t*> g_streams;
std::map<void*, size_t> g_device, g_pinned;
ihipStream_t* g_null = nullptr;
std::atomic<long> g_errors{0};

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

ihipStream_t* new_stream() {
  auto* s = new ihipStream_t();
  s->th = std::thread([s] { s->run(); });
  std::lock_guard<std::mutex> lk(g_mu);
  g_streams.insert(s);
  return s;
}

ihipStream_t* resolve(hipStream_t s) {
  if (s) return s;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_null) {
    g_null = new ihipStream_t();
    g_null->th = std::thread([p = g_null] { p->run(); });
    g_streams.insert(g_null);
  }
  return g_null;
}

void* track(std::map<void*, size_t>& m, size_t n) {
  void* p = std::malloc(n ? n : 1);
  if (!p) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  m[p] = n;
  return p;
}

hipError_t untrack(std::map<void*, size_t>& m, void* p, const char* what) {
  if (!p) return hipSuccess;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = m.find(p);
    if (it == m.end()) {
      std::fprintf(stderr, "hip stub: %s of a pointer it never returned: %p\n", what, p);
      g_errors.fetch_add(1);
      return hipErrorInvalidValue;
    }
    m.erase(it);
  }
  std::free(p);
  return hipSuccess;
}

}  // namespace

// Enqueue one operation on a stream (or record it into the stream's capture).
hipError_t stub_enqueue(hipStream_t sh, std::function<void()> op) {
  ihipStream_t* s = resolve(sh);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->capture) {
      if (s->capture_thread != std::this_thread::get_id()) return hipErrorStreamCaptureImplicit;
      s->capture->ops.push_back(std::move(op));
      return hipSuccess;
    }
  }
  s->push(std::move(op));
  return hipSuccess;
}

long stub_errors() { return g_errors.load(); }

void stub_report(const char* msg) {
  std::fprintf(stderr, "hip stub: %s\n", msg);
  g_errors.fetch_add(1);
}

size_t stub_live_device_bytes() {
  std::lock_guard<std::mutex> lk(g_mu);
  size_t n = 0;
  for (const auto& kv : g_device) n += kv.second;
  return n;
}

size_t stub_live_allocations() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_device.size() + g_pinned.size();
}

extern "C" {

const char* hipGetErrorString(hipError_t e) {
  switch (e) {
    case hipSuccess: return "no error";
    case hipErrorInvalidValue: return "invalid argument";
    case hipErrorOutOfMemory: return "out of memory";
    case hipErrorNotReady: return "not ready";
    case hipErrorStreamCaptureImplicit: return "capture from another thread";
    default: return "stub error";
  }
}

hipError_t hipSetDevice(int dev) { return dev == 0 ? hipSuccess : hipErrorInvalidDevice; }

hipError_t hipGetDevice(int* dev) {
  *dev = 0;
  return hipSuccess;
}

hipError_t hipGetDeviceProperties(hipDeviceProp_t* prop, int dev) {
  if (dev != 0) return hipErrorInvalidDevice;
  std::memset(prop, 0, sizeof *prop);
  std::snprintf(prop->name, sizeof prop->name, "CPU stand-in");
  std::snprintf(prop->gcnArchName, sizeof prop->gcnArchName, "gfx950:sramecc+:xnack-");
  prop->multiProcessorCount = 256;
  prop->warpSize = 64;
  prop->totalGlobalMem = size_t(288) << 30;
  prop->sharedMemPerBlock = 160 * 1024;
  return hipSuccess;
}

hipError_t hipMalloc(void** p, size_t n) {
  *p = track(g_device, n);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}

hipError_t hipFree(void* p) { return untrack(g_device, p, "hipFree"); }

hipError_t hipHostMalloc(void** p, size_t n, unsigned int) {
  *p = track(g_pinned, n);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}

hipError_t hipHostFree(void* p) { return untrack(g_pinned, p, "hipHostFree"); }

hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind) {
  (void)hipDeviceSynchronize();
  if (n) std::memcpy(dst, src, n);
  return hipSuccess;
}

hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t s) {
  return stub_enqueue(s, [dst, src, n] {
    if (n) std::memcpy(dst, src, n);
  });
}

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
  *s = new_stream();
  return hipSuccess;
}

hipError_t hipStreamDestroy(hipStream_t s) {
  if (!s) return hipErrorInvalidValue;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_streams.erase(s)) return hipErrorInvalidValue;
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->work_cv.notify_one();
  }
  s->th.join();
  delete s;
  return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t s) {
  resolve(s)->drain();
  return hipSuccess;
}

hipError_t hipStreamQuery(hipStream_t sh) {
  ihipStream_t* s = resolve(sh);
  std::lock_guard<std::mutex> lk(s->mu);
  return s->q.empty() && !s->busy ? hipSuccess : hipErrorNotReady;
}

hipError_t hipDeviceSynchronize(void) {
  std::vector<ihipStream_t*> all;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    all.assign(g_streams.begin(), g_streams.end());
  }
  // streams are destroyed only by their owners, after they stop using them
  for (ihipStream_t* s : all) s->drain();
  return hipSuccess;
}

hipError_t hipLaunchHostFunc(hipStream_t s, hipHostFn_t fn, void* user) {
  return stub_enqueue(s, [fn, user] { fn(user); });
}

hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
  *e = new ihipEvent_t();
  return hipSuccess;
}

hipError_t hipEventDestroy(hipEvent_t e) {
  if (!e) return hipErrorInvalidValue;
  {
    std::unique_lock<std::mutex> lk(e->mu);
    e->cv.wait(lk, [&] { return e->pending == 0; });
  }
  delete e;
  return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  {
    std::lock_guard<std::mutex> lk(e->mu);
    ++e->pending;
  }
  return stub_enqueue(s, [e] {
    std::lock_guard<std::mutex> lk(e->mu);
    e->t = now_s();
    --e->pending;
    e->cv.notify_all();
  });
}

hipError_t hipEventSynchronize(hipEvent_t e) {
  std::unique_lock<std::mutex> lk(e->mu);
  e->cv.wait(lk, [&] { return e->pending == 0; });
  return hipSuccess;
}

hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  double ta, tb;
  {
    std::lock_guard<std::mutex> lk(a->mu);
    if (a->pending) return hipErrorNotReady;
    ta = a->t;
  }
  {
    std::lock_guard<std::mutex> lk(b->mu);
    if (b->pending) return hipErrorNotReady;
    tb = b->t;
  }
  *ms = (float)((tb - ta) * 1e3);
  return hipSuccess;
}

hipError_t hipStreamBeginCapture(hipStream_t sh, hipStreamCaptureMode) {
  if (!sh) return hipErrorInvalidValue;   // the legacy stream cannot be captured
  std::lock_guard<std::mutex> lk(sh->mu);
  if (sh->capture) return hipErrorIllegalState;
  sh->capture = new ihipGraph();
  sh->capture_thread = std::this_thread::get_id();
  return hipSuccess;
}

hipError_t hipStreamEndCapture(hipStream_t sh, hipGraph_t* g) {
  std::lock_guard<std::mutex> lk(sh->mu);
  if (!sh->capture) return hipErrorIllegalState;
  *g = sh->capture;
  sh->capture = nullptr;
  return hipSuccess;
}

hipError_t hipGraphDestroy(hipGraph_t g) {
  delete g;
  return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  *x = new hipGraphExec();
  (*x)->ops = g->ops;
  return hipSuccess;
}

hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
  for (const auto& op : x->ops) {
    hipError_t e = stub_enqueue(s, op);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
  delete x;
  return hipSuccess;
}

}  // extern "C"
