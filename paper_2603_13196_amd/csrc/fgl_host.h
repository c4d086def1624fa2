// Host-side model object shared by the C-ABI (fgl_host.cpp) and the serving
// loop (fgl_serve.cpp).  Internal; the public interface is include/fgl.h.
#pragma once
#include "../../include/fgl.h"
#include "fgl_internal.h"

#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

namespace fgl {

// Workspace bound to one stream of one model.
struct WorkBuf {
  Work w{};
  int cap_rows = 0;
  double* d_theta = nullptr;   // staging for host-pointer calls
  double* d_out = nullptr;
  double* h_theta = nullptr;   // pinned
  double* h_out = nullptr;     // pinned
  bool stream_synced_free = false;  // old buffers may be freed at once
  size_t gpart_bytes = 0;      // capacity of w.gpart
  double* d_grad = nullptr;    // gradient staging for host-pointer calls
  double* h_grad = nullptr;    // pinned
  size_t grad_bytes = 0;       // capacity of d_grad / h_grad
};

// A captured call: host-pointer calls run on the model's staging buffers
// (theta, out and stream NULL); device-pointer calls also key on the
// caller's buffers and stream.
struct GraphKey {
  int kind, B, waves, fc, occ;
  const void* theta = nullptr;
  const void* out = nullptr;
  const void* stream = nullptr;
  bool operator<(const GraphKey& o) const {
    if (kind != o.kind) return kind < o.kind;
    if (B != o.B) return B < o.B;
    if (waves != o.waves) return waves < o.waves;
    if (fc != o.fc) return fc < o.fc;
    if (occ != o.occ) return occ < o.occ;
    if (theta != o.theta) return theta < o.theta;
    if (out != o.out) return out < o.out;
    return stream < o.stream;
  }
};

struct GraphEntry {
  hipGraphExec_t exec = nullptr;
};

struct Model {
  int dev = 0;
  int N = 0, F = 0, T = 0, P = 0;
  double nu_ref = 0.0, t_cmb = 0.0;
  unsigned flags = 0;
  DevModel dm{};
  bool resident = false;
  bool autotune = false;
  bool use_graphs = true;       // host-pointer calls: replay captured graphs
  bool device_graphs = false;   // device-pointer calls too (FGL_DEVICE_GRAPHS=1)
  bool async_calls = false;     // a device-pointer call was made (eviction then waits)
  hipStream_t stream = nullptr;
  std::mutex mu;                        // serialises calls on this model
  std::atomic<int> inflight{0};         // synchronous calls in progress
  std::atomic<int> served{0};           // serving requests not yet done
  std::atomic<bool> dying{false};
  std::map<hipStream_t, WorkBuf> work;  // per-stream workspaces
  std::vector<WorkBuf> retired;         // outgrown workspaces (freed at destroy)
  std::map<GraphKey, GraphEntry> graphs;
  std::unordered_map<uint64_t, Tile> tiles;  // tuned tiles per (kind, B bucket)
  std::unordered_map<uint64_t, uint64_t> tc_miss;  // tuner-cache misses, by cache generation
  std::string arch;                           // device architecture, e.g. gfx950
  // host copies of the device layouts (re-uploaded after an eviction)
  std::vector<int8_t> h_kd;
  std::vector<int32_t> h_eK;
  std::vector<float> h_k32, h_k64, h_kthin;
  std::vector<double> h_nl64, h_nl2, h_nu, h_D, h_tab;
  std::vector<int8_t> h_rd;                  // projected form (empty if unused)
  std::vector<int32_t> h_eR;
  std::vector<double> h_tg, h_dbar, h_pk;
  std::vector<double> h_pa64, h_pt64;        // projected rows in FP64 (gradient)
  std::vector<float> h_r32;                  // projected rows in FP32 (FGL_PLAIN_PROJECTED)
  // serving bookkeeping
  uint64_t last_use = 0;
  // kernel timing (fgl_kernel_timing): 0 off, n > 0 events around every
  // n-th launch (timing_n counts the launches since it was set)
  int timing = 0;
  uint64_t timing_n = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used, ev_free;
};

struct InflightGuard {
  Model* m;
  explicit InflightGuard(Model* mm) : m(mm) { m->inflight.fetch_add(1); }
  ~InflightGuard() { m->inflight.fetch_sub(1); }
};

int set_err(int code, const char* fmt, ...);
int hip_err(hipError_t e, const char* what);
const char* last_error();
int check_device(int* dev_out);   // current device, gfx950 required

size_t resident_bytes(const Model* m);
int make_resident(Model* m);
void evict(Model* m);
int ensure_work(Model* m, WorkBuf& wb, int B, int ngroups, bool host_io);
Kind kind_of(int prec, const DevModel& d);
int group_of(Kind k, const DevModel& d);
std::vector<Tile> candidates(Kind k, const DevModel& d);
Tile default_tile(Kind k, const DevModel& d, int B);
Tile tile_for(Model* m, Kind k, int B);
int bucket_of(int B);
int enqueue(Model* m, Kind k, const Tile& tile, WorkBuf& wb,
            const double* d_theta, int B, double* d_out, hipStream_t s);
int enqueue_partials(Model* m, Kind k, const Tile& tile, WorkBuf& wb,
                     const double* d_theta, int B, hipStream_t s);
// The likelihood kernel alone, on rows whose records the caller has already
// prepared (the chain kernels prepare their proposals' rows themselves).
int enqueue_main(Model* m, Kind k, const Tile& tile, WorkBuf& wb, hipStream_t s);
int tune(Model* m, Kind k, WorkBuf& wb, const double* d_theta, int B,
         double* d_out, hipStream_t s);
void drop_stream_work(hipStream_t s);   // fgl_host.cpp
int tune_cache_set(const char* path);   // fgl_host.cpp
void serve_forget_model(Model* m);      // fgl_serve.cpp

// A roctx range around a library call, for rocprofv3 --marker-trace (or
// --sys-trace / --runtime-trace): active only when the environment sets
// FGL_ROCTX=1 at the first call, and then only if the roctx library can be
// loaded (it is looked up at run time; nothing links against it).  The
// label is formatted only when active.
class TraceRange {
 public:
  explicit TraceRange(const char* fmt, ...) __attribute__((format(printf, 2, 3)));
  ~TraceRange();
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;

 private:
  bool on_;
};

}  // namespace fgl
