// The likelihood's device entry point without allocation
// (fgl_loglike_batch_device_noalloc in include/fgl.h).
//
// fgl_loglike_batch_device keeps a workspace per (model, stream) and grows
// it with hipMalloc.  Callers that cannot allocate (code under stream
// capture, tight serving loops, harnesses that forbid it) call this variant
// instead: the same row preparation, likelihood kernel and finalize, with the
// workspace carved out of one file-scope device array per GPU.
//
// The workspace holds, for B rows padded to Bpad: the transposed spectral
// indices (and log2 amplitude scales), one row record per row and one
// chi-square partial per (reduction group, row).  Every one of them is
// written for all Bpad rows by the preparation and likelihood kernels before
// it is read, so nothing has to start at zero and the contents a previous
// call left behind never matter.  Calls that overlap on one GPU share the
// array and race; the caller orders them (one stream, or events).
#include "fgl_host.h"

#include <mutex>

namespace fgl {

constexpr size_t kScratchBytes = size_t(64) << 20;   // per GPU
constexpr size_t kAlign = 256;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of this GPU's scratch array, looked up once per device
// with that device current (the array's name in host code is only a stand-in
// for the symbol, not an address).
int scratch_for(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return set_err(FGL_EDEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_err(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
  return FGL_OK;
}

size_t round_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

}  // namespace

}  // namespace fgl

using namespace fgl;

extern "C" int fgl_loglike_batch_device_noalloc(fgl_model* mh, const double* d_theta, int B,
                                                double* d_out, int prec, void* hip_stream) {
  TraceRange tr("fgl_loglike_batch_device_noalloc prec=%d B=%d", prec, B);
  Model* m = reinterpret_cast<Model*>(mh);
  if (!m) return set_err(FGL_EINVAL, "model is NULL");
  if (B < 0 || B > kMaxRows) return set_err(FGL_EINVAL, "B=%d outside 0..2^26", B);
  if (prec != FGL_PREC_MIXED && prec != FGL_PREC_FP32 && prec != FGL_PREC_FP64)
    return set_err(FGL_EINVAL, "unknown precision %d", prec);
  if (m->dying.load()) return set_err(FGL_EBUSY, "model is being destroyed");
  if (B == 0) return FGL_OK;
  if (!d_theta || !d_out) return set_err(FGL_EINVAL, "d_theta and d_out must be non-NULL");
  InflightGuard guard(m);
  std::lock_guard<std::mutex> lk(m->mu);
  m->async_calls = true;
  hipError_t e = hipSetDevice(m->dev);
  if (e != hipSuccess) return hip_err(e, "hipSetDevice");
  if (!m->resident)
    return set_err(FGL_EAGAIN, "the model is not resident on the device (a server evicted it); "
                               "an allocating call makes it resident again");
  const Kind k = kind_of(prec, m->dm);
  const Tile tile = tile_for(m, k, B);
  // the workspace of B rows, as ensure_work lays it out (rows padded to a
  // multiple of 256)
  const int Bpad = std::max(256, (B + 255) / 256 * 256);
  const int betaRows = m->dm.KC * 32;
  const int ngroups = n_groups(m->dm, tile);
  const size_t b_beta = round_up((size_t)betaRows * Bpad * 8);
  const size_t b_off = m->dm.NA > 0 ? b_beta : 0;
  const size_t b_rows = round_up((size_t)Bpad * sizeof(RowParams));
  const size_t b_part = round_up((size_t)ngroups * Bpad * 8);
  const size_t need = b_beta + b_off + b_rows + b_part;
  if (need > kScratchBytes) {
    const size_t per_row = (size_t)betaRows * 8 * (m->dm.NA > 0 ? 2 : 1) + sizeof(RowParams) +
                           (size_t)ngroups * 8;
    return set_err(FGL_EINVAL,
                   "B=%d on this model needs %zu bytes of workspace; the allocation-free call "
                   "has %zu per GPU (about %zu rows of this model)",
                   B, need, kScratchBytes, kScratchBytes / per_row / 256 * 256);
  }
  unsigned char* base = nullptr;
  int rc = scratch_for(m->dev, &base);
  if (rc != FGL_OK) return rc;
  Work w{};
  w.B = B;
  w.Bpad = Bpad;
  w.betaT = reinterpret_cast<double*>(base);
  w.offT = m->dm.NA > 0 ? reinterpret_cast<double*>(base + b_beta) : nullptr;
  w.rows = reinterpret_cast<RowParams*>(base + b_beta + b_off);
  w.partial = reinterpret_cast<double*>(base + b_beta + b_off + b_rows);
  w.ngroup_cap = ngroups;
  w.gpart = nullptr;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  if ((e = launch_prep(m->dm, d_theta, B, w, betaRows, s)) != hipSuccess)
    return hip_err(e, "prep kernel");
  if ((e = launch_main(k, m->dm, w, tile, s)) != hipSuccess)
    return hip_err(e, "likelihood kernel");
  if ((e = launch_finalize(k, m->dm, w, tile, d_out, s)) != hipSuccess)
    return hip_err(e, "finalize kernel");
  return FGL_OK;
}
