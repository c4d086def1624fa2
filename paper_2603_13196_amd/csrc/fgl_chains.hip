// Device-resident slice-sampling chains for batched nested sampling.
//
// One call advances n hit-and-run slice chains, each by `steps` steps under
// the constraint lnL > lnL* inside the prior box (the replacement step of
// nested slice sampling, Tutt et al. Sec. 3.1.2 and 3.1.3).  Every round
// proposes one point per chain (k_chain_propose), evaluates all n rows with
// the model's likelihood kernels, and advances each chain's state machine
// (k_chain_update):
//   stepping out:  the interval ends move out by one unit (in the geometry
//                  whitened by the caller's Cholesky factor) while they are
//                  inside the constrained region;
//   shrinking:     a uniform point of the interval is accepted if inside,
//                  otherwise the interval is cut at it.
// A chain that has finished its steps keeps its point and proposes nothing
// new.  Rounds are captured once into a hipGraph (R rounds per graph) and
// replayed; the host reads the chains' stages after each replay and stops
// when every chain is done.
//
// Coordinates: the sampler works in z = [beta.., A, nu21, w, log sigma] (or
// [beta.., log sigma] without the 21-cm term), uniform over the box; the
// likelihood row is z with its last entry exponentiated.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC 2011), keyed by the seed, with the
// chain index and a per-chain counter as the counter block; the counters
// start at zero when the engine is created and keep counting across calls,
// so no draw is ever repeated.  Uniforms take 53 bits, normals come from the
// Box-Muller transform.
#include "fgl_host.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace fgl {

namespace {

constexpr int kLeft = 0, kRight = 1, kShrink = 2, kDone = 3;
constexpr int kMaxExpand = 64;
constexpr int kRoundsPerGraph = 32;

struct ChainState {
  int n, P;
  double* x;        // [n][P] current points (sampler coordinates)
  double* dir;      // [n][P] step directions
  double* a;        // [n] interval, in units of dir
  double* b;
  double* t;        // [n] last proposal's position
  double* lx;       // [n] lnL at x
  int* stage;       // [n]
  int* done;        // [n] finished steps
  int* expand;      // [n] expansions of the current side
  int* evals;       // [n] in-box proposals evaluated
  unsigned long long* ctr;   // [n] Philox counter
  double* theta;    // [n][P] likelihood rows of the proposals
  int* inbox;       // [n]
  double* lnl;      // [n] likelihood of the proposals
  const double* chol;  // [P][P] lower-triangular whitening factor
  const double* lo;    // [P]
  const double* hi;    // [P]
  const double* lstar; // the constraint lnL > *lstar (device memory, so a
                       // captured graph stays valid across iterations)
  unsigned long long seed;
  int steps;
};

// --- Philox4x32-10 --------------------------------------------------------

__device__ inline void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)M0 * c[0];
    const uint64_t p1 = (uint64_t)M1 * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0;
    const uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += W0;
    k1 += W1;
  }
}

// Two uniforms in [0, 1) with 53 random bits each, from one Philox block.
__device__ inline void uniform2(const ChainState& s, int i, double& u0, double& u1) {
  const unsigned long long c = s.ctr[i]++;
  uint32_t v[4] = {(uint32_t)c, (uint32_t)(c >> 32), (uint32_t)i, 0x5eed5eedu};
  philox(v, (uint32_t)s.seed, (uint32_t)(s.seed >> 32));
  const uint64_t a = ((uint64_t)v[0] << 32 | v[1]) >> 11;
  const uint64_t b = ((uint64_t)v[2] << 32 | v[3]) >> 11;
  u0 = (double)a * 0x1.0p-53;
  u1 = (double)b * 0x1.0p-53;
}

// A new slice step: direction uniform on the unit sphere in whitened
// coordinates, mapped by the Cholesky factor; unit interval at a random
// offset around the current point.
__device__ void new_step(const ChainState& s, int i) {
  const int P = s.P;
  double* d = s.dir + (size_t)i * P;
  double nrm = 0.0;
  // the direction needs randomness, not precision: the Box-Muller pairs are
  // formed with the FP32 hardware transcendentals
  for (int k = 0; k < P; k += 2) {
    double u0, u1;
    uniform2(s, i, u0, u1);
    const float v = (float)(1.0 - u0);                  // in (0, 1]
    const float rad = __builtin_sqrtf(-2.0f * __logf(v));
    const float ang = 6.2831853f * (float)u1;
    const double z0 = (double)(rad * __cosf(ang)), z1 = (double)(rad * __sinf(ang));
    d[k] = z0;
    nrm += z0 * z0;
    if (k + 1 < P) {
      d[k + 1] = z1;
      nrm += z1 * z1;
    }
  }
  const double inv = 1.0 / sqrt(nrm);
  // dir = L u, L lower triangular; walk rows from the bottom so each u_k is
  // read before it is overwritten
  for (int j = P - 1; j >= 0; --j) {
    double acc = 0.0;
    for (int k = 0; k <= j; ++k) acc += s.chol[(size_t)j * P + k] * d[k];
    d[j] = acc * inv;
  }
  double r, unused;
  uniform2(s, i, r, unused);
  s.a[i] = -r;
  s.b[i] = 1.0 - r;
  s.stage[i] = kLeft;
  s.expand[i] = 0;
}

__global__ void k_chain_init(ChainState s, const double* x0, const double* l0) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.n) return;
  for (int k = 0; k < s.P; ++k) s.x[(size_t)i * s.P + k] = x0[(size_t)i * s.P + k];
  s.lx[i] = l0[i];
  s.done[i] = 0;
  s.evals[i] = 0;
  s.t[i] = 0.0;                   // ctr keeps counting across calls: fresh numbers every call
  if (s.steps > 0)
    new_step(s, i);
  else
    s.stage[i] = kDone;
}

// The likelihood row of a point: z with log sigma exponentiated.
__device__ inline void write_row(const ChainState& s, int i, const double* z) {
  double* th = s.theta + (size_t)i * s.P;
  for (int k = 0; k < s.P - 1; ++k) th[k] = z[k];
  th[s.P - 1] = exp(z[s.P - 1]);
}

__global__ void k_chain_propose(ChainState s) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.n) return;
  const int P = s.P;
  const double* x = s.x + (size_t)i * P;
  const int st = s.stage[i];
  if (st == kDone) {
    write_row(s, i, x);
    s.inbox[i] = 0;
    return;
  }
  double t;
  if (st == kShrink) {
    double u, unused;
    uniform2(s, i, u, unused);
    t = s.a[i] + (s.b[i] - s.a[i]) * u;
  } else {
    t = st == kLeft ? s.a[i] : s.b[i];
  }
  s.t[i] = t;
  const double* d = s.dir + (size_t)i * P;
  double* th = s.theta + (size_t)i * P;
  int in = 1;
  for (int k = 0; k < P; ++k) {
    const double p = x[k] + t * d[k];
    in &= (p >= s.lo[k]) & (p <= s.hi[k]);
    th[k] = p;
  }
  if (in)
    th[P - 1] = exp(th[P - 1]);
  else
    write_row(s, i, x);        // a valid row; its result is ignored
  s.inbox[i] = in;
}

__device__ inline void finish_step(const ChainState& s, int i) {
  s.done[i] += 1;
  if (s.done[i] >= s.steps)
    s.stage[i] = kDone;
  else
    new_step(s, i);
}

__global__ void k_chain_update(ChainState s) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.n) return;
  const double lstar = *s.lstar;
  const int st = s.stage[i];
  if (st == kDone) return;
  const double lp = s.lnl[i];
  const bool in = s.inbox[i] != 0;
  if (in) s.evals[i] += 1;
  const bool inside = in && (lp > lstar);          // NaN and -inf are outside
  if (st == kLeft || st == kRight) {
    if (inside && s.expand[i] < kMaxExpand) {
      if (st == kLeft)
        s.a[i] -= 1.0;
      else
        s.b[i] += 1.0;
      s.expand[i] += 1;
    } else {
      s.stage[i] = st == kLeft ? kRight : kShrink;
      s.expand[i] = 0;
    }
    return;
  }
  // shrinking
  const double t = s.t[i];
  if (inside) {
    const int P = s.P;
    double* x = s.x + (size_t)i * P;
    const double* d = s.dir + (size_t)i * P;
    for (int k = 0; k < P; ++k) x[k] = x[k] + t * d[k];    // the proposal, recomputed exactly
    s.lx[i] = lp;
    finish_step(s, i);
    return;
  }
  if (t < 0.0)
    s.a[i] = t;
  else
    s.b[i] = t;
  // an interval shrunk to nothing (a likelihood plateau at lnL*): keep the point
  if (s.b[i] - s.a[i] < 1e-12) finish_step(s, i);
}

}  // namespace

// ---------------------------------------------------------------------------
// host engine

struct Chains {
  Model* m = nullptr;
  int cap = 0, P = 0;
  ChainState st{};
  double *d_x0 = nullptr, *d_l0 = nullptr, *d_chol = nullptr, *d_lo = nullptr, *d_hi = nullptr;
  double* d_lstar = nullptr;
  int* h_stage = nullptr;                       // pinned
  std::vector<double> lo, hi;
  unsigned long long seed = 0;
  unsigned long long calls = 0;
  hipStream_t s = nullptr;
  // graph of kRoundsPerGraph rounds; rebuilt when the chain count, the
  // precision, the steps or any buffer it captured changes
  hipGraphExec_t graph = nullptr;
  int g_n = -1, g_prec = -1, g_steps = -1;
  const void* g_model = nullptr;      // model buffers at capture (eviction moves them)
  const void* g_work = nullptr;       // likelihood workspace at capture
  Tile g_tile{};
};

static void chains_free(Chains* c) {
  void* ps[] = {c->st.x, c->st.dir, c->st.a, c->st.b, c->st.t, c->st.lx, c->st.stage,
                c->st.done, c->st.expand, c->st.evals, c->st.ctr, c->st.theta, c->st.inbox,
                c->st.lnl, c->d_x0, c->d_l0, c->d_chol, c->d_lo, c->d_hi, c->d_lstar};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  if (c->h_stage) (void)hipHostFree(c->h_stage);
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  if (c->s) (void)hipStreamDestroy(c->s);
}

template <typename T>
static hipError_t dalloc(T** p, size_t n) {
  return hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(n * sizeof(T), 16));
}

}  // namespace fgl

using namespace fgl;

extern "C" {

int fgl_chains_create(fgl_model* mh, int max_chains, const double* lo, const double* hi,
                      uint64_t seed, fgl_chains** out) {
  if (!out) return set_err(FGL_EINVAL, "out is NULL");
  *out = nullptr;
  Model* m = reinterpret_cast<Model*>(mh);
  if (!m || !lo || !hi) return set_err(FGL_EINVAL, "model, lo and hi must be non-NULL");
  if (max_chains < 1) return set_err(FGL_EINVAL, "max_chains=%d < 1", max_chains);
  const int P = m->P;
  for (int k = 0; k < P; ++k)
    if (!std::isfinite(lo[k]) || !std::isfinite(hi[k]) || !(lo[k] < hi[k]))
      return set_err(FGL_EINVAL, "box coordinate %d: need finite lo < hi", k);
  Chains* c = new (std::nothrow) Chains();
  if (!c) return set_err(FGL_ENOMEM, "host allocation");
  c->m = m;
  c->cap = max_chains;
  c->P = P;
  c->lo.assign(lo, lo + P);
  c->hi.assign(hi, hi + P);
  c->seed = seed;
  hipError_t e = hipSetDevice(m->dev);
  const size_t n = (size_t)max_chains;
  ChainState& s = c->st;
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->s, hipStreamNonBlocking);
  if (e == hipSuccess) e = dalloc(&s.x, n * P);
  if (e == hipSuccess) e = dalloc(&s.dir, n * P);
  if (e == hipSuccess) e = dalloc(&s.a, n);
  if (e == hipSuccess) e = dalloc(&s.b, n);
  if (e == hipSuccess) e = dalloc(&s.t, n);
  if (e == hipSuccess) e = dalloc(&s.lx, n);
  if (e == hipSuccess) e = dalloc(&s.stage, n);
  if (e == hipSuccess) e = dalloc(&s.done, n);
  if (e == hipSuccess) e = dalloc(&s.expand, n);
  if (e == hipSuccess) e = dalloc(&s.evals, n);
  if (e == hipSuccess) e = dalloc(&s.ctr, n);
  if (e == hipSuccess) e = dalloc(&s.theta, n * P);
  if (e == hipSuccess) e = dalloc(&s.inbox, n);
  if (e == hipSuccess) e = dalloc(&s.lnl, n);
  if (e == hipSuccess) e = dalloc(&c->d_x0, n * P);
  if (e == hipSuccess) e = dalloc(&c->d_l0, n);
  if (e == hipSuccess) e = dalloc(&c->d_chol, (size_t)P * P);
  if (e == hipSuccess) e = dalloc(&c->d_lo, (size_t)P);
  if (e == hipSuccess) e = dalloc(&c->d_hi, (size_t)P);
  if (e == hipSuccess) e = dalloc(&c->d_lstar, 1);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&c->h_stage), n * sizeof(int), hipHostMallocDefault);
  if (e == hipSuccess) e = hipMemset(s.ctr, 0, n * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMemcpy(c->d_lo, lo, P * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->d_hi, hi, P * 8, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    chains_free(c);
    delete c;
    return hip_err(e, "allocating chain state");
  }
  s.P = P;
  s.chol = c->d_chol;
  s.lo = c->d_lo;
  s.hi = c->d_hi;
  s.lstar = c->d_lstar;
  s.seed = seed;
  m->served.fetch_add(1);       // the model stays alive while the engine exists
  *out = reinterpret_cast<fgl_chains*>(c);
  return FGL_OK;
}

int fgl_chains_run(fgl_chains* ch, const double* x0, const double* l0, int n, double lstar,
                   const double* chol, int steps, int prec, double* x_out, double* l_out,
                   int64_t* evals, int64_t* rounds) {
  Chains* c = reinterpret_cast<Chains*>(ch);
  if (!c || !x0 || !l0 || !chol || !x_out || !l_out)
    return set_err(FGL_EINVAL, "NULL argument");
  if (n < 1 || n > c->cap) return set_err(FGL_EINVAL, "n=%d outside 1..%d", n, c->cap);
  if (steps < 0) return set_err(FGL_EINVAL, "steps=%d < 0", steps);
  if (prec != FGL_PREC_MIXED && prec != FGL_PREC_FP32 && prec != FGL_PREC_FP64)
    return set_err(FGL_EINVAL, "unknown precision %d", prec);
  if (std::isnan(lstar)) return set_err(FGL_EINVAL, "lstar is NaN");
  Model* m = c->m;
  const int P = c->P;
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < P; ++k) {
      const double v = x0[(size_t)i * P + k];
      if (!(v >= c->lo[k] && v <= c->hi[k]))
        return set_err(FGL_EINVAL, "start point %d is outside the box (coordinate %d)", i, k);
    }
  InflightGuard guard(m);
  std::lock_guard<std::mutex> lk(m->mu);
  hipError_t e = hipSetDevice(m->dev);
  if (e != hipSuccess) return hip_err(e, "hipSetDevice");
  int rc = make_resident(m);
  if (rc != FGL_OK) return rc;
  hipStream_t s = c->s;
  ChainState st = c->st;
  st.n = n;
  st.steps = steps;
  if ((e = hipMemcpyAsync(c->d_x0, x0, (size_t)n * P * 8, hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(c->d_l0, l0, (size_t)n * 8, hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(c->d_chol, chol, (size_t)P * P * 8, hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(c->d_lstar, &lstar, 8, hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_err(e, "copy chain inputs");
  const int threads = 128, blocks = (n + threads - 1) / threads;
  hipLaunchKernelGGL(k_chain_init, dim3(blocks), dim3(threads), 0, s, st, c->d_x0, c->d_l0);
  if ((e = hipGetLastError()) != hipSuccess) return hip_err(e, "chain init");
  // the likelihood's workspace for n rows on this stream, fixed before capture
  const Kind k = kind_of(prec);
  const Tile tile = tile_for(m, k, n);
  WorkBuf& wb = m->work[s];
  wb.stream_synced_free = true;
  if ((rc = ensure_work(m, wb, n, n_groups(m->dm, tile), false)) != FGL_OK) return rc;
  auto round = [&]() -> int {
    hipLaunchKernelGGL(k_chain_propose, dim3(blocks), dim3(threads), 0, s, st);
    hipError_t e2 = hipGetLastError();
    if (e2 != hipSuccess) return hip_err(e2, "chain proposal");
    int rc2 = enqueue(m, k, tile, wb, st.theta, n, st.lnl, s);
    if (rc2 != FGL_OK) return rc2;
    hipLaunchKernelGGL(k_chain_update, dim3(blocks), dim3(threads), 0, s, st);
    e2 = hipGetLastError();
    return e2 == hipSuccess ? FGL_OK : hip_err(e2, "chain update");
  };
  // one eager round (it also sets the kernels' launch attributes outside
  // any capture), then kRoundsPerGraph rounds captured once and replayed
  if ((rc = round()) != FGL_OK) return rc;
  long long done_rounds = 1;
  const void* model_buf = m->dm.proj ? (const void*)m->dm.rd : (const void*)m->dm.kd;
  if (c->graph && (c->g_n != n || c->g_prec != prec || c->g_steps != steps ||
                   c->g_model != model_buf || c->g_work != (const void*)wb.w.partial ||
                   c->g_tile.waves != tile.waves || c->g_tile.fc != tile.fc ||
                   c->g_tile.occ != tile.occ)) {
    (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
  }
  const bool timing = m->timing;
  if (!c->graph && !timing) {
    hipGraph_t g = nullptr;
    if ((e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return hip_err(e, "begin capture");
    int crc = FGL_OK;
    for (int r = 0; r < kRoundsPerGraph && crc == FGL_OK; ++r) crc = round();
    e = hipStreamEndCapture(s, &g);
    if (crc != FGL_OK) {
      if (g) (void)hipGraphDestroy(g);
      return crc;
    }
    if (e != hipSuccess) return hip_err(e, "end capture");
    e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      c->graph = nullptr;
      return hip_err(e, "graph instantiate");
    }
    c->g_n = n;
    c->g_prec = prec;
    c->g_steps = steps;
    c->g_model = model_buf;
    c->g_work = wb.w.partial;
    c->g_tile = tile;
  }
  // replay until every chain is done; the bound covers steps of at most
  // 2 kMaxExpand + 64 rounds each
  const long long max_rounds = (long long)std::max(steps, 1) * (2 * kMaxExpand + 66);
  while (done_rounds < max_rounds) {
    if (c->graph) {
      if ((e = hipGraphLaunch(c->graph, s)) != hipSuccess) return hip_err(e, "graph launch");
    } else {
      for (int r = 0; r < kRoundsPerGraph; ++r)
        if ((rc = round()) != FGL_OK) return rc;
    }
    done_rounds += kRoundsPerGraph;
    if ((e = hipMemcpyAsync(c->h_stage, st.stage, (size_t)n * sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
      return hip_err(e, "chain progress");
    bool all = true;
    for (int i = 0; i < n && all; ++i) all = c->h_stage[i] == kDone;
    if (all) break;
  }
  std::vector<int> ev(n);
  if ((e = hipMemcpyAsync(x_out, st.x, (size_t)n * P * 8, hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipMemcpyAsync(l_out, st.lx, (size_t)n * 8, hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipMemcpyAsync(ev.data(), st.evals, (size_t)n * sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return hip_err(e, "copy chain results");
  bool all = true;
  for (int i = 0; i < n && all; ++i) all = c->h_stage[i] == kDone;
  if (!all) return set_err(FGL_EAGAIN, "chains did not finish within %lld rounds", max_rounds);
  if (evals) {
    int64_t sum = 0;
    for (int v : ev) sum += v;
    *evals = sum;
  }
  if (rounds) *rounds = done_rounds;
  c->calls++;
  return FGL_OK;
}

int fgl_chains_destroy(fgl_chains* ch) {
  Chains* c = reinterpret_cast<Chains*>(ch);
  if (!c) return set_err(FGL_EINVAL, "chains is NULL");
  (void)hipSetDevice(c->m->dev);
  if (c->s) (void)hipStreamSynchronize(c->s);
  if (c->s) drop_stream_work(c->s);
  chains_free(c);
  c->m->served.fetch_sub(1);
  delete c;
  return FGL_OK;
}

}  // extern "C"
