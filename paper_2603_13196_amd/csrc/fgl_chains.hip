// Device-resident slice-sampling chains for batched nested sampling.
//
// One call advances n hit-and-run slice chains, each by `steps` steps under
// the constraint lnL > lnL* inside the prior box (the replacement step of
// nested slice sampling, Tutt et al. Sec. 3.1.2 and 3.1.3).  A round is the
// model's row preparation and likelihood kernel over the n proposal rows,
// then k_chain_step, one wavefront per chain, which
//   * forms each row's lnL from the likelihood kernel's partial sums, in the
//     order and arithmetic of the library's finalize (so it equals what
//     fgl_loglike_batch returns for that row, bit for bit),
//   * advances the chain's state machine:
//       stepping out:  the interval ends move out by one unit (in the
//                      geometry whitened by the caller's Cholesky factor)
//                      while they are inside the constrained region;
//       shrinking:     a uniform point of the interval is accepted if
//                      inside, otherwise the interval is cut at it,
//   * and writes the chain's next proposal row.
// The lanes of a chain's wavefront share its coordinates (directions,
// Cholesky product, proposal) and its lnL reduction.  A chain that has
// finished its steps keeps its point and proposes nothing new.  Rounds are
// captured once into a hipGraph (R rounds per graph) and replayed; the host
// reads the chains' stages after each replay and stops when every chain is
// done.
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
#include "fgl_philox.h"

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
  // the likelihood's row records and transposed indices of the proposals,
  // written by the chain kernels themselves (the model's N = NA' NB regions,
  // NA' = max(NA, 1), betaRows = 32 KC transposed rows)
  RowParams* rows;
  double* betaT;
  double* offT;
  int Bpad, N, NA, NB, betaRows;
  unsigned flags;
};

// Two uniforms in [0, 1) with 53 random bits each, from Philox block c of
// chain i.
__device__ inline void uniform2(const ChainState& s, int i, unsigned long long c, double& u0,
                                double& u1) {
  uint32_t v[4] = {(uint32_t)c, (uint32_t)(c >> 32), (uint32_t)i, 0x5eed5eedu};
  philox4x32(v, (uint32_t)s.seed, (uint32_t)(s.seed >> 32));
  const uint64_t a = ((uint64_t)v[0] << 32 | v[1]) >> 11;
  const uint64_t b = ((uint64_t)v[2] << 32 | v[3]) >> 11;
  u0 = (double)a * 0x1.0p-53;
  u1 = (double)b * 0x1.0p-53;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

constexpr int kMaxP = 160;            // parameters a chain's LDS direction holds
constexpr int kWaves = 4;             // chains (wavefronts) per workgroup

// Per-chain scalars, held in registers (uniform across the wavefront) while a
// kernel works on the chain and written back by lane 0.
struct Scal {
  double a, b, t, lx;
  int stage, done, expand, evals;
  unsigned long long ctr;
};

__device__ inline Scal load_scal(const ChainState& s, int i) {
  return Scal{s.a[i], s.b[i], s.t[i], s.lx[i], s.stage[i], s.done[i], s.expand[i], s.evals[i],
              s.ctr[i]};
}

__device__ inline void store_scal(const ChainState& s, int i, const Scal& c, int lane) {
  if (lane != 0) return;
  s.a[i] = c.a;
  s.b[i] = c.b;
  s.t[i] = c.t;
  s.lx[i] = c.lx;
  s.stage[i] = c.stage;
  s.done[i] = c.done;
  s.expand[i] = c.expand;
  s.evals[i] = c.evals;
  s.ctr[i] = c.ctr;
}

// A new slice step: direction uniform on the unit sphere in whitened
// coordinates, mapped by the Cholesky factor; unit interval at a random
// offset around the current point.  Lane k/2 draws the normal pair of
// coordinates k, k + 1 (Philox block ctr + k/2); the pairs go through LDS
// so that lane j can form row j of the Cholesky product.
__device__ void new_step(const ChainState& s, int i, Scal& c, int lane, double* u) {
  const int P = s.P, np = (P + 1) / 2;
  double nrm = 0.0;
  // the direction needs randomness, not precision: the Box-Muller pairs are
  // formed with the FP32 hardware transcendentals
  for (int pr = lane; pr < np; pr += 64) {
    double u0, u1;
    uniform2(s, i, c.ctr + pr, u0, u1);
    const float v = (float)(1.0 - u0);                  // in (0, 1]
    const float rad = __builtin_sqrtf(-2.0f * __logf(v));
    const float ang = 6.2831853f * (float)u1;
    const double z0 = (double)(rad * __cosf(ang)), z1 = (double)(rad * __sinf(ang));
    u[2 * pr] = z0;
    nrm += z0 * z0;
    if (2 * pr + 1 < P) {
      u[2 * pr + 1] = z1;
      nrm += z1 * z1;
    }
  }
  nrm = wave_sum(nrm);
  __builtin_amdgcn_wave_barrier();                      // u written by all lanes
  const double inv = 1.0 / sqrt(nrm);
  double* d = s.dir + (size_t)i * P;
  for (int j = lane; j < P; j += 64) {                  // dir = L u, L lower triangular
    double acc = 0.0;
    for (int k = 0; k <= j; ++k) acc += s.chol[(size_t)j * P + k] * u[k];
    d[j] = acc * inv;
  }
  __builtin_amdgcn_wave_barrier();                      // u read by all lanes
  double r, unused;
  uniform2(s, i, c.ctr + np, r, unused);
  c.ctr += np + 1;
  c.a = -r;
  c.b = 1.0 - r;
  c.stage = kLeft;
  c.expand = 0;
}

// The row record and the transposed spectral indices (and log2 alpha) of
// likelihood row i, from the row's entries held by the chain's wavefront
// (v[q] is entry lane + 64 q), with the row-preparation kernel's rules:
// finite entries, |beta| <= 64, alpha in [2^-32, 2^32], sigma > 0 and
// w > 0; extremes of beta and log2 alpha; fills of the row's minimum for
// padded regions (zero for an invalid row).
__device__ void prep_row(const ChainState& s, int i, int lane, const double (&v)[3]) {
  const int P = s.P, NB = s.NB, NA = s.NA;
  const bool no21 = s.flags & 1u;
  int ok = 1;
  double bmin = INFINITY, bmax = -INFINITY, omin = INFINITY, omax = -INFINITY;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int k = lane + 64 * q;
    if (k < P) {
      const double x = v[q];
      ok = ok && isfinite(x);
      if (k < NB) {
        ok = ok && fabs(x) <= 64.0;
        bmin = fmin(bmin, x);
        bmax = fmax(bmax, x);
      } else if (k < NB + NA) {
        ok = ok && x >= 0x1p-32 && x <= 0x1p32;
        const double o = log2(x);
        omin = fmin(omin, o);
        omax = fmax(omax, o);
      }
    }
  }
  ok = __builtin_amdgcn_ballot_w64(!ok) == 0;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    bmin = fmin(bmin, __shfl_xor(bmin, m));
    bmax = fmax(bmax, __shfl_xor(bmax, m));
    omin = fmin(omin, __shfl_xor(omin, m));
    omax = fmax(omax, __shfl_xor(omax, m));
  }
  // entry k of the row (k may differ between lanes; every lane takes part)
  auto entry = [&](int k) {
    const double a0 = __shfl(v[0], k & 63), a1 = __shfl(v[1], k & 63);
    const double a2 = __shfl(v[2], k & 63);
    return k < 64 ? a0 : (k < 128 ? a1 : a2);
  };
  const double sig = entry(P - 1);
  const double wd = entry(no21 ? P - 1 : P - 2);
  const double amp = entry(no21 ? P - 1 : P - 4);
  const double nu0 = entry(no21 ? P - 1 : P - 3);
  if (ok) {
    ok = sig > 0.0;
    if (!no21) ok = ok && wd > 0.0;
  }
  if (!ok) bmin = bmax = 0.0;
  if (!ok || NA == 0) omin = omax = 0.0;
  if (lane == 0) {
    RowParams rp;
    rp.valid = ok ? 1 : 0;
    rp.pad = 0;
    rp.A = 0.0;
    rp.nu0 = 0.0;
    rp.inv_w = 1.0;
    rp.sigma = 1.0;
    rp.t21 = no21 ? 0.0 : 1.0;
    if (ok) {
      rp.sigma = sig;
      if (!no21) {
        rp.A = amp;
        rp.nu0 = nu0;
        rp.inv_w = 1.0 / wd;
      }
    }
    rp.bmin = bmin;
    rp.bmax = bmax;
    rp.omin = omin;
    rp.omax = omax;
    s.rows[i] = rp;
  }
  const int nq = (s.betaRows + 63) / 64;
  for (int q = 0; q < nq; ++q) {
    const int r = lane + 64 * q;
    const int ia = r / NB, jb = r - ia * NB;
    const bool real = ok && r < s.N;
    const double bv = entry(min(jb, P - 1));
    const double av = NA > 0 ? entry(min(NB + ia, P - 1)) : 1.0;
    if (r < s.betaRows) {
      s.betaT[(size_t)r * s.Bpad + i] = real ? bv : bmin;
      if (NA > 0) s.offT[(size_t)r * s.Bpad + i] = real ? log2(av) : omin;
    }
  }
}

// The chain's next likelihood row: the proposal x + t dir when it is inside
// the box, else (and for a finished chain) the chain's point itself, whose
// result is ignored.  The last coordinate is log sigma.  The row's record
// and transposed indices are prepared here too.
__device__ void propose(const ChainState& s, int i, Scal& c, int lane) {
  const int P = s.P;
  const double* x = s.x + (size_t)i * P;
  double* th = s.theta + (size_t)i * P;
  double v[3] = {0.0, 0.0, 0.0};
  if (c.stage == kDone) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int k = lane + 64 * q;
      if (k < P) {
        v[q] = k == P - 1 ? exp(x[k]) : x[k];
        th[k] = v[q];
      }
    }
    if (lane == 0) s.inbox[i] = 0;
    prep_row(s, i, lane, v);
    return;
  }
  double t;
  if (c.stage == kShrink) {
    double u, unused;
    uniform2(s, i, c.ctr, u, unused);
    c.ctr += 1;
    t = c.a + (c.b - c.a) * u;
  } else {
    t = c.stage == kLeft ? c.a : c.b;
  }
  c.t = t;
  const double* d = s.dir + (size_t)i * P;
  int out = 0;
  for (int k = lane; k < P; k += 64) {
    const double p = x[k] + t * d[k];
    out |= !((p >= s.lo[k]) & (p <= s.hi[k]));
  }
  const bool in = __builtin_amdgcn_ballot_w64(out != 0) == 0;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int k = lane + 64 * q;
    if (k < P) {
      const double p = in ? x[k] + t * d[k] : x[k];
      v[q] = k == P - 1 ? exp(p) : p;
      th[k] = v[q];
    }
  }
  if (lane == 0) s.inbox[i] = in ? 1 : 0;
  prep_row(s, i, lane, v);
}

__device__ inline void finish_step(const ChainState& s, int i, Scal& c, int lane, double* u) {
  c.done += 1;
  if (c.done >= s.steps)
    c.stage = kDone;
  else
    new_step(s, i, c, lane, u);
}

// The likelihood kernel's partial sums of row b, reduced as the library's
// finalize does (sixteen strided sums, then an xor tree).
struct RowSums {
  const double* partial;
  const RowParams* rows;
  int ngroup, Bpad;
  double nFT, chi0;
};

__device__ inline double row_lnl(const RowSums& r, int b, int lane) {
  double acc = 0.0;
  if (lane < 16)
    for (int c = lane; c < r.ngroup; c += 16) acc += r.partial[(size_t)c * r.Bpad + b];
  acc += __shfl_xor(acc, 8);
  acc += __shfl_xor(acc, 4);
  acc += __shfl_xor(acc, 2);
  acc += __shfl_xor(acc, 1);
  acc = __shfl(acc, 0);
  const RowParams rp = r.rows[b];
  if (!rp.valid) return -INFINITY;
  const double s2 = rp.sigma * rp.sigma;
  return -0.5 * (acc + r.chi0) / s2 - 0.5 * r.nFT * log(2.0 * M_PI * s2);
}

// Start: copy the starting points, draw every chain's first step and write
// its first proposal.
__global__ __launch_bounds__(64 * kWaves) void k_chain_start(ChainState s, const double* x0,
                                                             const double* l0) {
  __shared__ double s_u[kWaves][kMaxP];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = blockIdx.x * kWaves + wv;
  if (i >= s.n) return;
  const int P = s.P;
  for (int k = lane; k < P; k += 64) s.x[(size_t)i * P + k] = x0[(size_t)i * P + k];
  Scal c = load_scal(s, i);             // ctr keeps counting across calls: fresh numbers
  c.lx = l0[i];
  c.done = 0;
  c.evals = 0;
  c.t = 0.0;
  if (s.steps > 0)
    new_step(s, i, c, lane, s_u[wv]);
  else
    c.stage = kDone;
  propose(s, i, c, lane);
  store_scal(s, i, c, lane);
}

// One round's update from the likelihood of the last proposals, then the
// next proposal.
__global__ __launch_bounds__(64 * kWaves) void k_chain_step(ChainState s, RowSums rs) {
  __shared__ double s_u[kWaves][kMaxP];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = blockIdx.x * kWaves + wv;
  if (i >= s.n) return;
  const double lstar = *s.lstar;
  Scal c = load_scal(s, i);
  if (c.stage == kDone) return;
  const double lp = row_lnl(rs, i, lane);
  if (lane == 0) s.lnl[i] = lp;
  const bool in = s.inbox[i] != 0;
  if (in) c.evals += 1;
  const bool inside = in && (lp > lstar);          // NaN and -inf are outside
  if (c.stage == kLeft || c.stage == kRight) {
    if (inside && c.expand < kMaxExpand) {
      if (c.stage == kLeft)
        c.a -= 1.0;
      else
        c.b += 1.0;
      c.expand += 1;
    } else {
      c.stage = c.stage == kLeft ? kRight : kShrink;
      c.expand = 0;
    }
  } else if (inside) {                             // shrinking: accepted
    const int P = s.P;
    double* x = s.x + (size_t)i * P;
    const double* d = s.dir + (size_t)i * P;
    for (int k = lane; k < P; k += 64) x[k] = x[k] + c.t * d[k];   // the proposal, exactly
    c.lx = lp;
    finish_step(s, i, c, lane, s_u[wv]);
  } else {                                         // shrinking: cut the interval
    if (c.t < 0.0)
      c.a = c.t;
    else
      c.b = c.t;
    // an interval shrunk to nothing (a likelihood plateau at lnL*): keep the point
    if (c.b - c.a < 1e-12) finish_step(s, i, c, lane, s_u[wv]);
  }
  propose(s, i, c, lane);
  store_scal(s, i, c, lane);
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

// The chains' generator on its own: one thread per counter block.
__global__ void k_philox(const uint32_t* __restrict__ ctr, int n, uint32_t k0, uint32_t k1,
                         uint32_t* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  uint32_t c[4] = {ctr[4 * j], ctr[4 * j + 1], ctr[4 * j + 2], ctr[4 * j + 3]};
  philox4x32(c, k0, k1);
#pragma unroll
  for (int q = 0; q < 4; ++q) out[4 * j + q] = c[q];
}

constexpr int kPhiloxMaxBlocks = 1 << 24;

}  // namespace fgl

using namespace fgl;

extern "C" {

int fgl_chains_create(fgl_model* mh, int max_chains, const double* lo, const double* hi,
                      uint64_t seed, fgl_chains** out) {
  if (!out) return set_err(FGL_EINVAL, "out is NULL");
  *out = nullptr;
  Model* m = reinterpret_cast<Model*>(mh);
  if (!m || !lo || !hi) return set_err(FGL_EINVAL, "model, lo and hi must be non-NULL");
  if (max_chains < 1 || max_chains > kMaxRows)
    return set_err(FGL_EINVAL, "max_chains=%d outside 1..2^26", max_chains);
  const int P = m->P;
  if (P > kMaxP) return set_err(FGL_EINVAL, "P=%d exceeds the chains' %d parameters", P, kMaxP);
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
  TraceRange tr("fgl_chains_run n=%d steps=%d prec=%d", n, steps, prec);
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
  if (P > kMaxP) return set_err(FGL_EINVAL, "P=%d exceeds the chains' %d parameters", P, kMaxP);
  const int blocks = (n + kWaves - 1) / kWaves;
  // the likelihood's workspace for n rows on this stream, fixed before the
  // start kernel (which writes the first proposals' row records into it)
  // and before capture
  const Kind k = kind_of(prec, m->dm);
  const Tile tile = tile_for(m, k, n);
  WorkBuf& wb = m->work[s];
  wb.stream_synced_free = true;
  if ((rc = ensure_work(m, wb, n, n_groups(m->dm, tile), false)) != FGL_OK) return rc;
  st.rows = wb.w.rows;
  st.betaT = wb.w.betaT;
  st.offT = wb.w.offT;
  st.Bpad = wb.w.Bpad;
  st.N = m->dm.N;
  st.NA = m->dm.NA;
  st.NB = m->dm.NB;
  st.betaRows = m->dm.KC * 32;
  st.flags = m->dm.flags;
  hipLaunchKernelGGL(k_chain_start, dim3(blocks), dim3(64 * kWaves), 0, s, st, c->d_x0, c->d_l0);
  if ((e = hipGetLastError()) != hipSuccess) return hip_err(e, "chain start");
  // the padding rows up to Bpad (and the first proposals again, with the
  // same result) by the row-preparation kernel, once per call; later rounds
  // take the records the step kernel writes with each proposal
  if ((e = launch_prep(m->dm, st.theta, n, wb.w, m->dm.KC * 32, s)) != hipSuccess)
    return hip_err(e, "prep kernel");
  RowSums rs{wb.w.partial, wb.w.rows, n_groups(m->dm, tile), wb.w.Bpad,
             (double)m->dm.F * (double)m->dm.T,
             chi0_of(k, m->dm)};
  auto round = [&]() -> int {
    int rc2 = enqueue_main(m, k, tile, wb, s);
    if (rc2 != FGL_OK) return rc2;
    hipLaunchKernelGGL(k_chain_step, dim3(blocks), dim3(64 * kWaves), 0, s, st, rs);
    hipError_t e2 = hipGetLastError();
    return e2 == hipSuccess ? FGL_OK : hip_err(e2, "chain step");
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

int fgl_chains_philox(const uint32_t* ctr, int n, uint32_t k0, uint32_t k1, uint32_t* out) {
  if (!ctr || !out) return set_err(FGL_EINVAL, "ctr and out must be non-NULL");
  if (n < 1 || n > kPhiloxMaxBlocks)
    return set_err(FGL_EINVAL, "n=%d outside 1..%d", n, kPhiloxMaxBlocks);
  int dev = 0;
  int rc = check_device(&dev);
  if (rc != FGL_OK) return rc;
  const size_t bytes = (size_t)n * 16;
  uint32_t *d_in = nullptr, *d_out = nullptr;
  hipStream_t s = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&d_in), bytes);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&d_out), bytes);
  if (e == hipSuccess) e = hipMemcpyAsync(d_in, ctr, bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_philox, dim3((n + 255) / 256), dim3(256), 0, s, d_in, n, k0, k1, d_out);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(out, d_out, bytes, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (s) (void)hipStreamSynchronize(s);
  if (d_in) (void)hipFree(d_in);
  if (d_out) (void)hipFree(d_out);
  if (s) (void)hipStreamDestroy(s);
  return e == hipSuccess ? FGL_OK : hip_err(e, "Philox kernel");
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
