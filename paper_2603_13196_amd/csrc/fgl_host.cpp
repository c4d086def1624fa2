// Host side of the C-ABI: model residency, per-stream workspaces, tile
// choice and tuning, hipGraph replay of the per-call launch sequence.
#include "fgl_host.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <string>

#include <dlfcn.h>
#include <unistd.h>

namespace fgl {

// ---------------------------------------------------------------------------
// errors

static thread_local std::string g_err;

int set_err(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_err(hipError_t e, const char* what) {
  return set_err(e == hipErrorOutOfMemory ? FGL_ENOMEM : FGL_EDEVICE,
                 "%s: %s", what, hipGetErrorString(e));
}

const char* last_error() { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// roctx ranges (FGL_ROCTX=1)

namespace {

struct Roctx {
  int (*push)(const char*) = nullptr;
  int (*pop)() = nullptr;
};

const Roctx& roctx() {
  static const Roctx r = [] {
    Roctx x;
    const char* e = std::getenv("FGL_ROCTX");
    if (!e || e[0] != '1') return x;
    for (const char* lib : {"librocprofiler-sdk-roctx.so.1", "libroctx64.so.4"}) {
      void* h = dlopen(lib, RTLD_NOW | RTLD_GLOBAL);
      if (!h) continue;
      auto push = reinterpret_cast<int (*)(const char*)>(dlsym(h, "roctxRangePushA"));
      auto pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
      if (push && pop) {
        x.push = push;
        x.pop = pop;
        break;
      }
    }
    return x;
  }();
  return r;
}

}  // namespace

TraceRange::TraceRange(const char* fmt, ...) : on_(roctx().push != nullptr) {
  if (!on_) return;
  char buf[160];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  roctx().push(buf);
}

TraceRange::~TraceRange() {
  if (on_) roctx().pop();
}

// ---------------------------------------------------------------------------
// live models (so that a server can drop the workspaces of its streams)

static std::mutex g_models_mu;
static std::vector<Model*> g_models;

static void register_model(Model* m) {
  std::lock_guard<std::mutex> g(g_models_mu);
  g_models.push_back(m);
}

static void unregister_model(Model* m) {
  std::lock_guard<std::mutex> g(g_models_mu);
  g_models.erase(std::remove(g_models.begin(), g_models.end(), m), g_models.end());
}

// ---------------------------------------------------------------------------
// device check

int check_device(int* dev_out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_err(e, "hipGetDevice");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return hip_err(e, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return set_err(FGL_EDEVICE, "device %d is %s; this library is built for gfx950",
                   dev, prop.gcnArchName);
  *dev_out = dev;
  return FGL_OK;
}

// ---------------------------------------------------------------------------
// host-side layouts (built once per model)

// Balanced base-256 digits of a signed integer q with q + 0x808080 < 2^31:
// byte 3 of the result is the most significant digit, every byte read as
// int8 is a digit, and q = sum_L digit_L 2^(8(3-L)) with L = 3 - byte index.
static inline uint32_t digits4(int32_t q) {
  return ((uint32_t)q + 0x808080u) ^ 0x808080u;
}

static void build_projected(Model* m, const float* K, const double* data);


// 2^(r/64) on |r| <= 1/2 for the mixed kernel: the degree-4 polynomial that
// interpolates it at the five Chebyshev nodes (monomial coefficients q[0..4],
// solved in long double).  Its largest relative error is 2^-48.5, against
// 4e-17 for the fifth-order Taylor series the FP64 kernels use; the mixed
// kernel rounds its powers to 47 bits, and a digit-level emulation of its
// arithmetic gives the same margins on the posterior shells with either.
static void cheb_pow2(double q[5]) {
  constexpr int n = 5;
  long double a[n][n + 1];
  for (int k = 0; k < n; ++k) {
    const long double x = 0.5L * std::cos((2.0L * k + 1.0L) * 3.14159265358979323846264338L /
                                          (2.0L * n));
    long double xp = 1.0L;
    for (int j = 0; j < n; ++j, xp *= x) a[k][j] = xp;
    a[k][n] = std::exp2(x / 64.0L);
  }
  for (int c = 0; c < n; ++c) {                     // Gaussian elimination, partial pivoting
    int pr = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[r][c]) > std::fabs(a[pr][c])) pr = r;
    for (int j = 0; j <= n; ++j) std::swap(a[c][j], a[pr][j]);
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const long double f = a[r][c] / a[c][c];
      for (int j = c; j <= n; ++j) a[r][j] -= f * a[c][j];
    }
  }
  for (int j = 0; j < n; ++j) q[j] = (double)(a[j][n] / a[j][j]);
}

static void build_layouts(Model* m, const float* K, const double* freqs,
                          const double* data) {
  const int N = m->N, F = m->F, T = m->T;
  const int TT = m->dm.TT, TT16 = m->dm.TT16, KC = m->dm.KC;
  const int NP2 = m->dm.NP2, NQ = m->dm.NQ;
  auto Kat = [&](int i, int f, int t) -> float {
    return K[((size_t)i * F + f) * T + t];
  };
  // mixed digits [F][4][KC][TT][64][16] and per-channel exponents: K at
  // channel f is scaled by 2^(31 - eK) (|K| < 2^eK), rounded, and cut into
  // four balanced digits whose top digit must stay within [-125, 125] (the
  // bound behind the int32 level sums of the mixed kernel); if rounding
  // reaches 126 2^24 the channel uses eK + 1.  K values within 2^8 of the
  // channel's largest are exact.
  m->h_kd.assign((size_t)F * 4 * KC * TT * 1024, 0);
  m->h_eK.assign(F, 0);
  for (int f = 0; f < F; ++f) {
    float mx = 0.0f;
    for (int i = 0; i < N; ++i)
      for (int t = 0; t < T; ++t) mx = std::max(mx, std::fabs(Kat(i, f, t)));
    int ek = 0;
    if (mx > 0.0f) std::frexp((double)mx, &ek);   // mx < 2^ek
    for (;; ++ek) {
      const double q = std::nearbyint(std::ldexp((double)mx, 31 - ek));
      if (q + (double)0x808080 < 126.0 * 16777216.0) break;   // top digit <= 125
    }
    m->h_eK[f] = ek;
    int8_t* base = m->h_kd.data() + (size_t)f * 4 * KC * TT * 1024;
    for (int kc = 0; kc < KC; ++kc)
      for (int tt = 0; tt < TT; ++tt)
        for (int lane = 0; lane < 64; ++lane)
          for (int j = 0; j < 16; ++j) {
            const int i = kc * 32 + (lane >> 5) * 16 + j;
            const int t = tt * 32 + (lane & 31);
            uint32_t d = 0x00000000u;
            if (i < N && t < T) {
              const double v = std::ldexp((double)Kat(i, f, t), 31 - ek);
              d = digits4((int32_t)std::nearbyint(v));
            }
            for (int L = 0; L < 4; ++L) {
              const int8_t dig = (int8_t)(uint8_t)(d >> (8 * (3 - L)));
              base[(((size_t)L * KC + kc) * TT + tt) * 1024 + lane * 16 + j] = dig;
            }
          }
  }
  // FP32 A operands [F][NP2][TT][64]: lane -> (t = tt*32 + lane%32,
  // i = 2k + lane/32); regions >= N and times >= T are zero
  m->h_k32.assign((size_t)F * NP2 * TT * 64, 0.0f);
  for (int f = 0; f < F; ++f)
    for (int k = 0; k < NP2; ++k)
      for (int tt = 0; tt < TT; ++tt)
        for (int lane = 0; lane < 64; ++lane) {
          const int i = 2 * k + (lane >> 5), t = tt * 32 + (lane & 31);
          const float v = (t < T && i < N) ? Kat(i, f, t) : 0.0f;
          m->h_k32[(((size_t)f * NP2 + k) * TT + tt) * 64 + lane] = v;
        }
  // thin-kernel K [F][T][NT], zero padded in regions
  if (m->dm.thin) {
    const int NT = m->dm.NT;
    m->h_kthin.assign((size_t)F * T * NT, 0.0f);
    for (int f = 0; f < F; ++f)
      for (int t = 0; t < T; ++t)
        for (int i = 0; i < N; ++i) m->h_kthin[((size_t)f * T + t) * NT + i] = Kat(i, f, t);
  }
  // FP64 A operands (exact FP32 values) [F][NQ][TT16][64]: lane ->
  // (t = tt*16 + lane%16, i = 4k + lane/16); regions >= N are zero
  m->h_k64.assign((size_t)F * NQ * TT16 * 64, 0.0f);
  for (int f = 0; f < F; ++f)
    for (int k = 0; k < NQ; ++k)
      for (int tt = 0; tt < TT16; ++tt)
        for (int lane = 0; lane < 64; ++lane) {
          const int i = 4 * k + (lane >> 4), t = tt * 16 + (lane & 15);
          const float v = (t < T && i < N) ? Kat(i, f, t) : 0.0f;
          m->h_k64[(((size_t)f * NQ + k) * TT16 + tt) * 64 + lane] = v;
        }
  // per-channel constants
  m->h_nl64.resize(F);
  m->h_nl2.resize(F);
  m->h_nu.assign(freqs, freqs + F);
  for (int f = 0; f < F; ++f) {
    const double l2 = std::log2(freqs[f] / m->nu_ref);
    m->h_nl2[f] = -l2;
    m->h_nl64[f] = -64.0 * l2;
  }
  // data [F][TT*32], zero padded in t
  m->h_D.assign((size_t)F * TT * 32, 0.0);
  for (int f = 0; f < F; ++f)
    for (int t = 0; t < T; ++t) m->h_D[(size_t)f * TT * 32 + t] = data[(size_t)f * T + t];
  // exponent tables: Q 2^((k - kTabLo)/64) with Q = 2^47 - 2^41, then
  // 2^(m/64) / (1 - 2^-6) (the unit of the level-0 digit product)
  const long double Q = 140737488355328.0L - 2199023255552.0L;
  m->h_tab.resize(kTabSize + 2 * kFracSize);
  for (int k = 0; k < kTabSize; ++k)
    m->h_tab[k] = (double)(Q * std::exp2((long double)(k - kTabLo) / 64.0L));
  for (int k = 0; k < kFracSize; ++k) {
    const long double u = std::exp2((long double)k / 64.0L) / (1.0L - 1.0L / 64.0L);
    m->h_tab[kTabSize + k] = (double)u;
    m->h_tab[kTabSize + kFracSize + k] = (double)(1.0L / u);
  }
  const long double c1 = std::log(2.0L) / 64.0L;
  m->dm.c1 = (double)c1;
  m->dm.c2 = (double)(c1 * c1 / 2.0L);
  m->dm.c3 = (double)(c1 * c1 * c1 / 6.0L);
  m->dm.c4 = (double)(c1 * c1 * c1 * c1 / 24.0L);
  m->dm.c5 = (double)(c1 * c1 * c1 * c1 * c1 / 120.0L);
  cheb_pow2(m->dm.q);
  if (m->dm.proj) build_projected(m, K, data);
}

// Projected form of the mixed kernel.  Per channel, with Kbar_i and Dbar
// the time means and K~, D~ the centred series (T x N and T), a Householder
// QR K~ = Q R in long double gives the N x N upper-triangular R and
// z = Q^T D~.  The matrix rows are [sqrt(T) Kbar ; R] (the last row of R is
// left out and stored in pk when N is a multiple of 32), the targets are
// [(row 0 is formed per parameter row) ; z_0 .. z_{N-1}], and the constant
// sum_{k >= N} z_k^2 over all channels is chi0.
static inline void digits6(long long q, int8_t out[6]) {
  // balanced base-256 digits, out[0] most significant: the low five bytes
  // of q + 0x8080808080 are digit + 128, the rest is the top digit
  const long long u = q + 0x8080808080LL;
  for (int L = 1; L < 6; ++L)
    out[L] = (int8_t)((uint8_t)((u >> (8 * (5 - L))) & 0xff) ^ 0x80);
  out[0] = (int8_t)(u >> 40);
}

static void build_projected(Model* m, const float* K, const double* data) {
  const int N = m->N, F = m->F, T = m->T;
  DevModel& d = m->dm;
  const int KC = d.KC, RT = d.RT;
  const int rows = d.peel ? N : N + 1;              // rows in MFMA tiles
  const long double sT = std::sqrt((long double)T);
  m->h_rd.assign((size_t)F * kProjDigits * KC * RT * 1024, 0);
  if (d.pplain) m->h_r32.assign((size_t)F * d.NP2 * RT * 64, 0.0f);
  m->h_eR.assign(F, 0);
  m->h_tg.assign((size_t)F * RT * 32, 0.0);
  m->h_dbar.assign(F, 0.0);
  m->h_pk.assign((size_t)F * 2, 0.0);
  const int NQ = d.NQ, RT16 = (N + 1 + 15) / 16;
  d.RT16 = RT16;
  m->h_pa64.assign((size_t)F * NQ * RT16 * 64, 0.0);
  m->h_pt64.assign((size_t)F * RT16 * 16, 0.0);
  long double chi0 = 0.0L;
  std::vector<long double> A((size_t)N * T), z(T), mat((size_t)rows * N);
  for (int f = 0; f < F; ++f) {
    // centred columns, column-major: A[i*T + t]
    for (int i = 0; i < N; ++i) {
      long double s = 0.0L;
      const float* Ki = K + ((size_t)i * F + f) * T;
      for (int t = 0; t < T; ++t) s += Ki[t];
      const long double mean = s / T;
      mat[i] = sT * mean;                            // row 0: sqrt(T) Kbar
      for (int t = 0; t < T; ++t) A[(size_t)i * T + t] = (long double)Ki[t] - mean;
    }
    long double sd = 0.0L;
    const double* Df = data + (size_t)f * T;
    for (int t = 0; t < T; ++t) sd += Df[t];
    const long double dmean = sd / T;
    for (int t = 0; t < T; ++t) z[t] = (long double)Df[t] - dmean;
    // Householder QR of the T x N centred block (T >= N + 1)
    for (int j = 0; j < N; ++j) {
      long double* a = &A[(size_t)j * T];
      long double nrm = 0.0L;
      for (int t = j; t < T; ++t) nrm += a[t] * a[t];
      nrm = std::sqrt(nrm);
      if (nrm == 0.0L) continue;                     // column already in span
      const long double alpha = a[j] > 0.0L ? -nrm : nrm;
      // v = a[j:] - alpha e_j, stored in place; v^T v = 2 nrm (nrm + |a_j|)
      const long double vj = a[j] - alpha;
      const long double vtv = 2.0L * nrm * (nrm + std::fabs(a[j]));
      a[j] = vj;
      auto reflect = [&](long double* x) {
        long double s = 0.0L;
        for (int t = j; t < T; ++t) s += a[t] * x[t];
        const long double k = 2.0L * s / vtv;
        for (int t = j; t < T; ++t) x[t] -= k * a[t];
      };
      for (int k = j + 1; k < N; ++k) reflect(&A[(size_t)k * T]);
      reflect(z.data());
      a[j] = alpha;                                  // R[j][j]
      for (int t = j + 1; t < T; ++t) a[t] = 0.0L;
    }
    // rows 1.. of the matrix: R[k][i] = A[i*T + k] for i >= k
    for (int k = 0; k + 1 < rows; ++k)
      for (int i = 0; i < N; ++i) mat[(size_t)(k + 1) * N + i] = i >= k ? A[(size_t)i * T + k] : 0.0L;
    long double e2 = 0.0L;
    for (int t = N; t < T; ++t) e2 += z[t] * z[t];
    chi0 += e2;
    if (d.peel) {
      m->h_pk[2 * f] = (double)A[(size_t)(N - 1) * T + (N - 1)];
      m->h_pk[2 * f + 1] = (double)z[N - 1];
    }
    m->h_dbar[f] = (double)(sT * dmean);
    for (int k = 1; k < rows; ++k) m->h_tg[(size_t)f * RT * 32 + k] = (double)z[k - 1];
    // FP64 operands of all N + 1 rows: row 0 sqrt(T) Kbar, row k >= 1 R[k-1]
    auto full = [&](int k, int i) -> long double {
      if (k == 0) return mat[i];
      return i >= k - 1 ? A[(size_t)i * T + (k - 1)] : 0.0L;
    };
    for (int q = 0; q < NQ; ++q)
      for (int tt = 0; tt < RT16; ++tt)
        for (int lane = 0; lane < 64; ++lane) {
          const int k = tt * 16 + (lane & 15), i = 4 * q + (lane >> 4);
          const double v = (k <= N && i < N) ? (double)full(k, i) : 0.0;
          m->h_pa64[(((size_t)f * NQ + q) * RT16 + tt) * 64 + lane] = v;
        }
    m->h_pt64[(size_t)f * RT16 * 16] = (double)(sT * dmean);
    for (int k = 1; k <= N; ++k) m->h_pt64[(size_t)f * RT16 * 16 + k] = (double)z[k - 1];
    // per-channel fixed point and digits [kProjDigits][KC][RT][64][16]
    long double mx = 0.0L;
    for (size_t k = 0; k < (size_t)rows * N; ++k) mx = std::max(mx, std::fabs(mat[k]));
    int er = 0;
    if (mx > 0.0L) std::frexp((double)mx, &er);
    if (mx > 0.0L && std::ldexp((long double)1.0L, er) <= mx) ++er;   // mx < 2^er
    m->h_eR[f] = er;
    if (d.pplain)
      for (int p = 0; p < d.NP2; ++p)
        for (int rt = 0; rt < RT; ++rt)
          for (int lane = 0; lane < 64; ++lane) {
            const int i = 2 * p + (lane >> 5), k = rt * 32 + (lane & 31);
            m->h_r32[(((size_t)f * d.NP2 + p) * RT + rt) * 64 + lane] =
                (i < N && k < rows) ? (float)mat[(size_t)k * N + i] : 0.0f;
          }
    int8_t* base = m->h_rd.data() + (size_t)f * kProjDigits * KC * RT * 1024;
    for (int kc = 0; kc < KC; ++kc)
      for (int rt = 0; rt < RT; ++rt)
        for (int lane = 0; lane < 64; ++lane)
          for (int j = 0; j < 16; ++j) {
            const int i = kc * 32 + (lane >> 5) * 16 + j;
            const int k = rt * 32 + (lane & 31);
            int8_t dg[6] = {0, 0, 0, 0, 0, 0};
            if (i < N && k < rows) {
              const long double v = std::ldexp(mat[(size_t)k * N + i], kProjBits - er);
              digits6(std::llrint(v), dg);
            }
            for (int L = 0; L < kProjDigits; ++L)
              base[(((size_t)L * KC + kc) * RT + rt) * 1024 + lane * 16 + j] = dg[L];
          }
  }
  d.chi0 = (double)chi0;
  d.sqrtT = (double)sT;
}

// ---------------------------------------------------------------------------
// residency

template <typename T>
static hipError_t upload(T** dptr, const std::vector<T>& h) {
  const size_t bytes = std::max<size_t>(h.size() * sizeof(T), 16);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(dptr), bytes);
  if (e != hipSuccess) return e;
  if (!h.empty()) e = hipMemcpy(*dptr, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

size_t resident_bytes(const Model* m) {
  return m->h_kd.size() + m->h_eK.size() * 4 + m->h_k32.size() * 4 +
         m->h_k64.size() * 4 + m->h_kthin.size() * 4 + (m->h_nl64.size() + m->h_nl2.size() + m->h_nu.size()) * 8 +
         m->h_D.size() * 8 + m->h_tab.size() * 8 + m->h_rd.size() + m->h_eR.size() * 4 +
         (m->h_tg.size() + m->h_dbar.size() + m->h_pk.size()) * 8 +
         (m->h_pa64.size() + m->h_pt64.size()) * 8 + m->h_r32.size() * 4;
}

int make_resident(Model* m) {
  if (m->resident) return FGL_OK;
  hipError_t e = hipSetDevice(m->dev);
  if (e != hipSuccess) return hip_err(e, "hipSetDevice");
  int8_t *kd = nullptr, *rd = nullptr;
  int32_t *eK = nullptr, *eR = nullptr;
  float *k32 = nullptr, *k64 = nullptr, *kthin = nullptr, *r32 = nullptr;
  double *nl64 = nullptr, *nl2 = nullptr, *nu = nullptr, *D = nullptr, *tab = nullptr;
  double *tg = nullptr, *dbar = nullptr, *pk = nullptr, *pa64 = nullptr, *pt64 = nullptr;
  if ((e = upload(&kd, m->h_kd)) != hipSuccess || (e = upload(&eK, m->h_eK)) != hipSuccess ||
      (e = upload(&pa64, m->h_pa64)) != hipSuccess || (e = upload(&pt64, m->h_pt64)) != hipSuccess ||
      (e = upload(&k32, m->h_k32)) != hipSuccess || (e = upload(&k64, m->h_k64)) != hipSuccess ||
      (e = upload(&kthin, m->h_kthin)) != hipSuccess || (e = upload(&r32, m->h_r32)) != hipSuccess ||
      (e = upload(&nl64, m->h_nl64)) != hipSuccess || (e = upload(&nl2, m->h_nl2)) != hipSuccess ||
      (e = upload(&nu, m->h_nu)) != hipSuccess || (e = upload(&D, m->h_D)) != hipSuccess ||
      (e = upload(&tab, m->h_tab)) != hipSuccess || (e = upload(&rd, m->h_rd)) != hipSuccess ||
      (e = upload(&eR, m->h_eR)) != hipSuccess || (e = upload(&tg, m->h_tg)) != hipSuccess ||
      (e = upload(&dbar, m->h_dbar)) != hipSuccess || (e = upload(&pk, m->h_pk)) != hipSuccess) {
    void* ps[] = {kd, eK, k32, k64, nl64, nl2, nu, D, tab, rd, eR, tg, dbar, pk, pa64, pt64, kthin,
                  r32};
    for (void* p : ps)
      if (p) (void)hipFree(p);
    return hip_err(e, "uploading model");
  }
  m->dm.rd = rd;
  m->dm.eR = eR;
  m->dm.tg = tg;
  m->dm.dbar = dbar;
  m->dm.pk = pk;
  m->dm.pa64 = pa64;
  m->dm.pt64 = pt64;
  m->dm.kd = kd;
  m->dm.eK = eK;
  m->dm.k32 = k32;
  m->dm.k64 = k64;
  m->dm.kthin = kthin;
  m->dm.r32 = r32;
  m->dm.nl64 = nl64;
  m->dm.nl2 = nl2;
  m->dm.nu = nu;
  m->dm.D = D;
  m->dm.tab = tab;
  m->resident = true;
  return FGL_OK;
}

void evict(Model* m) {
  if (!m->resident) return;
  (void)hipSetDevice(m->dev);
  // device-pointer calls return before their kernels finish; a model only
  // used by synchronous calls and servers (which evict a model only when
  // none of its requests is in flight) has nothing left to wait for
  if (m->async_calls) (void)hipDeviceSynchronize();
  const void* ps[] = {m->dm.kd, m->dm.eK, m->dm.k32, m->dm.k64, m->dm.nl64,
                      m->dm.nl2, m->dm.nu, m->dm.D, m->dm.tab, m->dm.rd,
                      m->dm.eR, m->dm.tg, m->dm.dbar, m->dm.pk, m->dm.pa64, m->dm.pt64,
                      m->dm.kthin, m->dm.r32};
  for (const void* p : ps)
    if (p) (void)hipFree(const_cast<void*>(p));
  m->dm.rd = nullptr;
  m->dm.eR = nullptr;
  m->dm.tg = m->dm.dbar = m->dm.pk = m->dm.pa64 = m->dm.pt64 = nullptr;
  m->dm.kd = nullptr;
  m->dm.eK = nullptr;
  m->dm.k32 = m->dm.k64 = m->dm.kthin = m->dm.r32 = nullptr;
  m->dm.nl64 = m->dm.nl2 = m->dm.nu = m->dm.D = m->dm.tab = nullptr;
  m->resident = false;
  // graphs captured against the old buffers are stale
  for (auto& kv : m->graphs) {
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
  }
  m->graphs.clear();
}

// ---------------------------------------------------------------------------
// workspaces

static void free_work(WorkBuf& wb) {
  if (wb.w.betaT) (void)hipFree(wb.w.betaT);
  if (wb.w.offT) (void)hipFree(wb.w.offT);
  if (wb.w.rows) (void)hipFree(wb.w.rows);
  if (wb.w.partial) (void)hipFree(wb.w.partial);
  if (wb.d_theta) (void)hipFree(wb.d_theta);
  if (wb.d_out) (void)hipFree(wb.d_out);
  if (wb.h_theta) (void)hipHostFree(wb.h_theta);
  if (wb.h_out) (void)hipHostFree(wb.h_out);
  if (wb.w.gpart) (void)hipFree(wb.w.gpart);
  if (wb.d_grad) (void)hipFree(wb.d_grad);
  if (wb.h_grad) (void)hipHostFree(wb.h_grad);
  wb = WorkBuf();
}

static int padded_rows(int B) { return std::max(256, (B + 255) / 256 * 256); }

// Free the workspaces every live model keeps for stream s (the stream is
// about to be destroyed).
void drop_stream_work(hipStream_t s) {
  (void)hipStreamSynchronize(s);
  std::lock_guard<std::mutex> g(g_models_mu);
  for (Model* m : g_models) {
    std::lock_guard<std::mutex> lk(m->mu);
    auto it = m->work.find(s);
    if (it != m->work.end()) {
      free_work(it->second);
      m->work.erase(it);
    }
  }
}

int ensure_work(Model* m, WorkBuf& wb, int B, int ngroups, bool host_io) {
  const int Bpad = padded_rows(B);
  const int betaRows = m->dm.KC * 32;
  const bool grow_rows = Bpad > wb.cap_rows;
  const bool grow_groups = grow_rows || ngroups > wb.w.ngroup_cap;
  const bool grow_io = host_io && (grow_rows || !wb.h_theta);
  if (!grow_rows && !grow_groups && !grow_io) {
    wb.w.B = B;
    wb.w.Bpad = Bpad;
    return FGL_OK;
  }
  // drop graphs that captured the old pointers
  for (auto& kv : m->graphs)
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
  m->graphs.clear();
  const int rows = std::max(padded_rows(bucket_of(B)), wb.cap_rows);
  const int groups = std::max(ngroups, wb.w.ngroup_cap);
  WorkBuf nw;
  hipError_t e;
  if ((e = hipMalloc(reinterpret_cast<void**>(&nw.w.betaT), (size_t)betaRows * rows * 8)) != hipSuccess ||
      (m->dm.NA > 0 &&
       (e = hipMalloc(reinterpret_cast<void**>(&nw.w.offT), (size_t)betaRows * rows * 8)) != hipSuccess) ||
      (e = hipMalloc(reinterpret_cast<void**>(&nw.w.rows), (size_t)rows * sizeof(RowParams))) != hipSuccess ||
      (e = hipMalloc(reinterpret_cast<void**>(&nw.w.partial), (size_t)groups * rows * 8)) != hipSuccess) {
    free_work(nw);
    return hip_err(e, "allocating workspace");
  }
  if (host_io || wb.h_theta) {
    const size_t tb = (size_t)rows * m->P * 8, ob = (size_t)rows * 8;
    if ((e = hipMalloc(reinterpret_cast<void**>(&nw.d_theta), tb)) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void**>(&nw.d_out), ob)) != hipSuccess ||
        (e = hipHostMalloc(reinterpret_cast<void**>(&nw.h_theta), tb, hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc(reinterpret_cast<void**>(&nw.h_out), ob, hipHostMallocDefault)) != hipSuccess) {
      free_work(nw);
      return hip_err(e, "allocating staging buffers");
    }
  }
  // the old buffers may still be read by work queued on this stream
  if (wb.stream_synced_free) {
    free_work(wb);
  } else {
    m->retired.push_back(wb);
    wb = WorkBuf();
  }
  nw.cap_rows = rows;
  nw.w.ngroup_cap = groups;
  nw.w.B = B;
  nw.w.Bpad = Bpad;
  nw.stream_synced_free = wb.stream_synced_free;
  wb = nw;
  return FGL_OK;
}

// ---------------------------------------------------------------------------
// tiles

// Kernel family of a precision on a model: thin models evaluate the mixed
// (unless the direct digit form is forced) and FP64 precisions per row in
// FP64, which is exact and cheaper than MFMA tiles holding a few time bins.
Kind kind_of(int prec, const DevModel& d) {
  if (prec == FGL_PREC_FP32) return kFP32;
  if (d.thin && (prec == FGL_PREC_FP64 || !(d.flags & FGL_MIXED_DIRECT))) return kThin;
  return prec == FGL_PREC_FP64 ? kFP64 : kMixed;
}

// Largest wave count whose kernel fits in registers without spilling.
static int max_waves(Kind k, const DevModel& d) {
  if (k == kThin) return 4;
  if (k == kMixed) return d.KC <= 2 ? 8 : 4;
  if (k == kFP32) return 8;
  return 8;
}

// Channels of one reduction group: fixed per (model, precision).  Up to four
// channels, as many as fit in half a CU's LDS (two workgroups per CU).
int group_of(Kind k, const DevModel& d) {
  for (int g = 4; g >= 1; --g) {
    Tile t{4, g, g, 2};
    if (lds_bytes(k, d, t) <= max_lds_bytes() / 2) return g;
  }
  Tile t{4, 1, 1, 2};
  return lds_bytes(k, d, t) <= max_lds_bytes() ? 1 : 0;
}

// Candidate tiles for the tuner: waves in {4, 8} (within register limits),
// channels per workgroup a multiple of the group fitting in LDS, and for the
// projected mixed kernel with one region chunk also the variant compiled for
// three waves per SIMD (with the LDS of the workgroups that then share a CU).
std::vector<Tile> candidates(Kind k, const DevModel& d) {
  std::vector<Tile> out;
  const int G = group_of(k, d);
  if (G == 0) return out;
  const bool occ3 = k == kMixed && mixed_occ3(d);
  const std::vector<int> waves = k == kThin ? std::vector<int>{1, 2, 4} : std::vector<int>{4, 8};
  std::vector<int> occs{2};
  if (occ3) occs.push_back(3);
  for (int w : waves) {
    if (w > max_waves(k, d)) continue;
    for (int occ : occs) {
      const int per_cu = occ == 3 ? std::max(1, 12 / w) : 1;
      for (int mult = 1; mult <= 8; ++mult) {
        Tile t{w, G * mult, G, occ};
        if (lds_bytes(k, d, t) * per_cu > max_lds_bytes()) break;
        if (mult <= 2 || mult == 4 || mult == 8) out.push_back(t);
      }
    }
  }
  return out;
}

// Heuristic tile when no measurement is cached: as many waves as registers
// allow (the projected mixed kernel with one region chunk in its
// three-waves-per-SIMD variant), and the largest channel block whose LDS
// still lets the workgroups that registers allow on a CU be resident (the
// mixed kernel's 8-wave workgroups run one per CU; the plain kernels are
// given two workgroups per CU), with >= 2048 workgroups in flight.
Tile default_tile(Kind k, const DevModel& d, int B) {
  const int G = group_of(k, d);
  int W = max_waves(k, d);
  // the thin kernel on small batches: fewer waves per workgroup until the
  // row tiles times the channel groups give ~1024 workgroups
  if (k == kThin)
    while (W > 1 && (padded_rows(B) / (64 * W)) * ((d.F + G - 1) / G) < 1024) W /= 2;
  const int occ = (k == kMixed && mixed_occ3(d)) ? 3 : 2;
  Tile best{W, G, G, occ};
  const int cols = cols_per_wave(k) * W;
  const int nb = padded_rows(B) / cols;
  const int per_cu = k == kMixed ? std::max(1, 4 * occ / W) : 2;   // workgroups per CU
  const int lds_cap = max_lds_bytes() / per_cu;
  for (int mult = 1; mult <= 8; mult *= 2) {
    Tile t{W, G * mult, G, occ};
    if (lds_bytes(k, d, t) > lds_cap) break;
    const int blocks = nb * ((d.F + t.fc - 1) / t.fc);
    if (mult > 1 && blocks < 2048) break;
    best = t;
  }
  return best;
}

// ---------------------------------------------------------------------------
// one call: prep -> main -> finalize on stream s

int enqueue(Model* m, Kind k, const Tile& tile, WorkBuf& wb, const double* d_theta,
            int B, double* d_out, hipStream_t s) {
  const int rc = enqueue_partials(m, k, tile, wb, d_theta, B, s);
  if (rc != FGL_OK) return rc;
  hipError_t e;
  if ((e = launch_finalize(k, m->dm, wb.w, tile, d_out, s)) != hipSuccess)
    return hip_err(e, "finalize kernel");
  return FGL_OK;
}

// prep -> main: the likelihood kernel's per-(group, row) partial sums in
// wb.w.partial (the chain engine reduces them itself)
// Events that only time kernels: recorded without the system-scope fence
// (a cache write-back and invalidate that otherwise adds ~5.5 us before and
// after the timed kernel on this device).  Results are read only after a
// stream or device synchronisation, never through these events.
static hipError_t timing_event(hipEvent_t* ev) {
  return hipEventCreateWithFlags(ev, hipEventDisableSystemFence);
}

int enqueue_partials(Model* m, Kind k, const Tile& tile, WorkBuf& wb, const double* d_theta,
                     int B, hipStream_t s) {
  hipError_t e;
  if ((e = launch_prep(m->dm, d_theta, B, wb.w, m->dm.KC * 32, s)) != hipSuccess)
    return hip_err(e, "prep kernel");
  return enqueue_main(m, k, tile, wb, s);
}

int enqueue_main(Model* m, Kind k, const Tile& tile, WorkBuf& wb, hipStream_t s) {
  hipError_t e;
  std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
  const bool rec = m->timing > 0 && m->timing_n++ % (uint64_t)m->timing == 0;
  if (rec) {
    if (!m->ev_free.empty()) {
      ev = m->ev_free.back();
      m->ev_free.pop_back();
    } else if ((e = timing_event(&ev.first)) != hipSuccess ||
               (e = timing_event(&ev.second)) != hipSuccess) {
      return hip_err(e, "hipEventCreate");
    }
    if ((e = hipEventRecord(ev.first, s)) != hipSuccess) return hip_err(e, "hipEventRecord");
  }
  if ((e = launch_main(k, m->dm, wb.w, tile, s)) != hipSuccess)
    return hip_err(e, "likelihood kernel");
  if (rec) {
    if ((e = hipEventRecord(ev.second, s)) != hipSuccess) return hip_err(e, "hipEventRecord");
    m->ev_used.push_back(ev);
  }
  return FGL_OK;
}

// Gradient partials for B rows (after ensure_work has set the row padding):
// grow w.gpart, retiring the old buffer when queued work may still use it.
static int ensure_gpart(Model* m, WorkBuf& wb, const GradShape& gs) {
  const size_t need = (size_t)grad_slots(m->dm) * gs.chunks * wb.w.Bpad * 8;
  if (wb.gpart_bytes >= need) return FGL_OK;
  if (wb.w.gpart) {
    if (wb.stream_synced_free) {
      (void)hipFree(wb.w.gpart);
    } else {
      WorkBuf old;
      old.w.gpart = wb.w.gpart;
      m->retired.push_back(old);
    }
    wb.w.gpart = nullptr;
    wb.gpart_bytes = 0;
  }
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&wb.w.gpart), need);
  if (e != hipSuccess) {
    wb.w.gpart = nullptr;
    return hip_err(e, "allocating gradient partials");
  }
  wb.gpart_bytes = need;
  return FGL_OK;
}

// one gradient call: prep -> gradient kernel -> gradient finalize on stream s
int enqueue_grad(Model* m, WorkBuf& wb, const double* d_theta, int B, double* d_out,
                 double* d_grad, hipStream_t s) {
  const GradShape gs = grad_shape(m->dm, wb.w.Bpad);
  int rc = ensure_gpart(m, wb, gs);
  if (rc != FGL_OK) return rc;
  hipError_t e;
  if ((e = launch_prep(m->dm, d_theta, B, wb.w, m->dm.KC * 32, s)) != hipSuccess)
    return hip_err(e, "prep kernel");
  std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
  const bool rec = m->timing > 0 && m->timing_n++ % (uint64_t)m->timing == 0;
  if (rec) {
    if (!m->ev_free.empty()) {
      ev = m->ev_free.back();
      m->ev_free.pop_back();
    } else if ((e = timing_event(&ev.first)) != hipSuccess ||
               (e = timing_event(&ev.second)) != hipSuccess) {
      return hip_err(e, "hipEventCreate");
    }
    if ((e = hipEventRecord(ev.first, s)) != hipSuccess) return hip_err(e, "hipEventRecord");
  }
  if ((e = launch_grad(m->dm, wb.w, gs, s)) != hipSuccess) return hip_err(e, "gradient kernel");
  if (rec) {
    if ((e = hipEventRecord(ev.second, s)) != hipSuccess) return hip_err(e, "hipEventRecord");
    m->ev_used.push_back(ev);
  }
  if ((e = launch_grad_finalize(m->dm, wb.w, gs, d_theta, d_out, d_grad, s)) != hipSuccess)
    return hip_err(e, "gradient finalize");
  return FGL_OK;
}

// ---------------------------------------------------------------------------
// tuner cache: tuned tiles by (architecture, kernel family, model shape and
// form, batch bucket), shared by the models of a process and kept in a file
// of one JSON object per line (fgl_tune_cache or FGL_TUNE_CACHE), so that
// later processes start from the tiles earlier ones measured.

namespace {

std::mutex g_tc_mu;
std::map<std::string, Tile> g_tc;          // process cache
std::string g_tc_path;                     // file ("" = not persisted)
bool g_tc_env_done = false;
std::atomic<uint64_t> g_tc_gen{1};         // bumped whenever the cache changes

// The fields that fix a model's candidate tiles and their speeds.
std::string tc_key(const Model* m, Kind k, int bucket) {
  const DevModel& d = m->dm;
  char buf[256];
  std::snprintf(buf, sizeof buf,
                "\"arch\":\"%s\",\"kind\":%d,\"N\":%d,\"NA\":%d,\"F\":%d,\"T\":%d,"
                "\"proj\":%d,\"pplain\":%d,\"thin\":%d,\"bucket\":%d",
                m->arch.c_str(), (int)k, d.N, d.NA, d.F, d.T, d.proj, d.pplain,
                d.thin, bucket);
  return buf;
}

// One line per entry: {<key fields>,"waves":w,"fc":c,"occ":o}.  Lines that
// do not parse are skipped.
void tc_load_file(const std::string& path) {
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return;
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    std::string l(line);
    const size_t w = l.find(",\"waves\":");
    if (l.size() < 2 || l[0] != '{' || w == std::string::npos) continue;
    Tile t{0, 0, 0, 0};
    if (std::sscanf(l.c_str() + w, ",\"waves\":%d,\"fc\":%d,\"occ\":%d}", &t.waves, &t.fc,
                    &t.occ) != 3)
      continue;
    g_tc[l.substr(1, w - 1)] = t;
  }
  std::fclose(f);
  ++g_tc_gen;
}

// Write the whole cache (a temporary file renamed over the old one, so a
// reader never sees half a file).  Best effort: a failure leaves the file
// as it was.
void tc_save_file() {
  if (g_tc_path.empty()) return;
  const std::string tmp = g_tc_path + ".tmp" + std::to_string((long)getpid());
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  bool ok = true;
  for (const auto& kv : g_tc)
    ok = ok && std::fprintf(f, "{%s,\"waves\":%d,\"fc\":%d,\"occ\":%d}\n", kv.first.c_str(),
                            kv.second.waves, kv.second.fc, kv.second.occ) > 0;
  ok = (std::fclose(f) == 0) && ok;
  if (!ok || std::rename(tmp.c_str(), g_tc_path.c_str()) != 0) std::remove(tmp.c_str());
}

void tc_env_once() {
  if (g_tc_env_done) return;
  g_tc_env_done = true;
  const char* p = std::getenv("FGL_TUNE_CACHE");
  if (p && p[0]) {
    g_tc_path = p;
    tc_load_file(g_tc_path);
  }
}

}  // namespace

int tune_cache_set(const char* path) {
  std::lock_guard<std::mutex> lk(g_tc_mu);
  g_tc_env_done = true;
  g_tc_path = path ? path : "";
  if (!g_tc_path.empty()) tc_load_file(g_tc_path);
  return FGL_OK;
}

// A tile from the process cache, if one was measured for this model's shape
// and is still a candidate for it.
static bool tc_lookup(Model* m, Kind k, int bucket, Tile* out) {
  std::lock_guard<std::mutex> lk(g_tc_mu);
  tc_env_once();
  auto it = g_tc.find(tc_key(m, k, bucket));
  if (it == g_tc.end()) return false;
  for (const Tile& t : candidates(k, m->dm))
    if (t.waves == it->second.waves && t.fc == it->second.fc && t.occ == it->second.occ) {
      *out = t;
      return true;
    }
  return false;
}

static void tc_store(Model* m, Kind k, int bucket, const Tile& t) {
  std::lock_guard<std::mutex> lk(g_tc_mu);
  tc_env_once();
  g_tc[tc_key(m, k, bucket)] = t;
  ++g_tc_gen;
  tc_save_file();
}

Tile tile_for(Model* m, Kind k, int B) {
  const uint64_t key = ((uint64_t)k << 32) | (uint32_t)bucket_of(B);
  auto it = m->tiles.find(key);
  if (it != m->tiles.end()) return it->second;
  // the cache is consulted again only after it changed
  const uint64_t gen = g_tc_gen.load();
  auto miss = m->tc_miss.find(key);
  if (miss == m->tc_miss.end() || miss->second != gen) {
    Tile t;
    if (tc_lookup(m, k, bucket_of(B), &t)) {
      m->tiles[key] = t;
      return t;
    }
    m->tc_miss[key] = gen;
  }
  return default_tile(k, m->dm, B);
}

int bucket_of(int B) {
  int b = 256;
  while (b < B) b *= 2;
  return b;
}

// Time every candidate tile on the rows already staged in wb (device theta)
// and remember the fastest for this (precision, B bucket).
int tune(Model* m, Kind k, WorkBuf& wb, const double* d_theta, int B,
         double* d_out, hipStream_t s) {
  std::vector<Tile> cand = candidates(k, m->dm);
  if (cand.empty()) return set_err(FGL_EINVAL, "no tile fits this model");
  hipEvent_t e0, e1;
  hipError_t e;
  if ((e = timing_event(&e0)) != hipSuccess) return hip_err(e, "hipEventCreate");
  if ((e = timing_event(&e1)) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_err(e, "hipEventCreate");
  }
  // three sweeps over the candidates; in each, a candidate is timed over
  // enough calls to span >= 3 ms (5 to 40, from a timed warm-up call) and
  // its time is the mean per call of its fastest sweep.  Shorter windows let
  // clock ramps and co-scheduled work decide between tiles 2-3% apart.
  std::vector<float> best_of(cand.size(), std::numeric_limits<float>::max());
  int rc = FGL_OK;
  for (int sweep = 0; sweep < 3 && rc == FGL_OK; ++sweep) {
    for (size_t c = 0; c < cand.size(); ++c) {
      const Tile& t = cand[c];
      rc = ensure_work(m, wb, B, n_groups(m->dm, t), false);
      if (rc != FGL_OK) break;
      (void)hipEventRecord(e0, s);
      rc = enqueue(m, k, t, wb, d_theta, B, d_out, s);  // warm-up
      (void)hipEventRecord(e1, s);
      if (rc != FGL_OK) break;
      if ((e = hipEventSynchronize(e1)) != hipSuccess) {
        rc = hip_err(e, "tuning run");
        break;
      }
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      const int reps = ms > 0.0f ? std::max(5, std::min(40, (int)std::ceil(3.0f / ms))) : 5;
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < reps && rc == FGL_OK; ++r)
        rc = enqueue(m, k, t, wb, d_theta, B, d_out, s);
      (void)hipEventRecord(e1, s);
      if ((e = hipEventSynchronize(e1)) != hipSuccess) {
        rc = hip_err(e, "tuning run");
        break;
      }
      ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      best_of[c] = std::min(best_of[c], ms / reps);
    }
  }
  const Tile best =
      cand[std::min_element(best_of.begin(), best_of.end()) - best_of.begin()];
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == FGL_OK) {
    const uint64_t key = ((uint64_t)k << 32) | (uint32_t)bucket_of(B);
    m->tiles[key] = best;
    tc_store(m, k, bucket_of(B), best);
  }
  return rc;
}

}  // namespace fgl

// ===========================================================================
// C-ABI

using namespace fgl;

extern "C" {

const char* fgl_last_error(void) { return last_error(); }

// Model with NA amplitude masks (0: none, alpha = 1) and NB spectral-index
// masks; the two C entry points below differ only in NA.
static int create_model(const float* K, const double* freqs, const double* data,
                        double nu_ref, int NA, int NB, int F, int T, double t_cmb,
                        unsigned flags, fgl_model** out) {
  TraceRange tr("fgl_model_create N=%d F=%d T=%d", std::max(NA, 1) * NB, F, T);
  if (!out) return set_err(FGL_EINVAL, "out is NULL");
  *out = nullptr;
  if (!K || !freqs || !data) return set_err(FGL_EINVAL, "K, freqs and data must be non-NULL");
  if (NA < 0 || NB < 1 || (long)std::max(NA, 1) * NB > kMixedMaxN)
    return set_err(FGL_EINVAL, "masks n_alpha=%d, n_beta=%d: need n_beta >= 1 and %d regions at most",
                   NA, NB, kMixedMaxN);
  const int N = std::max(NA, 1) * NB;
  if (F < 1 || T < 1) return set_err(FGL_EINVAL, "F=%d and T=%d must be >= 1", F, T);
  if (flags & ~(FGL_NO_21CM | FGL_MIXED_DIRECT | FGL_PLAIN_PROJECTED))
    return set_err(FGL_EINVAL, "unknown flags 0x%x", flags);
  if (!(nu_ref > 0.0) || !std::isfinite(nu_ref)) return set_err(FGL_EINVAL, "nu_ref must be finite and > 0");
  if (!std::isfinite(t_cmb)) return set_err(FGL_EINVAL, "t_cmb must be finite");
  for (int f = 0; f < F; ++f) {
    const double r = freqs[f] / nu_ref;
    if (!std::isfinite(freqs[f]) || !(freqs[f] > 0.0) || r < 1.0 / 256.0 || r > 256.0)
      return set_err(FGL_EINVAL, "freqs[%d]=%g: need finite, > 0, within 2^-8..2^8 of nu_ref", f, freqs[f]);
  }
  for (size_t k = 0; k < (size_t)N * F * T; ++k)
    if (!std::isfinite(K[k])) return set_err(FGL_EINVAL, "K[%zu] is not finite", k);
  for (size_t k = 0; k < (size_t)F * T; ++k)
    if (!std::isfinite(data[k])) return set_err(FGL_EINVAL, "data[%zu] is not finite", k);
  int dev = 0;
  int rc = check_device(&dev);
  if (rc != FGL_OK) return rc;

  Model* m = new (std::nothrow) Model();
  if (!m) return set_err(FGL_ENOMEM, "host allocation");
  m->dev = dev;
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
      m->arch = prop.gcnArchName;
      const size_t c = m->arch.find(':');
      if (c != std::string::npos) m->arch.resize(c);
    }
  }
  m->N = N;
  m->F = F;
  m->T = T;
  m->P = NB + NA + ((flags & FGL_NO_21CM) ? 1 : 4);
  m->nu_ref = nu_ref;
  m->t_cmb = t_cmb;
  m->flags = flags;
  DevModel& d = m->dm;
  d.N = N;
  d.NA = NA;
  d.NB = NB;
  d.F = F;
  d.T = T;
  d.P = m->P;
  d.TT = (T + 31) / 32;
  d.TT16 = (T + 15) / 16;
  d.KC = (N + 31) / 32;
  d.NP2 = fp32_slots(N);
  d.NQ = fp64_slots(N);
  d.thin = thin_model(N, T) ? 1 : 0;
  d.NT = d.thin ? thin_slots(N) : 0;
  d.t_cmb = t_cmb;
  d.flags = flags;
  // the projected form when its N + 1 rows take fewer 32-row tiles than T
  d.proj = d.RT = d.peel = 0;
  if (!(flags & FGL_MIXED_DIRECT) && N <= kProjMaxN && T >= N + 1) {
    const int peel = N % 32 == 0 ? 1 : 0;
    const int RT = (N + 1 - peel + 31) / 32;
    if (RT < d.TT) {
      d.proj = 1;
      d.RT = RT;
      d.peel = peel;
    }
  }
  d.pplain = (d.proj && (flags & FGL_PLAIN_PROJECTED)) ? 1 : 0;
  for (Kind k : {kMixed, kFP32, kFP64, kThin}) {
    if (k == kThin && !d.thin) continue;
    if (group_of(k, d) == 0) {
      delete m;
      return set_err(FGL_EINVAL, "T=%d with N=%d does not fit one channel in LDS", T, N);
    }
  }
  try {
    build_layouts(m, K, freqs, data);
  } catch (const std::bad_alloc&) {
    delete m;
    return set_err(FGL_ENOMEM, "host allocation for layouts");
  }
  hipError_t e = hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete m;
    return hip_err(e, "hipStreamCreate");
  }
  rc = make_resident(m);
  if (rc != FGL_OK) {
    (void)hipStreamDestroy(m->stream);
    delete m;
    return rc;
  }
  const char* tune_env = std::getenv("FGL_TUNE");
  m->autotune = tune_env && tune_env[0] == '1';
  const char* graph_env = std::getenv("FGL_NO_GRAPH");
  m->use_graphs = !(graph_env && graph_env[0] == '1');
  const char* dgraph_env = std::getenv("FGL_DEVICE_GRAPHS");
  m->device_graphs = m->use_graphs && dgraph_env && dgraph_env[0] == '1';
  register_model(m);
  *out = reinterpret_cast<fgl_model*>(m);
  return FGL_OK;
}

int fgl_model_create(const float* K, const double* freqs, const double* data,
                     double nu_ref, int N, int F, int T, double t_cmb,
                     unsigned flags, fgl_model** out) {
  if (N < 1 || N > kMixedMaxN) {
    if (out) *out = nullptr;
    return set_err(FGL_EINVAL, "N=%d outside 1..%d", N, kMixedMaxN);
  }
  return create_model(K, freqs, data, nu_ref, 0, N, F, T, t_cmb, flags, out);
}

int fgl_model_create_masks(const float* K, const double* freqs, const double* data,
                           double nu_ref, int n_alpha, int n_beta, int F, int T,
                           double t_cmb, unsigned flags, fgl_model** out) {
  if (n_alpha < 1) {
    if (out) *out = nullptr;
    return set_err(FGL_EINVAL, "n_alpha=%d: need at least one amplitude mask", n_alpha);
  }
  return create_model(K, freqs, data, nu_ref, n_alpha, n_beta, F, T, t_cmb, flags, out);
}

int fgl_model_nparams(const fgl_model* mh) {
  return mh ? reinterpret_cast<const Model*>(mh)->P : -1;
}

size_t fgl_model_bytes(const fgl_model* mh) {
  return mh ? resident_bytes(reinterpret_cast<const Model*>(mh)) : 0;
}

static int check_call(Model* m, int B, int prec) {
  if (!m) return set_err(FGL_EINVAL, "model is NULL");
  if (B < 0 || B > kMaxRows) return set_err(FGL_EINVAL, "B=%d outside 0..2^26", B);
  if (prec != FGL_PREC_MIXED && prec != FGL_PREC_FP32 && prec != FGL_PREC_FP64)
    return set_err(FGL_EINVAL, "unknown precision %d", prec);
  if (m->dying.load()) return set_err(FGL_EBUSY, "model is being destroyed");
  return FGL_OK;
}

int fgl_loglike_batch(fgl_model* mh, const double* theta, int B, double* out, int prec) {
  TraceRange tr("fgl_loglike_batch prec=%d B=%d", prec, B);
  Model* m = reinterpret_cast<Model*>(mh);
  int rc = check_call(m, B, prec);
  if (rc != FGL_OK) return rc;
  if (B == 0) return FGL_OK;
  if (!theta || !out) return set_err(FGL_EINVAL, "theta and out must be non-NULL");
  InflightGuard guard(m);
  std::lock_guard<std::mutex> lk(m->mu);
  hipError_t e = hipSetDevice(m->dev);
  if (e != hipSuccess) return hip_err(e, "hipSetDevice");
  if ((rc = make_resident(m)) != FGL_OK) return rc;
  const Kind k = kind_of(prec, m->dm);
  hipStream_t s = m->stream;
  WorkBuf& wb = m->work[s];
  wb.stream_synced_free = true;   // this stream is synchronised after every call
  Tile tile = tile_for(m, k, B);
  if ((rc = ensure_work(m, wb, B, n_groups(m->dm, tile), true)) != FGL_OK) return rc;
  const size_t tb = (size_t)B * m->P * 8;
  std::memcpy(wb.h_theta, theta, tb);
  const uint64_t tkey = ((uint64_t)k << 32) | (uint32_t)bucket_of(B);
  if (m->autotune && !m->tiles.count(tkey)) {
    if ((e = hipMemcpyAsync(wb.d_theta, wb.h_theta, tb, hipMemcpyHostToDevice, s)) != hipSuccess)
      return hip_err(e, "copy theta");
    if ((rc = tune(m, k, wb, wb.d_theta, B, wb.d_out, s)) != FGL_OK) return rc;
    tile = tile_for(m, k, B);
    if ((rc = ensure_work(m, wb, B, n_groups(m->dm, tile), true)) != FGL_OK) return rc;
    std::memcpy(wb.h_theta, theta, tb);
  }
  // graph replay for a (precision, B, tile) seen before; eager otherwise
  const GraphKey gk{k, B, tile.waves, tile.fc, tile.occ};
  auto it = m->graphs.find(gk);
  const bool graphs = m->use_graphs && !m->timing;
  if (graphs && it != m->graphs.end() && it->second.exec) {
    if ((e = hipGraphLaunch(it->second.exec, s)) != hipSuccess) return hip_err(e, "hipGraphLaunch");
  } else {
    const bool capture = graphs && it != m->graphs.end();  // second sighting
    hipGraph_t graph = nullptr;
    if (capture && (e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return hip_err(e, "hipStreamBeginCapture");
    rc = FGL_OK;
    if ((e = hipMemcpyAsync(wb.d_theta, wb.h_theta, tb, hipMemcpyHostToDevice, s)) != hipSuccess)
      rc = hip_err(e, "copy theta");
    if (rc == FGL_OK) rc = enqueue(m, k, tile, wb, wb.d_theta, B, wb.d_out, s);
    if (rc == FGL_OK && (e = hipMemcpyAsync(wb.h_out, wb.d_out, (size_t)B * 8, hipMemcpyDeviceToHost, s)) != hipSuccess)
      rc = hip_err(e, "copy out");
    if (capture) {
      hipError_t ee = hipStreamEndCapture(s, &graph);
      if (rc == FGL_OK && ee != hipSuccess) rc = hip_err(ee, "hipStreamEndCapture");
      if (rc == FGL_OK) {
        hipGraphExec_t exec = nullptr;
        if ((e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0)) != hipSuccess)
          rc = hip_err(e, "hipGraphInstantiate");
        else if ((e = hipGraphLaunch(exec, s)) != hipSuccess)
          rc = hip_err(e, "hipGraphLaunch");
        m->graphs[gk].exec = exec;
      }
      if (graph) (void)hipGraphDestroy(graph);
      if (rc != FGL_OK) return rc;
    } else {
      if (rc != FGL_OK) return rc;
      m->graphs[gk];   // remember the sighting
    }
  }
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_err(e, "hipStreamSynchronize");
  std::memcpy(out, wb.h_out, (size_t)B * 8);
  return FGL_OK;
}

// Device-call graphs a model keeps before dropping them all.
constexpr size_t kMaxDeviceGraphs = 16;

int fgl_loglike_batch_device(fgl_model* mh, const double* d_theta, int B,
                             double* d_out, int prec, void* hip_stream) {
  TraceRange tr("fgl_loglike_batch_device prec=%d B=%d", prec, B);
  Model* m = reinterpret_cast<Model*>(mh);
  int rc = check_call(m, B, prec);
  if (rc != FGL_OK) return rc;
  if (B == 0) return FGL_OK;
  if (!d_theta || !d_out) return set_err(FGL_EINVAL, "d_theta and d_out must be non-NULL");
  InflightGuard guard(m);
  std::lock_guard<std::mutex> lk(m->mu);
  m->async_calls = true;
  hipError_t e = hipSetDevice(m->dev);
  if (e != hipSuccess) return hip_err(e, "hipSetDevice");
  if ((rc = make_resident(m)) != FGL_OK) return rc;
  const Kind k = kind_of(prec, m->dm);
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  WorkBuf& wb = m->work[s];
  const uint64_t tkey = ((uint64_t)k << 32) | (uint32_t)bucket_of(B);
  if (m->autotune && !m->tiles.count(tkey)) {
    if ((rc = tune(m, k, wb, d_theta, B, d_out, s)) != FGL_OK) return rc;
  }
  const Tile tile = tile_for(m, k, B);
  if ((rc = ensure_work(m, wb, B, n_groups(m->dm, tile), false)) != FGL_OK) return rc;
  // With FGL_DEVICE_GRAPHS=1: graph replay of prep, likelihood kernel and
  // finalize for a (precision, B, tile, buffers, stream) seen before,
  // captured on the model's own stream (the caller's may be the legacy
  // default stream, which cannot be captured) and launched on the caller's.
  // Off by default: one hipGraphLaunch costs the host more than the three
  // kernel launches it replaces (measured: back-to-back calls of a 1000-row
  // model take 22 us per call with graphs, 12 us without).  Calls whose
  // kernel the timing option records run eagerly.
  const bool rec_next = m->timing > 0 && m->timing_n % (uint64_t)m->timing == 0;
  if (!m->device_graphs || rec_next) return enqueue(m, k, tile, wb, d_theta, B, d_out, s);
  GraphKey gk{k, B, tile.waves, tile.fc, tile.occ};
  gk.theta = d_theta;
  gk.out = d_out;
  gk.stream = s;
  auto it = m->graphs.find(gk);
  if (it != m->graphs.end() && it->second.exec) {
    if (m->timing > 0) ++m->timing_n;
    if ((e = hipGraphLaunch(it->second.exec, s)) != hipSuccess) return hip_err(e, "hipGraphLaunch");
    return FGL_OK;
  }
  if (it == m->graphs.end()) {                     // first sighting: eager
    if ((rc = enqueue(m, k, tile, wb, d_theta, B, d_out, s)) != FGL_OK) return rc;
    // bound the device-call graphs a model keeps (each holds buffers' addresses)
    size_t dev_graphs = 0;
    for (const auto& kv : m->graphs) dev_graphs += kv.first.theta != nullptr;
    if (dev_graphs >= kMaxDeviceGraphs) {
      for (auto g = m->graphs.begin(); g != m->graphs.end();) {
        if (g->first.theta) {
          if (g->second.exec) (void)hipGraphExecDestroy(g->second.exec);
          g = m->graphs.erase(g);
        } else {
          ++g;
        }
      }
    }
    m->graphs[gk];
    return FGL_OK;
  }
  // second sighting: capture on the model's stream, then launch on s
  hipStream_t cs = m->stream;
  if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess)
    return hip_err(e, "hipStreamBeginCapture");
  const int erc = enqueue(m, k, tile, wb, d_theta, B, d_out, cs);
  hipGraph_t graph = nullptr;
  const hipError_t ee = hipStreamEndCapture(cs, &graph);
  if (erc != FGL_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return erc;
  }
  if (ee != hipSuccess) return hip_err(ee, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_err(e, "hipGraphInstantiate");
  it->second.exec = exec;
  if (m->timing > 0) ++m->timing_n;
  if ((e = hipGraphLaunch(exec, s)) != hipSuccess) return hip_err(e, "hipGraphLaunch");
  return FGL_OK;
}

static int check_grad(Model* m, int B, int prec) {
  int rc = check_call(m, B, prec);
  if (rc != FGL_OK) return rc;
  if (prec != FGL_PREC_FP64)
    return set_err(FGL_EINVAL, "gradients are evaluated in FP64 only (prec=%d)", prec);
  return FGL_OK;
}

int fgl_loglike_grad_batch(fgl_model* mh, const double* theta, int B, double* out,
                           double* grad, int prec) {
  TraceRange tr("fgl_loglike_grad_batch B=%d", B);
  Model* m = reinterpret_cast<Model*>(mh);
  int rc = check_grad(m, B, prec);
  if (rc != FGL_OK) return rc;
  if (B == 0) return FGL_OK;
  if (!theta || !out || !grad) return set_err(FGL_EINVAL, "theta, out and grad must be non-NULL");
  InflightGuard guard(m);
  std::lock_guard<std::mutex> lk(m->mu);
  hipError_t e = hipSetDevice(m->dev);
  if (e != hipSuccess) return hip_err(e, "hipSetDevice");
  if ((rc = make_resident(m)) != FGL_OK) return rc;
  hipStream_t s = m->stream;
  WorkBuf& wb = m->work[s];
  wb.stream_synced_free = true;   // this stream is synchronised after every call
  if ((rc = ensure_work(m, wb, B, 1, true)) != FGL_OK) return rc;
  const size_t tb = (size_t)B * m->P * 8;
  if (wb.grad_bytes < tb) {
    if (wb.d_grad) (void)hipFree(wb.d_grad);
    if (wb.h_grad) (void)hipHostFree(wb.h_grad);
    wb.d_grad = wb.h_grad = nullptr;
    wb.grad_bytes = 0;
    const size_t cap = (size_t)wb.cap_rows * m->P * 8;
    if ((e = hipMalloc(reinterpret_cast<void**>(&wb.d_grad), cap)) != hipSuccess ||
        (e = hipHostMalloc(reinterpret_cast<void**>(&wb.h_grad), cap, hipHostMallocDefault)) != hipSuccess) {
      if (wb.d_grad) (void)hipFree(wb.d_grad);
      wb.d_grad = nullptr;
      wb.h_grad = nullptr;
      return hip_err(e, "allocating gradient staging");
    }
    wb.grad_bytes = cap;
  }
  std::memcpy(wb.h_theta, theta, tb);
  if ((e = hipMemcpyAsync(wb.d_theta, wb.h_theta, tb, hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_err(e, "copy theta");
  if ((rc = enqueue_grad(m, wb, wb.d_theta, B, wb.d_out, wb.d_grad, s)) != FGL_OK) return rc;
  if ((e = hipMemcpyAsync(wb.h_out, wb.d_out, (size_t)B * 8, hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_err(e, "copy out");
  if ((e = hipMemcpyAsync(wb.h_grad, wb.d_grad, tb, hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_err(e, "copy grad");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_err(e, "hipStreamSynchronize");
  std::memcpy(out, wb.h_out, (size_t)B * 8);
  std::memcpy(grad, wb.h_grad, tb);
  return FGL_OK;
}

int fgl_loglike_grad_batch_device(fgl_model* mh, const double* d_theta, int B,
                                  double* d_out, double* d_grad, int prec,
                                  void* hip_stream) {
  TraceRange tr("fgl_loglike_grad_batch_device B=%d", B);
  Model* m = reinterpret_cast<Model*>(mh);
  int rc = check_grad(m, B, prec);
  if (rc != FGL_OK) return rc;
  if (B == 0) return FGL_OK;
  if (!d_theta || !d_out || !d_grad)
    return set_err(FGL_EINVAL, "d_theta, d_out and d_grad must be non-NULL");
  InflightGuard guard(m);
  std::lock_guard<std::mutex> lk(m->mu);
  m->async_calls = true;
  hipError_t e = hipSetDevice(m->dev);
  if (e != hipSuccess) return hip_err(e, "hipSetDevice");
  if ((rc = make_resident(m)) != FGL_OK) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  WorkBuf& wb = m->work[s];
  if ((rc = ensure_work(m, wb, B, 1, false)) != FGL_OK) return rc;
  return enqueue_grad(m, wb, d_theta, B, d_out, d_grad, s);
}

int fgl_mixed_form(const fgl_model* mh) {
  if (!mh) return set_err(FGL_EINVAL, "model is NULL");
  const Model* m = reinterpret_cast<const Model*>(mh);
  if (kind_of(FGL_PREC_MIXED, m->dm) == kThin) return FGL_FORM_THIN;
  return m->dm.proj ? FGL_FORM_PROJECTED : FGL_FORM_DIRECT;
}

int fgl_get_tile(fgl_model* mh, int B, int prec, int* waves, int* chans, int* occupancy) {
  Model* m = reinterpret_cast<Model*>(mh);
  int rc = check_call(m, B, prec);
  if (rc != FGL_OK) return rc;
  std::lock_guard<std::mutex> lk(m->mu);
  const Tile t = tile_for(m, kind_of(prec, m->dm), std::max(B, 1));
  if (waves) *waves = t.waves;
  if (chans) *chans = t.fc;
  if (occupancy) *occupancy = t.occ;
  return FGL_OK;
}

int fgl_set_tile(fgl_model* mh, int B, int prec, int waves, int chans, int occupancy) {
  Model* m = reinterpret_cast<Model*>(mh);
  int rc = check_call(m, B, prec);
  if (rc != FGL_OK) return rc;
  std::lock_guard<std::mutex> lk(m->mu);
  const Kind k = kind_of(prec, m->dm);
  for (const Tile& t : candidates(k, m->dm)) {
    if (t.waves == waves && t.fc == chans && t.occ == occupancy) {
      const uint64_t key = ((uint64_t)k << 32) | (uint32_t)bucket_of(std::max(B, 1));
      m->tiles[key] = t;
      return FGL_OK;
    }
  }
  return set_err(FGL_EINVAL, "tile (waves=%d, chans=%d, occupancy=%d) is not a candidate for "
                 "this model and precision", waves, chans, occupancy);
}

int fgl_tune_cache(const char* path) { return tune_cache_set(path); }

int fgl_tune(fgl_model* mh, int B, int prec) {
  TraceRange tr("fgl_tune prec=%d B=%d", prec, B);
  Model* m = reinterpret_cast<Model*>(mh);
  int rc = check_call(m, B, prec);
  if (rc != FGL_OK) return rc;
  if (B < 1) return set_err(FGL_EINVAL, "B must be >= 1 to tune");
  InflightGuard guard(m);
  std::lock_guard<std::mutex> lk(m->mu);
  hipError_t e = hipSetDevice(m->dev);
  if (e != hipSuccess) return hip_err(e, "hipSetDevice");
  if ((rc = make_resident(m)) != FGL_OK) return rc;
  hipStream_t s = m->stream;
  WorkBuf& wb = m->work[s];
  wb.stream_synced_free = true;
  if ((rc = ensure_work(m, wb, B, n_groups(m->dm, default_tile(kind_of(prec, m->dm), m->dm, B)), true)) != FGL_OK)
    return rc;
  // tune on prior-like rows: beta uniform in [2, 3.5], alpha in [0.8, 1.2]
  // (from the splitmix64 finaliser, so neighbouring rows differ as sampled
  // rows do: the table lookups of the mixed kernel see realistic address
  // spreads), A = -0.1, nu0 = 100, w = 15, sigma = 0.025
  auto unit = [](uint64_t x) {
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    x ^= x >> 31;
    return (double)(x >> 11) * 0x1.0p-53;
  };
  for (int b = 0; b < B; ++b) {
    double* row = wb.h_theta + (size_t)b * m->P;
    const int NB = m->dm.NB, NA = m->dm.NA;
    for (int j = 0; j < NB; ++j) row[j] = 2.0 + 1.5 * unit((uint64_t)b * 4099 + j);
    for (int i = 0; i < NA; ++i) row[NB + i] = 0.8 + 0.4 * unit((uint64_t)b * 4099 + 2048 + i);
    if (!(m->flags & FGL_NO_21CM)) {
      row[m->P - 4] = -0.1;
      row[m->P - 3] = 100.0;
      row[m->P - 2] = 15.0;
    }
    row[m->P - 1] = 0.025;
  }
  if ((e = hipMemcpyAsync(wb.d_theta, wb.h_theta, (size_t)B * m->P * 8, hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_err(e, "copy theta");
  rc = tune(m, kind_of(prec, m->dm), wb, wb.d_theta, B, wb.d_out, s);
  if (rc != FGL_OK) return rc;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_err(e, "hipStreamSynchronize");
  return FGL_OK;
}

int fgl_kernel_timing(fgl_model* mh, int enable) {
  Model* m = reinterpret_cast<Model*>(mh);
  if (!m) return set_err(FGL_EINVAL, "model is NULL");
  std::lock_guard<std::mutex> lk(m->mu);
  for (auto& ev : m->ev_used) {
    (void)hipEventSynchronize(ev.second);
    m->ev_free.push_back(ev);
  }
  m->ev_used.clear();
  if (enable < 0) return set_err(FGL_EINVAL, "enable=%d: need 0 (off) or n >= 1 (every n-th launch)", enable);
  m->timing = enable;
  m->timing_n = 0;
  return FGL_OK;
}

int fgl_kernel_time(fgl_model* mh, double* total_ms, int64_t* launches) {
  Model* m = reinterpret_cast<Model*>(mh);
  if (!m || !total_ms || !launches) return set_err(FGL_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(m->mu);
  double tot = 0.0;
  for (auto& ev : m->ev_used) {
    hipError_t e = hipEventSynchronize(ev.second);
    if (e != hipSuccess) return hip_err(e, "hipEventSynchronize");
    float ms = 0.0f;
    if ((e = hipEventElapsedTime(&ms, ev.first, ev.second)) != hipSuccess)
      return hip_err(e, "hipEventElapsedTime");
    tot += ms;
  }
  *total_ms = tot;
  *launches = (int64_t)m->ev_used.size();
  return FGL_OK;
}

int fgl_model_destroy(fgl_model* mh) {
  Model* m = reinterpret_cast<Model*>(mh);
  if (!m) return set_err(FGL_EINVAL, "model is NULL");
  if (m->inflight.load() != 0 || m->served.load() != 0)
    return set_err(FGL_EBUSY, "model has %d calls and %d served requests in flight",
                   m->inflight.load(), m->served.load());
  bool expected = false;
  if (!m->dying.compare_exchange_strong(expected, true))
    return set_err(FGL_EBUSY, "model is already being destroyed");
  if (m->inflight.load() != 0 || m->served.load() != 0) {
    m->dying.store(false);
    return set_err(FGL_EBUSY, "model became busy");
  }
  unregister_model(m);
  serve_forget_model(m);
  (void)hipSetDevice(m->dev);
  // work may still be queued on caller streams (device-pointer calls)
  (void)hipDeviceSynchronize();
  for (auto& kv : m->graphs)
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
  m->graphs.clear();
  for (auto& kv : m->work) free_work(kv.second);
  for (auto& wb : m->retired) free_work(wb);
  for (auto* v : {&m->ev_used, &m->ev_free})
    for (auto& ev : *v) {
      (void)hipEventDestroy(ev.first);
      (void)hipEventDestroy(ev.second);
    }
  evict(m);
  (void)hipStreamDestroy(m->stream);
  delete m;
  return FGL_OK;
}

}  // extern "C"
