// Driver of the host code under the sanitizers, on the CPU stand-in of the
// HIP runtime (hip_stub.cpp) and of the kernel launchers (launch_stub.cpp).
// Test infrastructure only.
//
// It checks the likelihood launch's chunk plans and block map, then runs
// the library's host paths the GPU tests run, with every row's
// result predicted exactly (the launcher stand-ins compute
// lnL' = sum_k (k + 1) theta_k + D[0]):
//   1. model creation in every form (direct, projected, thin, crossed masks,
//      plain-projected, no 21-cm term): the real layout builders;
//   2. synchronous calls, three times each (eager, captured, replayed);
//   3. device-pointer calls on user streams and the legacy stream, with and
//      without graph replay; the allocation-free path is not built here;
//   4. gradients, host and device pointers;
//   5. the tuner with events and a persisted tuner cache, kernel timing;
//   6. eight threads calling two models each, synchronous and device calls;
//   7. serving: 16 clients with up to four requests each in flight, with and
//      without launches shared across models, with and without an HBM
//      budget that forces eviction; a held queue released at once;
//      cancellation, the wait limit and the budget from the environment; a forced
//      request failure; destroying a busy model and a busy server;
//   8. after destroying everything, no device or pinned allocation is live.
// Exit status 0 when every check passed and the stand-ins reported nothing.
#include <unistd.h>

#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "../../include/fgl.h"
#include "../../paper_2603_13196_amd/csrc/fgl_internal.h"
#include "hip_stub.h"

namespace {

std::atomic<long> g_fail{0};
std::mutex g_print_mu;

#define CHECK(cond, ...)                                    \
  do {                                                      \
    if (!(cond)) {                                          \
      std::lock_guard<std::mutex> lk_(g_print_mu);          \
      std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
      std::fprintf(stderr, __VA_ARGS__);                    \
      std::fprintf(stderr, " (%s)\n", fgl_last_error());    \
      g_fail.fetch_add(1);                                  \
    }                                                       \
  } while (0)

void step(const char* what) {
  std::lock_guard<std::mutex> lk(g_print_mu);
  std::printf("-- %s\n", what);
  std::fflush(stdout);
}

struct TM {
  fgl_model* h = nullptr;
  int P = 0;
  double d0 = 0.0;
  const char* name = "";
};

TM make(const char* name, int NA, int NB, int F, int T, unsigned flags, uint64_t seed) {
  std::mt19937_64 rng(seed);
  std::uniform_real_distribution<double> u(0.1, 1.0);
  const int N = (NA > 0 ? NA : 1) * NB;
  std::vector<float> K((size_t)N * F * T);
  for (auto& k : K) k = (float)u(rng);
  std::vector<double> freqs(F), data((size_t)F * T);
  for (int f = 0; f < F; ++f) freqs[f] = 50.0 + 150.0 * f / std::max(1, F - 1);
  for (auto& d : data) d = 2.725 + u(rng);
  TM m;
  m.name = name;
  const int rc = NA > 0 ? fgl_model_create_masks(K.data(), freqs.data(), data.data(), 100.0, NA,
                                                 NB, F, T, 2.725, flags, &m.h)
                        : fgl_model_create(K.data(), freqs.data(), data.data(), 100.0, NB, F, T,
                                           2.725, flags, &m.h);
  CHECK(rc == FGL_OK, "create %s", name);
  m.P = fgl_model_nparams(m.h);
  m.d0 = data[0];
  return m;
}

std::vector<double> rows(int B, int P, uint64_t seed, bool with_invalid) {
  std::mt19937_64 rng(seed);
  std::uniform_real_distribution<double> u(-1.0, 1.0);
  std::vector<double> th((size_t)B * P);
  for (auto& x : th) x = u(rng);
  if (with_invalid && B > 2) th[(size_t)(B / 2) * P] = NAN;
  return th;
}

double want(const TM& m, const double* row) {
  double v = 0.0;
  for (int k = 0; k < m.P; ++k) {
    if (!std::isfinite(row[k])) return -INFINITY;
    v += (double)(k + 1) * row[k];
  }
  return v + m.d0;
}

long mismatches(const TM& m, const std::vector<double>& th, const double* out, int B) {
  long bad = 0;
  for (int b = 0; b < B; ++b) {
    const double w = want(m, &th[(size_t)b * m.P]);
    if (!(out[b] == w)) ++bad;
  }
  return bad;
}

const int kPrecs[3] = {FGL_PREC_MIXED, FGL_PREC_FP32, FGL_PREC_FP64};

void sync_calls(const TM& m) {
  for (int B : {1, 37, 300, 1000, 4100}) {
    for (int prec : kPrecs) {
      const auto th = rows(B, m.P, 1000u + B + prec, true);
      std::vector<double> out(B);
      for (int rep = 0; rep < 3; ++rep) {
        std::fill(out.begin(), out.end(), 0.0);
        const int rc = fgl_loglike_batch(m.h, th.data(), B, out.data(), prec);
        CHECK(rc == FGL_OK, "%s sync B=%d prec=%d rep=%d", m.name, B, prec, rep);
        CHECK(mismatches(m, th, out.data(), B) == 0, "%s sync B=%d prec=%d rep=%d values",
              m.name, B, prec, rep);
      }
    }
  }
}

void device_calls(const TM& m, hipStream_t s) {
  for (int B : {5, 700, 2100}) {
    const auto th = rows(B, m.P, 77u + B, false);
    double *d_th = nullptr, *d_out = nullptr;
    CHECK(hipMalloc(reinterpret_cast<void**>(&d_th), th.size() * 8) == hipSuccess, "alloc");
    CHECK(hipMalloc(reinterpret_cast<void**>(&d_out), (size_t)B * 8) == hipSuccess, "alloc");
    CHECK(hipMemcpy(d_th, th.data(), th.size() * 8, hipMemcpyHostToDevice) == hipSuccess, "copy");
    for (int prec : kPrecs)
      for (int rep = 0; rep < 3; ++rep) {
        CHECK(fgl_loglike_batch_device(m.h, d_th, B, d_out, prec, s) == FGL_OK,
              "%s device B=%d prec=%d", m.name, B, prec);
        std::vector<double> out(B);
        CHECK(hipMemcpyAsync(out.data(), d_out, (size_t)B * 8, hipMemcpyDeviceToHost, s) ==
                  hipSuccess, "copy back");
        CHECK(hipStreamSynchronize(s) == hipSuccess, "sync");
        CHECK(mismatches(m, th, out.data(), B) == 0, "%s device B=%d prec=%d rep=%d values",
              m.name, B, prec, rep);
      }
    (void)hipFree(d_th);
    (void)hipFree(d_out);
  }
}

void grad_calls(const TM& m) {
  const int B = 333;
  const auto th = rows(B, m.P, 5, true);
  std::vector<double> out(B), grad((size_t)B * m.P);
  CHECK(fgl_loglike_grad_batch(m.h, th.data(), B, out.data(), grad.data(), FGL_PREC_FP64) ==
            FGL_OK, "%s grad", m.name);
  CHECK(mismatches(m, th, out.data(), B) == 0, "%s grad values", m.name);
  for (int b = 0; b < B; ++b)
    if (std::isfinite(out[b]))
      for (int k = 0; k < m.P; ++k)
        CHECK(grad[(size_t)b * m.P + k] == k + 1, "%s grad row %d entry %d", m.name, b, k);
  CHECK(fgl_loglike_grad_batch(m.h, th.data(), B, out.data(), grad.data(), FGL_PREC_MIXED) ==
            FGL_EINVAL, "%s grad in mixed precision must be refused", m.name);
  double *d_th, *d_out, *d_grad;
  (void)hipMalloc(reinterpret_cast<void**>(&d_th), th.size() * 8);
  (void)hipMalloc(reinterpret_cast<void**>(&d_out), (size_t)B * 8);
  (void)hipMalloc(reinterpret_cast<void**>(&d_grad), grad.size() * 8);
  (void)hipMemcpy(d_th, th.data(), th.size() * 8, hipMemcpyHostToDevice);
  CHECK(fgl_loglike_grad_batch_device(m.h, d_th, B, d_out, d_grad, FGL_PREC_FP64, nullptr) ==
            FGL_OK, "%s grad device", m.name);
  std::vector<double> out2(B);
  (void)hipMemcpy(out2.data(), d_out, (size_t)B * 8, hipMemcpyDeviceToHost);
  CHECK(mismatches(m, th, out2.data(), B) == 0, "%s grad device values", m.name);
  (void)hipFree(d_th);
  (void)hipFree(d_out);
  (void)hipFree(d_grad);
}

// a client of a server: `n` requests, at most `depth` in flight
void client(fgl_server* srv, const std::vector<TM>& ms, int id, int n, int depth,
            std::atomic<long>* failed_polls) {
  std::mt19937_64 rng(9000 + id);
  struct Pending {
    uint64_t ticket;
    int mi, B;
    std::vector<double> th, out;
  };
  std::vector<Pending> fly;
  int sent = 0;
  while (sent < n || !fly.empty()) {
    while (sent < n && (int)fly.size() < depth) {
      Pending p;
      p.mi = (int)(rng() % ms.size());
      p.B = 1 + (int)(rng() % 3000);
      p.th = rows(p.B, ms[p.mi].P, rng(), rng() % 4 == 0);
      p.out.assign(p.B, 0.0);
      const int prec = kPrecs[rng() % 3];
      const int rc = fgl_serve_submit(srv, ms[p.mi].h, p.th.data(), p.B, p.out.data(), prec,
                                      &p.ticket);
      CHECK(rc == FGL_OK, "client %d submit", id);
      if (rc != FGL_OK) return;
      fly.push_back(std::move(p));
      ++sent;
    }
    for (size_t i = 0; i < fly.size();) {
      int done = 0;
      double us = 0.0;
      const int rc = fgl_serve_poll(srv, fly[i].ticket, &done, &us);
      if (!done) {
        CHECK(rc == FGL_OK, "client %d poll", id);
        ++i;
        continue;
      }
      if (rc != FGL_OK) {
        failed_polls->fetch_add(1);
      } else {
        CHECK(mismatches(ms[fly[i].mi], fly[i].th, fly[i].out.data(), fly[i].B) == 0,
              "client %d ticket %llu model %s B=%d values", id,
              (unsigned long long)fly[i].ticket, ms[fly[i].mi].name, fly[i].B);
      }
      fly.erase(fly.begin() + (long)i);
    }
    std::this_thread::yield();
  }
}

void serve_round(const std::vector<TM>& ms, size_t budget, int slots, int share, int clients,
                 int per_client) {
  char what[160];
  std::snprintf(what, sizeof what, "serving: budget %zu, %d slots, sharing %d, %d clients",
                budget, slots, share, clients);
  step(what);
  fgl_server* srv = nullptr;
  CHECK(fgl_serve_create(budget, slots, &srv) == FGL_OK, "serve_create");
  CHECK(fgl_serve_set_sharing(srv, share) == FGL_OK, "set_sharing");
  std::atomic<long> failed{0};
  std::vector<std::thread> th;
  for (int c = 0; c < clients; ++c)
    th.emplace_back(client, srv, std::cref(ms), c, per_client, 4, &failed);
  for (auto& t : th) t.join();
  CHECK(failed.load() == 0, "no request may fail here");
  CHECK(fgl_serve_drain(srv) == FGL_OK, "drain");
  uint64_t launches = 0, shared = 0, groups = 0;
  CHECK(fgl_serve_stats(srv, &launches, &shared, &groups) == FGL_OK, "stats");
  std::printf("   launches %llu, shared %llu carrying %llu groups\n",
              (unsigned long long)launches, (unsigned long long)shared,
              (unsigned long long)groups);
  CHECK(launches > 0, "launches");
  CHECK(fgl_serve_destroy(srv) == FGL_OK, "serve_destroy");
}

}  // namespace

// The likelihood launch's channel chunks (fgl::chunk_plan) and its block
// map (fgl::map_block_split): the chunks tile [0, F) at multiples of the
// reduction group, and the map sends the launch's block ids one to one onto
// (row tile, chunk), with every XCD's large chunks ahead of its small ones.
void chunk_plans() {
  using namespace fgl;
  long plans = 0, split = 0;
  for (int F : {1, 5, 64, 301, 401, 1000})
    for (int KC : {1, 2})
      for (int proj : {0, 1})
        for (int G : {1, 2, 4})
          for (int mult : {1, 2, 4})
            for (int W : {4, 8})
              for (int occ : {2, 3})
                for (int nb : {1, 3, 64, 128, 511}) {
                  DevModel m{};
                  m.F = F;
                  m.KC = KC;
                  m.proj = proj;
                  m.RT = 2;
                  m.TT = 3;
                  const Tile t{W, G * mult, G, occ};
                  if (lds_bytes(kMixed, m, t) > max_lds_bytes()) continue;
                  const Chunks c = chunk_plan(kMixed, m, t, nb);
                  ++plans;
                  CHECK(c.fc == t.fc && c.fs >= 1 && c.fs <= c.fc && c.fs % G == 0 &&
                            c.nbig >= 1 && c.nbig <= c.nc,
                        "plan F=%d fc=%d: fc %d fs %d nbig %d nc %d", F, t.fc, c.fc, c.fs,
                        c.nbig, c.nc);
                  const int nsmall = c.nc - c.nbig;
                  split += nsmall > 0;
                  // chunk ch covers [f0, f0 + fn): contiguous, in order, ending at F
                  int next = 0;
                  for (int ch = 0; ch < c.nc; ++ch) {
                    const bool big = ch < c.nbig;
                    const int f0 = big ? ch * c.fc : c.nbig * c.fc + (ch - c.nbig) * c.fs;
                    const int fn = std::min(big ? c.fc : c.fs, F - f0);
                    CHECK(f0 == next && fn >= 1 && f0 % G == 0, "chunk %d of F=%d", ch, F);
                    next = f0 + fn;
                  }
                  CHECK(next == F, "chunks end at %d, F=%d", next, F);
                  CHECK(nsmall == 0 || (long)nb * nsmall >= 8, "too few small pairs");
                  const long total = (long)nb * c.nc;
                  if (total > 200000) continue;
                  std::vector<char> seen(total, 0);
                  std::vector<char> small_seen(8, 0);
                  bool order = true, onto = true;
                  for (long id = 0; id < total; ++id) {
                    int bt = -1, ch = -1;
                    map_block_split((int)id, nb, c.nbig, nsmall, bt, ch);
                    if (bt < 0 || bt >= nb || ch < 0 || ch >= c.nc || seen[(long)bt * c.nc + ch]) {
                      onto = false;
                      break;
                    }
                    seen[(long)bt * c.nc + ch] = 1;
                    const int x = (int)(id & 7);
                    if (ch >= c.nbig) small_seen[x] = 1;
                    else if (small_seen[x]) order = false;
                  }
                  CHECK(onto, "block map not one to one: F=%d nb=%d plan %d/%d/%d/%d", F, nb,
                        c.fc, c.fs, c.nbig, c.nc);
                  CHECK(order, "small chunk ahead of a large one: F=%d nb=%d", F, nb);
                }
  // the headline shape: N32 F301, 8 waves of 32 rows, B = 16384 (64 row tiles)
  DevModel h{};
  h.F = 301;
  h.KC = 1;
  h.proj = 1;
  h.RT = 1;
  const Chunks c = chunk_plan(kMixed, h, Tile{8, 8, 4, 3}, 64);
  CHECK(c.fc == 8 && c.fs == 4 && c.nbig == 36 && c.nc == 40, "headline plan %d/%d/%d/%d",
        c.fc, c.fs, c.nbig, c.nc);
  // N64 F401 in the direct form, B = 65536 in 2-channel chunks: the split
  // would move one channel per row tile (401 against 402 per CU), under the
  // 2% it has to gain, so the chunks stay uniform
  DevModel l{};
  l.F = 401;
  l.KC = 2;
  l.TT = 8;
  const Chunks d = chunk_plan(kMixed, l, Tile{8, 2, 1, 2}, 256);
  CHECK(d.nbig == d.nc && d.nc == 201, "N64 F401 direct plan %d/%d/%d/%d", d.fc, d.fs, d.nbig,
        d.nc);
  const Chunks p = chunk_plan(kFP32, h, Tile{8, 8, 4, 2}, 64);
  CHECK(p.nbig == p.nc && p.fs == p.fc, "plain kernels keep uniform chunks");
  std::printf("   %ld plans, %ld with small chunks\n", plans, split);
}

int main() {
  setvbuf(stdout, nullptr, _IOLBF, 0);
  step("chunk plans and the likelihood block map");
  chunk_plans();
  step("models in every form");
  std::vector<TM> ms;
  ms.push_back(make("direct", 0, 8, 20, 40, FGL_MIXED_DIRECT, 1));
  ms.push_back(make("projected", 0, 8, 20, 96, 0, 2));
  ms.push_back(make("thin", 0, 4, 15, 6, 0, 3));
  ms.push_back(make("masks", 2, 4, 10, 40, 0, 4));
  ms.push_back(make("plain-projected", 0, 6, 12, 80, FGL_PLAIN_PROJECTED, 5));
  ms.push_back(make("no21", 0, 3, 11, 4, FGL_NO_21CM, 6));
  ms.push_back(make("projected-b", 0, 8, 24, 96, 0, 7));    // same variant as "projected"
  ms.push_back(make("thin-b", 0, 3, 9, 5, 0, 8));           // same variant as "thin"
  for (const TM& m : ms) {
    std::printf("   %-16s P=%d form=%d bytes=%zu\n", m.name, m.P, fgl_mixed_form(m.h),
                fgl_model_bytes(m.h));
  }

  step("synchronous calls (eager, captured, replayed)");
  for (const TM& m : ms) sync_calls(m);

  step("device-pointer calls");
  hipStream_t us = nullptr;
  (void)hipStreamCreateWithFlags(&us, hipStreamNonBlocking);
  for (const TM& m : ms) device_calls(m, us);
  device_calls(ms[1], nullptr);
  setenv("FGL_DEVICE_GRAPHS", "1", 1);
  TM g = make("device-graphs", 0, 8, 20, 96, 0, 9);
  unsetenv("FGL_DEVICE_GRAPHS");
  device_calls(g, us);

  step("gradients");
  for (const TM& m : ms) grad_calls(m);

  step("tuner, tuner cache, kernel timing");
  char path[] = "/tmp/fgl_tc_XXXXXX";
  const int fd = mkstemp(path);
  CHECK(fd >= 0, "temp file");
  close(fd);
  CHECK(fgl_tune_cache(path) == FGL_OK, "tune_cache");
  CHECK(fgl_tune(ms[1].h, 1000, FGL_PREC_MIXED) == FGL_OK, "tune");
  int waves = 0, chans = 0, occ = 0;
  CHECK(fgl_get_tile(ms[1].h, 1000, FGL_PREC_MIXED, &waves, &chans, &occ) == FGL_OK, "get_tile");
  FILE* f = std::fopen(path, "r");
  char line[512] = {0};
  CHECK(f && std::fgets(line, sizeof line, f), "the tuner cache file holds an entry");
  if (f) std::fclose(f);
  std::printf("   tuned waves=%d chans=%d occ=%d; cache: %s", waves, chans, occ, line);
  CHECK(fgl_tune_cache(nullptr) == FGL_OK, "tune_cache off");
  std::remove(path);
  sync_calls(ms[1]);
  CHECK(fgl_kernel_timing(ms[0].h, 1) == FGL_OK, "timing on");
  for (int r = 0; r < 4; ++r) {
    const auto th = rows(64, ms[0].P, r, false);
    std::vector<double> out(64);
    CHECK(fgl_loglike_batch(ms[0].h, th.data(), 64, out.data(), FGL_PREC_MIXED) == FGL_OK, "timed");
  }
  double ms_total = 0.0;
  int64_t launches = 0;
  CHECK(fgl_kernel_time(ms[0].h, &ms_total, &launches) == FGL_OK && launches == 4,
        "kernel_time launches=%lld", (long long)launches);
  CHECK(fgl_kernel_timing(ms[0].h, 0) == FGL_OK, "timing off");

  step("eight threads on shared models");
  {
    std::vector<std::thread> th;
    for (int t = 0; t < 8; ++t)
      th.emplace_back([&, t] {
        hipStream_t s = nullptr;
        (void)hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        std::mt19937_64 rng(t);
        for (int i = 0; i < 30; ++i) {
          const TM& m = ms[(t + i) % 4];
          const int B = 1 + (int)(rng() % 2000);
          const int prec = kPrecs[rng() % 3];
          const auto th2 = rows(B, m.P, rng(), false);
          std::vector<double> out(B);
          if (i % 3 == 2) {
            double *d_th, *d_out;
            (void)hipMalloc(reinterpret_cast<void**>(&d_th), th2.size() * 8);
            (void)hipMalloc(reinterpret_cast<void**>(&d_out), (size_t)B * 8);
            (void)hipMemcpyAsync(d_th, th2.data(), th2.size() * 8, hipMemcpyHostToDevice, s);
            CHECK(fgl_loglike_batch_device(m.h, d_th, B, d_out, prec, s) == FGL_OK, "thread device");
            (void)hipMemcpyAsync(out.data(), d_out, (size_t)B * 8, hipMemcpyDeviceToHost, s);
            (void)hipStreamSynchronize(s);
            (void)hipFree(d_th);
            (void)hipFree(d_out);
          } else {
            CHECK(fgl_loglike_batch(m.h, th2.data(), B, out.data(), prec) == FGL_OK, "thread sync");
          }
          CHECK(mismatches(m, th2, out.data(), B) == 0, "thread %d call %d %s values", t, i, m.name);
        }
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
      });
    for (auto& x : th) x.join();
  }

  // serving, on models that only the servers use (eviction then does not
  // wait for the device: a server evicts only models with no request in
  // flight); the models without amplitude masks share launches when their
  // variants match; the budget below holds about half of the models
  step("models for serving");
  std::vector<TM> sv;
  sv.push_back(make("s-direct", 0, 8, 20, 40, FGL_MIXED_DIRECT, 11));
  sv.push_back(make("s-projected", 0, 8, 20, 96, 0, 12));
  sv.push_back(make("s-projected-b", 0, 8, 24, 96, 0, 13));
  sv.push_back(make("s-thin", 0, 4, 15, 6, 0, 14));
  sv.push_back(make("s-thin-b", 0, 3, 9, 5, 0, 15));
  sv.push_back(make("s-masks", 2, 4, 10, 40, 0, 16));
  sv.push_back(make("s-no21", 0, 3, 11, 4, FGL_NO_21CM, 17));
  size_t all = 0;
  for (const TM& m : sv) all += fgl_model_bytes(m.h);
  serve_round(sv, 0, 3, 1, 16, 40);
  serve_round(sv, 0, 2, 8, 16, 40);
  serve_round(sv, 0, 1, 16, 16, 40);
  serve_round(sv, all / 2, 2, 1, 12, 30);
  serve_round(sv, all / 2, 3, 8, 12, 30);
  serve_round(sv, all / 3, 4, 8, 16, 30);

  step("serving: a held queue released at once");
  {
    fgl_server* srv = nullptr;
    CHECK(fgl_serve_create(0, 2, &srv) == FGL_OK, "create");
    CHECK(fgl_serve_set_sharing(srv, 16) == FGL_OK, "sharing");
    CHECK(fgl_serve_hold(srv, 1) == FGL_OK, "hold");
    const int n = 48;
    std::vector<std::vector<double>> th(n), out(n);
    std::vector<uint64_t> tk(n);
    for (int i = 0; i < n; ++i) {
      const TM& m = sv[i % 5];                     // models without amplitude masks
      const int B = 50 + 37 * i;
      th[i] = rows(B, m.P, 700 + i, false);
      out[i].assign(B, 0.0);
      CHECK(fgl_serve_submit(srv, m.h, th[i].data(), B, out[i].data(), FGL_PREC_MIXED, &tk[i]) ==
                FGL_OK, "submit held");
    }
    CHECK(fgl_serve_drain(srv) == FGL_EAGAIN, "drain of a held queue");
    CHECK(fgl_serve_destroy(srv) == FGL_EBUSY, "destroy of a held queue");
    CHECK(fgl_serve_hold(srv, 0) == FGL_OK, "release");
    CHECK(fgl_serve_drain(srv) == FGL_OK, "drain");
    for (int i = 0; i < n; ++i) {
      int done = 0;
      double us2 = 0.0;
      CHECK(fgl_serve_poll(srv, tk[i], &done, &us2) == FGL_OK && done == 1, "held ticket %d", i);
      CHECK(mismatches(sv[i % 5], th[i], out[i].data(), (int)out[i].size()) == 0,
            "held ticket %d values", i);
    }
    uint64_t launches = 0, shared = 0, groups = 0;
    CHECK(fgl_serve_stats(srv, &launches, &shared, &groups) == FGL_OK, "stats");
    std::printf("   launches %llu, shared %llu carrying %llu groups\n",
                (unsigned long long)launches, (unsigned long long)shared,
                (unsigned long long)groups);
    CHECK(shared >= 1 && launches < (uint64_t)n, "a released queue is merged and shared");
    CHECK(fgl_serve_destroy(srv) == FGL_OK, "destroy");
  }

  step("serving: cancellation, wait limit, budget from the environment");
  {
    fgl_server* srv = nullptr;
    CHECK(fgl_serve_create(0, 2, &srv) == FGL_OK, "create");
    const TM& m = sv[0];
    auto submit = [&](std::vector<double>& th, std::vector<double>& out, int B, int seed,
                      uint64_t* t) {
      th = rows(B, m.P, seed, false);
      out.assign(B, -1.0);
      return fgl_serve_submit(srv, m.h, th.data(), B, out.data(), FGL_PREC_MIXED, t);
    };
    std::vector<double> th[4], out[4];
    uint64_t tk[4] = {0, 0, 0, 0};
    int done = 0;
    double us2 = 0.0;
    // a queued request is cancelled; the others complete
    CHECK(fgl_serve_hold(srv, 1) == FGL_OK, "hold");
    for (int i = 0; i < 3; ++i) CHECK(submit(th[i], out[i], 100 + i, 900 + i, &tk[i]) == FGL_OK, "submit");
    CHECK(fgl_serve_cancel(srv, tk[1]) == FGL_OK, "cancel a queued request");
    CHECK(fgl_serve_cancel(srv, tk[1]) == FGL_EBUSY, "cancel twice");
    CHECK(fgl_serve_poll(srv, tk[1], &done, &us2) == FGL_ECANCELED && done == 1, "cancelled poll");
    CHECK(out[1][0] == -1.0, "a cancelled request writes nothing");
    CHECK(fgl_serve_cancel(srv, tk[1]) == FGL_EINVAL, "cancel a retired ticket");
    CHECK(fgl_serve_hold(srv, 0) == FGL_OK, "release");
    CHECK(fgl_serve_drain(srv) == FGL_OK, "drain");
    CHECK(fgl_serve_cancel(srv, tk[0]) == FGL_EBUSY, "cancel a completed request");
    for (int i : {0, 2}) {
      CHECK(fgl_serve_poll(srv, tk[i], &done, &us2) == FGL_OK && done == 1, "ticket %d", i);
      CHECK(mismatches(m, th[i], out[i].data(), (int)out[i].size()) == 0, "ticket %d values", i);
    }
    // queued past the wait limit (held, so nothing launches): timed out
    CHECK(fgl_serve_set_timeout(srv, -1.0) == FGL_EINVAL, "negative wait limit");
    CHECK(fgl_serve_set_timeout(srv, 2000.0) == FGL_OK, "wait limit");
    CHECK(fgl_serve_hold(srv, 1) == FGL_OK, "hold");
    for (int i = 0; i < 2; ++i) CHECK(submit(th[i], out[i], 64, 950 + i, &tk[i]) == FGL_OK, "submit");
    for (int i = 0; i < 2; ++i) {
      int spins = 0;
      int rc = FGL_OK;
      done = 0;
      while (!done && spins++ < 2000) {
        rc = fgl_serve_poll(srv, tk[i], &done, &us2);
        if (!done) usleep(1000);
      }
      CHECK(done == 1 && rc == FGL_ETIMEDOUT && us2 >= 2000.0, "timed out (rc %d, %g us)", rc, us2);
      CHECK(out[i][0] == -1.0, "a timed-out request writes nothing");
    }
    CHECK(fgl_serve_hold(srv, 0) == FGL_OK, "release");
    CHECK(fgl_serve_set_timeout(srv, 0.0) == FGL_OK, "no wait limit");
    CHECK(submit(th[3], out[3], 80, 990, &tk[3]) == FGL_OK, "submit");
    CHECK(fgl_serve_drain(srv) == FGL_OK, "drain");
    CHECK(fgl_serve_poll(srv, tk[3], &done, &us2) == FGL_OK && done == 1, "after the limit");
    CHECK(mismatches(m, th[3], out[3].data(), (int)out[3].size()) == 0, "values after the limit");
    CHECK(fgl_serve_destroy(srv) == FGL_OK, "destroy");
    // a budget of 0.1 MiB from FGL_HBM_BUDGET_MB is below the model's bytes
    setenv("FGL_HBM_BUDGET_MB", "0.1", 1);
    CHECK(fgl_serve_create(0, 1, &srv) == FGL_OK, "create with FGL_HBM_BUDGET_MB");
    unsetenv("FGL_HBM_BUDGET_MB");
    CHECK(submit(th[0], out[0], 10, 999, &tk[0]) == FGL_EAGAIN, "budget from the environment");
    CHECK(fgl_serve_destroy(srv) == FGL_OK, "destroy");
  }

  step("serving: forced failure, busy model and server");
  {
    setenv("FGL_SERVE_FAIL_TICKET", "3", 1);
    fgl_server* srv = nullptr;
    CHECK(fgl_serve_create(0, 1, &srv) == FGL_OK, "create");
    unsetenv("FGL_SERVE_FAIL_TICKET");
    const int n = 40, B = 4000;
    std::vector<std::vector<double>> th(n), out(n, std::vector<double>(B));
    std::vector<uint64_t> tk(n);
    for (int i = 0; i < n; ++i) {
      th[i] = rows(B, ms[1].P, 500 + i, false);
      CHECK(fgl_serve_submit(srv, ms[1].h, th[i].data(), B, out[i].data(), FGL_PREC_MIXED,
                             &tk[i]) == FGL_OK, "submit");
    }
    const int drc = fgl_model_destroy(ms[1].h);
    const int src = fgl_serve_destroy(srv);
    std::printf("   model destroy with queued work: %d, server destroy: %d\n", drc, src);
    CHECK(drc == FGL_EBUSY || drc == FGL_OK, "model destroy");
    if (drc == FGL_OK) ms[1].h = nullptr;
    CHECK(src == FGL_EBUSY || src == FGL_OK, "server destroy");
    if (src == FGL_EBUSY) {
      CHECK(fgl_serve_drain(srv) == FGL_OK, "drain");
      int failed = 0;
      for (int i = 0; i < n; ++i) {
        int done = 0;
        double us2 = 0.0;
        const int rc = fgl_serve_poll(srv, tk[i], &done, &us2);
        CHECK(done == 1, "ticket %d done after drain", i);
        if (rc != FGL_OK) {
          ++failed;
          CHECK(tk[i] == 3 && rc == FGL_EDEVICE, "only ticket 3 fails (ticket %llu rc %d)",
                (unsigned long long)tk[i], rc);
        } else {
          CHECK(ms[1].h == nullptr || mismatches(ms[1], th[i], out[i].data(), B) == 0,
                "ticket %d values", i);
        }
      }
      CHECK(failed == 1, "one forced failure, saw %d", failed);
      CHECK(fgl_serve_destroy(srv) == FGL_OK, "destroy after drain");
    }
  }

  step("teardown");
  (void)hipStreamDestroy(us);
  for (auto* v : {&ms, &sv})
    for (TM& m : *v)
      if (m.h) CHECK(fgl_model_destroy(m.h) == FGL_OK, "destroy %s", m.name);
  CHECK(fgl_model_destroy(g.h) == FGL_OK, "destroy device-graphs");
  const size_t live = stub_live_allocations();
  CHECK(live == 0, "%zu device or pinned allocations still live after teardown", live);
  const long stub = stub_errors();
  std::printf("checks failed: %ld, stand-in reports: %ld\n", g_fail.load(), stub);
  return g_fail.load() == 0 && stub == 0 ? 0 : 1;
}
