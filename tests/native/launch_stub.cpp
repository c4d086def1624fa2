// CPU stand-ins for the kernel launchers of fgl_kernels.hip, for the
// sanitizer build of the host code (with hip_stub.cpp).  Test infrastructure
// only.
//
// Each launcher checks its arguments as the real one does and enqueues, on
// the same stream, a closure that touches what the real kernel touches:
//  * row preparation writes the row record and the transposed indices of
//    every padded row (so a workspace smaller than the kernel's writes is an
//    out-of-bounds write);
//  * the likelihood launch reads the first and last element of each model
//    buffer its kernel family reads (so a launch on an evicted model is a
//    use after free) and writes every reduction group's partial of every row;
//  * finalize reads the partials and writes out[0..B).
// The value is not the likelihood but a stand-in that the driver can
// predict exactly for every row:
//   lnL'(theta) = sum_k (k + 1) theta_k + D[0]
// (D[0] the model's first data value, read from its device buffer; -inf
// for a row with a non-finite entry), with gradient row (1, 2, .., P).
// A shared launch reads its group table from device memory when it runs
// (after the table's copy on the same stream) and checks that every group's
// workgroup ranges fit the grid, start on a multiple of eight and do not
// overlap, and that every group has the launch's compiled variant.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include "../../paper_2603_13196_amd/csrc/fgl_internal.h"
#include "hip_stub.h"

namespace fgl {

namespace {

thread_local volatile double g_sink;   // per stream thread: reads the compiler must keep

template <typename T>
void touch(const T* p, size_t n, const char* what) {
  if (!p) {
    char msg[160];
    std::snprintf(msg, sizeof msg, "a kernel read the model buffer %s, which is not resident", what);
    stub_report(msg);
    return;
  }
  g_sink = (double)p[0] + (double)p[n - 1];
}

void touch_model(Kind k, const DevModel& m) {
  touch(m.D, (size_t)m.F * m.TT * 32, "D");
  switch (k) {
    case kMixed:
      touch(m.tab, (size_t)kTabSize + 2 * kFracSize, "tab");
      if (m.proj)
        touch(m.rd, (size_t)m.F * kProjDigits * m.KC * m.RT * 1024, "rd");
      else
        touch(m.kd, (size_t)m.F * 4 * m.KC * m.TT * 1024, "kd");
      break;
    case kFP32:
      if (m.pplain)
        touch(m.r32, (size_t)m.F * m.NP2 * m.RT * 64, "r32");
      else
        touch(m.k32, (size_t)m.F * m.NP2 * m.TT * 64, "k32");
      break;
    case kFP64:
      if (m.pplain)
        touch(m.pa64, (size_t)m.F * m.NQ * m.RT16 * 64, "pa64");
      else
        touch(m.k64, (size_t)m.F * m.NQ * m.TT16 * 64, "k64");
      break;
    case kThin: touch(m.kthin, (size_t)m.F * m.T * m.NT, "kthin"); break;
  }
}

// row preparation of rows [0, Bpad)
void prep_rows(const DevModel& m, const double* theta, int B, const Work& w, int betaRows) {
  for (int b = 0; b < w.Bpad; ++b) {
    RowParams rp{};
    rp.valid = 0;
    if (b < B) {
      double v = 0.0;
      bool ok = true;
      for (int k = 0; k < m.P; ++k) {
        const double x = theta[(size_t)b * m.P + k];
        ok = ok && std::isfinite(x);
        v += (double)(k + 1) * x;
      }
      rp.valid = ok ? 1 : 0;
      rp.A = v;
    }
    w.rows[b] = rp;
    for (int r = 0; r < betaRows; ++r) {
      const bool real = b < B && r < m.N;
      w.betaT[(size_t)r * w.Bpad + b] = real ? theta[(size_t)b * m.P + r % m.NB] : 0.0;
      if (m.NA > 0) w.offT[(size_t)r * w.Bpad + b] = 0.0;
    }
  }
}

void main_rows(Kind k, const DevModel& m, const Work& w, int ngroups) {
  touch_model(k, m);
  const double d0 = m.D ? m.D[0] : 0.0;
  for (int g = 0; g < ngroups; ++g)
    for (int b = 0; b < w.Bpad; ++b)
      w.partial[(size_t)g * w.Bpad + b] = g == 0 ? w.rows[b].A + d0 : 0.0;
}

void finalize_rows(const Work& w, int ngroups, double* out) {
  for (int b = 0; b < w.B; ++b) {
    double acc = 0.0;
    for (int g = 0; g < ngroups; ++g) acc += w.partial[(size_t)g * w.Bpad + b];
    out[b] = w.rows[b].valid ? acc : -INFINITY;
  }
}

hipError_t check_main(Kind k, const DevModel& m, const Work& w, const Tile& tile) {
  const int cols = cols_per_wave(k) * tile.waves;
  if (w.Bpad % cols != 0 || n_groups(m, tile) > w.ngroup_cap || tile.group < 1 ||
      tile.fc % tile.group != 0 || lds_bytes(k, m, tile) > max_lds_bytes())
    return hipErrorInvalidValue;
  if (k == kThin && (!m.thin || !(tile.waves == 1 || tile.waves == 2 || tile.waves == 4)))
    return hipErrorInvalidValue;
  if (k != kThin && tile.waves != 4 && tile.waves != 8) return hipErrorInvalidValue;
  return hipSuccess;
}

}  // namespace

hipError_t launch_prep(const DevModel& m, const double* theta, int B, const Work& w,
                       int betaRows, hipStream_t s) {
  if (betaRows != m.KC * 32) return hipErrorInvalidValue;
  return stub_enqueue(s, [m, theta, B, w, betaRows] { prep_rows(m, theta, B, w, betaRows); });
}

hipError_t launch_main(Kind k, const DevModel& m, const Work& w, const Tile& tile,
                       hipStream_t s) {
  const hipError_t e = check_main(k, m, w, tile);
  if (e != hipSuccess) return e;
  const int ng = n_groups(m, tile);
  return stub_enqueue(s, [k, m, w, ng] { main_rows(k, m, w, ng); });
}

hipError_t launch_finalize(Kind, const DevModel& m, const Work& w, const Tile& tile,
                           double* out, hipStream_t s) {
  const int ng = n_groups(m, tile);
  return stub_enqueue(s, [w, ng, out] { finalize_rows(w, ng, out); });
}

hipError_t launch_groups(Kind k, const DevModel& m0, const Tile& tile, const GroupDesc* d, int n,
                         const int grid[3], int lds, hipStream_t s) {
  if (n < 1 || n > kMaxGroups || variant_of(k, m0, tile) == 0 || lds > max_lds_bytes())
    return hipErrorInvalidValue;
  const int g0 = grid[0], g1 = grid[1], g2 = grid[2];
  const uint64_t var = variant_of(k, m0, tile);
  return stub_enqueue(s, [k, tile, d, n, g0, g1, g2, lds, var] {
    int end[3] = {0, 0, 0};
    for (int j = 0; j < n; ++j) {
      const GroupDesc g = d[j];                     // the table, as the kernels read it
      const Tile tj{tile.waves, g.fc, g.G, tile.occ};
      const int cols = cols_per_wave(k) * tile.waves;
      const int len[3] = {g.nb * g.nc, (g.w.Bpad + kPrepRows - 1) / kPrepRows,
                          (g.w.B * 16 + 255) / 256};
      const int lim[3] = {g0, g1, g2};
      bool ok = variant_of(k, g.m, tj) == var && g.start[0] % 8 == 0 &&
                g.nb == g.w.Bpad / cols && g.nc == n_chunks(g.m, tj) &&
                g.ngroups == n_groups(g.m, tj) && lds_bytes(k, g.m, tj) <= lds &&
                check_main(k, g.m, g.w, tj) == hipSuccess;
      for (int q = 0; q < 3; ++q) {
        ok = ok && g.start[q] >= end[q] && g.start[q] + len[q] <= lim[q];
        end[q] = g.start[q] + len[q];
      }
      if (!ok) {
        char msg[120];
        std::snprintf(msg, sizeof msg, "shared launch: group %d of %d does not fit its plan", j, n);
        stub_report(msg);
        continue;
      }
      prep_rows(g.m, g.theta, g.w.B, g.w, g.m.KC * 32);
      main_rows(k, g.m, g.w, g.ngroups);
      finalize_rows(g.w, g.ngroups, g.out);
    }
  });
}

hipError_t launch_grad(const DevModel& m, const Work& w, const GradShape& g, hipStream_t s) {
  if (w.Bpad % 64 != 0 || g.lds > max_lds_bytes() || !w.gpart) return hipErrorInvalidValue;
  return stub_enqueue(s, [m, w, g] {
    touch(m.D, (size_t)m.F * m.TT * 32, "D");
    if (m.proj)
      touch(m.pa64, (size_t)m.F * m.NQ * m.RT16 * 64, "pa64");
    else
      touch(m.k64, (size_t)m.F * m.NQ * m.TT16 * 64, "k64");
    const size_t n = (size_t)grad_slots(m) * g.chunks * w.Bpad;
    for (size_t i = 0; i < n; ++i) w.gpart[i] = 0.0;
  });
}

hipError_t launch_grad_finalize(const DevModel& m, const Work& w, const GradShape& g,
                                const double* theta, double* out, double* grad, hipStream_t s) {
  return stub_enqueue(s, [m, w, g, theta, out, grad] {
    const double d0 = m.D ? m.D[0] : 0.0;
    g_sink = theta[0] + w.gpart[(size_t)grad_slots(m) * g.chunks * w.Bpad - 1];
    for (int b = 0; b < w.B; ++b) {
      const bool ok = w.rows[b].valid != 0;
      out[b] = ok ? w.rows[b].A + d0 : -INFINITY;
      for (int k = 0; k < m.P; ++k) grad[(size_t)b * m.P + k] = ok ? (double)(k + 1) : NAN;
    }
  });
}

}  // namespace fgl
