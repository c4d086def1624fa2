// Launch planning: host-side shape arithmetic of the kernels in
// fgl_kernels.hip (the LDS a tile stages, the reduction groups and channel
// chunks of a launch, the workgroup ranges of a launch shared by several
// models, the gradient kernel's chunking).  No device code: the library
// compiles it with hipcc, and the sanitizer build of the host code on the
// CPU compiles the same file with g++.
#include "fgl_internal.h"

#include <algorithm>

namespace fgl {

int cols_per_wave(Kind k) { return k == kFP64 ? 16 : (k == kThin ? 64 : 32); }

int max_lds_bytes() { return 160 * 1024; }

int lds_bytes(Kind k, const DevModel& m, const Tile& t) {
  const int d = t.fc * m.TT * 32 * 8;
  switch (k) {
    case kMixed:
      if (m.proj)
        return t.fc * (kProjDigits * m.KC * m.RT * 1024 + m.RT * 32 * 8) +
               (kTabSize + 2 * kFracSize) * 8;
      return t.fc * 4 * m.KC * m.TT * 1024 + d + (kTabSize + 2 * kFracSize) * 8;
    case kFP32:
      if (m.pplain) return t.fc * (m.NP2 * m.RT * 64 * 4 + m.RT * 32 * 8);
      return t.fc * m.NP2 * m.TT * 64 * 4 + d;
    case kThin: return 512 + t.fc * m.T * m.NT * 4 + d;
    default:
      if (m.pplain) return 512 + t.fc * (m.NQ * m.RT16 * 64 * 8 + m.RT16 * 16 * 8);
      return 512 + t.fc * m.NQ * m.TT16 * 64 * 4 + d;
  }
}

int n_chunks(const DevModel& m, const Tile& t) { return (m.F + t.fc - 1) / t.fc; }

// A round is one workgroup on every slot of the chip: the CUs times the
// workgroups that registers (four SIMDs of `occ` waves) and LDS let share a
// CU.  With uniform chunks the last round of a launch can be nearly empty
// (at N32 F301 B16384, eight-channel chunks make 9.5 rounds of 256
// workgroups).  Whole rounds of large chunks followed by half-size chunks
// cut the busiest CU's channels from ceil(rounds) * fc toward the mean
// (there from 80 to 76, against 75.25).
Chunks chunk_plan(Kind k, const DevModel& m, const Tile& t, int nb) {
  const int nc = n_chunks(m, t);
  const Chunks even{t.fc, t.fc, nc, nc};
  if (k != kMixed || nb < 1) return even;
  const int fs = std::max(t.group, t.fc / 2 / t.group * t.group);
  if (fs >= t.fc) return even;
  const int per_cu = std::max(1, std::min(4 * t.occ / t.waves,
                                          max_lds_bytes() / lds_bytes(k, m, t)));
  const long slots = (long)kCUs * per_cu;
  const long rounds = (long)nb * (m.F / t.fc) / slots;
  if (rounds == 0) return even;
  const int nbig = (int)(rounds * slots / nb);
  const int nsmall = (m.F - nbig * t.fc + fs - 1) / fs;
  auto up = [&](long wg) { return (wg + slots - 1) / slots; };
  const long now = up((long)nb * nc) * t.fc;
  const long split = up((long)nb * nbig) * t.fc + up((long)nb * nsmall) * fs;
  // only where it cuts the busiest CU's share by 2% or more; and the block
  // map needs at least one small chunk per XCD
  if (nbig < 1 || 50 * (now - split) < now || (long)nb * nsmall < 8) return even;
  return Chunks{t.fc, fs, nbig, nbig + nsmall};
}

int n_groups(const DevModel& m, const Tile& t) {
  return (m.F + t.group - 1) / t.group;
}

uint64_t variant_of(Kind k, const DevModel& m, const Tile& t) {
  if (m.NA != 0) return 0;
  if (k == kMixed) {
    if (t.waves != 8 || m.KC > 2 || (t.occ == 3 && !(m.proj && m.KC == 1))) return 0;
    return 1ull | (uint64_t)m.KC << 8 | (uint64_t)m.proj << 12 | (uint64_t)t.occ << 16;
  }
  if (k == kThin) return 2ull | (uint64_t)m.NT << 8 | (uint64_t)t.waves << 16;
  return 0;
}

void plan_groups(Kind k, const Tile& tile, GroupDesc* h, int n, int grid[3], int* lds) {
  const int cols = cols_per_wave(k) * tile.waves;
  int main = 0, prep = 0, fin = 0, l = 0;
  for (int j = 0; j < n; ++j) {
    GroupDesc& g = h[j];
    const Tile tj{tile.waves, g.fc, g.G, tile.occ};
    g.nb = g.w.Bpad / cols;
    g.nc = n_chunks(g.m, tj);
    main = (main + 7) & ~7;
    g.start[0] = main;
    main += g.nb * g.nc;
    g.start[1] = prep;
    prep += (g.w.Bpad + kPrepRows - 1) / kPrepRows;
    g.start[2] = fin;
    fin += (g.w.B * 16 + 255) / 256;
    l = std::max(l, lds_bytes(k, g.m, tj));
  }
  grid[0] = main;
  grid[1] = prep;
  grid[2] = fin;
  *lds = l;
}

// 4-wave workgroups (64 rows); chunks of kGradChunk channels, fixed per
// model so that a row's sums do not depend on the batch it came in; as many
// channels staged at once as fit in 40 KB (at least one; measured faster than
// 24 KB or 64 KB at the headline shape, for the workgroups it lets share a CU).
constexpr int kGradChunk = 16;

GradShape grad_shape(const DevModel& m, int Bpad) {
  GradShape g;
  g.nb = Bpad / 64;
  const int per_ch = m.proj ? m.NQ * m.RT16 * 64 * 8 + m.RT16 * 16 * 8
                           : m.NQ * m.TT16 * 64 * 4 + m.TT * 32 * 8;
  g.per = std::min(m.F, kGradChunk);
  g.chunks = (m.F + g.per - 1) / g.per;
  // stages of <= 40 KB with the power table (four workgroups per CU)
  g.fs = std::max(1, std::min(g.per, (40 * 1024 - 512) / per_ch));
  g.lds = 512 + g.fs * per_ch;
  return g;
}

}  // namespace fgl
