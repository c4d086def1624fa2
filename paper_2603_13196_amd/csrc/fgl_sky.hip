// Region construction and chromatic response functions (Tutt et al.,
// Sec. 4 and Eq. chromatic_function) on an equirectangular sky.
//
// Pixels are rings (declination) x columns (right ascension), with solid
// angle omega[ring] (divided by 4 pi).  Sky-frame maps: t_ex = T_base -
// T_CMB and the spectral index beta.  Antenna-frame maps (declination x hour
// angle): the beam D(nu) and the horizon H.  At LST step t the sky pixel
// (ring, ra) sits at the antenna pixel (ring, (ra - s_t) mod nlon).
//
// Every quantity here is a cyclic correlation along the columns of each
// ring, summed over rings:
//   Z(nu, t)  = sum_q omega a(q, nu) b(nu, p_t(q))        (normalisers)
//   I(q)      = sum_{nu, t} omega a(q, nu) b(nu, p_t(q)) / Z(nu, t)
//   K_j(nu, t) = sum_{q in region j} omega t_ex(q) D(nu, p_t(q))
// with a = T_sky (Eq. skyapproximation) or 1 and b = D H or H by scheme.
// k_sky_corr computes Z: one workgroup per (block of four channels, chunk of
// four rings), two lanes per time step, the ring's b window and weights
// staged in LDS.  k_sky_k
// computes K: four channels per workgroup and a balanced run of rings of
// one group of regions (details at the kernel).  Every sum has a fixed
// order.  k_sky_importance computes I: one thread per pixel, looping over
// blocks of four channels with the ring's b row and 1/Z(nu, .) of the block
// in LDS.  The partition
// (Algs. method1 and method2) is a short sequential computation on the
// host.
#include "fgl_host.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <vector>

namespace fgl {

namespace {

constexpr int kRingChunk = 4;          // rings per k_sky_corr workgroup (more workgroups: measured faster than 8 or 32)

struct SkyDev {
  int nlat, nlon, F;
  double t_cmb;
  const double* omega;   // [nlat]
  const double* t_ex;    // [nlat][nlon]
  const double* beta;    // [nlat][nlon]
  const float* beam;     // [F][nlat][nlon]
  const uint8_t* hor;    // [nlat][nlon]
  const double* lr;      // [F] log2(nu / nu0)
  const float4* beam4;   // [ceil(F / 4)][nlat][nlon]: channels 4 b .. 4 b + 3 of a
                         // pixel side by side (zero past the last channel)
};

enum Corr { kCorrBeam = 1, kCorrSky = 2, kCorrHorizon = 3 };

// weight a(q, nu) of a sky pixel, omega included
template <int MODE>
__device__ inline double aval(const SkyDev& s, int f, int ring, int ra) {
  const size_t px = (size_t)ring * s.nlon + ra;
  if constexpr (MODE == kCorrHorizon) return s.omega[ring];
  // Eq. skyapproximation
  return s.omega[ring] * fma(s.t_ex[px], exp2(-s.beta[px] * s.lr[f]), s.t_cmb);
}

// b(nu, ring, ha) of the four channels 4 fb .. 4 fb + 3 for a weighting (zero
// past the last channel)
template <int MODE>
__device__ inline float4 bval4(const SkyDev& s, int fb, int ring, int ha) {
  const size_t px = (size_t)ring * s.nlon + ha;
  if (!s.hor[px]) return make_float4(0.f, 0.f, 0.f, 0.f);
  if constexpr (MODE == kCorrBeam) return s.beam4[((size_t)fb * s.nlat) * s.nlon + px];
  return make_float4(1.f, 1.f, 1.f, 1.f);
}

// The normalisers: partial[(chunk * F + f) * T + t] = the sum over the
// chunk's rings of sum_ra a(ra) b(ra - s_t), for four channels per workgroup
// and two lanes per time step (lane 2t + h: channels 2h and 2h + 1 of the
// block at step t0 + t), so that T = 96 steps fill three waves.  Per ring the
// block's b values sit in LDS as a window of four-channel columns (entry e
// holds column (e + nlon - smax) mod nlon, so column ra at step t is entry
// ra + smax - s_t with no wrap test, and a lane reads its two channels with
// one 8-byte gather), beside the weights of the four channels (zero-padded
// to Lz columns, a multiple of eight).  A lane keeps eight partial sums per
// channel over the columns ra = u mod 8 and adds them in a fixed tree after
// each ring.
template <int MODE>
__global__ __launch_bounds__(256) void k_sky_corr(SkyDev s, const int* __restrict__ shifts,
                                                  int T, int t0, int smax, int Lz,
                                                  double* __restrict__ partial) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int fb = blockIdx.x, f0 = 4 * fb, chunk = blockIdx.y;
  const int nlon = s.nlon, nwin = nlon + smax + 8, wbase = nlon - smax;
  double* s_a = reinterpret_cast<double*>(smem);                    // [Lz][4]
  float4* s_b = reinterpret_cast<float4*>(s_a + 4 * (size_t)Lz);   // [nwin]
  const int tl = threadIdx.x, tb = blockDim.x;
  const int h = tl & 1, t = t0 + (tl >> 1);
  const bool live = t < T;
  const unsigned char* bo = reinterpret_cast<const unsigned char*>(s_b) +
                            (smax - (live ? shifts[t] : 0)) * 16 + 8 * h;
  const double* ao = s_a + 2 * h;
  double acc0 = 0.0, acc1 = 0.0;
  const int r0 = chunk * kRingChunk, r1 = min(s.nlat, r0 + kRingChunk);
  for (int ring = r0; ring < r1; ++ring) {
    __syncthreads();
    for (int e = tl; e < nwin; e += tb) {
      const int c = (e + wbase) % nlon;
      s_b[e] = bval4<MODE>(s, fb, ring, c);
    }
    for (int k = tl; k < 4 * Lz; k += tb) {
      const int q = k >> 2, f = f0 + (k & 3);
      s_a[k] = q < nlon && f < s.F ? aval<MODE>(s, f, ring, q) : 0.0;
    }
    __syncthreads();
    if (!live) continue;
    double c0[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double c1[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < Lz; k += 8) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const float2 b = *reinterpret_cast<const float2*>(bo + (size_t)(k + u) * 16);
        const double2 a = *reinterpret_cast<const double2*>(ao + (size_t)(k + u) * 4);
        c0[u] = fma(a.x, (double)b.x, c0[u]);
        c1[u] = fma(a.y, (double)b.y, c1[u]);
      }
    }
    acc0 += ((c0[0] + c0[1]) + (c0[2] + c0[3])) + ((c0[4] + c0[5]) + (c0[6] + c0[7]));
    acc1 += ((c1[0] + c1[1]) + (c1[2] + c1[3])) + ((c1[4] + c1[5]) + (c1[6] + c1[7]));
  }
  if (!live) return;
  const int f = f0 + 2 * h;
  if (f < s.F) partial[((size_t)chunk * s.F + f) * T + t] = acc0;
  if (f + 1 < s.F) partial[((size_t)chunk * s.F + f + 1) * T + t] = acc1;
}

// K of up to kRegionsPerGroup regions for four channels: one workgroup per
// (channel block, work item), two lanes per time step, each taking two of
// the four channels (lane 2t + h: channels 2h and 2h + 1 at step t0 + t).
// A work item is a region group and a run of consecutive rings whose
// estimated cost (the group's pixels, plus a fixed cost per ring for the
// staging and the barrier) is about that of every other item: the partition
// makes regions of very different sizes, so fixed ring chunks would leave the
// workgroups of the largest regions running alone at the end.
//
// Per ring the block's beam rows sit in LDS as the interleaved device copy
// holds them, four channels of a column side by side, over the window of the
// doubled row (as above) that the steps' shifts reach, so a lane reads its
// two channels of a pixel with one 8-byte gather;
// the group's columns (stored as byte offsets) and weights omega t_ex sit
// beside them and are read with same-address loads.  All of it is
// double-buffered: the next ring is read from global memory into registers
// before the current ring's sums and written to the other buffers after
// them, one barrier per ring.  Each (region, channel) sum stays in a
// register across the item's rings, pixels in the ring's region order,
// rings in order.  Region runs are padded to a multiple of four with
// weight-zero entries.
constexpr int kRegionsPerGroup = 8;     // regions per workgroup of the K kernels
constexpr int kSkyPrefetchCols = 4;     // beam columns a thread prefetches per ring
constexpr int kSkyPrefetchIds = 4;      // columns (and weights) a thread prefetches per ring

__global__ __launch_bounds__(256) void k_sky_k(SkyDev s, const int* __restrict__ shifts, int T,
                                               int t0, int smax, const int* __restrict__ order,
                                               const double* __restrict__ asort,
                                               const int* __restrict__ seg, int NJ, int L,
                                               int Lg, const int4* __restrict__ items,
                                               double* __restrict__ partial) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int fb = blockIdx.x, f0 = 4 * fb, item = blockIdx.y;
  const int4 it = items[item];                       // (region group, first ring, end ring)
  const int j0 = it.x * kRegionsPerGroup, nj = min(kRegionsPerGroup, NJ - j0);
  const int nlon = s.nlon;
  // the window of the doubled row that some step reads: entries
  // nlon - smax .. 2 nlon - 1 (entry e holds column e mod nlon)
  const int nwin = nlon + smax, wbase = nlon - smax;
  double* s_w = reinterpret_cast<double*>(smem);                 // [2][Lg]
  int* s_id = reinterpret_cast<int*>(s_w + 2 * (size_t)Lg);      // [2][Lg] byte offsets
  float4* s_b = reinterpret_cast<float4*>(s_id + 2 * (size_t)Lg);  // [2][nwin]
  // the two lanes of a step are neighbours, so a wave's gathers read whole
  // 16-byte column entries side by side (no bank conflicts)
  const int tl = threadIdx.x, tb = blockDim.x;
  const int h = tl & 1, t = t0 + (tl >> 1);
  const bool live = t < T;
  // byte offset of this lane's channel pair in window entry smax - s_t
  const int o = (smax - (live ? shifts[t] : 0)) * 16 + 8 * h;
  const int r0 = it.y, r1 = it.z;
  const float4* b4 = s.beam4 + (size_t)fb * s.nlat * nlon;
  // window entry q of `ring` (column (wbase + q) mod nlon)
  auto col_of = [&](int q) { const int e = wbase + q; return e < nlon ? e : e - nlon; };
  auto slice = [&](int ring, int& first, int& len) {   // the group's part of the ring's list
    const int* sg = seg + (size_t)ring * (NJ + 1);
    first = sg[j0];
    len = sg[j0 + nj] - first;
  };
  {
    int kb, kl;
    slice(r0, kb, kl);
    for (int q = tl; q < nwin; q += tb) s_b[q] = b4[(size_t)r0 * nlon + col_of(q)];
    for (int k = tl; k < kl; k += tb) {
      s_id[k] = order[(size_t)r0 * L + kb + k] * 16;
      s_w[k] = asort[(size_t)r0 * L + kb + k];
    }
  }
  __syncthreads();
  double acc[kRegionsPerGroup][2];
#pragma unroll
  for (int j = 0; j < kRegionsPerGroup; ++j) acc[j][0] = acc[j][1] = 0.0;
  for (int ring = r0; ring < r1; ++ring) {
    const int cur = (ring - r0) & 1;
    const bool next = ring + 1 < r1;
    // the next ring's first window entries and slice entries, into
    // registers now and into the other buffers after this ring's sums
    int nb = 0, nl = 0;
    if (next) slice(ring + 1, nb, nl);
    float4 pf[kSkyPrefetchCols];
    int pi[kSkyPrefetchIds];
    double pw[kSkyPrefetchIds];
#pragma unroll
    for (int i = 0; i < kSkyPrefetchCols; ++i) {
      const int q = tl + i * tb;
      pf[i] = next && q < nwin ? b4[(size_t)(ring + 1) * nlon + col_of(q)]
                               : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int i = 0; i < kSkyPrefetchIds; ++i) {
      const int k = tl + i * tb;
      const bool in = k < nl;
      pi[i] = in ? order[(size_t)(ring + 1) * L + nb + k] * 16 : 0;
      pw[i] = in ? asort[(size_t)(ring + 1) * L + nb + k] : 0.0;
    }
    if (live) {
      const unsigned char* bo =
          reinterpret_cast<const unsigned char*>(s_b + (size_t)cur * nwin) + o;
      const int* li = s_id + (size_t)cur * Lg;
      const double* lw = s_w + (size_t)cur * Lg;
      int kb, kl;
      slice(ring, kb, kl);
      const int* sg = seg + (size_t)ring * (NJ + 1) + j0;
#pragma unroll
      for (int j = 0; j < kRegionsPerGroup; ++j) {
        if (j >= nj) break;
        const int k1 = sg[j + 1] - kb;
        int k = sg[j] - kb;
        if (k >= k1) continue;
        // software pipelined over groups of four pixels: the next group's
        // gathers and the columns and weights of the one after are in flight
        // while this group's FMAs run (LDS returns in order, so waiting for
        // this group's gathers never waits for the later reads)
        auto gather = [&](const int4 id, float2 (&b)[4]) {
          b[0] = *reinterpret_cast<const float2*>(bo + id.x);
          b[1] = *reinterpret_cast<const float2*>(bo + id.y);
          b[2] = *reinterpret_cast<const float2*>(bo + id.z);
          b[3] = *reinterpret_cast<const float2*>(bo + id.w);
        };
        int4 id = *reinterpret_cast<const int4*>(li + k);
        double2 wa = *reinterpret_cast<const double2*>(lw + k);
        double2 wb = *reinterpret_cast<const double2*>(lw + k + 2);
        float2 b[4];
        gather(id, b);
        int kn = k + 4 < k1 ? k + 4 : k;
        int4 idn = *reinterpret_cast<const int4*>(li + kn);
        double2 wan = *reinterpret_cast<const double2*>(lw + kn);
        double2 wbn = *reinterpret_cast<const double2*>(lw + kn + 2);
#pragma unroll 2
        for (; k < k1; k += 4) {
          float2 bn[4];
          gather(idn, bn);
          const int kq = kn + 4 < k1 ? kn + 4 : kn;
          const int4 idq = *reinterpret_cast<const int4*>(li + kq);
          const double2 waq = *reinterpret_cast<const double2*>(lw + kq);
          const double2 wbq = *reinterpret_cast<const double2*>(lw + kq + 2);
          acc[j][0] = fma(wa.x, (double)b[0].x, acc[j][0]);
          acc[j][1] = fma(wa.x, (double)b[0].y, acc[j][1]);
          acc[j][0] = fma(wa.y, (double)b[1].x, acc[j][0]);
          acc[j][1] = fma(wa.y, (double)b[1].y, acc[j][1]);
          acc[j][0] = fma(wb.x, (double)b[2].x, acc[j][0]);
          acc[j][1] = fma(wb.x, (double)b[2].y, acc[j][1]);
          acc[j][0] = fma(wb.y, (double)b[3].x, acc[j][0]);
          acc[j][1] = fma(wb.y, (double)b[3].y, acc[j][1]);
#pragma unroll
          for (int u = 0; u < 4; ++u) b[u] = bn[u];
          wa = wan;
          wb = wbn;
          idn = idq;
          wan = waq;
          wbn = wbq;
          kn = kq;
        }
      }
    }
    if (next) {
      const int nxt = cur ^ 1;
      float4* dst = s_b + (size_t)nxt * nwin;
#pragma unroll
      for (int i = 0; i < kSkyPrefetchCols; ++i) {
        const int q = tl + i * tb;
        if (q < nwin) dst[q] = pf[i];
      }
#pragma unroll
      for (int i = 0; i < kSkyPrefetchIds; ++i) {
        const int k = tl + i * tb;
        if (k < nl) {
          s_id[(size_t)nxt * Lg + k] = pi[i];
          s_w[(size_t)nxt * Lg + k] = pw[i];
        }
      }
      // what the registers did not hold (wide rings, long slices)
      for (int q = tl + kSkyPrefetchCols * tb; q < nwin; q += tb)
        dst[q] = b4[(size_t)(ring + 1) * nlon + col_of(q)];
      for (int k = tl + kSkyPrefetchIds * tb; k < nl; k += tb) {
        s_id[(size_t)nxt * Lg + k] = order[(size_t)(ring + 1) * L + nb + k] * 16;
        s_w[(size_t)nxt * Lg + k] = asort[(size_t)(ring + 1) * L + nb + k];
      }
    }
    __syncthreads();
  }
  if (!live) return;
#pragma unroll
  for (int j = 0; j < kRegionsPerGroup; ++j)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int f = f0 + 2 * h + c;
      if (j < nj && f < s.F)
        partial[(((size_t)item * kRegionsPerGroup + j) * s.F + f) * T + t] = acc[j][c];
    }
}

// The interleaved beam copy: out[b][p] = (beam[4 b][p] .. beam[4 b + 3][p]),
// zero past the last channel, for np pixels per channel.
__global__ __launch_bounds__(256) void k_beam_interleave(const float* __restrict__ beam, int F,
                                                         size_t np, size_t n,
                                                         float4* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const size_t b = i / np, p = i - b * np;
  float v[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const size_t f = 4 * b + c;
    v[c] = f < (size_t)F ? beam[f * np + p] : 0.0f;
  }
  out[i] = make_float4(v[0], v[1], v[2], v[3]);
}

// K[j][f][t] = sum over the work items of j's region group, in order, of the
// items' partial sums (first[g] .. first[g + 1] - 1 are group g's items).
__global__ __launch_bounds__(256) void k_sky_k_reduce(const double* __restrict__ partial,
                                                      const int* __restrict__ first, int NJ,
                                                      int F, int T, double* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t ft = (size_t)F * T;
  if (i >= (size_t)NJ * ft) return;
  const int j = (int)(i / ft);
  const size_t rest = i - (size_t)j * ft;
  const int g = j / kRegionsPerGroup, jj = j - g * kRegionsPerGroup;
  double acc = 0.0;
  for (int y = first[g]; y < first[g + 1]; ++y)
    acc += partial[((size_t)y * kRegionsPerGroup + jj) * ft + rest];
  out[i] = acc;
}

// out[i] = sum over chunks (in order) of partial[chunk * n + i]
__global__ __launch_bounds__(256) void k_sky_reduce(const double* __restrict__ partial,
                                                    int chunks, size_t n,
                                                    double* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int c = 0; c < chunks; ++c) acc += partial[(size_t)c * n + i];
  out[i] = acc;
}

// I(ring, ra) = sum_nu a(q, nu) sum_t b(nu, ring, ra - s_t) / Z(nu, t): one
// workgroup per (ring, chunk of four-channel blocks), one thread per column,
// four channels at a time.  Per block the b row (the four channels of a
// column side by side, the interleaved beam copy times the horizon, staged
// twice in a row so that column ra at step t is entry ra + nlon - s_t) and
// 1/Z of the four channels at every step sit in LDS: a thread gathers the
// four channels of a column with one 16-byte read per step and reads 1/Z
// with two same-address reads.  Per channel the sum over steps alternates
// two partial sums (even and odd t); their sum times a(q, nu) is added to
// the column's total in channel order.  The chunk's total is written to
// imp[(chunk * nlat + ring) * nlon + ra].
template <int MODE>
__global__ __launch_bounds__(256) void k_sky_importance(SkyDev s, const int* __restrict__ shifts,
                                                        int T, const double* __restrict__ Z,
                                                        int bper, double* __restrict__ imp) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int ring = blockIdx.x, chunk = blockIdx.y;
  const int nlon = s.nlon;
  double* s_iz = reinterpret_cast<double*>(smem);                  // [T][4]
  float4* s_b = reinterpret_cast<float4*>(s_iz + 4 * (size_t)T);   // [2 nlon]
  int* s_o = reinterpret_cast<int*>(s_b + 2 * (size_t)nlon);       // [T] nlon - s_t
  for (int t = threadIdx.x; t < T; t += blockDim.x) s_o[t] = nlon - shifts[t];
  const int nb = (s.F + 3) / 4;
  const int b0 = chunk * bper, b1 = min(nb, b0 + bper);
  for (int ra0 = 0; ra0 < nlon; ra0 += blockDim.x) {
    const int ra = ra0 + threadIdx.x;
    double total = 0.0;
    for (int fb = b0; fb < b1; ++fb) {
      __syncthreads();
      for (int k = threadIdx.x; k < 4 * T; k += blockDim.x) {
        const int f = 4 * fb + (k & 3);
        s_iz[k] = f < s.F ? 1.0 / Z[(size_t)f * T + (k >> 2)] : 0.0;
      }
      for (int k = threadIdx.x; k < nlon; k += blockDim.x) {
        const float4 v = bval4<MODE>(s, fb, ring, k);
        s_b[k] = v;
        s_b[k + nlon] = v;
      }
      __syncthreads();
      if (ra < nlon) {
        double ce[4] = {0.0, 0.0, 0.0, 0.0}, co[4] = {0.0, 0.0, 0.0, 0.0};
        const double2* iz = reinterpret_cast<const double2*>(s_iz);
        int t = 0;
        for (; t + 2 <= T; t += 2) {
          const float4 v0 = s_b[ra + s_o[t]];
          const float4 v1 = s_b[ra + s_o[t + 1]];
          const double2 a0 = iz[2 * t], a1 = iz[2 * t + 1];
          const double2 b0v = iz[2 * t + 2], b1v = iz[2 * t + 3];
          ce[0] = fma((double)v0.x, a0.x, ce[0]);
          ce[1] = fma((double)v0.y, a0.y, ce[1]);
          ce[2] = fma((double)v0.z, a1.x, ce[2]);
          ce[3] = fma((double)v0.w, a1.y, ce[3]);
          co[0] = fma((double)v1.x, b0v.x, co[0]);
          co[1] = fma((double)v1.y, b0v.y, co[1]);
          co[2] = fma((double)v1.z, b1v.x, co[2]);
          co[3] = fma((double)v1.w, b1v.y, co[3]);
        }
        if (t < T) {
          const float4 v0 = s_b[ra + s_o[t]];
          const double2 a0 = iz[2 * t], a1 = iz[2 * t + 1];
          ce[0] = fma((double)v0.x, a0.x, ce[0]);
          ce[1] = fma((double)v0.y, a0.y, ce[1]);
          ce[2] = fma((double)v0.z, a1.x, ce[2]);
          ce[3] = fma((double)v0.w, a1.y, ce[3]);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int f = 4 * fb + c;
          if (f < s.F) total = fma(aval<MODE>(s, f, ring, ra), ce[c] + co[c], total);
        }
      }
    }
    if (ra < nlon) imp[((size_t)chunk * s.nlat + ring) * nlon + ra] = total;
  }
}

// LDS of a k_sky_corr workgroup: the four channels' weights (Lz columns) and
// the window of nlon + smax + 8 four-channel b columns.
size_t corr_lds(int nlon, int smax, int Lz) {
  return (size_t)Lz * 32 + ((size_t)nlon + smax + 8) * 16;
}

int pad8(int n) { return (n + 7) / 8 * 8; }
int pad4(int n) { return (n + 3) / 4 * 4; }


struct Sky {
  int dev = 0;
  SkyDev d{};
  double nu0 = 0.0;
  hipStream_t stream = nullptr;
  std::vector<double> h_beta;      // for the masks of a partition
  std::vector<double> h_omega, h_tex;   // for the region-sorted pixel weights
  double last_ms = 0.0;            // last k_sky_corr duration (chromatic)
};

template <typename KernelT>
hipError_t set_lds(KernelT k) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

// Z partial sums and their chunk reduction into out (device, [F][T]).
template <int MODE>
int run_corr(Sky* sk, const int* d_shifts, int T, int smax, int Lz, double* d_out) {
  const SkyDev& d = sk->d;
  const int chunks = (d.nlat + kRingChunk - 1) / kRingChunk;
  const size_t n = (size_t)d.F * T;
  double* part = nullptr;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&part), n * chunks * 8);
  if (e != hipSuccess) return hip_err(e, "allocating partial sums");
  // two lanes per step: up to 128 steps per launch in up to 256 lanes
  const int tb = std::min(256, (2 * T + 63) / 64 * 64), TS = tb / 2;
  const size_t lds = corr_lds(d.nlon, smax, Lz);
  if ((e = set_lds(k_sky_corr<MODE>)) == hipSuccess) {
    for (int t0 = 0; t0 < T && e == hipSuccess; t0 += TS) {
      hipLaunchKernelGGL(k_sky_corr<MODE>, dim3((d.F + 3) / 4, chunks), dim3(tb), lds,
                         sk->stream, d, d_shifts, T, t0, smax, Lz, part);
      e = hipGetLastError();
    }
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_sky_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, sk->stream,
                       part, chunks, n, d_out);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(sk->stream);
  (void)hipFree(part);
  return e == hipSuccess ? FGL_OK : hip_err(e, "normaliser kernels");
}

// LDS of a k_sky_k workgroup: two buffers of the row window (nlon + smax
// four-channel columns) and of Lg columns and weights.
size_t k_lds(int nlon, int smax, int Lg) {
  return (size_t)32 * (nlon + smax) + (size_t)24 * Lg;
}

// K by k_sky_k over the work items (device int4 [n_items]: region group,
// first ring, end ring; group g's items are first[g] .. first[g + 1] - 1,
// device int [groups + 1]) and their reduction into d_out (device).
int run_k(Sky* sk, const int* d_shifts, int T, int smax, const int* d_order,
          const double* d_asort, const int* d_seg, int NJ, int L, int Lg, const int4* d_items,
          int n_items, const int* d_first, double* d_out, float* ms) {
  const SkyDev& d = sk->d;
  if (k_lds(d.nlon, smax, Lg) > 160 * 1024)
    return set_err(FGL_EINVAL, "nlon=%d does not fit one workgroup's LDS", d.nlon);
  // two lanes per step: T steps per launch in up to 256 lanes
  const int tb = std::min(256, (2 * T + 63) / 64 * 64), TS = tb / 2;  const size_t ft = (size_t)d.F * T;
  double* part = nullptr;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&part),
                           (size_t)n_items * kRegionsPerGroup * ft * 8);
  if (e != hipSuccess) return hip_err(e, "allocating partial sums");
  const size_t lds = k_lds(d.nlon, smax, Lg);
  const dim3 grid((d.F + 3) / 4, n_items);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ms) {
    // timing only: no system-scope fence around the kernel
    (void)hipEventCreateWithFlags(&e0, hipEventDisableSystemFence);
    (void)hipEventCreateWithFlags(&e1, hipEventDisableSystemFence);
    (void)hipEventRecord(e0, sk->stream);
  }
  e = set_lds(k_sky_k);
  for (int t0 = 0; t0 < T && e == hipSuccess; t0 += TS) {
    hipLaunchKernelGGL(k_sky_k, grid, dim3(tb), lds, sk->stream, d, d_shifts, T, t0, smax,
                       d_order, d_asort, d_seg, NJ, L, Lg, d_items, part);
    e = hipGetLastError();
  }
  if (ms && e == hipSuccess) (void)hipEventRecord(e1, sk->stream);
  if (e == hipSuccess) {
    const size_t n = (size_t)NJ * ft;
    hipLaunchKernelGGL(k_sky_k_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       sk->stream, part, d_first, NJ, d.F, T, d_out);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(sk->stream);
  if (ms && e == hipSuccess) (void)hipEventElapsedTime(ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(part);
  return e == hipSuccess ? FGL_OK : hip_err(e, "K kernels");
}

// Work items of the K kernel: each region group's rings cut into runs of
// about the same estimated cost, a ring costing its padded pixels of the
// group plus kRingCost (at least one ring per item).  Measured on the
// 256 x 512 benchmark sky (32 regions, 301 channels, 96 steps): 128 items
// beat 32 and 64 by 10 % and 4 %; a per-ring cost of 64, 256 or 1024 pixels
// changed nothing or made it slower.
constexpr int kRingCost = 0;            // pixels' worth of one ring's staging and barrier
constexpr int kItems = 128;             // work items aimed at per call
void k_items(const std::vector<int>& seg, int nlat, int NJ, std::vector<int4>& items,
             std::vector<int>& first) {
  const int groups = (NJ + kRegionsPerGroup - 1) / kRegionsPerGroup;
  auto px = [&](int g, int r) {
    const int* sg = &seg[(size_t)r * (NJ + 1)];
    return sg[std::min(NJ, (g + 1) * kRegionsPerGroup)] - sg[g * kRegionsPerGroup] + kRingCost;
  };
  long total = 0;
  for (int g = 0; g < groups; ++g)
    for (int r = 0; r < nlat; ++r) total += px(g, r);
  // about kItems items in all, each costing at least 512
  const long target = std::max<long>(512, (total + kItems - 1) / kItems);
  items.clear();
  first.assign(groups + 1, 0);
  for (int g = 0; g < groups; ++g) {
    first[g] = (int)items.size();
    int r0 = 0;
    long acc = 0;
    for (int r = 0; r < nlat; ++r) {
      acc += px(g, r);
      if (acc >= target || r == nlat - 1) {
        items.push_back(make_int4(g, r0, r + 1, 0));
        r0 = r + 1;
        acc = 0;
      }
    }
  }
  first[groups] = (int)items.size();
}

int check_shifts(const Sky* sk, const int32_t* shifts, int T) {
  if (!shifts || T < 1) return set_err(FGL_EINVAL, "need T >= 1 shifts");
  for (int t = 0; t < T; ++t)
    if (shifts[t] < 0 || shifts[t] >= sk->d.nlon)
      return set_err(FGL_EINVAL, "shifts[%d]=%d outside 0..%d", t, shifts[t], sk->d.nlon - 1);
  return FGL_OK;
}

// device buffer holding a host array
template <typename T>
int to_device(T** dst, const T* src, size_t count, const char* what) {
  hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), std::max<size_t>(count * sizeof(T), 16));
  if (e == hipSuccess && count) e = hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (*dst) (void)hipFree(*dst);
    *dst = nullptr;
    return hip_err(e, what);
  }
  return FGL_OK;
}

void free_sky(Sky* sk) {
  const void* ps[] = {sk->d.omega, sk->d.t_ex, sk->d.beta, sk->d.beam, sk->d.hor, sk->d.lr,
                      sk->d.beam4};
  for (const void* p : ps)
    if (p) (void)hipFree(const_cast<void*>(p));
  if (sk->stream) (void)hipStreamDestroy(sk->stream);
  delete sk;
}

}  // namespace

// Algs. method1 and method2 on the importance-weighted CDF (host).
int partition_host(const double* beta, const double* weight, int n, int n_regions, int method,
                   double* edges) {
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return beta[a] < beta[b]; });
  std::vector<double> xs(n), cs(n);
  double run = 0.0;
  for (int k = 0; k < n; ++k) {
    xs[k] = beta[order[k]];
    run += weight[order[k]];
    cs[k] = run;
  }
  const double total = cs[n - 1];
  if (!(total > 0.0)) return set_err(FGL_EINVAL, "the weights sum to zero");
  for (int k = 0; k < n; ++k) cs[k] = cs[k] / total;
  auto cdf_at = [&](double x) {
    const int k = (int)(std::upper_bound(xs.begin(), xs.end(), x) - xs.begin());
    return k == 0 ? 0.0 : cs[k - 1];
  };
  auto cdf_inv = [&](double c) {
    const int k = (int)(std::lower_bound(cs.begin(), cs.end(), c) - cs.begin());
    return xs[std::min(k, n - 1)];
  };
  std::vector<double> e;
  if (method == FGL_PARTITION_HIERARCHICAL) {
    int base = 1;
    while (base * 2 <= n_regions) base *= 2;
    e.push_back(xs[0]);
    for (int k = 1; k < base; ++k) e.push_back(cdf_inv((double)k / (double)base));
    e.push_back(xs[n - 1]);
    for (int r = base; r < n_regions; ++r) {
      int j = 0;
      double best = e[1] - e[0];
      for (int i = 1; i + 1 < (int)e.size(); ++i)
        if (e[i + 1] - e[i] > best) {
          best = e[i + 1] - e[i];
          j = i;
        }
      const double cm = 0.5 * (cdf_at(e[j]) + cdf_at(e[j + 1]));
      e.insert(e.begin() + j + 1, cdf_inv(cm));
    }
  } else {
    e = {xs[0], xs[n - 1]};
    while ((int)e.size() - 1 < n_regions) {
      const int nr = (int)e.size() - 1;
      int j = 0;
      double best = -1.0;
      for (int i = 0; i < nr; ++i) {
        const bool last = i == nr - 1;
        const int lo = (int)(std::lower_bound(xs.begin(), xs.end(), e[i]) - xs.begin());
        const int hi = last ? (int)(std::upper_bound(xs.begin(), xs.end(), e[i + 1]) - xs.begin())
                            : (int)(std::lower_bound(xs.begin(), xs.end(), e[i + 1]) - xs.begin());
        const double top = hi > 0 ? cs[hi - 1] : 0.0, bottom = lo > 0 ? cs[lo - 1] : 0.0;
        const double m = top - bottom;
        if (i == 0 || m > best) {
          best = m;
          j = i;
        }
      }
      e.insert(e.begin() + j + 1, 0.5 * (e[j] + e[j + 1]));
    }
  }
  std::copy(e.begin(), e.end(), edges);
  return FGL_OK;
}

}  // namespace fgl

using namespace fgl;

extern "C" {

int fgl_sky_create(int nlat, int nlon, int F, const double* omega, const double* t_ex,
                   const double* beta, const float* beam, const uint8_t* horizon,
                   const double* freqs, double nu0, double t_cmb, fgl_sky** out) {
  if (!out) return set_err(FGL_EINVAL, "out is NULL");
  *out = nullptr;
  if (nlat < 1 || nlon < 1 || F < 1) return set_err(FGL_EINVAL, "need nlat, nlon, F >= 1");
  if (!omega || !t_ex || !beta || !beam || !horizon || !freqs)
    return set_err(FGL_EINVAL, "array arguments must be non-NULL");
  if (!(nu0 > 0.0) || !std::isfinite(nu0) || !std::isfinite(t_cmb))
    return set_err(FGL_EINVAL, "nu0 must be finite and > 0, t_cmb finite");
  const size_t np = (size_t)nlat * nlon;
  for (int r = 0; r < nlat; ++r)
    if (!(omega[r] > 0.0) || !std::isfinite(omega[r])) return set_err(FGL_EINVAL, "omega[%d] must be finite and > 0", r);
  for (size_t k = 0; k < np; ++k)
    if (!std::isfinite(t_ex[k]) || !std::isfinite(beta[k]) || std::fabs(beta[k]) > 64.0)
      return set_err(FGL_EINVAL, "t_ex/beta[%zu] must be finite with |beta| <= 64", k);
  for (size_t k = 0; k < np * F; ++k)
    if (!std::isfinite(beam[k])) return set_err(FGL_EINVAL, "beam[%zu] is not finite", k);
  std::vector<double> lr(F);
  for (int f = 0; f < F; ++f) {
    if (!(freqs[f] > 0.0) || !std::isfinite(freqs[f])) return set_err(FGL_EINVAL, "freqs[%d] must be finite and > 0", f);
    lr[f] = std::log2(freqs[f] / nu0);
  }
  int dev = 0;
  int rc = check_device(&dev);
  if (rc != FGL_OK) return rc;
  Sky* sk = new (std::nothrow) Sky();
  if (!sk) return set_err(FGL_ENOMEM, "host allocation");
  sk->dev = dev;
  sk->nu0 = nu0;
  sk->d.nlat = nlat;
  sk->d.nlon = nlon;
  sk->d.F = F;
  sk->d.t_cmb = t_cmb;
  sk->h_beta.assign(beta, beta + np);
  sk->h_omega.assign(omega, omega + nlat);
  sk->h_tex.assign(t_ex, t_ex + np);
  double *om = nullptr, *tx = nullptr, *bt = nullptr, *l2 = nullptr;
  float* bm = nullptr;
  uint8_t* hz = nullptr;
  if ((rc = to_device(&om, omega, (size_t)nlat, "uploading omega")) != FGL_OK ||
      (rc = to_device(&tx, t_ex, np, "uploading t_ex")) != FGL_OK ||
      (rc = to_device(&bt, beta, np, "uploading beta")) != FGL_OK ||
      (rc = to_device(&bm, beam, np * F, "uploading the beam")) != FGL_OK ||
      (rc = to_device(&hz, horizon, np, "uploading the horizon")) != FGL_OK ||
      (rc = to_device(&l2, lr.data(), (size_t)F, "uploading frequencies")) != FGL_OK) {
    sk->d.omega = om; sk->d.t_ex = tx; sk->d.beta = bt; sk->d.beam = bm; sk->d.hor = hz; sk->d.lr = l2;
    free_sky(sk);
    return rc;
  }
  sk->d.omega = om;
  sk->d.t_ex = tx;
  sk->d.beta = bt;
  sk->d.beam = bm;
  sk->d.hor = hz;
  sk->d.lr = l2;
  hipError_t e = hipStreamCreateWithFlags(&sk->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    sk->stream = nullptr;
    free_sky(sk);
    return hip_err(e, "hipStreamCreate");
  }
  // the beam interleaved by four channels for the K kernel
  const size_t n4 = (size_t)((F + 3) / 4) * np;
  float4* b4 = nullptr;
  if ((e = hipMalloc(reinterpret_cast<void**>(&b4), n4 * sizeof(float4))) == hipSuccess) {
    sk->d.beam4 = b4;
    hipLaunchKernelGGL(k_beam_interleave, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0,
                       sk->stream, bm, F, np, n4, b4);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(sk->stream);
  }
  if (e != hipSuccess) {
    free_sky(sk);
    return hip_err(e, "interleaving the beam");
  }
  *out = reinterpret_cast<fgl_sky*>(sk);
  return FGL_OK;
}

int fgl_sky_importance(fgl_sky* sh, const int32_t* shifts, int T, int scheme, double* importance) {
  TraceRange tr("fgl_sky_importance scheme=%d T=%d", scheme, T);
  Sky* sk = reinterpret_cast<Sky*>(sh);
  if (!sk || !importance) return set_err(FGL_EINVAL, "sky and importance must be non-NULL");
  if (scheme < FGL_WEIGHT_HORIZON || scheme > FGL_WEIGHT_BEAM)
    return set_err(FGL_EINVAL, "unknown weighting scheme %d", scheme);
  int rc = check_shifts(sk, shifts, T);
  if (rc != FGL_OK) return rc;
  const int Lz = pad8(sk->d.nlon);
  const int smax = *std::max_element(shifts, shifts + T);
  if (corr_lds(sk->d.nlon, smax, Lz) > 160 * 1024)
    return set_err(FGL_EINVAL, "nlon=%d does not fit one workgroup's LDS", sk->d.nlon);
  hipError_t e = hipSetDevice(sk->dev);
  if (e != hipSuccess) return hip_err(e, "hipSetDevice");
  const SkyDev& d = sk->d;
  int* d_sh = nullptr;
  double *Z = nullptr, *imp = nullptr;
  if ((rc = to_device(&d_sh, shifts, (size_t)T, "uploading shifts")) != FGL_OK) return rc;
  if ((e = hipMalloc(reinterpret_cast<void**>(&Z), (size_t)d.F * T * 8)) != hipSuccess ||
      (e = hipMalloc(reinterpret_cast<void**>(&imp), (size_t)d.nlat * d.nlon * 8)) != hipSuccess) {
    rc = hip_err(e, "allocating importance buffers");
  }
  if (rc == FGL_OK) {
    rc = scheme == FGL_WEIGHT_BEAM ? run_corr<kCorrBeam>(sk, d_sh, T, smax, Lz, Z)
         : scheme == FGL_WEIGHT_SKY ? run_corr<kCorrSky>(sk, d_sh, T, smax, Lz, Z)
                                    : run_corr<kCorrHorizon>(sk, d_sh, T, smax, Lz, Z);
  }
  if (rc == FGL_OK) {
    std::vector<double> hz((size_t)d.F * T);
    if ((e = hipMemcpy(hz.data(), Z, hz.size() * 8, hipMemcpyDeviceToHost)) != hipSuccess)
      rc = hip_err(e, "copy normalisers");
    for (size_t k = 0; rc == FGL_OK && k < hz.size(); ++k)
      if (!(hz[k] > 0.0))
        rc = set_err(FGL_EINVAL, "the weight of channel %zu, step %zu integrates to %g",
                     k / T, k % T, hz[k]);
  }
  if (rc == FGL_OK) {
    const size_t lds = (size_t)T * 36 + (size_t)d.nlon * 32;
    // chunks of four-channel blocks: enough workgroups to fill the device,
    // summed in order
    const int nb = (d.F + 3) / 4;
    const int fchunks = std::max(1, std::min(nb, (2048 + d.nlat - 1) / d.nlat));
    const int bper = (nb + fchunks - 1) / fchunks;
    const int nch = (nb + bper - 1) / bper;
    const size_t np = (size_t)d.nlat * d.nlon;
    double* part = nullptr;
    if (lds > 160 * 1024) {
      rc = set_err(FGL_EINVAL, "T=%d and nlon=%d do not fit one workgroup's LDS", T, d.nlon);
    } else if ((e = hipMalloc(reinterpret_cast<void**>(&part), np * nch * 8)) != hipSuccess) {
      rc = hip_err(e, "allocating importance partials");
    } else {
      auto launch = [&](auto kern) {
        hipError_t ee = set_lds(kern);
        if (ee != hipSuccess) return ee;
        hipLaunchKernelGGL(kern, dim3(d.nlat, nch), dim3(256), lds, sk->stream, d, d_sh, T, Z,
                           bper, part);
        return hipGetLastError();
      };
      e = scheme == FGL_WEIGHT_BEAM ? launch(k_sky_importance<kCorrBeam>)
          : scheme == FGL_WEIGHT_SKY ? launch(k_sky_importance<kCorrSky>)
                                     : launch(k_sky_importance<kCorrHorizon>);
      if (e == hipSuccess) {
        hipLaunchKernelGGL(k_sky_reduce, dim3((unsigned)((np + 255) / 256)), dim3(256), 0,
                           sk->stream, part, nch, np, imp);
        e = hipGetLastError();
      }
      if (e == hipSuccess) e = hipStreamSynchronize(sk->stream);
      if (e == hipSuccess) e = hipMemcpy(importance, imp, np * 8, hipMemcpyDeviceToHost);
      if (e != hipSuccess) rc = hip_err(e, "importance kernel");
    }
    if (part) (void)hipFree(part);
  }
  if (d_sh) (void)hipFree(d_sh);
  if (Z) (void)hipFree(Z);
  if (imp) (void)hipFree(imp);
  return rc;
}

int fgl_partition(const double* beta, const double* weight, int n, int n_regions, int method,
                  double* edges) {
  if (!beta || !weight || !edges) return set_err(FGL_EINVAL, "arrays must be non-NULL");
  if (n < 1 || n_regions < 1) return set_err(FGL_EINVAL, "need n >= 1 and n_regions >= 1");
  if (method != FGL_PARTITION_HIERARCHICAL && method != FGL_PARTITION_RECURSIVE)
    return set_err(FGL_EINVAL, "unknown partition method %d", method);
  for (int k = 0; k < n; ++k)
    if (!std::isfinite(beta[k]) || !std::isfinite(weight[k]) || weight[k] < 0.0)
      return set_err(FGL_EINVAL, "beta[%d] must be finite and weight[%d] finite and >= 0", k, k);
  return partition_host(beta, weight, n, n_regions, method, edges);
}

int fgl_sky_chromatic(fgl_sky* sh, const double* edges, int n_regions, const int32_t* shifts,
                      int T, double* K) {
  TraceRange tr("fgl_sky_chromatic regions=%d T=%d", n_regions, T);
  Sky* sk = reinterpret_cast<Sky*>(sh);
  if (!sk || !edges || !K) return set_err(FGL_EINVAL, "sky, edges and K must be non-NULL");
  if (n_regions < 1 || n_regions > 1024) return set_err(FGL_EINVAL, "n_regions=%d outside 1..1024", n_regions);
  for (int j = 0; j <= n_regions; ++j)
    if (!std::isfinite(edges[j]) || (j > 0 && edges[j] < edges[j - 1]))
      return set_err(FGL_EINVAL, "edges must be finite and non-decreasing");
  int rc = check_shifts(sk, shifts, T);
  if (rc != FGL_OK) return rc;
  hipError_t e = hipSetDevice(sk->dev);
  if (e != hipSuccess) return hip_err(e, "hipSetDevice");
  const SkyDev& d = sk->d;
  const int N = n_regions, nlon = d.nlon;
  // masks: region j holds e_j <= beta < e_{j+1}, the last closed; then the
  // columns of each ring grouped by region (ascending column within one),
  // every region's run padded to a multiple of four with weight-zero entries
  std::vector<int> regs((size_t)d.nlat * nlon), counts((size_t)d.nlat * N, 0);
  int L = 8;
  for (int r = 0; r < d.nlat; ++r) {
    int len = 0;
    for (int c = 0; c < nlon; ++c) {
      const double b = sk->h_beta[(size_t)r * nlon + c];
      int j = (int)(std::upper_bound(edges, edges + N + 1, b) - edges) - 1;
      if (b == edges[N]) j = N - 1;
      if (b < edges[0] || b > edges[N]) j = -1;
      regs[(size_t)r * nlon + c] = j;
      if (j >= 0) ++counts[(size_t)r * N + j];
    }
    for (int j = 0; j < N; ++j) len += pad4(counts[(size_t)r * N + j]);
    L = std::max(L, len);
  }
  // longest slice of one region group's columns in a ring (a multiple of 4)
  int Lg = 8;
  for (int r = 0; r < d.nlat; ++r)
    for (int j0 = 0; j0 < N; j0 += kRegionsPerGroup) {
      int len = 0;
      for (int j = j0; j < std::min(N, j0 + kRegionsPerGroup); ++j)
        len += pad4(counts[(size_t)r * N + j]);
      Lg = std::max(Lg, len);
    }
  const int smax = *std::max_element(shifts, shifts + T);
  if (k_lds(nlon, smax, Lg) > 160 * 1024)
    return set_err(FGL_EINVAL, "nlon=%d does not fit one workgroup's LDS", nlon);
  std::vector<int> order((size_t)d.nlat * L, 0), seg((size_t)d.nlat * (N + 1));
  std::vector<double> asort((size_t)d.nlat * L, 0.0);
  for (int r = 0; r < d.nlat; ++r) {
    int* sg = &seg[(size_t)r * (N + 1)];
    sg[0] = 0;
    for (int j = 0; j < N; ++j) sg[j + 1] = sg[j] + pad4(counts[(size_t)r * N + j]);
    std::vector<int> fill(sg, sg + N);
    for (int c = 0; c < nlon; ++c) {
      const int j = regs[(size_t)r * nlon + c];
      if (j < 0) continue;
      const size_t at = (size_t)r * L + fill[j]++;
      order[at] = c;
      asort[at] = sk->h_omega[r] * sk->h_tex[(size_t)r * nlon + c];
    }
  }
  std::vector<int4> items;
  std::vector<int> first;
  k_items(seg, d.nlat, N, items, first);
  int *d_sh = nullptr, *d_order = nullptr, *d_seg = nullptr, *d_first = nullptr;
  int4* d_items = nullptr;
  double *d_K = nullptr, *d_as = nullptr;
  if ((rc = to_device(&d_sh, shifts, (size_t)T, "uploading shifts")) == FGL_OK &&
      (rc = to_device(&d_order, order.data(), order.size(), "uploading the region order")) == FGL_OK &&
      (rc = to_device(&d_as, asort.data(), asort.size(), "uploading pixel weights")) == FGL_OK &&
      (rc = to_device(&d_seg, seg.data(), seg.size(), "uploading region segments")) == FGL_OK &&
      (rc = to_device(&d_items, items.data(), items.size(), "uploading work items")) == FGL_OK &&
      (rc = to_device(&d_first, first.data(), first.size(), "uploading work items")) == FGL_OK) {
    if ((e = hipMalloc(reinterpret_cast<void**>(&d_K), (size_t)N * d.F * T * 8)) != hipSuccess)
      rc = hip_err(e, "allocating K");
  }
  float ms = 0.0f;
  if (rc == FGL_OK)
    rc = run_k(sk, d_sh, T, smax, d_order, d_as, d_seg, N, L, Lg, d_items, (int)items.size(),
               d_first, d_K, &ms);
  if (rc == FGL_OK) {
    sk->last_ms = ms;
    if ((e = hipMemcpy(K, d_K, (size_t)N * d.F * T * 8, hipMemcpyDeviceToHost)) != hipSuccess)
      rc = hip_err(e, "copy K");
  }
  const void* ps[] = {d_sh, d_order, d_seg, d_K, d_as, d_items, d_first};
  for (const void* p : ps)
    if (p) (void)hipFree(const_cast<void*>(p));
  return rc;
}

int fgl_sky_kernel_ms(const fgl_sky* sh, double* ms) {
  const Sky* sk = reinterpret_cast<const Sky*>(sh);
  if (!sk || !ms) return set_err(FGL_EINVAL, "sky and ms must be non-NULL");
  *ms = sk->last_ms;
  return FGL_OK;
}

int fgl_sky_destroy(fgl_sky* sh) {
  Sky* sk = reinterpret_cast<Sky*>(sh);
  if (!sk) return set_err(FGL_EINVAL, "sky is NULL");
  (void)hipSetDevice(sk->dev);
  if (sk->stream) (void)hipStreamSynchronize(sk->stream);
  free_sky(sk);
  return FGL_OK;
}

}  // extern "C"
