// Internal interface between the host library (fgl_host.cpp) and the device
// kernels (fgl_kernels.hip).  Not part of the public C-ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fgl {

// Exponent tables of the mixed kernel: tab[k] = Q 2^((k - kTabLo)/64) for
// k in [0, kTabSize), Q = 2^47 - 2^41 (forty-eight octaves below the row
// maximum, where the power's fixed point ends, up to the maximum itself),
// then frac[m] = 2^(m/64) / (1 - 2^-6) for m in [0, 64) at
// tab[kTabSize + m], then 1 / frac[m] at tab[kTabSize + kFracSize + m].
constexpr int kTabLo = 3072;
constexpr int kTabSize = 3074;
constexpr int kFracSize = 64;
constexpr int kTabBytes = (kTabSize + 2 * kFracSize) * 8;   // a multiple of 16
// Level sums are kept in int32 accumulators (see fgl_kernels.hip); their
// range bounds the region count of the mixed kernel: 128 for the direct
// form, 96 for the projected form (whose matrix has two more digits).
constexpr int kMixedMaxN = 128;
// Rows per call: keeps every grid and row index of the likelihood kernels
// far inside 32-bit work-item counts (2^26 rows of 36 parameters are 19 GB).
constexpr int kMaxRows = 1 << 26;
constexpr int kProjMaxN = 96;
// Digits of the projected-form matrix and its fixed-point scale: entries
// are scaled by 2^(kProjBits - eR(nu)) (|entry| < 2^eR) and cut into
// kProjDigits balanced base-256 digits.
constexpr int kProjDigits = 6;
constexpr int kProjBits = 46;

// Rows per workgroup of the row-preparation kernel (256 threads, sixteen per
// row).
constexpr int kPrepRows = 16;

// Per-row parameters written by the prep kernel (one 80-byte record per row).
struct RowParams {
  double bmin, bmax;   // extreme spectral indices of the row
  double omin, omax;   // extreme log2 amplitude scales (0 without amplitude masks)
  double A, nu0;       // 21-cm amplitude (K) and centre (MHz)
  double inv_w;        // 1 / width (1/MHz)
  double sigma;        // noise level (K)
  double t21;          // 1.0 with the 21-cm term, 0.0 without
  int32_t valid;       // 0: invalid row -> logL = -inf
  int32_t pad;
};

// Compiled operand slot counts of the plain kernels: region pairs (FP32) and
// region quads (FP64), rounded up; padded regions have K = 0.
inline int fp32_slots(int N) {
  const int n = (N + 1) / 2;
  for (int s : {2, 4, 8, 12, 16, 24, 32, 48, 64})
    if (n <= s) return s;
  return 0;
}
inline int fp64_slots(int N) {
  const int n = (N + 3) / 4;
  for (int s : {1, 2, 4, 6, 8, 12, 16, 24, 32})
    if (n <= s) return s;
  return 0;
}

// Kernel families behind one entry point.  kThin: small models evaluated
// per row in FP64 on the vector units; used for the mixed and FP64
// precisions of such models (thin_model below).
enum Kind { kMixed = 0, kFP32 = 1, kFP64 = 2, kThin = 3 };
constexpr int kThinMaxT = 64;
constexpr int kThinMaxN = 32;
constexpr int kThinCostDirect = 650;
constexpr int kThinCostProj = 580;

// Compiled region counts of the thin kernel (regions >= N have K = 0).
inline int thin_slots(int N) {
  for (int s : {4, 8, 12, 16, 24, 32})
    if (N <= s) return s;
  return 0;
}

// A row and channel cost the thin kernel about NT T + 12 NT + 2 T vector
// operations per lane (NT region slots: the model sums, the powers, the
// residuals), scaled by what the compiled slot count measured per operation
// (percent; 24 slots spill into more registers, 32 unroll best).  The digit
// kernel costs the same whatever the shape below one tile: its direct form
// (T <= 32) matched ~650 such operations, its projected form (always taken
// for 32 < T <= 64 since T > N) ~580.
inline int thin_scale(int nt) { return nt == 24 ? 117 : nt == 32 ? 90 : nt == 12 ? 97 : 100; }
inline bool thin_model(int N, int T) {
  const int nt = thin_slots(N);
  if (nt == 0 || T > kThinMaxT) return false;
  const int ops = nt * T + 12 * nt + 2 * T;
  return ops * thin_scale(nt) <= (T <= 32 ? kThinCostDirect : kThinCostProj) * 100;
}

// Tile configuration of one launch (chosen by the tuner).
// The channel sum of a row is cut into reduction groups of `group`
// consecutive channels; the workgroup of a row tile stages `fc` channels
// (a multiple of `group`) and writes one partial per group.  The group size
// is fixed per (model, precision), so results never depend on the tuned
// waves/fc.
struct Tile {
  int waves;   // waves per workgroup: 4 or 8
  int fc;      // frequency channels staged per workgroup
  int group;   // channels per reduction group
  int occ;     // waves per SIMD the kernel is compiled for (2 or 3)
};

// Channel chunks of a likelihood launch: `nbig` chunks of `fc` channels,
// then chunks of `fs` channels up to F, `nc` in all (fs <= fc, both
// multiples of the reduction group, so the partials do not depend on the
// chunking).  On each XCD every row tile's large chunks are dispatched
// before the small ones, which fill the last round of workgroups.
struct Chunks {
  int fc, fs, nbig, nc;
};

// Compute units of the device (MI355X: 8 XCDs of 32).
constexpr int kCUs = 256;

// Workgroup `id` of a likelihood launch -> (row tile bt, chunk ch).  Block
// ids go round-robin to the 8 XCDs; XCD xcd takes its share of the (row
// tile, large chunk) pairs first, then its share of the (row tile, small
// chunk) pairs, each a contiguous run in row-tile order, so that both cover
// the same row tiles (whose rows then stay in that XCD's L2) and the small
// chunks come last.  The small pairs are shared out so that each XCD's total
// is the round-robin count of its ids, which needs nb * nsmall >= 8 (or no
// small chunks: then this is the plain contiguous split).
__host__ __device__ inline void map_block_split(int id, int nb, int nbig, int nsmall, int& bt,
                                                int& ch) {
  const int total = nb * (nbig + nsmall), tb = nb * nbig;
  const int xcd = id & 7, k = id >> 3;
  const int q = total >> 3, rem = total & 7;
  const int qb = tb >> 3, rb = tb & 7;
  const int start_b = xcd * qb + (xcd < rb ? xcd : rb);
  const int n_b = qb + (xcd < rb ? 1 : 0);
  if (k < n_b) {
    const int L = start_b + k;
    bt = L / nbig;
    ch = L - bt * nbig;
  } else {
    const int L = xcd * q + (xcd < rem ? xcd : rem) - start_b + (k - n_b);
    bt = L / nsmall;
    ch = nbig + (L - bt * nsmall);
  }
}

// Device-side model (all pointers are device memory owned by the model).
struct DevModel {
  int N, F, T, P;
  // masks: NA amplitude masks (0: none, alpha = 1) crossed with NB
  // spectral-index masks; region r = i NB + j has alpha_i and beta_j, and
  // N = max(NA, 1) NB
  int NA, NB;
  int TT;            // 32-row time tiles (mixed, FP32)
  int TT16;          // 16-row time tiles (FP64)
  int KC;            // 32-region chunks (mixed)
  int NP2;           // region pairs, rounded up to a compiled size (FP32)
  int NQ;            // region quads, rounded up to a compiled size (FP64)
  double t_cmb;
  unsigned flags;
  const int8_t* kd;      // mixed digits [F][4][KC][TT][64][16]
  const int32_t* eK;     // [F] per-channel exponent of the digits
  const float* k32;      // FP32 A-operands [F][NP2][TT][64], zero-padded regions
  const float* k64;      // FP64 A-operands, as exact FP32 [F][NQ][TT16][64]
  const double* nl64;    // [F] -64 log2(nu/nu_ref)
  const double* nl2;     // [F] -log2(nu/nu_ref)
  const double* nu;      // [F] MHz
  const double* D;       // [F][TT*32] data, zero padded in t
  const double* tab;     // [kTabSize + 2 kFracSize] exponent tables
  double c1, c2, c3, c4; // Taylor coefficients of 2^(r/64)
  double c5;             // and its fifth-order term
  double q[5];           // the mixed kernel's 2^(r/64): degree 4, Chebyshev nodes
  // projected form of the mixed kernel (proj = 1): per channel, the rows
  // [sqrt(T) mean_t K ; R] where K~^T = Q R is the QR factorisation of the
  // time-centred responses, and targets [sqrt(T) mean_t D ; (Q^T D~)_0..]
  int proj;              // 1: the mixed kernel runs the projected form
  int RT;                // 32-row tiles of the projected matrix
  int peel;              // 1: the last row of R (one entry) is done in FP64
  double sqrtT;
  double chi0;           // sum over channels of the data's out-of-span part
  const int8_t* rd;      // digits [F][kProjDigits][KC][RT][64][16]
  // plain precisions in the projected form (FGL_PLAIN_PROJECTED): the same
  // rows in FP32 as A operands of the FP32 kernel, [F][NP2][RT][64]: lane ->
  // (row 32 rt + lane%32, region 2 p + lane/32); the FP64 kernel reads pa64
  int pplain;            // 1: the FP32 and FP64 kernels run the projected form
  const float* r32;
  const int32_t* eR;     // [F] per-channel exponent of the digits
  const double* tg;      // [F][RT*32] targets (row 0 is per parameter row)
  const double* dbar;    // [F] sqrt(T) mean_t D
  const double* pk;      // [F][2] peeled diagonal entry and its target
  // the same projected rows in FP64 for the gradient kernel: all N + 1 rows
  // (nothing peeled) in 16-row tiles, as FP64 MFMA A operands
  int RT16;              // 16-row tiles of the N + 1 rows
  const double* pa64;    // [F][NQ][RT16][64]: lane -> (row 16 tt + lane%16, region 4 q + lane/16)
  const double* pt64;    // [F][RT16*16] targets: row 0 sqrt(T) mean_t D, rows 1.. z
  // thin models (thin_model(N, T))
  int thin;              // 1: mixed (unless the direct form is forced) and FP64 use k_thin64
  int NT;                // regions rounded up to a compiled count
  const float* kthin;    // [F][T][NT] K, zero padded in regions
};

// Amplitude-mask mode of the mixed kernel: 0 without amplitude masks, 2 when
// the index masks come in multiples of 16 (a 16-region half chunk then lies
// within one amplitude mask, so a lane holds one alpha per chunk), else 1
// (one alpha per region).
inline int mixed_alpha_mode(const DevModel& d) {
  return d.NA == 0 ? 0 : (d.NB % 16 == 0 ? 2 : 1);
}
// The mixed kernel's three-waves-per-SIMD compile exists for the projected
// form with one region chunk and at most one alpha per lane and chunk.
inline bool mixed_occ3(const DevModel& d) {
  return d.proj && d.KC == 1 && mixed_alpha_mode(d) != 1;
}

// The constant chi-square of the data's part outside the span of the
// projected rows, added to every row's sum by the kernel families that run
// the projected form.
inline double chi0_of(Kind k, const DevModel& d) {
  if (k == kMixed) return d.proj ? d.chi0 : 0.0;
  if (k == kFP32 || k == kFP64) return d.pplain ? d.chi0 : 0.0;
  return 0.0;
}

// Per-call workspace (device memory owned by the model, per stream).
struct Work {
  int B, Bpad;           // rows and rows padded to the widest b-tile
  double* betaT;         // [KC*32 rounded][Bpad] sanitised spectral indices
  double* offT;          // [KC*32 rounded][Bpad] log2 alpha per region (NA > 0)
  RowParams* rows;       // [Bpad]
  double* partial;       // [ngroups][Bpad]
  int ngroup_cap;        // capacity of partial in groups
  double* gpart;         // gradient partials [chunks][grad_slots][Bpad]
};

// One model's rows in a launch shared by several models whose likelihood
// kernel is the same compiled variant (serving): its model, workspace and
// tile, and where its workgroups start in each of the three launches.
constexpr int kMaxGroups = 16;
struct GroupDesc {
  DevModel m;
  Work w;
  int fc, G, nb, nc;     // likelihood tile and grid (row tiles x channel chunks)
  int start[3];          // first workgroup in the likelihood, preparation and finalize launches
  int ngroups;           // partials per row
  const double* theta;   // [B][P] device
  double* out;           // [B] device
  double nFT, chi0;
};

// Gradient partials per (channel chunk, row): chi-square, the three 21-cm
// sums, then per region sum_nu (-log2(nu/nu_ref)) c u and, with amplitude
// masks, sum_nu c u (c: the region's coefficient, u: the region's row of
// K times the residual).
__host__ __device__ inline int grad_slots(const DevModel& m) { return 4 + m.N * (m.NA > 0 ? 2 : 1); }

// Launch shape of the gradient kernel for B rows: 4-wave workgroups of 64
// rows, `chunks` channel chunks of `per` channels, staged `fs` at a time.
struct GradShape {
  int nb, chunks, per, fs, lds;
};
GradShape grad_shape(const DevModel& m, int Bpad);

// Launchers (fgl_kernels.hip).  All enqueue on `s`; none synchronises.
// The launch planning below them (tile LDS, reduction groups, shared-launch
// plans, gradient shape) is host logic in fgl_plan.cpp.
hipError_t launch_prep(const DevModel& m, const double* theta, int B,
                       const Work& w, int betaRows, hipStream_t s);
hipError_t launch_main(Kind k, const DevModel& m, const Work& w,
                       const Tile& tile, hipStream_t s);
hipError_t launch_finalize(Kind k, const DevModel& m, const Work& w,
                           const Tile& tile, double* out, hipStream_t s);
// The three launches of groups that share a compiled likelihood variant:
// h[0..n) on the host (their start[] filled in here), copied by the caller
// to d (device) before these run; `k` and `tile` as for group 0.
void plan_groups(Kind k, const Tile& tile, GroupDesc* h, int n, int grid[3], int* lds);
hipError_t launch_groups(Kind k, const DevModel& m0, const Tile& tile, const GroupDesc* d,
                         int n, const int grid[3], int lds, hipStream_t s);
// The compiled likelihood variant of (kind, model, tile): launches of models
// with equal signatures can be shared.
uint64_t variant_of(Kind k, const DevModel& m, const Tile& tile);
// Gradient (FP64): the kernel writes w.gpart, the finalize lnL and the
// gradient rows.  w.gpart must hold grad_slots(m) * chunks * Bpad doubles.
hipError_t launch_grad(const DevModel& m, const Work& w, const GradShape& g,
                       hipStream_t s);
hipError_t launch_grad_finalize(const DevModel& m, const Work& w, const GradShape& g,
                                const double* theta, double* out, double* grad,
                                hipStream_t s);

// Shape helpers shared by host and launcher.
int lds_bytes(Kind k, const DevModel& m, const Tile& t);
int cols_per_wave(Kind k);
int n_chunks(const DevModel& m, const Tile& t);   // workgroups along nu
int n_groups(const DevModel& m, const Tile& t);   // partials per row
int max_lds_bytes();
// The likelihood launch's chunks over nb row tiles (uniform chunks of
// t.fc channels but for the mixed kernel, whose last round is filled with
// half-size chunks when that shortens the busiest CU's share).
Chunks chunk_plan(Kind k, const DevModel& m, const Tile& t, int nb);

}  // namespace fgl
