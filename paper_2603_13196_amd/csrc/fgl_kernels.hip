// Device kernels of the batched foreground log-likelihood, for CDNA4 (gfx950).
//
// Computed quantity (Tutt et al., Eqs. fast_forward_model, t21model and
// likelihood): for each parameter row b,
//   M[b,nu,t] = sum_i K[i,nu,t] (nu/nu_ref)^(-beta_bi) + T_CMB
//               + A_b exp(-(nu - nu0_b)^2 / (2 w_b^2))
//   lnL_b     = -sum_{nu,t} [ (D - M)^2 / (2 sigma_b^2) + ln(2 pi sigma_b^2)/2 ]
//
// Every kernel works in the transposed orientation M^T = K^T (T x N) P (N x B)
// per channel: MFMA rows are time bins, MFMA columns are parameter rows.  A
// wave owns one tile of parameter rows (its MFMA columns) for a range of
// channels, so each lane holds exactly one row b and all per-row constants
// are per-lane scalars; the time bins of a lane sit in its accumulator
// registers and the data D[nu, t] for them are broadcast reads from LDS.
//
// The workgroup stages the chromatic responses of a block of channels (and
// the data of those channels) in LDS once; its waves then run independently
// over the channels.  Each workgroup writes one chi-square partial per row
// and per reduction group of channels; a finalize kernel sums the partials
// of a row in channel order.  The group size is fixed per model, so results
// are bitwise reproducible, independent of the tuned tile and of what else
// runs on the device.
//
// Four arithmetic forms share that skeleton:
//   k_mixed: exact integer slicing.  The powers are computed in FP64,
//            rounded to 47-bit fixed point relative to the row's largest
//            power at the channel and cut into six signed 8-bit digits; the
//            matrix rows (K itself, or an orthonormal projection of it with
//            N + 1 rows when that is shorter than T) are cut into digits once,
//            at model creation.  The digit products run as
//            v_mfma_i32_32x32x32_i8 with exact int32 sums in three
//            accumulators, and the residual and the chi-square run in FP64.
//   k_fp32:  the model in FP32 (v_mfma_f32_32x32x2_f32, FP32 powers),
//            residual and chi-square in FP64.
//   k_fp64:  the model in FP64 (v_mfma_f64_16x16x4_f64, FP64 powers).
//   k_thin64: small models (few time bins and regions), where a matrix
//            tile would be mostly padding: each lane evaluates its row's
//            model values as FP64 sums on the vector units.
#include "fgl_internal.h"

#include <math.h>

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <set>

namespace fgl {

typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x16 __attribute__((ext_vector_type(16)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// shared helpers

// Workgroup id -> (row tile, channel chunk).  Consecutive workgroup ids go
// to different XCDs round-robin; the remap gives every XCD a contiguous run
// of row tiles, channel chunk fastest, so an XCD reads only its own rows'
// spectral indices and row records (which then stay in its L2 across all
// channel chunks) while the chunks of K, shared by all XCDs, are read once
// per XCD.
__device__ inline void map_block_id(int id, int nb, int nc, int& bt, int& ch) {
  const int total = nb * nc;
  const int xcd = id & 7, k = id >> 3;
  const int q = total >> 3, rem = total & 7;
  const int L = xcd * q + (xcd < rem ? xcd : rem) + k;
  bt = L / nc;
  ch = L - bt * nc;
}
__device__ inline void map_block(int nb, int nc, int& bt, int& ch) {
  map_block_id(blockIdx.x, nb, nc, bt, ch);
}

// Cooperative 16-byte copy global -> LDS (bytes is a multiple of 16).
__device__ inline void stage(void* dst, const void* src, int bytes) {
  const uint4* s = reinterpret_cast<const uint4*>(src);
  uint4* d = reinterpret_cast<uint4*>(dst);
  const int n = bytes >> 4;
  for (int k = threadIdx.x; k < n; k += blockDim.x) d[k] = s[k];
}

// 4x4 byte transpose: out[L] gathers byte (3-L) of v0..v3 (byte k of out[L]
// comes from v_k).  Eight v_perm_b32.
__device__ inline void transpose4(uint32_t v0, uint32_t v1, uint32_t v2,
                                  uint32_t v3, uint32_t out[4]) {
  const uint32_t a = __builtin_amdgcn_perm(v1, v0, 0x05010400u);
  const uint32_t b = __builtin_amdgcn_perm(v1, v0, 0x07030602u);
  const uint32_t c = __builtin_amdgcn_perm(v3, v2, 0x05010400u);
  const uint32_t d = __builtin_amdgcn_perm(v3, v2, 0x07030602u);
  out[3] = __builtin_amdgcn_perm(c, a, 0x05040100u);  // byte 0 of each
  out[2] = __builtin_amdgcn_perm(c, a, 0x07060302u);  // byte 1
  out[1] = __builtin_amdgcn_perm(d, b, 0x05040100u);  // byte 2
  out[0] = __builtin_amdgcn_perm(d, b, 0x07060302u);  // byte 3
}

// exp(-z^2/2) in FP32 for the 21-cm profile of the plain FP32 kernel.
__device__ inline double gauss21(double nu, const RowParams& rp) {
  const float z = (float)((nu - rp.nu0) * rp.inv_w);
  return (double)__builtin_amdgcn_exp2f(-0.7213475204444817f * z * z);
}

// FP64 powers of the plain-FP64, thin and gradient kernels: 2^(y/64) for
// |y| < 2^31 as 2^floor(j/64) (ldexp) times 2^((j mod 64)/64) from the
// 64-entry LDS table t64 times 2^(r/64), j = round(y), |r| <= 1/2, by its
// Taylor series to fifth order (truncation below 4e-17 relative).
__device__ inline void init_t64(double* t64) {
  if (threadIdx.x < 64) t64[threadIdx.x] = exp2((double)threadIdx.x * (1.0 / 64.0));
}
__device__ inline double pow2_64(double y, const double* t64, const DevModel& m) {
  const double MAGIC = 0x1.8p52;                  // rint via the low word
  const double t = y + MAGIC;
  const int j = (int)(uint32_t)__double_as_longlong(t);
  const double r = y - (t - MAGIC);               // |r| <= 1/2
  double p = fma(r, m.c5, m.c4);
  p = fma(r, p, m.c3);
  p = fma(r, p, m.c2);
  p = fma(r, p, m.c1);
  p = fma(r, p, 1.0);
  return ldexp(t64[j & 63] * p, j >> 6);
}

// ---------------------------------------------------------------------------
// mixed: exact int8 slices on MFMA
//
// Digits.  At channel nu a row's powers are normalised by 2^(ymax/64), the
// row's largest power rounded up to 1/64 octave (ymax from the extreme
// spectral index), so x_i = P_i / 2^(ymax/64) lies in (0, 1].  Each x_i is
// rounded to q_i = round(x_i Q), Q = 2^47 - 2^41, and written as six
// balanced base-256 digits d0..d5 (d0 in [0, 127], the others in
// [-128, 127]).  One FP64 fma produces all six: t = x Q + (2^52 + 2^39 +
// 2^31 + 2^23 + 2^15 + 2^7) is an integer-valued double whose low word
// holds d2..d5 offset by 128 and whose high word holds d1 + 128 (byte 0)
// and d0 (byte 1).  The powers need this width: a power's rounding error is
// shared by every time bin of the channel, so on rows near the posterior
// peak, whose residuals carry a coherent part of a few sigma, it adds up
// over t; 39 bits used most of the tolerance there.
//
// Two forms share the power-law code and the digit products.  S_l is the
// sum of the digit products of significance l = p + q (power digit p,
// matrix digit q); levels up to 5 are kept, in three accumulators
// acc0 = S0 2^8 + S1, acc1 = S2 2^8 + S3, acc2 = S4 2^8 + S5, whose int32
// sums are exact: each digit is within [-128, 127], d0 within [0, 127].
// Direct form, top K digit within [-125, 125]: |S4|, |S5| <= 65152 N, so
// |acc2| <= 257 65152 N + 2^15 < 2^31 for N <= 128 (acc0 and acc1 have
// more room).  Projected form, top matrix digit within [-64, 64]:
// |S4| <= 73600 N, |S5| <= 89984 N, so |acc2| < 2^31 for N <= 113.
//
// Direct form (the model on the time grid).  The MFMA rows are time bins:
// K at channel nu is scaled by 2^(31 - eK(nu)) and cut into four digits
// e0..e3 (e0 in [-125, 125]) once, at model creation.  The eighteen digit
// products with p + q <= 5 run on v_mfma_i32_32x32x32_i8; the constant
// T_CMB + A g of the row enters the three accumulators as digits through
// the shift-adds that combine levels.  Dropped products (significance
// >= 6) are below 2^-47 of the leading term, as is the power-law rounding
// relative to the row's largest power.
//
// Projected form (the residual in an orthonormal basis of each channel).
// With Kbar, Dbar the time means at channel nu and K~, D~ the centred
// series, the time sum of (D - M)^2 splits exactly into
//   T (Dbar - c - Kbar.P)^2 + |D~ - K~^T P|^2,
// and with the QR factorisation K~^T = Q R (R upper triangular, N x N) the
// second term is |Q^T D~ - R P|^2 over the first N coordinates plus the
// data's part outside the span of K~, a constant per model.  The MFMA rows
// are then the N + 1 rows [sqrt(T) Kbar ; R] instead of T time bins, and the
// residual of each row is its target [sqrt(T) (Dbar - c) ; (Q^T D~)_k]
// minus the row's product with P.  R is not exact in a few digits, so its
// rows are cut into six digits (46-bit fixed point per channel) and the
// twenty-one products of significance <= 5 run.  When N is a multiple of 32 the
// last row of R (a single diagonal entry) is evaluated in FP64 from the
// same rounded power, so the MFMA rows fill whole tiles.

// OCC: waves per SIMD the register allocation targets (2, or 3 for the
// projected form with one region chunk, which fits in 168 registers).
// The body of workgroup `block` of a launch on (m, w); the kernels below
// call it for one model (k_mixed) or for several that share the compiled
// variant (k_mixed_multi).
template <int W, int KC, bool PROJ, int OCC, int AM>
__device__ __forceinline__ void mixed_body(const DevModel& m, const Work& w, const Chunks& cp,
                                           int G, int nb, int block) {
  constexpr int ND = PROJ ? kProjDigits : 4;       // digits of the matrix rows
  constexpr int NP = 6;                            // digits of the powers
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int bt, ch;
  map_block_split(block, nb, cp.nbig, cp.nc - cp.nbig, bt, ch);
  const int TT = PROJ ? m.RT : m.TT;               // 32-row tiles
  const int fc = cp.fc;                            // LDS layout: the large chunk
  const bool big = ch < cp.nbig;
  const int f0 = big ? ch * fc : cp.nbig * fc + (ch - cp.nbig) * cp.fs;
  const int fn = min(big ? fc : cp.fs, m.F - f0);
  const int kbytes = ND * KC * TT * 1024;
  // LDS: the exponent tables at offset 0 (so a table byte offset is an LDS
  // address), then the channels' matrix digits and data
  double* s_tab = reinterpret_cast<double*>(smem);
  unsigned char* s_kd = smem + kTabBytes;
  double* s_D = reinterpret_cast<double*>(s_kd + (size_t)fc * kbytes);
  stage(s_tab, m.tab, kTabBytes);
  stage(s_kd, (PROJ ? m.rd : m.kd) + (size_t)f0 * kbytes, fn * kbytes);
  stage(s_D, (PROJ ? m.tg : m.D) + (size_t)f0 * TT * 32, fn * TT * 32 * 8);
  __syncthreads();
  const double* s_tab0 = s_tab + kTabLo;            // s_tab0[jj], jj in [-kTabLo, 0]
  const double* s_frac = s_tab + kTabSize;          // unit of the level-0 product
  const double* s_ifrac = s_frac + kFracSize;       // its reciprocal

  const int g = lane >> 5;
  const int b = bt * (W * 32) + wave * 32 + (lane & 31);
  const RowParams rp = w.rows[b];
  // amplitude masks (AM): 64 log2 alpha per region (AM = 1), or one value
  // per 16-region half chunk when the index masks come in multiples of 16,
  // so that each half chunk lies within one amplitude mask (AM = 2)
  constexpr bool AB = AM != 0;
  double beta[KC][16];
  double off[AM == 1 ? KC : 1][16];
  double off1[AM == 2 ? KC : 1];
#pragma unroll
  for (int kc = 0; kc < KC; ++kc)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const size_t at = (size_t)(kc * 32 + g * 16 + j) * w.Bpad + b;
      beta[kc][j] = w.betaT[at];
      if constexpr (AM == 1) off[kc][j] = 64.0 * w.offT[at];
      if constexpr (AM == 2)
        if (j == 0) off1[kc] = 64.0 * w.offT[at];
    }

  const double MAGIC = 0x1.8p52;                        // rint via the low word
  const double DIGITS = 0x1.0p52 + (double)0x8080808080ull;  // digit offsets
  double acc_a = 0.0, acc_b = 0.0;

  // Per-channel scalars (fetched ahead of use) and the row's state at one
  // channel: level units, the constant term's digits (direct form), the
  // target of the mean row and the last region's rounded power (projected
  // form), and the power-law digits, the MFMA B operands of this lane (row
  // b, 16 regions per 32-region chunk, five significance levels).
  struct Scal {
    double nl, nu;
    int ek;
  };
  struct Epi {                 // what the epilogue and the peeled row need
    double s0, t0, qlast;      // s0: unit of acc0 (acc1: s0 2^-16, acc2: s0 2^-32)
    int ey, fm;
  };
  struct Chan {
    Epi e;
    int c0, c1, c2;
    i32x4 B[KC][NP];
  };
  auto fetch = [&](int fi) {
    const int fx = min(fi, m.F - 1);
    return Scal{m.nl64[fx], m.nu[fx], PROJ ? m.eR[fx] : m.eK[fx]};
  };
  auto make = [&](const Scal& sc, int fi, Chan& C) {
    const double nl = sc.nl;
    // row constants at this channel: normalisation, level units, constant
    // term.  The 21-cm profile is FP64 (its error is shared by all time
    // bins): exp(-z^2/2) = 2^(y/64), y = -32 z^2 / ln 2, from the power
    // table and polynomial below (y is clamped at -4096, far below the
    // table, where the profile is < 2^-48 and takes the table's last entry).
    const double zg = (sc.nu - rp.nu0) * rp.inv_w;
    const double yg = fmax(zg * zg * (-32.0 / M_LN2), -4096.0);
    const double tg = yg + MAGIC;
    const double rg = yg - (tg - MAGIC);             // |rg| <= 1/2
    const int jg = max((int)(uint32_t)__double_as_longlong(tg), -kTabLo);
    double pg = fma(rg, m.q[4], m.q[3]);
    pg = fma(rg, pg, m.q[2]);
    pg = fma(rg, pg, m.q[1]);
    pg = fma(rg, pg, m.q[0]);
    // tab = Q 2^(j/64) with 1/Q = 2^-47 (64/63)
    const double c = fma(rp.A * (0x1.0p-47 * 64.0 / 63.0), s_tab0[jg] * pg, m.t_cmb);
    const double bext = nl > 0.0 ? rp.bmax : rp.bmin;
    // with amplitude masks the bound adds the row's largest 64 log2 alpha;
    // fl is monotone, so no region's rounded exponent exceeds it
    double ymax = AB ? ceil(fma(bext, nl, 64.0 * rp.omax)) : ceil(bext * nl);
    const int ey = (int)floor(ymax * (1.0 / 64.0));
    const int fm = (int)(ymax - 64.0 * ey);
    C.e.ey = ey;
    C.e.fm = fm;
    C.e.t0 = 0.0;
    C.c0 = C.c1 = C.c2 = 0;
    C.e.qlast = 0.0;
    if constexpr (PROJ) {
      // unit of the level-0 product: 2^(ymax/64) / Q times 2^(eR - 46)
      // times its weight 2^80
      const double u = ldexp(s_frac[fm], ey + sc.ek + 80 - kProjBits - 47);
      C.e.s0 = u * 0x1.0p-8;
      C.e.t0 = m.dbar[fi] - m.sqrtT * c;           // target of the mean row
    } else {
      // unit of the level-0 product: 2^(ymax/64) / Q times 2^(eK - 31)
      // times its weight 2^64, i.e. frac[fm] 2^(ey + eK - 14)
      int eu = ey + sc.ek - 14;
      double ic = c * ldexp(s_ifrac[fm], 8 - eu);   // ~ c / unit of acc0
      int ec;
      frexp(ic, &ec);                               // |ic| < 2^ec
      // constant term dominates: coarser power-law digits (branch-free)
      const int sh = max(ec - 29, 0);
      ymax += 64.0 * sh;
      eu += sh;
      ic = ldexp(ic, -sh);
      const double u0 = ldexp(s_frac[fm], eu);
      C.e.s0 = u0 * 0x1.0p-8;
      const double c0f = rint(ic);
      C.c0 = (int)c0f;
      // remainders by fma, in acc1 then acc2 units; c1, c2 in [-2^15, 2^15]
      const double r1 = fma(-c0f, C.e.s0, c);
      const double c1f = rint(r1 * ldexp(s_ifrac[fm], 24 - eu));
      C.c1 = (int)c1f;
      C.c2 = (int)rint(fma(-c1f, u0 * 0x1.0p-24, r1) * ldexp(s_ifrac[fm], 40 - eu));
    }
    // Powers 2^(y/64), y = 64 log2(x) <= 0, as tab[round(y)] 2^(r/64), the
    // latter by the degree-4 polynomial interpolating it at the Chebyshev
    // nodes of |r| <= 1/2 (relative error below 2^-48.5, under the 47-bit
    // rounding that follows).  Exponents below the table (x < 2^-48, all
    // digits zero) take its last entry, which rounds to zero digits for any
    // |r| <= 1/2.
    const double cm = MAGIC - ymax;                 // exact: ymax is an integer
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      uint32_t lo[16], hi[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        double t, r;
        if constexpr (AB) {
          const double y = fma(beta[kc][j], nl, AM == 1 ? off[kc][j] : off1[kc]) - ymax;
          t = y + MAGIC;
          r = y - (t - MAGIC);                     // |r| <= 1/2
        } else {
          // t = MAGIC + round(beta nl - ymax); u = that integer + ymax
          // (exact, same binade); r = beta nl - u with one rounding
          t = fma(beta[kc][j], nl, cm);
          const double u = t - cm;
          r = fma(beta[kc][j], nl, -u);            // |r| <= 1/2
        }
        const int jj = max((int)(uint32_t)__double_as_longlong(t), -kTabLo);
        const double T2 = s_tab0[jj];              // Q 2^(jj/64)
        double p = fma(r, m.q[4], m.q[3]);
        p = fma(r, p, m.q[2]);
        p = fma(r, p, m.q[1]);
        p = fma(r, p, m.q[0]);                     // 2^(r/64), degree 4
        const double q = fma(T2, p, DIGITS);       // 2^52 + q + offsets
        if (PROJ && kc == KC - 1 && j == 15) C.e.qlast = q - DIGITS;
        const unsigned long long bits = __double_as_longlong(q);
        lo[j] = (uint32_t)bits ^ 0x80808080u;      // digits d2 d3 d4 d5 (byte 3..0)
        hi[j] = (uint32_t)(bits >> 32);            // byte 1: d0, byte 0: d1 + 128
      }
#pragma unroll
      for (int m4 = 0; m4 < 4; ++m4) {
        uint32_t o[4];
        transpose4(lo[4 * m4], lo[4 * m4 + 1], lo[4 * m4 + 2], lo[4 * m4 + 3], o);
        // o[L] holds byte (3 - L) of the low words: d(L+2)
#pragma unroll
        for (int L = 0; L < 4; ++L) C.B[kc][L + 2][m4] = (int32_t)o[L];
        // bytes 0 and 1 of the four high words: x = [h0.0 h0.1 h1.0 h1.1],
        // y likewise for h2, h3; then d1 = [x.0 x.2 y.0 y.2] (offset 128
        // removed) and d0 = [x.1 x.3 y.1 y.3]
        const uint32_t x = __builtin_amdgcn_perm(hi[4 * m4 + 1], hi[4 * m4], 0x05040100u);
        const uint32_t y = __builtin_amdgcn_perm(hi[4 * m4 + 3], hi[4 * m4 + 2], 0x05040100u);
        C.B[kc][1][m4] = (int32_t)(__builtin_amdgcn_perm(y, x, 0x06040200u) ^ 0x80808080u);
        C.B[kc][0][m4] = (int32_t)__builtin_amdgcn_perm(y, x, 0x07050301u);
      }
    }
  };

  auto load_A = [&](int f, int tt, i32x4 (&A)[ND][KC]) {
    const unsigned char* kf = s_kd + (size_t)f * kbytes + lane * 16;
#pragma unroll
    for (int L = 0; L < ND; ++L)
#pragma unroll
      for (int kc = 0; kc < KC; ++kc)
        A[L][kc] = *reinterpret_cast<const i32x4*>(kf + ((L * KC + kc) * TT + tt) * 1024);
  };
  // MF(acc, q, p): the product of matrix digit q and power digit p
#define MF(acc, q, p) acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[q][kc], C.B[kc][p], acc, 0, 0, 0)
  // levels 0, 2 and 4 (no dependence on a shift)
  auto part1 = [&](const i32x4 (&A)[ND][KC], const Chan& C, i32x16& a0, i32x16& a1,
                   i32x16& a2) {
    a0 = i32x16{};
    a1 = i32x16{};
    a2 = i32x16{};
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      MF(a0, 0, 0);
      MF(a1, 0, 2); MF(a1, 1, 1); MF(a1, 2, 0);
      MF(a2, 0, 4); MF(a2, 1, 3); MF(a2, 2, 2); MF(a2, 3, 1);
      if constexpr (PROJ) MF(a2, 4, 0);
    }
  };
  // shift-adds (direct form: with the constant term's digits), then levels
  // 1, 3 and 5
  auto part2 = [&](const i32x4 (&A)[ND][KC], const Chan& C, i32x16& a0, i32x16& a1,
                   i32x16& a2) {
    if constexpr (PROJ) {
      a0 = (i32x16)((u32x16)a0 << 8u);
      a1 = (i32x16)((u32x16)a1 << 8u);
      a2 = (i32x16)((u32x16)a2 << 8u);
    } else {
      a0 = (i32x16)(((u32x16)a0 << 8u) + (uint32_t)C.c0);
      a1 = (i32x16)(((u32x16)a1 << 8u) + (uint32_t)C.c1);
      a2 = (i32x16)(((u32x16)a2 << 8u) + (uint32_t)C.c2);
    }
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      MF(a0, 0, 1); MF(a0, 1, 0);
      MF(a1, 0, 3); MF(a1, 1, 2); MF(a1, 2, 1); MF(a1, 3, 0);
      MF(a2, 0, 5); MF(a2, 1, 4); MF(a2, 2, 3); MF(a2, 3, 2);
      if constexpr (PROJ) {
        MF(a2, 4, 1); MF(a2, 5, 0);
      }
    }
  };
#undef MF
  auto epi = [&](int f, int tt, const Epi& C, const i32x16& a0, const i32x16& a1,
                 const i32x16& a2) {
    const double* Dt = s_D + (size_t)f * TT * 32 + g * 4 + tt * 32;
    const double s0 = C.s0, s1 = C.s0 * 0x1.0p-16, s2 = C.s0 * 0x1.0p-32;
    if (!PROJ && tt == TT - 1 && (m.T & 31)) {     // ragged last tile (uniform)
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        double r = fma(-s0, (double)a0[j], Dt[(j >> 2) * 8 + (j & 3)]);
        r = fma(-s1, (double)a1[j], r);
        r = fma(-s2, (double)a2[j], r);
        const int t = tt * 32 + (j >> 2) * 8 + g * 4 + (j & 3);
        r = t < m.T ? r : 0.0;
        if (j & 1) acc_b = fma(r, r, acc_b);
        else acc_a = fma(r, r, acc_a);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        double d = Dt[(j >> 2) * 8 + (j & 3)];
        // projected form: row 0 (element 0 of the first tile in lanes
        // 0..31) is the mean row, whose target depends on the row b
        if (PROJ && j == 0) d = (tt == 0 && g == 0) ? C.t0 : d;
        double r = fma(-s0, (double)a0[j], d);
        r = fma(-s1, (double)a1[j], r);
        r = fma(-s2, (double)a2[j], r);
        if (j & 1) acc_b = fma(r, r, acc_b);
        else acc_a = fma(r, r, acc_a);
      }
    }
  };
  // after a channel's last row tile: the peeled row, the partial
  auto tail = [&](int f, const Epi& C) {
    if constexpr (PROJ) {
      // peeled last row of R: R[N-1][N-1] P_{N-1}, P from the same rounding
      // (region N - 1 = 32 KC - 1 is element 15 of the last chunk, g = 1)
      if (m.peel) {
        const int fi = f0 + f;
        const double v = ldexp(s_frac[C.fm], C.ey - 47) * m.pk[2 * fi];
        const double r = fma(-v, C.qlast, m.pk[2 * fi + 1]);
        acc_a = fma(r, g ? r : 0.0, acc_a);
      }
    }
    // one partial per reduction group of G channels (f0 is a multiple of G)
    if ((f + 1) % G == 0 || f == fn - 1) {
      double acc = acc_a + acc_b;
      acc += __shfl_xor(acc, 32);
      if (g == 0) w.partial[(size_t)((f0 + f) / G) * w.Bpad + b] = acc;
      acc_a = 0.0;
      acc_b = 0.0;
    }
  };

  // A wave finishes one row tile before the next; the other waves of its
  // SIMD overlap their vector work with its matrix work.
  Scal sc = fetch(f0);
  for (int f = 0; f < fn; ++f) {
    const Scal cur = sc;
    sc = fetch(f0 + f + 1);                        // one channel ahead
    Chan C;
    make(cur, f0 + f, C);
    for (int tt = 0; tt < TT; ++tt) {
      i32x4 A[ND][KC];
      i32x16 x0, x1, x2;
      load_A(f, tt, A);
      part1(A, C, x0, x1, x2);
      part2(A, C, x0, x1, x2);
      epi(f, tt, C.e, x0, x1, x2);
    }
    tail(f, C.e);
  }
}

template <int W, int KC, bool PROJ, int OCC, int AM>
__global__ __launch_bounds__(W * 64)
__attribute__((amdgpu_waves_per_eu(OCC, OCC))) void k_mixed(DevModel m, Work w, Chunks cp,
                                                    int G, int nb) {
  mixed_body<W, KC, PROJ, OCC, AM>(m, w, cp, G, nb, blockIdx.x);
}

// The group of workgroup blockIdx.x in launch `which` (0 likelihood, 1 row
// preparation, 2 finalize).  In the likelihood launch groups start at
// multiples of eight, so each group's XCD-aware map sees the XCD numbering a
// launch of its own would.
__device__ inline int group_of_block(const GroupDesc* d, int n, int which) {
  int j = 0;
  while (j + 1 < n && (int)blockIdx.x >= d[j + 1].start[which]) ++j;
  return j;
}

template <int W, int KC, bool PROJ, int OCC, int AM>
__global__ __launch_bounds__(W * 64)
__attribute__((amdgpu_waves_per_eu(OCC, OCC))) void k_mixed_multi(const GroupDesc* __restrict__ d,
                                                          int n) {
  const int j = group_of_block(d, n, 0);
  const int local = (int)blockIdx.x - d[j].start[0];
  const int nb = d[j].nb, nc = d[j].nc;
  if (local >= nb * nc) return;                    // padding to a multiple of eight
  const DevModel m = d[j].m;
  const Work w = d[j].w;
  mixed_body<W, KC, PROJ, OCC, AM>(m, w, Chunks{d[j].fc, d[j].fc, nc, nc}, d[j].G, nb, local);
}

// ---------------------------------------------------------------------------
// plain FP32 model (FP64 residual and chi-square)
//
// The region sum runs as v_mfma_f32_32x32x2_f32 over NPB region pairs (the
// model's pair count rounded up to a compiled size; padded regions have
// K = 0 and unit powers).  The constant T_CMB + A g is added to the FP32 sum
// in the epilogue, then D - M and the chi-square run in FP64.  PROJ: the
// same on the projected rows [sqrt(T) Kbar ; R] held in FP32 (the form the
// mixed kernel describes above), each row's residual its target minus the
// FP32 row product, the peeled last row of R in FP64 from the FP32 power.

template <int W, int NPB, bool AB, bool PROJ>
__global__ __launch_bounds__(W * 64) void k_fp32(DevModel m, Work w, int fc, int G,
                                                 int nb, int nc) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int bt, ch;
  map_block(nb, nc, bt, ch);
  const int TT = PROJ ? m.RT : m.TT, N = m.N;      // 32-row tiles
  const int f0 = ch * fc;
  const int fn = min(fc, m.F - f0);
  const int kfl = NPB * TT * 64;            // floats per channel
  float* s_k = reinterpret_cast<float*>(smem);
  double* s_D = reinterpret_cast<double*>(smem + (size_t)fc * kfl * 4);
  stage(s_k, (PROJ ? m.r32 : m.k32) + (size_t)f0 * kfl, fn * kfl * 4);
  stage(s_D, (PROJ ? m.tg : m.D) + (size_t)f0 * TT * 32, fn * TT * 32 * 8);
  __syncthreads();

  const int g = lane >> 5;
  const int b = bt * (W * 32) + wave * 32 + (lane & 31);
  const RowParams rp = w.rows[b];
  float betaf[NPB];
  float offf[AB ? NPB : 1];                   // log2 alpha (AB)
#pragma unroll
  for (int k = 0; k < NPB; ++k) {
    const int i = 2 * k + g;
    betaf[k] = i < N ? (float)w.betaT[(size_t)i * w.Bpad + b] : 0.0f;
    if constexpr (AB) offf[k] = i < N ? (float)w.offT[(size_t)i * w.Bpad + b] : 0.0f;
  }
  double acc0 = 0.0, acc1 = 0.0;
  for (int f = 0; f < fn; ++f) {
    const int fi = f0 + f;
    const float nl = (float)m.nl2[fi];
    const double c64 = m.t_cmb + rp.A * gauss21(m.nu[fi], rp);
    const float c = (float)c64;
    float Bp[NPB];
#pragma unroll
    for (int k = 0; k < NPB; ++k)
      Bp[k] = __builtin_amdgcn_exp2f(AB ? fmaf(betaf[k], nl, offf[k]) : betaf[k] * nl);
    const float* kf = s_k + (size_t)f * kfl + lane;
    const double* Df = s_D + (size_t)f * TT * 32 + g * 4;
    // projected form: the target of the mean row (row 0, lanes 0..31)
    const double t0 = PROJ ? m.dbar[fi] - m.sqrtT * c64 : 0.0;
    for (int tt = 0; tt < TT; ++tt) {
      float Ak[NPB];
#pragma unroll
      for (int k = 0; k < NPB; ++k) Ak[k] = kf[(k * TT + tt) * 64];
      f32x16 a = {};
#pragma unroll
      for (int k = 0; k < NPB; ++k)
        a = __builtin_amdgcn_mfma_f32_32x32x2f32(Ak[k], Bp[k], a, 0, 0, 0);
      const double* Dt = Df + tt * 32;
      const bool ragged = !PROJ && (tt == TT - 1) && (m.T & 31);
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        double r;
        if constexpr (PROJ) {
          // padded rows have zero operands and zero targets
          double d = Dt[(j >> 2) * 8 + (j & 3)];
          if (j == 0) d = (tt == 0 && g == 0) ? t0 : d;
          r = d - (double)a[j];
        } else {
          r = Dt[(j >> 2) * 8 + (j & 3)] - (double)(a[j] + c);
        }
        if (ragged) {
          const int t = tt * 32 + (j >> 2) * 8 + g * 4 + (j & 3);
          r = t < m.T ? r : 0.0;
        }
        if (j & 1) acc1 = fma(r, r, acc1);
        else acc0 = fma(r, r, acc0);
      }
    }
    if constexpr (PROJ) {
      // peeled last row of R (N a multiple of 32): region N - 1 = 2 kl + 1
      // is pair kl of the lanes with g = 1
      if (m.peel) {
        const int kl = (N - 2) >> 1;
        float pl = 0.0f;
#pragma unroll
        for (int k = 0; k < NPB; ++k) pl = k == kl ? Bp[k] : pl;
        const double r = m.pk[2 * fi + 1] - m.pk[2 * fi] * (double)pl;
        acc0 = fma(r, g ? r : 0.0, acc0);
      }
    }
    // one partial per reduction group of G channels (f0 is a multiple of G)
    if ((f + 1) % G == 0 || f == fn - 1) {
      double acc = acc0 + acc1;
      acc += __shfl_xor(acc, 32);
      if (g == 0) w.partial[(size_t)((f0 + f) / G) * w.Bpad + b] = acc;
      acc0 = 0.0;
      acc1 = 0.0;
    }
  }
}

// ---------------------------------------------------------------------------
// plain FP64 model
//
// v_mfma_f64_16x16x4_f64 over NQB region quads (padded as above; K staged as
// its exact FP32 values and widened in registers), the constant term added in
// the FP64 epilogue.  PROJ: the projected rows (all N + 1 of them, in FP64,
// the gradient kernel's operands), each row's residual its target minus the
// row product.

template <int W, int NQB, bool AB, bool PROJ>
__global__ __launch_bounds__(W * 64) void k_fp64(DevModel m, Work w, int fc, int G,
                                                 int nb, int nc) {
  extern __shared__ __align__(16) unsigned char smem[];
  using AT = typename std::conditional<PROJ, double, float>::type;   // operand type
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int bt, ch;
  map_block(nb, nc, bt, ch);
  const int TT16 = PROJ ? m.RT16 : m.TT16, N = m.N;   // 16-row tiles
  const int drow = PROJ ? m.RT16 * 16 : m.TT * 32;    // targets per channel
  const int f0 = ch * fc;
  const int fn = min(fc, m.F - f0);
  const int kdl = NQB * TT16 * 64;          // values per channel
  double* s_t64 = reinterpret_cast<double*>(smem);                  // [64] 2^(m/64)
  AT* s_k = reinterpret_cast<AT*>(smem + 512);
  double* s_D = reinterpret_cast<double*>(smem + 512 + (size_t)fc * kdl * sizeof(AT));
  stage(s_k, (PROJ ? reinterpret_cast<const AT*>(m.pa64) : reinterpret_cast<const AT*>(m.k64)) +
                 (size_t)f0 * kdl,
        fn * kdl * (int)sizeof(AT));
  stage(s_D, (PROJ ? m.pt64 : m.D) + (size_t)f0 * drow, fn * drow * 8);
  init_t64(s_t64);
  __syncthreads();

  const int g = lane >> 4;                  // 0..3
  const int b = bt * (W * 16) + wave * 16 + (lane & 15);
  const RowParams rp = w.rows[b];
  double beta[NQB];
  double off[AB ? NQB : 1];                   // 64 log2 alpha (AB)
#pragma unroll
  for (int k = 0; k < NQB; ++k) {
    const int i = 4 * k + g;
    beta[k] = i < N ? w.betaT[(size_t)i * w.Bpad + b] : 0.0;
    if constexpr (AB) off[k] = i < N ? 64.0 * w.offT[(size_t)i * w.Bpad + b] : 0.0;
  }
  double acc0 = 0.0, acc1 = 0.0;
  for (int f = 0; f < fn; ++f) {
    const int fi = f0 + f;
    const double nl = m.nl64[fi];             // -64 log2(nu / nu_ref)
    const double z = (m.nu[fi] - rp.nu0) * rp.inv_w;
    const double c = m.t_cmb + rp.A * exp(-0.5 * z * z);
    double Bp[NQB];
#pragma unroll
    for (int k = 0; k < NQB; ++k)
      Bp[k] = pow2_64(AB ? fma(beta[k], nl, off[k]) : beta[k] * nl, s_t64, m);
    const AT* kf = s_k + (size_t)f * kdl + lane;
    // 16x16 FP64 MFMA output: register j of lane l holds row l/16 + 4 j
    const double* Df = s_D + (size_t)f * drow + g;
    // projected form: the target of the mean row (row 0: lanes 0..15, j = 0)
    const double t0 = PROJ ? s_D[(size_t)f * drow] - m.sqrtT * c : 0.0;
    for (int tt = 0; tt < TT16; ++tt) {
      AT Ak[NQB];
#pragma unroll
      for (int k = 0; k < NQB; ++k) Ak[k] = kf[(k * TT16 + tt) * 64];
      f64x4 a = {};
#pragma unroll
      for (int k = 0; k < NQB; ++k)
        a = __builtin_amdgcn_mfma_f64_16x16x4f64((double)Ak[k], Bp[k], a, 0, 0, 0);
      const double* Dt = Df + tt * 16;
      const bool ragged = !PROJ && (tt == TT16 - 1) && (m.T & 15);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        double r;
        if constexpr (PROJ) {
          // padded rows have zero operands and zero targets
          const double d = (j == 0 && tt == 0 && g == 0) ? t0 : Dt[4 * j];
          r = d - a[j];
        } else {
          r = (Dt[4 * j] - c) - a[j];
        }
        if (ragged) {
          const int t = tt * 16 + g + 4 * j;
          r = t < m.T ? r : 0.0;
        }
        if (j & 1) acc1 = fma(r, r, acc1);
        else acc0 = fma(r, r, acc0);
      }
    }
    if ((f + 1) % G == 0 || f == fn - 1) {
      double acc = acc0 + acc1;
      acc += __shfl_xor(acc, 16);
      acc += __shfl_xor(acc, 32);
      if (g == 0) w.partial[(size_t)((f0 + f) / G) * w.Bpad + b] = acc;
      acc0 = 0.0;
      acc1 = 0.0;
    }
  }
}

// ---------------------------------------------------------------------------
// thin models: FP64 on the vector units
//
// For small models (thin_model: few time bins and regions) the matrix tiles
// would be mostly padding, so the model is evaluated per parameter row on
// the vector units: one lane per row, the channel's N powers in FP64, then
// for each time bin the region sum (ascending i), the residual and the
// chi-square, all in FP64.  A power
// 2^y is 2^(j/64) 2^(r/64) with j = round(64 y): 2^floor(j/64) by ldexp,
// 2^((j mod 64)/64) from a 64-entry LDS table and 2^(r/64), |r| <= 1/2, by
// its Taylor series to fifth order (truncation below 4e-17 relative).  K and
// D of the workgroup's channels are staged in LDS and read as broadcasts
// (every lane takes the same channel and time bin).  One partial per row and
// reduction group, as the other kernels.

template <int NT, bool AB>
__device__ __forceinline__ void thin_body(const DevModel& m, const Work& w, int fc, int G,
                                          int nb, int nc, int block) {
  extern __shared__ __align__(16) unsigned char smem[];
  int bt, ch;
  map_block_id(block, nb, nc, bt, ch);
  const int T = m.T, TD = m.TT * 32, N = m.N;
  const int f0 = ch * fc;
  const int fn = min(fc, m.F - f0);
  double* s_t64 = reinterpret_cast<double*>(smem);                   // [64] 2^(m/64)
  float* s_k = reinterpret_cast<float*>(smem + 512);                 // [fc][T][NT]
  double* s_D = reinterpret_cast<double*>(smem + 512 + (size_t)fc * T * NT * 4);   // [fc][TD]
  stage(s_k, m.kthin + (size_t)f0 * T * NT, fn * T * NT * 4);
  stage(s_D, m.D + (size_t)f0 * TD, fn * TD * 8);
  init_t64(s_t64);
  __syncthreads();
  const int b = bt * blockDim.x + threadIdx.x;
  const RowParams rp = w.rows[b];
  double beta[NT];
  double off[AB ? NT : 1];                        // 64 log2 alpha (AB)
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    beta[i] = i < N ? w.betaT[(size_t)i * w.Bpad + b] : 0.0;
    if constexpr (AB) off[i] = i < N ? 64.0 * w.offT[(size_t)i * w.Bpad + b] : 0.0;
  }
  double acc = 0.0;
  for (int f = 0; f < fn; ++f) {
    const int fi = f0 + f;
    const double nl = m.nl64[fi];                 // -64 log2(nu / nu_ref)
    const double z = (m.nu[fi] - rp.nu0) * rp.inv_w;
    const double c = m.t_cmb + rp.A * exp(-0.5 * z * z);
    double P[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i)
      P[i] = pow2_64(AB ? fma(beta[i], nl, off[i]) : beta[i] * nl, s_t64, m);   // 64 log2 P
    const float* kf = s_k + (size_t)f * T * NT;
    const double* Df = s_D + (size_t)f * TD;
    for (int t = 0; t < T; ++t) {
      double msum = 0.0;
#pragma unroll
      for (int i = 0; i < NT; ++i) msum = fma((double)kf[t * NT + i], P[i], msum);
      const double r = (Df[t] - c) - msum;
      acc = fma(r, r, acc);
    }
    // one partial per reduction group of G channels (f0 is a multiple of G)
    if ((f + 1) % G == 0 || f == fn - 1) {
      w.partial[(size_t)((f0 + f) / G) * w.Bpad + b] = acc;
      acc = 0.0;
    }
  }
}

template <int NT, bool AB>
__global__ __launch_bounds__(256) void k_thin64(DevModel m, Work w, int fc, int G, int nb,
                                                int nc) {
  thin_body<NT, AB>(m, w, fc, G, nb, nc, blockIdx.x);
}

template <int NT, bool AB>
__global__ __launch_bounds__(256) void k_thin64_multi(const GroupDesc* __restrict__ d, int n) {
  const int j = group_of_block(d, n, 0);
  const int local = (int)blockIdx.x - d[j].start[0];
  const int nb = d[j].nb, nc = d[j].nc;
  if (local >= nb * nc) return;
  const DevModel m = d[j].m;
  const Work w = d[j].w;
  thin_body<NT, AB>(m, w, d[j].fc, d[j].G, nb, nc, local);
}

// ---------------------------------------------------------------------------
// gradient (FP64)
//
// d lnL / d theta by the chain rule through Eqs. likelihood,
// fast_forward_model and t21model.  With r = D - M on the time grid and
// c_i = alpha P_i the coefficient of region i at channel nu:
//   d lnL / d beta  = (1/sigma^2) sum_nu (-ln(nu/nu_ref)) c_i u_i,
//   d lnL / d alpha = (1/sigma^2) sum_nu P_i u_i,        u_i = sum_t K_i r,
//   d lnL / d A     = (1/sigma^2) sum_nu g rho,          rho = sum_t r,
//   d lnL / d nu21  = (A/(w^2 sigma^2)) sum_nu g (nu - nu21) rho,
//   d lnL / d w     = (A/(w^3 sigma^2)) sum_nu g (nu - nu21)^2 rho,
//   d lnL / d sigma = chi2/sigma^3 - F T/sigma.
// The kernel runs the model of k_fp64 (same operands, same FP64 MFMA) and,
// per 16-bin time tile, the transposed product u += K^T r on the same
// matrix cores: the four residual registers of a lane are the B operands of
// four v_mfma_f64_16x16x4_f64 whose K dimension is the lane group's time
// bins, and the output rows land on the regions whose powers the lane
// already holds (region 4q + g in register j = q mod 4 of group q / 4).  A
// workgroup owns 64 rows for a chunk of channels, restaging K and D every
// `fs` channels, and writes one set of partial sums per (chunk, row).

// Register budgets that compile without spills: three waves per SIMD up to
// 32 regions without amplitude masks, two up to 64 (48 with masks), else
// what the variant needs.
template <int NQB, bool AB>
constexpr int grad_waves() {
  return (!AB && NQB <= 8) ? 3 : (NQB <= (AB ? 12 : 16) ? 2 : 1);
}

template <int W, int NQB, bool AB, bool PROJ>
__global__ __launch_bounds__(W * 64)
__attribute__((amdgpu_waves_per_eu(grad_waves<NQB, AB>()))) void k_grad64(
    DevModel m, Work w, int per, int fs, int nb, int nc) {
  extern __shared__ __align__(16) unsigned char smem[];
  using AT = typename std::conditional<PROJ, double, float>::type;   // operand type
  constexpr int NU = (NQB + 3) / 4;         // 16-region output groups
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int bt, ch;
  map_block(nb, nc, bt, ch);
  const int TR = PROJ ? m.RT16 : m.TT16;    // 16-row tiles of the matrix
  const int N = m.N;
  const int kdl = NQB * TR * 64;            // operand values per channel
  const int drow = PROJ ? m.RT16 * 16 : m.TT * 32;   // targets per channel
  double* s_t64 = reinterpret_cast<double*>(smem);                  // [64] 2^(m/64)
  AT* s_k = reinterpret_cast<AT*>(smem + 512);
  double* s_D = reinterpret_cast<double*>(smem + 512 + (size_t)fs * kdl * sizeof(AT));
  init_t64(s_t64);                          // visible after the first stage's barrier
  const AT* kg = PROJ ? reinterpret_cast<const AT*>(m.pa64) : reinterpret_cast<const AT*>(m.k64);
  const double* dg = PROJ ? m.pt64 : m.D;
  const int g = lane >> 4;                  // 0..3
  const int b = bt * (W * 16) + wave * 16 + (lane & 15);
  const RowParams rp = w.rows[b];
  double beta[NQB];
  double off[AB ? NQB : 1];                 // 64 log2 alpha (AB)
#pragma unroll
  for (int k = 0; k < NQB; ++k) {
    const int i = 4 * k + g;
    beta[k] = i < N ? w.betaT[(size_t)i * w.Bpad + b] : 0.0;
    if constexpr (AB) off[k] = i < N ? 64.0 * w.offT[(size_t)i * w.Bpad + b] : 0.0;
  }
  double s1[NQB], s2[AB ? NQB : 1];
#pragma unroll
  for (int k = 0; k < NQB; ++k) {
    s1[k] = 0.0;
    if constexpr (AB) s2[k] = 0.0;
  }
  double chi_a = 0.0, chi_b = 0.0, h0 = 0.0, h1 = 0.0, h2 = 0.0;
  // the A operand of the transposed product: matrix row 16 tt + 4 j + g and
  // region 16 it + (lane & 15), read from the forward layout
  const int qsub = (lane & 15) >> 2;
  const int tsub = g + 16 * (lane & 3);
  const int c0 = ch * per, c1 = min(m.F, c0 + per);
  for (int cs = c0; cs < c1; cs += fs) {
    const int fn = min(fs, c1 - cs);
    __syncthreads();                        // the previous stage is consumed
    stage(s_k, kg + (size_t)cs * kdl, fn * kdl * (int)sizeof(AT));
    stage(s_D, dg + (size_t)cs * drow, fn * drow * 8);
    __syncthreads();
    for (int f = 0; f < fn; ++f) {
      const int fi = cs + f;
      const double nl = m.nl2[fi];
      const double nl64 = m.nl64[fi];       // 64 nl exactly
      const double dnu = m.nu[fi] - rp.nu0;
      const double z = dnu * rp.inv_w;
      const double gg = exp(-0.5 * z * z);
      const double c = m.t_cmb + rp.A * gg;
      double Bp[NQB];
#pragma unroll
      for (int k = 0; k < NQB; ++k)
        Bp[k] = pow2_64(AB ? fma(beta[k], nl64, off[k]) : beta[k] * nl64, s_t64, m);
      const AT* kf = s_k + (size_t)f * kdl;
      const double* Df = s_D + (size_t)f * drow + g;
      f64x4 u[NU];
#pragma unroll
      for (int it = 0; it < NU; ++it) u[it] = f64x4{0.0, 0.0, 0.0, 0.0};
      double rho = 0.0;
      // projected rows with N a multiple of 16 (and 4 NQB = N): the last row
      // (N) is alone in its tile and holds one entry, R[N-1][N-1] on region
      // N - 1 = 4 (NQB - 1) + 3; it is done in FP64 below instead of as a
      // tile of MFMAs
      const bool peel = PROJ && (N & 15) == 0 && 4 * NQB == N;
      const int TL = peel ? TR - 1 : TR;
      for (int tt = 0; tt < TL; ++tt) {
        AT Ak[NQB];
#pragma unroll
        for (int k = 0; k < NQB; ++k) Ak[k] = kf[(k * TR + tt) * 64 + lane];
        f64x4 a = {};
#pragma unroll
        for (int k = 0; k < NQB; ++k)
          a = __builtin_amdgcn_mfma_f64_16x16x4f64((double)Ak[k], Bp[k], a, 0, 0, 0);
        const double* Dt = Df + tt * 16;
        double r[4];
        if constexpr (PROJ) {
          // targets; row 0 (tile 0, group 0, register 0) is the mean row,
          // whose target sqrt(T) (Dbar - c) depends on the parameter row.
          // Padded rows have zero operands and targets: their e is 0.
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const bool mean_row = tt == 0 && g == 0 && j == 0;
            const double tgt = mean_row ? fma(-m.sqrtT, c, Dt[0]) : Dt[4 * j];
            r[j] = tgt - a[j];
            if (j & 1) chi_b = fma(r[j], r[j], chi_b);
            else chi_a = fma(r[j], r[j], chi_a);
            if (mean_row) rho = m.sqrtT * r[j];   // sum_t r = sqrt(T) e_0
          }
        } else {
          const bool ragged = (tt == TR - 1) && (m.T & 15);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            r[j] = (Dt[4 * j] - c) - a[j];
            if (ragged) {
              const int t = tt * 16 + g + 4 * j;
              r[j] = t < m.T ? r[j] : 0.0;
            }
            if (j & 1) chi_b = fma(r[j], r[j], chi_b);
            else chi_a = fma(r[j], r[j], chi_a);
            rho += r[j];
          }
        }
#pragma unroll
        for (int it = 0; it < NU; ++it) {
          const int q = 4 * it + qsub;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const double at = q < NQB ? (double)kf[(q * TR + tt) * 64 + 4 * j + tsub] : 0.0;
            u[it] = __builtin_amdgcn_mfma_f64_16x16x4f64(at, r[j], u[it], 0, 0, 0);
          }
        }
      }
      if (peel && g == 3) {
        // row N: target z_{N-1}; the entry is read from the forward layout
        // (tile TR - 1, lane 16 * 3: row 16 (TR - 1), region 4 (NQB - 1) + 3)
        const double rl = (double)kf[((NQB - 1) * TR + TR - 1) * 64 + 48];
        const double e = s_D[(size_t)f * drow + N] - rl * Bp[NQB - 1];
        chi_a = fma(e, e, chi_a);
        u[NU - 1][3] = fma(rl, e, u[NU - 1][3]);
      }
      // u[it][j] is region 16 it + 4 j + g = 4 q + g with q = 4 it + j
#pragma unroll
      for (int it = 0; it < NU; ++it)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int q = 4 * it + j;
          if (q < NQB) {
            const double cu = Bp[q] * u[it][j];
            s1[q] = fma(nl, cu, s1[q]);
            if constexpr (AB) s2[q] += cu;
          }
        }
      const double grho = gg * rho;
      h0 += grho;
      h1 = fma(grho, dnu, h1);
      h2 = fma(grho * dnu, dnu, h2);
    }
  }
  // the lane groups hold disjoint matrix rows: chi-square and the 21-cm sums
  // add over them; the region sums are per lane
  double chi = chi_a + chi_b;
  chi += __shfl_xor(chi, 16);
  chi += __shfl_xor(chi, 32);
  h0 += __shfl_xor(h0, 16);
  h0 += __shfl_xor(h0, 32);
  h1 += __shfl_xor(h1, 16);
  h1 += __shfl_xor(h1, 32);
  h2 += __shfl_xor(h2, 16);
  h2 += __shfl_xor(h2, 32);
  const int S = grad_slots(m);
  double* gp = w.gpart + (size_t)ch * S * w.Bpad + b;
  if (g == 0) {
    gp[0] = chi;
    gp[(size_t)1 * w.Bpad] = h0;
    gp[(size_t)2 * w.Bpad] = h1;
    gp[(size_t)3 * w.Bpad] = h2;
  }
#pragma unroll
  for (int q = 0; q < NQB; ++q) {
    const int i = 4 * q + g;
    if (i < N) {
      gp[(size_t)(4 + i) * w.Bpad] = s1[q];
      if constexpr (AB) gp[(size_t)(4 + N + i) * w.Bpad] = s2[q];
    }
  }
}

// Sum the chunk partials of every (slot, row) in chunk order into the
// first chunk's slab; one thread per (slot, row).
__global__ __launch_bounds__(256) void k_grad_reduce(Work w, int S, int chunks) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)S * w.Bpad) return;
  const size_t cs = (size_t)S * w.Bpad;
  double acc = 0.0;
  for (int c = 0; c < chunks; ++c) acc += w.gpart[c * cs + idx];
  w.gpart[idx] = acc;
}

// lnL and the gradient row from the reduced sums, one thread per row.
// Invalid rows get -inf and a NaN gradient.
__global__ __launch_bounds__(256) void k_grad_finalize(DevModel m, Work w, double chi0,
                                                       const double* __restrict__ theta,
                                                       double* __restrict__ out,
                                                       double* __restrict__ grad) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= w.B) return;
  const int P = m.P, N = m.N, NB = m.NB, NA = m.NA;
  const double* gp = w.gpart + b;
  double* gr = grad + (size_t)b * P;
  const RowParams rp = w.rows[b];
  if (!rp.valid) {
    out[b] = -INFINITY;
    for (int k = 0; k < P; ++k) gr[k] = NAN;
    return;
  }
  auto sum = [&](int slot) { return gp[(size_t)slot * w.Bpad]; };
  const double s2 = rp.sigma * rp.sigma;
  const double chi = sum(0) + chi0;
  const double nFT = (double)m.F * (double)m.T;
  out[b] = -0.5 * chi / s2 - 0.5 * nFT * log(2.0 * M_PI * s2);
  for (int k = 0; k < P; ++k) gr[k] = 0.0;
  const double kb = M_LN2 / s2;             // d/d beta: -ln(nu/nu_ref) = ln2 nl2
  for (int r = 0; r < N; ++r) {
    const int ia = r / NB, jb = r - ia * NB;
    gr[jb] += kb * sum(4 + r);
    if (NA > 0) gr[NB + ia] += sum(4 + N + r);
  }
  for (int i = 0; i < NA; ++i) gr[NB + i] = gr[NB + i] / (theta[(size_t)b * P + NB + i] * s2);
  if (!(m.flags & 1u)) {
    const double iw = rp.inv_w;
    gr[P - 4] = sum(1) / s2;
    gr[P - 3] = rp.A * iw * iw * sum(2) / s2;
    gr[P - 2] = rp.A * iw * iw * iw * sum(3) / s2;
  }
  gr[P - 1] = chi / (s2 * rp.sigma) - nFT / rp.sigma;
}

// ---------------------------------------------------------------------------
// row preparation and finalize

// Row preparation: validate, sanitise, expand the spectral indices (and,
// with amplitude masks, log2 of the amplitude scales) to one value per
// region, transposed to [i][b], and record the row constants.  A block of
// 256 threads takes 16 rows: the rows are read coalesced into LDS, sixteen
// threads per row check it and derive its bounds, one of them writes the
// row record, and all threads write the transposed indices in runs of 16
// consecutive rows.  Invalid rows are given harmless values (finalize
// writes -inf for them).

__device__ __forceinline__ void prep_body(const double* __restrict__ theta, int B, int Bpad,
                                          int N, int NA, int NB, int P, unsigned flags,
                                          int betaRows, double* __restrict__ betaT,
                                          double* __restrict__ offT,
                                          RowParams* __restrict__ rows, int block) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* s_th = reinterpret_cast<double*>(smem);                 // [rows][P]
  double* s_fill = s_th + (size_t)kPrepRows * P;                 // [rows] bmin or 0
  double* s_ofill = s_fill + kPrepRows;                          // [rows] omin or 0
  int* s_ok = reinterpret_cast<int*>(s_ofill + kPrepRows);       // [rows]
  const int b0 = block * kPrepRows;
  const int nrow = max(0, min(kPrepRows, B - b0));
  for (int k = threadIdx.x; k < nrow * P; k += blockDim.x)
    s_th[k] = theta[(size_t)b0 * P + k];
  __syncthreads();
  const bool no21 = flags & 1u;
  {
    // sixteen threads per row (r = t / 16): each checks and bounds the
    // entries q, q + 16, ... of the row; xor-shuffles within the sixteen
    // combine them (min, max and "and" do not depend on the order)
    static_assert(kPrepRows * 16 == 256, "sixteen threads per row");
    const int r = threadIdx.x >> 4, q = threadIdx.x & 15;
    const double* th = s_th + (size_t)r * P;
    int ok = r < nrow;
    double bmin = INFINITY, bmax = -INFINITY, omin = INFINITY, omax = -INFINITY;
    if (ok) {
      for (int k = q; k < P; k += 16) ok = ok && isfinite(th[k]);
      for (int j = q; j < NB; j += 16) {
        ok = ok && fabs(th[j]) <= 64.0;
        bmin = fmin(bmin, th[j]);
        bmax = fmax(bmax, th[j]);
      }
      for (int i = q; i < NA; i += 16) {
        ok = ok && th[NB + i] >= 0x1p-32 && th[NB + i] <= 0x1p32;
        const double o = log2(th[NB + i]);
        omin = fmin(omin, o);
        omax = fmax(omax, o);
      }
    }
#pragma unroll
    for (int sh = 8; sh >= 1; sh >>= 1) {
      ok = ok & __shfl_xor(ok, sh);
      bmin = fmin(bmin, __shfl_xor(bmin, sh));
      bmax = fmax(bmax, __shfl_xor(bmax, sh));
      omin = fmin(omin, __shfl_xor(omin, sh));
      omax = fmax(omax, __shfl_xor(omax, sh));
    }
    if (q == 0) {
      if (ok) {
        ok = th[P - 1] > 0.0;
        if (!no21) ok = ok && th[P - 2] > 0.0;
      }
      RowParams rp;
      rp.valid = ok ? 1 : 0;
      rp.pad = 0;
      rp.A = 0.0;
      rp.nu0 = 0.0;
      rp.inv_w = 1.0;
      rp.sigma = 1.0;
      rp.t21 = no21 ? 0.0 : 1.0;
      if (ok) {
        rp.sigma = th[P - 1];
        if (!no21) {
          rp.A = th[P - 4];
          rp.nu0 = th[P - 3];
          rp.inv_w = 1.0 / th[P - 2];
        }
      } else {
        bmin = bmax = 0.0;
      }
      if (!ok || NA == 0) omin = omax = 0.0;
      rp.bmin = bmin;
      rp.bmax = bmax;
      rp.omin = omin;
      rp.omax = omax;
      s_fill[r] = bmin;
      s_ofill[r] = omin;
      s_ok[r] = ok ? 1 : 0;
      if (b0 + r < Bpad) rows[b0 + r] = rp;
    }
  }
  __syncthreads();
  // betaT[i][b]: the index of region i's spectral-index mask for valid rows
  // and i < N, the row's minimum otherwise; offT[i][b] likewise with log2 of
  // the region's amplitude scale
  for (int k = threadIdx.x; k < betaRows * kPrepRows; k += blockDim.x) {
    const int i = k / kPrepRows, r = k - i * kPrepRows;
    if (b0 + r >= Bpad) continue;
    const bool real = s_ok[r] && i < N;
    const int ia = i / NB, jb = i - ia * NB;
    betaT[(size_t)i * Bpad + b0 + r] = real ? s_th[(size_t)r * P + jb] : s_fill[r];
    if (NA > 0)
      offT[(size_t)i * Bpad + b0 + r] = real ? log2(s_th[(size_t)r * P + NB + ia]) : s_ofill[r];
  }
}

__global__ __launch_bounds__(256) void k_prep(const double* __restrict__ theta, int B, int Bpad,
                                              int N, int NA, int NB, int P, unsigned flags,
                                              int betaRows, double* __restrict__ betaT,
                                              double* __restrict__ offT,
                                              RowParams* __restrict__ rows) {
  prep_body(theta, B, Bpad, N, NA, NB, P, flags, betaRows, betaT, offT, rows, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_prep_multi(const GroupDesc* __restrict__ d, int n) {
  const int j = group_of_block(d, n, 1);
  const GroupDesc& g = d[j];
  prep_body(g.theta, g.w.B, g.w.Bpad, g.m.N, g.m.NA, g.m.NB, g.m.P, g.m.flags, g.m.KC * 32,
            g.w.betaT, g.w.offT, g.w.rows, (int)blockIdx.x - g.start[1]);
}

// lnL_b = -chi2_b / (2 sigma^2) - (F T / 2) ln(2 pi sigma^2), with chi2_b
// the sum of the row's partials plus chi0 (a per-model constant of the
// projected form, 0 otherwise).  Sixteen sums per row: sum s adds the
// partials of groups s, s+16, ... in order; then a fixed tree adds the
// sixteen (s with s + 8, then + 4, + 2, + 1), so the result does not depend
// on timing.  (The chain-step kernel adds a row the same way.)  A
// workgroup takes 16 rows: thread t sums s = t / 16 for row t % 16, so a
// wave's loads are runs of 16 consecutive rows.
__device__ __forceinline__ void finalize_body(const double* __restrict__ partial, int ngroup,
                                              int Bpad, const RowParams* __restrict__ rows,
                                              int B, double nFT, double chi0,
                                              double* __restrict__ out, int block) {
  __shared__ double s_acc[16][16];                 // [s][row]
  const int bl = threadIdx.x & 15, s = threadIdx.x >> 4;
  const int b = block * 16 + bl;
  double acc = 0.0;
  if (b < B)
    for (int c = s; c < ngroup; c += 16) acc += partial[(size_t)c * Bpad + b];
  s_acc[s][bl] = acc;
  __syncthreads();
  if (threadIdx.x >= 16 || b >= B) return;
  double v[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = s_acc[k][bl];
#pragma unroll
  for (int h = 8; h >= 1; h >>= 1)
#pragma unroll
    for (int k = 0; k < h; ++k) v[k] = v[k] + v[k + h];
  acc = v[0];
  const RowParams rp = rows[b];
  if (!rp.valid) {
    out[b] = -INFINITY;
    return;
  }
  const double s2 = rp.sigma * rp.sigma;
  out[b] = -0.5 * (acc + chi0) / s2 - 0.5 * nFT * log(2.0 * M_PI * s2);
}

__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ partial, int ngroup,
                                                  int Bpad, const RowParams* __restrict__ rows,
                                                  int B, double nFT, double chi0,
                                                  double* __restrict__ out) {
  finalize_body(partial, ngroup, Bpad, rows, B, nFT, chi0, out, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_finalize_multi(const GroupDesc* __restrict__ d, int n) {
  const int j = group_of_block(d, n, 2);
  const GroupDesc& g = d[j];
  finalize_body(g.w.partial, g.ngroups, g.w.Bpad, g.w.rows, g.w.B, g.nFT, g.chi0, g.out,
                (int)blockIdx.x - g.start[2]);
}

// ---------------------------------------------------------------------------
// launchers

namespace {

std::mutex g_attr_mu;
std::set<const void*> g_attr_done;

// Raise a kernel's dynamic-LDS limit once per process.  The first launch of
// every kernel is eager (graphs capture only repeated calls), so this never
// runs during stream capture.
hipError_t allow_lds(const void* fp) {
  std::lock_guard<std::mutex> lk(g_attr_mu);
  if (g_attr_done.count(fp)) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(fp, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     max_lds_bytes());
  if (e == hipSuccess) g_attr_done.insert(fp);
  return e;
}

// Launch with dynamic LDS.
template <typename KernelT>
hipError_t go(KernelT kern, int blocks, int threads, int lds, hipStream_t s,
              const DevModel& m, const Work& w, int fc, int G, int nb, int nc) {
  hipError_t e = allow_lds(reinterpret_cast<const void*>(kern));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(threads), lds, s, m, w, fc, G, nb, nc);
  return hipGetLastError();
}

// Launch the mixed kernel: nb row tiles times cp.nc channel chunks.
template <typename KernelT>
hipError_t go_mixed(KernelT kern, int nb, int lds, hipStream_t s, const DevModel& m,
                    const Work& w, const Chunks& cp, int G, int threads) {
  hipError_t e = allow_lds(reinterpret_cast<const void*>(kern));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(nb * cp.nc), dim3(threads), lds, s, m, w, cp, G, nb);
  return hipGetLastError();
}

template <int W, int AM>
hipError_t mixed_wa(const DevModel& m, const Work& w, const Chunks& cp, int G, int nb,
                    int occ, int lds, hipStream_t s) {
  const int th = W * 64;
  if (m.proj) {
    switch (m.KC) {
      case 1:
        if constexpr (AM != 1)
          if (occ == 3)
            return go_mixed(k_mixed<W, 1, true, 3, AM>, nb, lds, s, m, w, cp, G, th);
        return go_mixed(k_mixed<W, 1, true, 2, AM>, nb, lds, s, m, w, cp, G, th);
      case 2: return go_mixed(k_mixed<W, 2, true, 2, AM>, nb, lds, s, m, w, cp, G, th);
      case 3: return go_mixed(k_mixed<W, 3, true, 2, AM>, nb, lds, s, m, w, cp, G, th);
      default: return hipErrorInvalidValue;
    }
  }
  switch (m.KC) {
    case 1: return go_mixed(k_mixed<W, 1, false, 2, AM>, nb, lds, s, m, w, cp, G, th);
    case 2: return go_mixed(k_mixed<W, 2, false, 2, AM>, nb, lds, s, m, w, cp, G, th);
    case 3: return go_mixed(k_mixed<W, 3, false, 2, AM>, nb, lds, s, m, w, cp, G, th);
    case 4: return go_mixed(k_mixed<W, 4, false, 2, AM>, nb, lds, s, m, w, cp, G, th);
    default: return hipErrorInvalidValue;
  }
}

template <int W>
hipError_t mixed_w(const DevModel& m, const Work& w, const Chunks& cp, int G, int nb,
                   int occ, int lds, hipStream_t s) {
  if (occ == 3 && !mixed_occ3(m)) return hipErrorInvalidValue;
  switch (mixed_alpha_mode(m)) {
    case 0: return mixed_wa<W, 0>(m, w, cp, G, nb, occ, lds, s);
    case 1: return mixed_wa<W, 1>(m, w, cp, G, nb, occ, lds, s);
    default: return mixed_wa<W, 2>(m, w, cp, G, nb, occ, lds, s);
  }
}

// The projected form needs N <= 96: region pairs up to 48, quads up to 24.
template <int W, bool AB, bool PROJ>
hipError_t fp32_wap(const DevModel& m, const Work& w, int fc, int G, int nb,
                    int nc, int lds, hipStream_t s) {
  const int blocks = nb * nc, th = W * 64;
  switch (m.NP2) {
    case 2: return go(k_fp32<W, 2, AB, PROJ>, blocks, th, lds, s, m, w, fc, G, nb, nc);
    case 4: return go(k_fp32<W, 4, AB, PROJ>, blocks, th, lds, s, m, w, fc, G, nb, nc);
    case 8: return go(k_fp32<W, 8, AB, PROJ>, blocks, th, lds, s, m, w, fc, G, nb, nc);
    case 12: return go(k_fp32<W, 12, AB, PROJ>, blocks, th, lds, s, m, w, fc, G, nb, nc);
    case 16: return go(k_fp32<W, 16, AB, PROJ>, blocks, th, lds, s, m, w, fc, G, nb, nc);
    case 24: return go(k_fp32<W, 24, AB, PROJ>, blocks, th, lds, s, m, w, fc, G, nb, nc);
    case 32: return go(k_fp32<W, 32, AB, PROJ>, blocks, th, lds, s, m, w, fc, G, nb, nc);
    case 48: return go(k_fp32<W, 48, AB, PROJ>, blocks, th, lds, s, m, w, fc, G, nb, nc);
    case 64:
      if constexpr (!PROJ)
        return go(k_fp32<W, 64, AB, false>, blocks, th, lds, s, m, w, fc, G, nb, nc);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template <int W>
hipError_t fp32_w(const DevModel& m, const Work& w, int fc, int G, int nb,
                  int nc, int lds, hipStream_t s) {
  if (m.pplain)
    return m.NA > 0 ? fp32_wap<W, true, true>(m, w, fc, G, nb, nc, lds, s)
                    : fp32_wap<W, false, true>(m, w, fc, G, nb, nc, lds, s);
  return m.NA > 0 ? fp32_wap<W, true, false>(m, w, fc, G, nb, nc, lds, s)
                  : fp32_wap<W, false, false>(m, w, fc, G, nb, nc, lds, s);
}

template <int W, bool AB, bool PROJ>
hipError_t fp64_wap(const DevModel& m, const Work& w, int fc, int G, int nb,
                    int nc, int lds, hipStream_t s) {
  const int blocks = nb * nc, th = W * 64;
  switch (m.NQ) {
    case 1: return go(k_fp64<W, 1, AB, PROJ>, blocks, th, lds, s, m, w, fc, G, nb, nc);
    case 2: return go(k_fp64<W, 2, AB, PROJ>, blocks, th, lds, s, m, w, fc, G, nb, nc);
    case 4: return go(k_fp64<W, 4, AB, PROJ>, blocks, th, lds, s, m, w, fc, G, nb, nc);
    case 6: return go(k_fp64<W, 6, AB, PROJ>, blocks, th, lds, s, m, w, fc, G, nb, nc);
    case 8: return go(k_fp64<W, 8, AB, PROJ>, blocks, th, lds, s, m, w, fc, G, nb, nc);
    case 12: return go(k_fp64<W, 12, AB, PROJ>, blocks, th, lds, s, m, w, fc, G, nb, nc);
    case 16: return go(k_fp64<W, 16, AB, PROJ>, blocks, th, lds, s, m, w, fc, G, nb, nc);
    case 24: return go(k_fp64<W, 24, AB, PROJ>, blocks, th, lds, s, m, w, fc, G, nb, nc);
    case 32:
      if constexpr (!PROJ)
        return go(k_fp64<W, 32, AB, false>, blocks, th, lds, s, m, w, fc, G, nb, nc);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template <int W>
hipError_t fp64_w(const DevModel& m, const Work& w, int fc, int G, int nb,
                  int nc, int lds, hipStream_t s) {
  if (m.pplain)
    return m.NA > 0 ? fp64_wap<W, true, true>(m, w, fc, G, nb, nc, lds, s)
                    : fp64_wap<W, false, true>(m, w, fc, G, nb, nc, lds, s);
  return m.NA > 0 ? fp64_wap<W, true, false>(m, w, fc, G, nb, nc, lds, s)
                  : fp64_wap<W, false, false>(m, w, fc, G, nb, nc, lds, s);
}

template <bool AB>
hipError_t thin_wa(const DevModel& m, const Work& w, int fc, int G, int nb, int nc, int lds,
                   hipStream_t s, int threads) {
  const int blocks = nb * nc;
  switch (m.NT) {
    case 4: return go(k_thin64<4, AB>, blocks, threads, lds, s, m, w, fc, G, nb, nc);
    case 8: return go(k_thin64<8, AB>, blocks, threads, lds, s, m, w, fc, G, nb, nc);
    case 12: return go(k_thin64<12, AB>, blocks, threads, lds, s, m, w, fc, G, nb, nc);
    case 16: return go(k_thin64<16, AB>, blocks, threads, lds, s, m, w, fc, G, nb, nc);
    case 24: return go(k_thin64<24, AB>, blocks, threads, lds, s, m, w, fc, G, nb, nc);
    case 32: return go(k_thin64<32, AB>, blocks, threads, lds, s, m, w, fc, G, nb, nc);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_prep(const DevModel& m, const double* theta, int B,
                       const Work& w, int betaRows, hipStream_t s) {
  const int blocks = (w.Bpad + kPrepRows - 1) / kPrepRows;
  const int lds = kPrepRows * (m.P + 2) * 8 + kPrepRows * 4;
  hipError_t e = allow_lds(reinterpret_cast<const void*>(k_prep));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_prep, dim3(blocks), dim3(256), lds, s, theta, B,
                     w.Bpad, m.N, m.NA, m.NB, m.P, m.flags, betaRows, w.betaT, w.offT,
                     w.rows);
  return hipGetLastError();
}

hipError_t launch_main(Kind k, const DevModel& m, const Work& w,
                       const Tile& tile, hipStream_t s) {
  const int cols = cols_per_wave(k) * tile.waves;
  const int nb = w.Bpad / cols;
  const int nc = n_chunks(m, tile);
  const int lds = lds_bytes(k, m, tile);
  if (w.Bpad % cols != 0 || n_groups(m, tile) > w.ngroup_cap ||
      tile.group < 1 || tile.fc % tile.group != 0 || lds > max_lds_bytes())
    return hipErrorInvalidValue;
  if (k == kThin) {
    // one, two or four waves of 64 rows per workgroup (small batches take
    // fewer, so that more workgroups share the channels)
    if (!m.thin || !(tile.waves == 1 || tile.waves == 2 || tile.waves == 4))
      return hipErrorInvalidValue;
    const int th = 64 * tile.waves;
    return m.NA > 0 ? thin_wa<true>(m, w, tile.fc, tile.group, nb, nc, lds, s, th)
                    : thin_wa<false>(m, w, tile.fc, tile.group, nb, nc, lds, s, th);
  }
  if (k == kMixed) {
    const Chunks cp = chunk_plan(k, m, tile, nb);
    return tile.waves == 8 ? mixed_w<8>(m, w, cp, tile.group, nb, tile.occ, lds, s)
                           : mixed_w<4>(m, w, cp, tile.group, nb, tile.occ, lds, s);
  } else if (k == kFP32) {
    return tile.waves == 8 ? fp32_w<8>(m, w, tile.fc, tile.group, nb, nc, lds, s)
                           : fp32_w<4>(m, w, tile.fc, tile.group, nb, nc, lds, s);
  }
  return tile.waves == 8 ? fp64_w<8>(m, w, tile.fc, tile.group, nb, nc, lds, s)
                         : fp64_w<4>(m, w, tile.fc, tile.group, nb, nc, lds, s);
}

hipError_t launch_finalize(Kind k, const DevModel& m, const Work& w,
                           const Tile& tile, double* out, hipStream_t s) {
  const int threads = 256;
  const int blocks = (w.B * 16 + threads - 1) / threads;
  const double chi0 = chi0_of(k, m);
  hipLaunchKernelGGL(k_finalize, dim3(blocks), dim3(threads), 0, s, w.partial,
                     n_groups(m, tile), w.Bpad, w.rows, w.B,
                     (double)m.F * (double)m.T, chi0, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// launches shared by several models (serving)
//
// Models whose likelihood kernel is the same compiled variant share one
// launch of each of the three kernels; every workgroup finds its group in
// the descriptor table and runs what a launch of its own would run, so each
// row's result is bitwise the one it gets alone.  Sharing covers the
// variants the default tiles of models without amplitude masks use: the
// mixed kernel with 8 waves and one or two region chunks (both forms, both
// register budgets) and the thin kernel.

namespace {

template <typename KernelT>
hipError_t go_multi(KernelT kern, int blocks, int threads, int lds, hipStream_t s,
                    const GroupDesc* d, int n) {
  hipError_t e = allow_lds(reinterpret_cast<const void*>(kern));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(threads), lds, s, d, n);
  return hipGetLastError();
}

hipError_t main_multi(Kind k, const DevModel& m, const Tile& t, const GroupDesc* d, int n,
                      int blocks, int lds, hipStream_t s) {
  if (k == kMixed) {
    const int th = 8 * 64;
    if (m.proj && m.KC == 1 && t.occ == 3)
      return go_multi(k_mixed_multi<8, 1, true, 3, 0>, blocks, th, lds, s, d, n);
    if (m.proj && m.KC == 1) return go_multi(k_mixed_multi<8, 1, true, 2, 0>, blocks, th, lds, s, d, n);
    if (m.proj) return go_multi(k_mixed_multi<8, 2, true, 2, 0>, blocks, th, lds, s, d, n);
    if (m.KC == 1) return go_multi(k_mixed_multi<8, 1, false, 2, 0>, blocks, th, lds, s, d, n);
    return go_multi(k_mixed_multi<8, 2, false, 2, 0>, blocks, th, lds, s, d, n);
  }
  const int th = 64 * t.waves;
  switch (m.NT) {
    case 4: return go_multi(k_thin64_multi<4, false>, blocks, th, lds, s, d, n);
    case 8: return go_multi(k_thin64_multi<8, false>, blocks, th, lds, s, d, n);
    case 12: return go_multi(k_thin64_multi<12, false>, blocks, th, lds, s, d, n);
    case 16: return go_multi(k_thin64_multi<16, false>, blocks, th, lds, s, d, n);
    case 24: return go_multi(k_thin64_multi<24, false>, blocks, th, lds, s, d, n);
    case 32: return go_multi(k_thin64_multi<32, false>, blocks, th, lds, s, d, n);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_groups(Kind k, const DevModel& m0, const Tile& tile, const GroupDesc* d,
                         int n, const int grid[3], int lds, hipStream_t s) {
  if (n < 1 || n > kMaxGroups || variant_of(k, m0, tile) == 0 || lds > max_lds_bytes())
    return hipErrorInvalidValue;
  // row preparation: the LDS of the widest row (at most 128 + 4 parameters)
  const int plds = kPrepRows * ((kMixedMaxN + 4) + 2) * 8 + kPrepRows * 4;
  hipError_t e = go_multi(k_prep_multi, grid[1], 256, plds, s, d, n);
  if (e != hipSuccess) return e;
  if ((e = main_multi(k, m0, tile, d, n, grid[0], lds, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_finalize_multi, dim3(grid[2]), dim3(256), 0, s, d, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// gradient launchers

namespace {

template <bool AB, bool PROJ>
hipError_t grad_wa(const DevModel& m, const Work& w, const GradShape& gs, hipStream_t s) {
  const int blocks = gs.nb * gs.chunks, th = 4 * 64;
#define G64(Q)                                                                            \
  case Q: {                                                                               \
    hipError_t e = allow_lds(reinterpret_cast<const void*>(k_grad64<4, Q, AB, PROJ>));    \
    if (e != hipSuccess) return e;                                                        \
    hipLaunchKernelGGL((k_grad64<4, Q, AB, PROJ>), dim3(blocks), dim3(th), gs.lds, s, m,  \
                       w, gs.per, gs.fs, gs.nb, gs.chunks);                               \
    return hipGetLastError();                                                             \
  }
  switch (m.NQ) {
    G64(1) G64(2) G64(4) G64(6) G64(8) G64(12) G64(16) G64(24) G64(32)
    default: return hipErrorInvalidValue;
  }
#undef G64
}

}  // namespace

hipError_t launch_grad(const DevModel& m, const Work& w, const GradShape& g, hipStream_t s) {
  if (w.Bpad % 64 != 0 || g.lds > max_lds_bytes() || !w.gpart) return hipErrorInvalidValue;
  if (m.proj)
    return m.NA > 0 ? grad_wa<true, true>(m, w, g, s) : grad_wa<false, true>(m, w, g, s);
  return m.NA > 0 ? grad_wa<true, false>(m, w, g, s) : grad_wa<false, false>(m, w, g, s);
}

hipError_t launch_grad_finalize(const DevModel& m, const Work& w, const GradShape& g,
                                const double* theta, double* out, double* grad,
                                hipStream_t s) {
  const int S = grad_slots(m);
  const size_t n = (size_t)S * w.Bpad;
  hipLaunchKernelGGL(k_grad_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, S,
                     g.chunks);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int blocks = (w.B + 255) / 256;
  const double chi0 = m.proj ? m.chi0 : 0.0;
  hipLaunchKernelGGL(k_grad_finalize, dim3(blocks), dim3(256), 0, s, m, w, chi0, theta, out,
                     grad);
  return hipGetLastError();
}

}  // namespace fgl
