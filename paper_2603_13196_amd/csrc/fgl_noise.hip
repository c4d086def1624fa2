// Residual-likelihood reference distribution of the accuracy criterion
// (Tutt et al., Sec. 5): the likelihood of Eq. likelihood over data sets that
// the model describes exactly up to uncorrelated Gaussian noise, and the
// lower-tail fraction q of a fit's median likelihood within it.
//
// For data = M(theta) + e the residual at theta is e itself, so realisation r
// has lnL_r = -(sigma_noise^2 / (2 sigma_like^2)) S_r - (n/2) ln(2 pi
// sigma_like^2) with S_r = sum_k z_rk^2 over its n standard normals.  The
// normals come from Philox4x32-10 (Salmon et al., SC 2011; key (seed low
// word, seed high word), block b of stream s on counter (b, r, s, 'nois'))
// through the Box-Muller transform with 32-bit uniforms: pair j takes u1 from
// word j % 4 of stream-0 block j / 4 and u2 from the same word of stream 1.
// The two normals of a pair have z0^2 + z1^2 = -2 ln u1, so a full pair adds
// -2 ln u1 to S and needs neither u2 nor any trigonometry: only the stream-0
// words are drawn, four pairs (eight normals) per block, and stream 1 and the
// cosine are touched only for a pair cut by the end of an odd-length
// realisation.
//
// k_noise_lnl: one workgroup per realisation.  Each thread walks its
// stream-0 blocks keeping the product of its u1 values as mantissa and
// binary exponent (frexp after every block; u1 >= 2^-32, so four factors
// never underflow) and takes one logarithm at the end: per block the work
// is the generator (twenty 32x32-bit products) and four multiplies.  The
// per-thread sums meet in a fixed shuffle-and-LDS tree.  Nothing is read
// from memory; the kernel is bound by the generator's integer multiplies.
//
// k_noise_q: one workgroup per fit; its threads count the reference values at
// or below the fit's lnL in a fixed tree, and q = count / R.
#include "fgl_host.h"
#include "fgl_philox.h"

#include <cmath>

namespace fgl {

namespace {

constexpr int kNoiseThreads = 256;
constexpr int kNoiseMaxGroups = 1 << 23;           // R and nb: grids well below 2^32 work-items
constexpr int64_t kNoiseMaxN = (int64_t)1 << 31;    // residuals per data set
constexpr double kNoiseMaxNormals = 1099511627776.0;  // 2^40 per call: about 2 s of work
constexpr uint32_t kNoiseTag = 0x6e6f6973u;          // counter word 3 ('nois')

// Block b of stream s of realisation r.
__device__ inline void noise_block(uint32_t b, uint32_t r, uint32_t s, uint64_t seed,
                                   uint32_t x[4]) {
  x[0] = b;
  x[1] = r;
  x[2] = s;
  x[3] = kNoiseTag;
  philox4x32(x, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// word j (0..3) of a block, without indexing the array at run time
__device__ inline uint32_t word(const uint32_t x[4], int j) {
  return j == 0 ? x[0] : j == 1 ? x[1] : j == 2 ? x[2] : x[3];
}

__device__ inline double u_open0(uint32_t w) {   // (0, 1]
  return ((double)w + 1.0) * 0x1p-32;
}
__device__ inline double u_open1(uint32_t w) {   // [0, 1)
  return (double)w * 0x1p-32;
}

// lnL of realisations 0..R-1, one per workgroup.
__global__ __launch_bounds__(kNoiseThreads) void k_noise_lnl(int64_t n, uint64_t seed,
                                                             double sigma_noise,
                                                             double sigma_like, double* out) {
  const uint64_t r = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t npair = n >> 1;                 // pairs whose two normals both count
  const int64_t nfull = npair >> 2;             // stream-0 blocks of four such pairs
  double p = 1.0;                               // product of u1, times 2^-e
  int e = 0;
  for (int64_t b = tid; b < nfull; b += kNoiseThreads) {
    uint32_t x[4];
    noise_block((uint32_t)b, (uint32_t)r, 0u, seed, x);
    // u1 = (w + 1) 2^-32: p (w + 1) as one fma, the 2^-32 in the exponent
    // (scaling by a power of two does not change a rounding)
    p = fma(p, (double)x[0], p);
    p = fma(p, (double)x[1], p);
    p = fma(p, (double)x[2], p);
    p = fma(p, (double)x[3], p);
    int ex;
    p = frexp(p, &ex);
    e += ex - 128;
  }
  // S contribution of the full pairs: -2 sum ln u1
  double s = -2.0 * (log(p) + (double)e * 0.69314718055994530942);
  const int rem = (int)(npair & 3);             // full pairs in the last block
  const bool odd = n & 1;                       // and a pair cut in half
  if ((rem || odd) && tid == 0) {
    uint32_t x[4];
    noise_block((uint32_t)nfull, (uint32_t)r, 0u, seed, x);
    for (int j = 0; j < rem; ++j) s += -2.0 * log(u_open0(word(x, j)));
    if (odd) {
      uint32_t y[4];
      noise_block((uint32_t)nfull, (uint32_t)r, 1u, seed, y);
      const double c = cospi(2.0 * u_open1(word(y, rem)));
      s += -2.0 * log(u_open0(word(x, rem))) * c * c;
    }
  }
  for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m);
  __shared__ double part[kNoiseThreads / 64];
  if ((tid & 63) == 0) part[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) {
    const double S = (part[0] + part[1]) + (part[2] + part[3]);
    const double v = sigma_like * sigma_like;
    out[r] = -(sigma_noise * sigma_noise) / (2.0 * v) * S -
             0.5 * (double)n * log(6.28318530717958647693 * v);
  }
}

// q[i] = #{r : ref[r] <= lbar[i]} / R, one workgroup per i.
__global__ __launch_bounds__(kNoiseThreads) void k_noise_q(const double* __restrict__ ref, int R,
                                                           const double* __restrict__ lbar,
                                                           double* __restrict__ q) {
  const int i = blockIdx.x, tid = threadIdx.x;
  const double x = lbar[i];
  int c = 0;
  for (int64_t r = tid; r < R; r += kNoiseThreads) c += ref[r] <= x ? 1 : 0;
  for (int m = 32; m >= 1; m >>= 1) c += __shfl_xor(c, m);
  __shared__ int part[kNoiseThreads / 64];
  if ((tid & 63) == 0) part[tid >> 6] = c;
  __syncthreads();
  if (tid == 0) q[i] = (double)((part[0] + part[1]) + (part[2] + part[3])) / (double)R;
}

// Device buffers and a stream for one synchronous call.
struct Call {
  hipStream_t s = nullptr;
  void* buf[3] = {nullptr, nullptr, nullptr};
  ~Call() {
    if (s) (void)hipStreamSynchronize(s);
    for (void* b : buf)
      if (b) (void)hipFree(b);
    if (s) (void)hipStreamDestroy(s);
  }
  int open() {
    int dev = 0;
    const int rc = check_device(&dev);
    if (rc != FGL_OK) return rc;
    const hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) {
      s = nullptr;
      return hip_err(e, "hipStreamCreate");
    }
    return FGL_OK;
  }
  int alloc(int k, size_t bytes) {
    const hipError_t e = hipMalloc(&buf[k], bytes);
    if (e != hipSuccess) {
      buf[k] = nullptr;
      return hip_err(e, "hipMalloc");
    }
    return FGL_OK;
  }
};

}  // namespace

}  // namespace fgl

using namespace fgl;

extern "C" {

int fgl_noise_loglike(int64_t n, int R, double sigma_noise, double sigma_like, uint64_t seed,
                      double* lnl, double* kernel_ms) {
  TraceRange tr("fgl_noise_loglike n=%lld R=%d", (long long)n, R);
  if (!lnl) return set_err(FGL_EINVAL, "lnl is NULL");
  if (n < 1 || n > kNoiseMaxN) return set_err(FGL_EINVAL, "n=%lld outside 1..2^31", (long long)n);
  if (R < 1 || R > kNoiseMaxGroups)
    return set_err(FGL_EINVAL, "R=%d outside 1..%d", R, kNoiseMaxGroups);
  if ((double)n * (double)R > kNoiseMaxNormals)
    return set_err(FGL_EINVAL, "n R = %.3g normals exceeds 2^40 in one call", (double)n * R);
  if (!(sigma_noise >= 0.0) || !std::isfinite(sigma_noise) || !(sigma_like > 0.0) ||
      !std::isfinite(sigma_like))
    return set_err(FGL_EINVAL, "need finite sigma_noise >= 0 and sigma_like > 0");
  Call c;
  int rc = c.open();
  if (rc == FGL_OK) rc = c.alloc(0, (size_t)R * 8);
  if (rc != FGL_OK) return rc;
  double* d_out = static_cast<double*>(c.buf[0]);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (kernel_ms) {
    // timing only: no system-scope fence around the kernel
    (void)hipEventCreateWithFlags(&e0, hipEventDisableSystemFence);
    (void)hipEventCreateWithFlags(&e1, hipEventDisableSystemFence);
    (void)hipEventRecord(e0, c.s);
  }
  hipLaunchKernelGGL(k_noise_lnl, dim3(R), dim3(kNoiseThreads), 0, c.s, n, seed, sigma_noise,
                     sigma_like, d_out);
  hipError_t e = hipGetLastError();
  if (kernel_ms && e == hipSuccess) (void)hipEventRecord(e1, c.s);
  if (e == hipSuccess) e = hipMemcpyAsync(lnl, d_out, (size_t)R * 8, hipMemcpyDeviceToHost, c.s);
  if (e == hipSuccess) e = hipStreamSynchronize(c.s);
  if (kernel_ms && e == hipSuccess) {
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    *kernel_ms = ms;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return e == hipSuccess ? FGL_OK : hip_err(e, "noise likelihood kernel");
}

int fgl_noise_quantile(const double* lnl_noise, int R, const double* lbar, int nb, double* q) {
  if (!lnl_noise || !lbar || !q) return set_err(FGL_EINVAL, "arrays must be non-NULL");
  if (R < 1 || nb < 1 || nb > kNoiseMaxGroups)
    return set_err(FGL_EINVAL, "need R >= 1 and nb in 1..%d", kNoiseMaxGroups);
  Call c;
  int rc = c.open();
  if (rc == FGL_OK) rc = c.alloc(0, (size_t)R * 8);
  if (rc == FGL_OK) rc = c.alloc(1, (size_t)nb * 8);
  if (rc == FGL_OK) rc = c.alloc(2, (size_t)nb * 8);
  if (rc != FGL_OK) return rc;
  double* d_ref = static_cast<double*>(c.buf[0]);
  double* d_lbar = static_cast<double*>(c.buf[1]);
  double* d_q = static_cast<double*>(c.buf[2]);
  hipError_t e = hipMemcpyAsync(d_ref, lnl_noise, (size_t)R * 8, hipMemcpyHostToDevice, c.s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_lbar, lbar, (size_t)nb * 8, hipMemcpyHostToDevice, c.s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_noise_q, dim3(nb), dim3(kNoiseThreads), 0, c.s, d_ref, R, d_lbar, d_q);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(q, d_q, (size_t)nb * 8, hipMemcpyDeviceToHost, c.s);
  if (e == hipSuccess) e = hipStreamSynchronize(c.s);
  return e == hipSuccess ? FGL_OK : hip_err(e, "noise quantile kernel");
}

}  // extern "C"
