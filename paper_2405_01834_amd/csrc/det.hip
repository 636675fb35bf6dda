// det.hip -- the order-independent accumulation of the J and K builds and
// of the gradient.
// Every image v reaching an element of K' or J' is scaled by a power of two
// s and held as the fixed-point number floor(v s) + f 2^-32, f = the rounded
// fraction, in two 64-bit integer words that integer atomics add; integer
// sums are associative, so the result does not depend on which wave adds
// first.  s is chosen so that the sum of the magnitudes reaching one element
// stays below 2^62: |(ab|cd)| <= Q_ab Q_cd <= Q_max^2 (Cauchy-Schwarz), each
// element of K' or J' collects at most twice sum_bd |(ab|cd)| |D_bd| (weights
// of the permutational images at most 1, both images of a pair), so B =
// 4 Q_max^2 sum |D| bounds it and s = 2^(62 - ceil(log2 B)).
#include <cmath>

#include "device_common.h"

namespace mderi {

namespace {

constexpr int kDetBlocks = 512;
constexpr int kDetThreads = 256;

// Fixed-order tree sum over a workgroup of kDetThreads lanes.
__device__ double block_sum(double v, double *lds) {
  lds[threadIdx.x] = v;
  __syncthreads();
  for (int h = kDetThreads / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) lds[threadIdx.x] += lds[threadIdx.x + h];
    __syncthreads();
  }
  return lds[0];
}

__global__ void __launch_bounds__(kDetThreads) abs_partial_kernel(size_t n, const double *__restrict__ D,
                                                                  double *__restrict__ work) {
  __shared__ double lds[kDetThreads];
  double s = 0.0;
  for (size_t e = (size_t)blockIdx.x * kDetThreads + threadIdx.x; e < n; e += (size_t)kDetBlocks * kDetThreads)
    s += fabs(D[e]);
  const double t = block_sum(s, lds);
  if (threadIdx.x == 0) work[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kDetThreads) det_scale_kernel(const double *__restrict__ work, double qmax,
                                                                double *__restrict__ scale) {
  __shared__ double lds[kDetThreads];
  double s = 0.0;
  for (int b = threadIdx.x; b < kDetBlocks; b += kDetThreads) s += work[b];
  const double sum = block_sum(s, lds);
  if (threadIdx.x != 0) return;
  const double B = 4.0 * qmax * qmax * sum;
  double sc = 1.0;
  if (B > 0.0 && B <= 1.7e308) {
    int E;
    const double m = frexp(B, &E);          // B = m 2^E, m in [0.5, 1)
    const int c = (m == 0.5) ? E - 1 : E;   // ceil(log2 B)
    sc = ldexp(1.0, min(1000, max(-1000, 62 - c)));
  }
  scale[0] = sc;
}

// The value of one fixed-point pair: floor words and fraction words are
// summed separately; the fraction sum's carries move into the integer part.
__device__ __forceinline__ double fixed_value(const unsigned long long *p) {
  const unsigned long long lo = p[1];
  const long long hi = (long long)p[0] + (long long)(lo >> 32);
  return (double)hi + (double)(lo & 0xffffffffull) * 0x1p-32;
}

__global__ void __launch_bounds__(256) symmetrize_fixed_kernel(int n, const unsigned long long *__restrict__ in,
                                                               const double *__restrict__ scale,
                                                               double *__restrict__ out) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * n) return;
  const size_t r = e / n, c = e - r * n;
  const double inv = 1.0 / scale[0];  // a power of two: exact
  out[e] = (fixed_value(in + 2 * e) + fixed_value(in + 2 * (c * n + r))) * inv;
}

// Gradient copies in four-digit fixed point (digit k of weight 2^(32 k - 80),
// each word the signed sum of that digit over the adds): the copies are
// summed word by word as integers, the carries moved up (arithmetic shifts),
// a negative total negated digit-wise so its magnitude is a sum of
// non-negative terms, and the magnitude rounded once to double.
__global__ void __launch_bounds__(256) sum_copies_fixed_kernel(int n, int copies,
                                                               const unsigned long long *__restrict__ in,
                                                               double *__restrict__ out, int accumulate) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  long long w[4] = {0, 0, 0, 0};
  for (int c = 0; c < copies; ++c)
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] += (long long)in[4 * ((size_t)c * n + i) + k];
  const long long m32 = 0xffffffffll;
  auto carry = [&]() {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      w[k + 1] += w[k] >> 32;
      w[k] &= m32;
    }
  };
  carry();  // w[0..2] in [0, 2^32), w[3] signed
  const bool neg = w[3] < 0;
  if (neg) {
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = -w[k];
    carry();
  }
  const double mag = (double)w[3] * 0x1p16 + (double)w[2] * 0x1p-16 + (double)w[1] * 0x1p-48 + (double)w[0] * 0x1p-80;
  const double v = neg ? -mag : mag;
  out[i] = accumulate ? out[i] + v : v;
}

__global__ void zero_u64_kernel(size_t n, unsigned long long *__restrict__ x) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    x[e] = 0ull;
}

}  // namespace

size_t det_scale_work_doubles() { return kDetBlocks; }

hipError_t launch_det_scale(size_t n, const double *D, double qmax, double *work, double *scale, hipStream_t s) {
  hipLaunchKernelGGL(abs_partial_kernel, dim3(kDetBlocks), dim3(kDetThreads), 0, s, n, D, work);
  hipLaunchKernelGGL(det_scale_kernel, dim3(1), dim3(kDetThreads), 0, s, (const double *)work, qmax, scale);
  return hipGetLastError();
}

hipError_t launch_symmetrize_fixed(int n, const unsigned long long *in, const double *scale, double *out,
                                   hipStream_t s) {
  const size_t tot = (size_t)n * n;
  if (!tot) return hipSuccess;
  hipLaunchKernelGGL(symmetrize_fixed_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, in, scale,
                     out);
  return hipGetLastError();
}

hipError_t launch_sum_copies_fixed(int n, int copies, const unsigned long long *in, double *out, int accumulate,
                                   hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(sum_copies_fixed_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, copies, in, out, accumulate);
  return hipGetLastError();
}

hipError_t launch_zero_u64(size_t n, unsigned long long *x, hipStream_t s) {
  if (!n) return hipSuccess;
  const size_t blocks = (n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536;
  hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)blocks), dim3(256), 0, s, n, x);
  return hipGetLastError();
}

}  // namespace mderi
