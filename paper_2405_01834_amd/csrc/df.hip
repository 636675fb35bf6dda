// df.hip -- the contractions of density-fitted Coulomb (the use of 3-centre
// integrals that Sec. 1 motivates): with B the (ab|P) matrix (rows = AO pairs
// of the canonical shell pairs, columns = auxiliary AOs, column-major) and M
// the metric (P|Q),
//   gamma_Q = sum_rows B[row][Q] w_row D[a_row][b_row]      (the fitted charge)
//   c = M^{-1} gamma                                        (library Cholesky)
//   J[a][b] = J[b][a] = sum_Q B[row][Q] c_Q                 (every pair row)
// and for density-fitted exchange the solved B' = B L^{-T} (M = L L^T)
// spread over all AO pairs (df_expand) for the two GEMMs of the K build.
// w_row = 2 for rows of a pair of two different shells (the pair stands for
// both orders), 1 on a diagonal shell pair.
#include <algorithm>

#include "device_common.h"

namespace mderi {

namespace {

constexpr int kDfThreads = 256;

// dvec[row] = w_row D[a][b]
__global__ void __launch_bounds__(kDfThreads) df_dvec_kernel(int nrow, const int2 *ab, const double *w,
                                                            const double *D, int nao, double *dvec) {
  const int r = blockIdx.x * kDfThreads + threadIdx.x;
  if (r >= nrow) return;
  const int2 x = ab[r];
  dvec[r] = w[r] * D[(size_t)x.x * nao + x.y];
}

// gamma[col] = sum_row B[row + nrow col] dvec[row]: one workgroup per column,
// consecutive rows across the workgroup's threads (each wave reads 512
// contiguous bytes per step), four independent partial sums per thread so
// that four loads are in flight, then a fixed-order tree in LDS.
__global__ void __launch_bounds__(kDfThreads) df_gamma_kernel(int nrow, const double *B, const double *dvec,
                                                             double *gamma) {
  __shared__ double part[kDfThreads];
  const int col = blockIdx.x;
  const double *Bc = B + (size_t)nrow * col;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  constexpr int step = 4 * kDfThreads;
  int r = threadIdx.x;
  for (; r + 3 * kDfThreads < nrow; r += step) {
    s0 = fma(Bc[r], dvec[r], s0);
    s1 = fma(Bc[r + kDfThreads], dvec[r + kDfThreads], s1);
    s2 = fma(Bc[r + 2 * kDfThreads], dvec[r + 2 * kDfThreads], s2);
    s3 = fma(Bc[r + 3 * kDfThreads], dvec[r + 3 * kDfThreads], s3);
  }
  for (; r < nrow; r += kDfThreads) s0 = fma(Bc[r], dvec[r], s0);
  part[threadIdx.x] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  for (int h = kDfThreads / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) gamma[col] = part[0];
}

// J rows: jr = sum_col B[row + nrow col] c[col], then J[a][b] = J[b][a] = jr
// from the rows with a >= b (a diagonal shell pair holds both (a, b) and
// (b, a), equal up to rounding; the other pairs have a > b throughout), so
// every element has one writer and J is exactly symmetric.  A workgroup takes
// kJRows consecutive rows; its kJParts waves split the columns (wave w takes
// col = w mod kJParts, two partial sums each) and the parts are added in a
// fixed order.
constexpr int kJRows = 64, kJParts = kDfThreads / kJRows;

__global__ void __launch_bounds__(kDfThreads) df_j_kernel(int nrow, int ncol, const double *B, const double *c,
                                                         const int2 *ab, double *J, int nao) {
  __shared__ double part[kJParts][kJRows];
  const int lane = threadIdx.x % kJRows, w = threadIdx.x / kJRows;
  const int r = blockIdx.x * kJRows + lane;
  double s0 = 0.0, s1 = 0.0;
  if (r < nrow) {
    const double *Br = B + r;
    int k = w;
    for (; k + kJParts < ncol; k += 2 * kJParts) {
      s0 = fma(Br[(size_t)nrow * k], c[k], s0);
      s1 = fma(Br[(size_t)nrow * (k + kJParts)], c[k + kJParts], s1);
    }
    if (k < ncol) s0 = fma(Br[(size_t)nrow * k], c[k], s0);
  }
  part[w][lane] = s0 + s1;
  __syncthreads();
  if (w != 0 || r >= nrow) return;
  double s = part[0][lane];
  for (int q = 1; q < kJParts; ++q) s += part[q][lane];
  const int2 x = ab[r];
  if (x.x < x.y) return;
  J[(size_t)x.x * nao + x.y] = s;
  J[(size_t)x.y * nao + x.x] = s;
}

// One class batch of the metric, V[i + na (ma + Na (mc + Nc k))], into the
// column-major metric M[row + n col] (row = first AO of shell A_i + ma, col =
// first AO of shell C_k + mc).
__global__ void __launch_bounds__(kDfThreads) df_scatter_kernel(int na, int Na, int nc, int Nc, const double *V,
                                                               const int *shells_a, const int *shells_c,
                                                               const int *ao_off, double *M, int n) {
  const long total = (long)na * Na * Nc * nc;
  for (long e = (long)blockIdx.x * kDfThreads + threadIdx.x; e < total; e += (long)gridDim.x * kDfThreads) {
    long q = e;
    const int i = (int)(q % na);
    q /= na;
    const int ma = (int)(q % Na);
    q /= Na;
    const int mc = (int)(q % Nc);
    const int k = (int)(q / Nc);
    M[(size_t)(ao_off[shells_a[i]] + ma) + (size_t)n * (ao_off[shells_c[k]] + mc)] = V[e];
  }
}

// The solved (ab|P) matrix B' (column-major, rows = AO pairs of the
// canonical shell pairs) spread over all AO pairs: Bt[(a naux + Q) nao + b] =
// B'[row of (a, b)][Q], and the transposed element too for the rows of a pair
// of two shells (w = 2; a diagonal shell pair holds both orders as rows).
__global__ void __launch_bounds__(kDfThreads) df_expand_kernel(int nrow, int ncol, const double *B, const int2 *ab,
                                                              const double *w, int nao, double *Bt) {
  const size_t total = (size_t)nrow * ncol;
  for (size_t e = (size_t)blockIdx.x * kDfThreads + threadIdx.x; e < total; e += (size_t)gridDim.x * kDfThreads) {
    const int r = (int)(e % nrow), q = (int)(e / nrow);
    const int2 x = ab[r];
    const double v = B[e];
    Bt[((size_t)x.x * ncol + q) * nao + x.y] = v;
    if (w[r] > 1.0) Bt[((size_t)x.y * ncol + q) * nao + x.x] = v;
  }
}

}  // namespace

hipError_t launch_df_expand(int nrow, int ncol, const double *B, const int2 *ab, const double *w, int nao, double *Bt,
                            hipStream_t s) {
  const size_t total = (size_t)nrow * ncol;
  if (!total) return hipSuccess;
  const int grid = (int)std::min<size_t>(65536, (total + kDfThreads - 1) / kDfThreads);
  hipLaunchKernelGGL(df_expand_kernel, dim3(grid), dim3(kDfThreads), 0, s, nrow, ncol, B, ab, w, nao, Bt);
  return hipGetLastError();
}

hipError_t launch_df_dvec(int nrow, const int2 *ab, const double *w, const double *D, int nao, double *dvec,
                          hipStream_t s) {
  if (nrow <= 0) return hipSuccess;
  hipLaunchKernelGGL(df_dvec_kernel, dim3((nrow + kDfThreads - 1) / kDfThreads), dim3(kDfThreads), 0, s, nrow, ab, w,
                     D, nao, dvec);
  return hipGetLastError();
}

hipError_t launch_df_gamma(int nrow, int ncol, const double *B, const double *dvec, double *gamma, hipStream_t s) {
  if (ncol <= 0) return hipSuccess;
  hipLaunchKernelGGL(df_gamma_kernel, dim3(ncol), dim3(kDfThreads), 0, s, nrow, B, dvec, gamma);
  return hipGetLastError();
}

hipError_t launch_df_j(int nrow, int ncol, const double *B, const double *c, const int2 *ab, double *J, int nao,
                       hipStream_t s) {
  if (nrow <= 0) return hipSuccess;
  hipLaunchKernelGGL(df_j_kernel, dim3((nrow + kJRows - 1) / kJRows), dim3(kDfThreads), 0, s, nrow, ncol, B, c, ab, J,
                     nao);
  return hipGetLastError();
}

hipError_t launch_df_scatter(int na, int Na, int nc, int Nc, const double *V, const int *shells_a, const int *shells_c,
                             const int *ao_off, double *M, int n, hipStream_t s) {
  const long total = (long)na * Na * Nc * nc;
  if (total <= 0) return hipSuccess;
  const int grid = (int)std::min<long>(4096, (total + kDfThreads - 1) / kDfThreads);
  hipLaunchKernelGGL(df_scatter_kernel, dim3(grid), dim3(kDfThreads), 0, s, na, Na, nc, Nc, V, shells_a, shells_c,
                     ao_off, M, n);
  return hipGetLastError();
}

}  // namespace mderi
