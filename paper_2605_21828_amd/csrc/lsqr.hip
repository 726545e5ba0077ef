// Vector kernels of the LSQR least-squares iteration (Paige and Saunders'
// bidiagonalization) that solves the inverse transform min ||Phi~ c - f||_2
// column by column (Sec. 7.1, eq. inverse-MHT).  The matrix products are the
// butterfly applies; these kernels carry the per-column recurrences so that a
// whole solve is enqueued on one stream with no host synchronization.
//
// Every vector is row-major (rows x b, ld = b unless stated) and every scalar
// is an array of b, one per right-hand side.  Column norms are deterministic:
// per-block partial sums in a fixed order, then one workgroup per column
// reduces its column's partial sums with a fixed tree.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "bfmht_internal.h"

namespace bfmht {

constexpr int kLsqrThreads = 256;
constexpr int kCols = 64;                         // columns per block (one per lane of a wave)
constexpr int kPhases = kLsqrThreads / kCols;     // rows in flight per block step

// u = y - coef[j] u (or u = y when coef is null), and partial[blk][j] = sum of
// u[r][j]^2 over the rows this block visits.
template <typename T>
__global__ __launch_bounds__(kLsqrThreads) void sub_partial_kernel(const T *y, int64_t ldy, int64_t rows, int b,
                                                                   const T *coef, T *u, T *partial) {
  __shared__ T red[kLsqrThreads];
  const int j = blockIdx.y * kCols + (threadIdx.x % kCols);
  const int ph = threadIdx.x / kCols;
  T acc = 0;
  if (j < b) {
    const T cj = coef ? coef[j] : T(0);
    for (int64_t r = (int64_t)blockIdx.x * kPhases + ph; r < rows; r += (int64_t)gridDim.x * kPhases) {
      const T v = y[r * ldy + j] - (coef ? cj * u[r * b + j] : T(0));
      u[r * b + j] = v;
      acc += v * v;
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  if (ph == 0 && j < b) {
    T s = red[threadIdx.x];
#pragma unroll
    for (int q = 1; q < kPhases; ++q) s += red[threadIdx.x + q * kCols];
    partial[(int64_t)blockIdx.x * b + j] = s;
  }
}

// norm[j] = sqrt(sum over blocks of partial[blk][j]); inv[j] = 1 / norm[j] (0 for a zero column).
// One workgroup per column: thread t sums blocks t, t + 256, ... in order, then a
// fixed halving tree in LDS, so the result does not depend on timing.
template <typename T>
__global__ __launch_bounds__(kLsqrThreads) void finish_norm_kernel(const T *partial, int nblk, int b, T *norm, T *inv) {
  __shared__ T red[kLsqrThreads];
  const int j = blockIdx.x;
  T s = 0;
  for (int k = threadIdx.x; k < nblk; k += kLsqrThreads) s += partial[(int64_t)k * b + j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = kLsqrThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const T nv = sqrt(red[0]);
    norm[j] = nv;
    inv[j] = nv > T(0) ? T(1) / nv : T(0);
  }
}

// u[r][j] *= inv[j]
template <typename T>
__global__ __launch_bounds__(kLsqrThreads) void scale_cols_kernel(T *u, int64_t rows, int b, const T *inv) {
  const int64_t total = rows * b;
  for (int64_t e = (int64_t)blockIdx.x * kLsqrThreads + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * kLsqrThreads)
    u[e] *= inv[e % b];
}

// The plane rotation of one LSQR step, per column (alpha = alpha_{i+1}, beta =
// beta_{i+1}; rhobar and phibar advance in place):
//   rho = sqrt(rhobar^2 + beta^2), c = rhobar / rho, s = beta / rho,
//   theta = s alpha, rhobar' = -c alpha, phi = c phibar, phibar' = s phibar,
//   cx = phi / rho (step along w), cw = theta / rho (w update), rnorm = |phibar'|.
// rho = 0 means rhobar = beta = 0: A^T r = 0 and the bidiagonalization has
// ended, so the column keeps its iterate (cx = 0, and w = v = 0 from then on)
// and its residual estimate phibar.
template <typename T>
__global__ void rotate_kernel(int b, const T *alpha, const T *beta, T *rhobar, T *phibar, T *cx, T *cw, T *rnorm) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= b) return;
  const T rb = rhobar[j], be = beta[j], al = alpha[j], pb = phibar[j];
  const T rho = sqrt(rb * rb + be * be);
  const bool live = rho > T(0);
  const T c = live ? rb / rho : T(1), s = live ? be / rho : T(0);
  const T theta = s * al, phi = c * pb;
  const T pb1 = live ? s * pb : pb;
  rhobar[j] = live ? -c * al : rb;
  phibar[j] = pb1;
  cx[j] = live ? phi / rho : T(0);
  cw[j] = live ? theta / rho : T(0);
  if (rnorm) rnorm[j] = fabs(pb1);
}

// x += cx[j] w; w = v - cw[j] w   (x with its own leading dimension)
template <typename T>
__global__ __launch_bounds__(kLsqrThreads) void update_kernel(T *x, int64_t ldx, T *w, const T *v, int64_t rows,
                                                             int b, const T *cx, const T *cw) {
  const int64_t total = rows * b;
  for (int64_t e = (int64_t)blockIdx.x * kLsqrThreads + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * kLsqrThreads) {
    const int64_t r = e / b;
    const int j = (int)(e % b);
    const T we = w[e];
    x[r * ldx + j] += cx[j] * we;
    w[e] = v[e] - cw[j] * we;
  }
}

// x[r][j] = 0 (x with its own leading dimension), w = v
template <typename T>
__global__ __launch_bounds__(kLsqrThreads) void init_kernel(T *x, int64_t ldx, T *w, const T *v, int64_t rows, int b) {
  const int64_t total = rows * b;
  for (int64_t e = (int64_t)blockIdx.x * kLsqrThreads + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * kLsqrThreads) {
    x[(e / b) * ldx + e % b] = T(0);
    w[e] = v[e];
  }
}

namespace {
unsigned grid_for(int64_t total) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + kLsqrThreads - 1) / kLsqrThreads, 4096));
}
}  // namespace

int lsqr_norm_blocks(int64_t rows) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((rows + kPhases - 1) / kPhases, kLsqrMaxBlocks));
}

template <typename T>
static int normalize_t(const void *y, int64_t ldy, int64_t rows, int b, const void *coef, void *u, void *partial,
                       void *norm, void *inv, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  const int nblk = lsqr_norm_blocks(rows);
  hipLaunchKernelGGL((sub_partial_kernel<T>), dim3(nblk, (b + kCols - 1) / kCols), dim3(kLsqrThreads), 0, s,
                     static_cast<const T *>(y), ldy, rows, b, static_cast<const T *>(coef), static_cast<T *>(u),
                     static_cast<T *>(partial));
  hipLaunchKernelGGL((finish_norm_kernel<T>), dim3(b), dim3(kLsqrThreads), 0, s, static_cast<const T *>(partial),
                     nblk, b, static_cast<T *>(norm), static_cast<T *>(inv));
  hipLaunchKernelGGL((scale_cols_kernel<T>), dim3(grid_for(rows * b)), dim3(kLsqrThreads), 0, s, static_cast<T *>(u),
                     rows, b, static_cast<const T *>(inv));
  return (int)hipGetLastError();
}

int lsqr_normalize(int esz, const void *y, int64_t ldy, int64_t rows, int b, const void *coef, void *u,
                   void *partial, void *norm, void *inv, void *stream) {
  return esz == 8 ? normalize_t<double>(y, ldy, rows, b, coef, u, partial, norm, inv, stream)
                  : normalize_t<float>(y, ldy, rows, b, coef, u, partial, norm, inv, stream);
}

int lsqr_rotate(int esz, int b, const void *alpha, const void *beta, void *rhobar, void *phibar, void *cx, void *cw,
                void *rnorm, void *stream) {
  const dim3 g((b + 63) / 64), t(64);
  if (esz == 8)
    hipLaunchKernelGGL((rotate_kernel<double>), g, t, 0, (hipStream_t)stream, b, static_cast<const double *>(alpha),
                       static_cast<const double *>(beta), static_cast<double *>(rhobar),
                       static_cast<double *>(phibar), static_cast<double *>(cx), static_cast<double *>(cw),
                       static_cast<double *>(rnorm));
  else
    hipLaunchKernelGGL((rotate_kernel<float>), g, t, 0, (hipStream_t)stream, b, static_cast<const float *>(alpha),
                       static_cast<const float *>(beta), static_cast<float *>(rhobar), static_cast<float *>(phibar),
                       static_cast<float *>(cx), static_cast<float *>(cw), static_cast<float *>(rnorm));
  return (int)hipGetLastError();
}

int lsqr_update(int esz, void *x, int64_t ldx, void *w, const void *v, int64_t rows, int b, const void *cx,
                const void *cw, void *stream) {
  const dim3 g(grid_for(rows * b)), t(kLsqrThreads);
  if (esz == 8)
    hipLaunchKernelGGL((update_kernel<double>), g, t, 0, (hipStream_t)stream, static_cast<double *>(x), ldx,
                       static_cast<double *>(w), static_cast<const double *>(v), rows, b,
                       static_cast<const double *>(cx), static_cast<const double *>(cw));
  else
    hipLaunchKernelGGL((update_kernel<float>), g, t, 0, (hipStream_t)stream, static_cast<float *>(x), ldx,
                       static_cast<float *>(w), static_cast<const float *>(v), rows, b,
                       static_cast<const float *>(cx), static_cast<const float *>(cw));
  return (int)hipGetLastError();
}

int lsqr_init(int esz, void *x, int64_t ldx, void *w, const void *v, int64_t rows, int b, void *stream) {
  const dim3 g(grid_for(rows * b)), t(kLsqrThreads);
  if (esz == 8)
    hipLaunchKernelGGL((init_kernel<double>), g, t, 0, (hipStream_t)stream, static_cast<double *>(x), ldx,
                       static_cast<double *>(w), static_cast<const double *>(v), rows, b);
  else
    hipLaunchKernelGGL((init_kernel<float>), g, t, 0, (hipStream_t)stream, static_cast<float *>(x), ldx,
                       static_cast<float *>(w), static_cast<const float *>(v), rows, b);
  return (int)hipGetLastError();
}

}  // namespace bfmht
