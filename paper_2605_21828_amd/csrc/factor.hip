// Device side of the butterfly factorization: blocks of Phi formed from
// tables, and their column interpolative decompositions (FP64).
//
// Every block the factorization compresses is a submatrix of Phi (Sec. 2,
// Alg. "Butterfly factorization", with column IDs: the previous level's column
// basis restricted to a space node is Phi at the previous skeleton columns), so
// a level is a batch of independent tall blocks of uneven size.  Three calls:
//
//   bfmht_form_blocks       writes each block column-major into one buffer,
//                           entry (t, s) = tab0[ta_s][row0 + t] * tab1[tb_s][row0 + t]
//                           (a product of two table entries covers the Fourier
//                           matrix, cos/sin of k x per coordinate, and a dense
//                           Phi with a row of ones as the second table);
//   bfmht_column_id         column-pivoted Householder QR of each block, one
//                           workgroup per block, stopped at the first pivot
//                           whose column is shorter than tol |R_00|;
//   bfmht_id_coefficients   P = [I  R11^-1 R12] Pi^T of each block by back
//                           substitution, written row-major.
//
// Pivoting (Businger-Golub): at step j the remaining column with the largest
// sum of squares over rows j..M-1 is taken, the first in the current column
// order on ties; the sums are recomputed exactly from the updated entries in
// the same pass that applies the reflector (no downdating).  The reflector is
// H = I - tau v v^T with v_0 = 1, beta = -sign(alpha) |x|, tau = (beta - alpha) / beta,
// R_jj = beta (tau = 0 when the part below the diagonal is zero).
//
// Metadata (block shapes and offsets, per-column table rows) comes from host
// arrays, is checked there, and is staged into the caller's workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/bfmht.h"
#include "bfmht_internal.h"

namespace {

constexpr int kIdThreads = 512;       // 8 waves per block
constexpr int kIdWaves = kIdThreads / 64;
constexpr int kFormThreads = 256;
constexpr int kCoefThreads = 256;

int64_t round256(int64_t x) { return (x + 255) & ~int64_t(255); }

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Larger value wins; on equal values the smaller column index.
__device__ __forceinline__ void better(double &v, int &i, double v2, int i2) {
  if (v2 > v || (v2 == v && i2 < i)) {
    v = v2;
    i = i2;
  }
}

// Block of global column g: the largest b with col_off[b] <= g.
__device__ __forceinline__ int block_of(const int64_t *col_off, int count, int64_t g) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (col_off[mid] <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Staged metadata: per block row0, rows, col_off (count + 1), a_off; per column ta, tb.
struct Meta {
  const int64_t *row0, *rows, *col_off, *a_off;
  const int32_t *ta, *tb;
};

__global__ __launch_bounds__(kFormThreads) void form_blocks_kernel(Meta md, int count, const double *__restrict__ tab0,
                                                                   int64_t ld0, const double *__restrict__ tab1,
                                                                   int64_t ld1, double *__restrict__ a) {
  const int64_t g = blockIdx.x;
  const int b = block_of(md.col_off, count, g);
  const int64_t s = g - md.col_off[b];
  const int64_t M = md.rows[b], r0 = md.row0[b];
  const double *t0 = tab0 + (int64_t)md.ta[g] * ld0 + r0;
  const double *t1 = tab1 + (int64_t)md.tb[g] * ld1 + r0;
  double *out = a + md.a_off[b] + s * M;
  for (int64_t i = threadIdx.x; i < M; i += kFormThreads) out[i] = t0[i] * t1[i];
}

// Column-pivoted QR of one block per workgroup, in place.  LDS: the column
// sums of squares (K doubles), the logical-to-stored column map (K ints), the
// reflector below the diagonal (up to vcap doubles; beyond that it is read back
// from the block), and the reduction slots.  R > 0: every block has at most
// 64 R + 1 rows and its whole reflector fits vcap, so a wave keeps the column
// it updates in R registers per lane (one read and one write per step);
// R = 0: the column is read twice per step.
template <int R>
__global__ __launch_bounds__(kIdThreads) void cpqr_kernel(Meta md, int kmax, int vcap, double *__restrict__ a, double tol,
                                                          int32_t *__restrict__ rank_out, int32_t *__restrict__ piv_out) {
  extern __shared__ double lds[];
  double *nrm = lds;                                        // [kmax]
  double *vl = nrm + kmax;                                  // [vcap]
  double *red = vl + vcap;                                  // [2 * kIdWaves]
  int *redi = reinterpret_cast<int *>(red + 2 * kIdWaves);  // [kIdWaves]
  int *colmap = redi + kIdWaves;                            // [kmax]

  const int b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t M = md.rows[b];
  const int64_t c0 = md.col_off[b];
  const int K = (int)(md.col_off[b + 1] - c0);
  double *A = a + md.a_off[b];

  for (int c = tid; c < K; c += kIdThreads) colmap[c] = c;
  for (int c = wave; c < K; c += kIdWaves) {
    const double *col = A + (int64_t)c * M;
    double s = 0.0;
    for (int64_t i = lane; i < M; i += 64) s = fma(col[i], col[i], s);
    s = wave_sum(s);
    if (lane == 0) nrm[c] = s;
  }
  __syncthreads();

  const int steps = (int)std::min<int64_t>(M, K);
  int k = steps;
  double d0 = 0.0;
  for (int j = 0; j < steps; ++j) {
    // pivot: the largest remaining sum of squares, first index on ties
    double bv = -1.0;
    int bi = K;
    for (int c = j + tid; c < K; c += kIdThreads) better(bv, bi, nrm[c], c);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) better(bv, bi, __shfl_xor(bv, o, 64), __shfl_xor(bi, o, 64));
    if (lane == 0) {
      red[wave] = bv;
      redi[wave] = bi;
    }
    __syncthreads();
    bv = red[0];
    bi = redi[0];
    for (int w = 1; w < kIdWaves; ++w) better(bv, bi, red[w], redi[w]);
    const double pn = std::sqrt(bv);
    if (j == 0) d0 = pn;
    if (!(pn > tol * d0) || d0 == 0.0) {   // uniform over the workgroup
      k = j;
      break;
    }
    __syncthreads();   // every thread has read nrm and the slots
    if (tid == 0 && bi != j) {
      const int tc = colmap[j];
      colmap[j] = colmap[bi];
      colmap[bi] = tc;
      const double tn = nrm[j];
      nrm[j] = nrm[bi];
      nrm[bi] = tn;
    }
    __syncthreads();

    // reflector of the pivot column, rows j..M-1
    double *pcol = A + (int64_t)colmap[j] * M;
    const double alpha = pcol[j];
    double s = 0.0;
    for (int64_t i = j + 1 + tid; i < M; i += kIdThreads) s = fma(pcol[i], pcol[i], s);
    s = wave_sum(s);
    if (lane == 0) red[kIdWaves + wave] = s;
    __syncthreads();
    s = 0.0;
    for (int w = 0; w < kIdWaves; ++w) s += red[kIdWaves + w];
    double tau = 0.0, beta = alpha, scal = 0.0;
    if (s > 0.0) {
      beta = -std::copysign(std::sqrt(alpha * alpha + s), alpha);
      tau = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    const int64_t nv = M - j - 1;
    for (int64_t i = tid; i < nv; i += kIdThreads) {
      const double v = pcol[j + 1 + i] * scal;
      pcol[j + 1 + i] = v;
      if (i < vcap) vl[i] = v;
    }
    __syncthreads();   // the reflector is in LDS and in the block; beta is not yet stored
    if (tid == 0) pcol[j] = beta;

    // apply H to every remaining column and recompute its sum of squares below row j
    for (int c = j + 1 + wave; c < K; c += kIdWaves) {
      double *col = A + (int64_t)colmap[c] * M;
      double *cb = col + j + 1;
      double w = 0.0, s2 = 0.0;
      if constexpr (R > 0) {
        // the column below row j stays in registers from the dot product to the update
        double x[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int64_t i = lane + 64 * r;
          x[r] = i < nv ? cb[i] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int64_t i = lane + 64 * r;
          if (i < nv) w = fma(vl[i], x[r], w);
        }
        w = wave_sum(w) + col[j];
        const double tw = tau * w;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int64_t i = lane + 64 * r;
          if (i < nv) {
            const double y = x[r] - tw * vl[i];
            cb[i] = y;
            s2 = fma(y, y, s2);
          }
        }
        s2 = wave_sum(s2);
        if (lane == 0) {
          col[j] -= tw;
          nrm[c] = s2;
        }
      } else {
#pragma unroll 4
        for (int64_t i = lane; i < nv; i += 64) {
          const double v = i < vcap ? vl[i] : pcol[j + 1 + i];
          w = fma(v, cb[i], w);
        }
        w = wave_sum(w) + col[j];
        const double tw = tau * w;
#pragma unroll 4
        for (int64_t i = lane; i < nv; i += 64) {
          const double v = i < vcap ? vl[i] : pcol[j + 1 + i];
          const double y = cb[i] - tw * v;
          cb[i] = y;
          s2 = fma(y, y, s2);
        }
        s2 = wave_sum(s2);
        if (lane == 0) {
          col[j] -= tw;
          nrm[c] = s2;
        }
      }
    }
    __syncthreads();
  }
  if (tid == 0) rank_out[b] = k;
  for (int c = tid; c < K; c += kIdThreads) piv_out[c0 + c] = colmap[c];
}

// P of one block (row-major k x K at p + p_off): positions s < k of the pivot
// order hold unit columns, positions s >= k the columns of T = R11^-1 R12.
// Workgroup (b, g) takes positions [g G, g G + G); its T columns are solved
// together in LDS, reading R11 column by column.
__global__ __launch_bounds__(kCoefThreads) void coef_kernel(Meta md, const int64_t *__restrict__ p_off,
                                                            const int32_t *__restrict__ rank, int G,
                                                            const double *__restrict__ a,
                                                            const int32_t *__restrict__ piv, double *__restrict__ p) {
  extern __shared__ double x[];   // [G][k]
  const int b = blockIdx.x;
  const int64_t po = p_off[b];
  if (po < 0) return;
  const int64_t M = md.rows[b];
  const int64_t c0 = md.col_off[b];
  const int K = (int)(md.col_off[b + 1] - c0);
  const int k = rank[b];
  const int s0 = blockIdx.y * G;
  if (s0 >= K) return;
  const int s1 = std::min(K, s0 + G);
  const double *A = a + md.a_off[b];
  const int32_t *pv = piv + c0;
  double *P = p + po;
  const int tid = threadIdx.x;

  // unit columns
  for (int s = std::max(s0, 0); s < std::min(s1, k); ++s)
    for (int i = tid; i < k; i += kCoefThreads) P[(int64_t)i * K + pv[s]] = (i == s) ? 1.0 : 0.0;

  const int t0 = std::max(s0, k);
  const int nt = s1 - t0;
  if (nt <= 0) return;
  for (int e = tid; e < nt * k; e += kCoefThreads) {
    const int g = e / k, i = e - g * k;
    x[g * k + i] = A[(int64_t)pv[t0 + g] * M + i];
  }
  __syncthreads();
  for (int i = k - 1; i >= 0; --i) {
    const double *ri = A + (int64_t)pv[i] * M;   // column i of R11 (rows 0..i)
    const double rii = ri[i];
    for (int e = tid; e < nt * i; e += kCoefThreads) {
      const int g = e / i, r = e - g * i;
      x[g * k + r] -= (x[g * k + i] / rii) * ri[r];
    }
    __syncthreads();
    if (tid < nt) x[tid * k + i] /= rii;
    __syncthreads();
  }
  for (int e = tid; e < nt * k; e += kCoefThreads) {
    const int g = e / k, i = e - g * k;
    P[(int64_t)i * K + pv[t0 + g]] = x[g * k + i];
  }
}

int max_lds_bytes() {
  static int v = -1;
  if (v < 0) {
    int dev = 0, bytes = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      bytes = 65536;
    v = bytes;
  }
  return v;
}

// Check the host metadata of a batch: block b covers a[a_off[b], a_off[b] + rows[b] * K_b)
// inside a_len, its rows [row0, row0 + rows) inside both tables' ld, col_off
// nondecreasing from 0.  Also returns the largest K and rows.
bfmht_status check_blocks(const char *who, int32_t count, const int64_t *row0, const int64_t *rows,
                          const int64_t *col_off, const int64_t *a_off, int64_t a_len, int64_t ld_rows,
                          int64_t *kmax, int64_t *mmax) {
  const std::string w(who);
  if (count < 0) return bfmht::set_error(BFMHT_EINVAL, w + ": count < 0");
  if (count == 0) return BFMHT_OK;
  if (!rows || !col_off || !a_off) return bfmht::set_error(BFMHT_EINVAL, w + ": NULL metadata array");
  if (col_off[0] != 0) return bfmht::set_error(BFMHT_EINVAL, w + ": col_off[0] != 0");
  *kmax = 0;
  *mmax = 0;
  for (int32_t b = 0; b < count; ++b) {
    const int64_t K = col_off[b + 1] - col_off[b];
    if (K < 0) return bfmht::set_error(BFMHT_EINVAL, w + ": col_off decreases at block " + std::to_string(b));
    if (rows[b] < 0 || rows[b] > (int64_t(1) << 31))
      return bfmht::set_error(BFMHT_EINVAL, w + ": bad row count at block " + std::to_string(b));
    if (a_off[b] < 0 || (K > 0 && rows[b] > 0 && (a_len - a_off[b]) / K < rows[b]) ||
        (a_off[b] > a_len))
      return bfmht::set_error(BFMHT_EINVAL, w + ": block " + std::to_string(b) + " lies outside a");
    if (row0) {
      if (row0[b] < 0 || row0[b] + rows[b] > ld_rows)
        return bfmht::set_error(BFMHT_EINVAL, w + ": rows of block " + std::to_string(b) + " outside the tables");
    }
    *kmax = std::max(*kmax, K);
    *mmax = std::max(*mmax, rows[b]);
  }
  if (col_off[count] > (int64_t(1) << 31) - 1) return bfmht::set_error(BFMHT_EINVAL, w + ": too many columns");
  return BFMHT_OK;
}

// Layout of the metadata workspace: per block row0, rows, col_off (count + 1),
// a_off (int64); then p_off (int64) and rank (int32) per block; then the
// per-column table rows ta, tb (int32).
struct MetaLayout {
  int64_t poff, rank, ta, tb, total;
  MetaLayout(int64_t count, int64_t tc) {
    poff = round256((4 * count + 1) * 8);
    rank = poff + round256(count * 8);
    ta = rank + round256(count * 4);
    tb = ta + round256(tc * 4);
    total = tb + round256(tc * 4);
  }
};

// Stage the metadata into ws and wait for the copies (the host arrays may be
// freed on return).  Optional parts are NULL.
bfmht_status stage_meta(const char *who, int32_t count, const int64_t *row0, const int64_t *rows, const int64_t *col_off,
                        const int64_t *a_off, const int64_t *p_off, const int32_t *rank, const int32_t *ta,
                        const int32_t *tb, void *ws, int64_t ws_bytes, hipStream_t st, Meta *md,
                        int64_t **d_poff = nullptr, int32_t **d_rank = nullptr) {
  const int64_t tc = col_off[count];
  const MetaLayout lay(count, tc);
  const int64_t need = ta ? lay.total : lay.ta;   // the per-column part only when there are table rows
  if (!ws || ws_bytes < need)
    return bfmht::set_error(BFMHT_ENOSPACE, std::string(who) + ": metadata workspace smaller than " +
                                                std::to_string(need) + " bytes");
  std::vector<int64_t> h(4 * (size_t)count + 1, 0);
  for (int32_t b = 0; b < count; ++b) {
    h[b] = row0 ? row0[b] : 0;
    h[count + b] = rows[b];
    h[3 * (size_t)count + 1 + b] = a_off[b];
  }
  for (int32_t b = 0; b <= count; ++b) h[2 * (size_t)count + b] = col_off[b];
  char *base = static_cast<char *>(ws);
  hipError_t e = hipMemcpyAsync(base, h.data(), h.size() * sizeof(int64_t), hipMemcpyHostToDevice, st);
  const int64_t *d = reinterpret_cast<const int64_t *>(base);
  md->row0 = d;
  md->rows = d + count;
  md->col_off = d + 2 * (size_t)count;
  md->a_off = d + 3 * (size_t)count + 1;
  md->ta = reinterpret_cast<const int32_t *>(base + lay.ta);
  md->tb = reinterpret_cast<const int32_t *>(base + lay.tb);
  if (e == hipSuccess && p_off) e = hipMemcpyAsync(base + lay.poff, p_off, (size_t)count * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && rank) e = hipMemcpyAsync(base + lay.rank, rank, (size_t)count * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && ta && tc > 0) e = hipMemcpyAsync(base + lay.ta, ta, tc * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && tb && tc > 0) e = hipMemcpyAsync(base + lay.tb, tb, tc * 4, hipMemcpyHostToDevice, st);
  if (d_poff) *d_poff = reinterpret_cast<int64_t *>(base + lay.poff);
  if (d_rank) *d_rank = reinterpret_cast<int32_t *>(base + lay.rank);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return bfmht::set_error(BFMHT_EHIP, std::string(who) + ": " + hipGetErrorString(e));
  return BFMHT_OK;
}

}  // namespace

extern "C" int64_t bfmht_factor_meta_bytes(int32_t count, int64_t total_cols) {
  if (count < 0 || total_cols < 0) return -1;
  return MetaLayout(count, total_cols).total;
}

extern "C" bfmht_status bfmht_form_blocks(int32_t count, const int64_t *row0, const int64_t *rows,
                                          const int64_t *col_off, const int32_t *ta, const int32_t *tb,
                                          const int64_t *a_off, const double *tab0, int64_t ld0, int64_t w0,
                                          const double *tab1, int64_t ld1, int64_t w1, double *a, int64_t a_len,
                                          void *ws, int64_t ws_bytes, void *stream) {
  const char *who = "bfmht_form_blocks";
  if (ld0 < 0 || ld1 < 0 || w0 < 0 || w1 < 0 || a_len < 0)
    return bfmht::set_error(BFMHT_EINVAL, std::string(who) + ": negative size");
  int64_t kmax = 0, mmax = 0;
  bfmht_status st = check_blocks(who, count, row0, rows, col_off, a_off, a_len, std::min(ld0, ld1), &kmax, &mmax);
  if (st != BFMHT_OK || count == 0) return st;
  if (!row0) return bfmht::set_error(BFMHT_EINVAL, std::string(who) + ": row0 is NULL");
  const int64_t tc = col_off[count];
  if (tc == 0 || mmax == 0) return BFMHT_OK;
  if (!ta || !tb || !tab0 || !tab1 || !a) return bfmht::set_error(BFMHT_EINVAL, std::string(who) + ": NULL pointer");
  for (int64_t g = 0; g < tc; ++g)
    if (ta[g] < 0 || ta[g] >= w0 || tb[g] < 0 || tb[g] >= w1)
      return bfmht::set_error(BFMHT_EINVAL, std::string(who) + ": table column out of range at column " + std::to_string(g));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Meta md;
  st = stage_meta(who, count, row0, rows, col_off, a_off, nullptr, nullptr, ta, tb, ws, ws_bytes, s, &md);
  if (st != BFMHT_OK) return st;
  hipLaunchKernelGGL(form_blocks_kernel, dim3((unsigned)tc), dim3(kFormThreads), 0, s, md, (int)count, tab0, ld0,
                     tab1, ld1, a);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return bfmht::set_error(BFMHT_EHIP, std::string(who) + ": " + hipGetErrorString(e));
  return BFMHT_OK;
}

extern "C" bfmht_status bfmht_column_id(int32_t count, const int64_t *rows, const int64_t *col_off, const int64_t *a_off,
                                        double *a, int64_t a_len, double tol, int32_t *rank, int32_t *piv, void *ws,
                                        int64_t ws_bytes, void *stream) {
  const char *who = "bfmht_column_id";
  if (!(tol >= 0.0)) return bfmht::set_error(BFMHT_EINVAL, std::string(who) + ": tol must be >= 0");
  int64_t kmax = 0, mmax = 0;
  bfmht_status st = check_blocks(who, count, nullptr, rows, col_off, a_off, a_len, 0, &kmax, &mmax);
  if (st != BFMHT_OK || count == 0) return st;
  if (!rank || (col_off[count] > 0 && (!piv || !a))) return bfmht::set_error(BFMHT_EINVAL, std::string(who) + ": NULL pointer");
  const int lds_max = max_lds_bytes();
  const int64_t fixed = kmax * 12 + 3 * kIdWaves * 8 + 64;
  if (fixed > lds_max)
    return bfmht::set_error(BFMHT_EINVAL, std::string(who) + ": " + std::to_string(kmax) +
                                              " columns in one block exceed the workgroup's local memory");
  const int64_t vcap = std::min<int64_t>(mmax, (lds_max - fixed) / 8);
  const int64_t lds = (kmax + vcap + 3 * kIdWaves) * 8 + kmax * 4;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Meta md;
  st = stage_meta(who, count, nullptr, rows, col_off, a_off, nullptr, nullptr, nullptr, nullptr, ws, ws_bytes, s, &md);
  if (st != BFMHT_OK) return st;
  // registers per lane for the cached column: the smallest R with 64 R >= the longest reflector
  const int64_t nvmax = std::max<int64_t>(mmax - 1, 0);
  const int R = nvmax > vcap ? 0 : nvmax <= 256 ? 4 : nvmax <= 1024 ? 16 : nvmax <= 2048 ? 32 : 0;
  const void *fn = R == 4    ? reinterpret_cast<const void *>(cpqr_kernel<4>)
                   : R == 16 ? reinterpret_cast<const void *>(cpqr_kernel<16>)
                   : R == 32 ? reinterpret_cast<const void *>(cpqr_kernel<32>)
                             : reinterpret_cast<const void *>(cpqr_kernel<0>);
  hipError_t e = hipSuccess;
  if (lds > 65536) e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess) {
    const dim3 grid((unsigned)count), block(kIdThreads);
    const int ik = (int)kmax, iv = (int)vcap;
    if (R == 4) hipLaunchKernelGGL(cpqr_kernel<4>, grid, block, (size_t)lds, s, md, ik, iv, a, tol, rank, piv);
    else if (R == 16) hipLaunchKernelGGL(cpqr_kernel<16>, grid, block, (size_t)lds, s, md, ik, iv, a, tol, rank, piv);
    else if (R == 32) hipLaunchKernelGGL(cpqr_kernel<32>, grid, block, (size_t)lds, s, md, ik, iv, a, tol, rank, piv);
    else hipLaunchKernelGGL(cpqr_kernel<0>, grid, block, (size_t)lds, s, md, ik, iv, a, tol, rank, piv);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return bfmht::set_error(BFMHT_EHIP, std::string(who) + ": " + hipGetErrorString(e));
  return BFMHT_OK;
}

extern "C" bfmht_status bfmht_id_coefficients(int32_t count, const int64_t *rows, const int64_t *col_off,
                                              const int64_t *a_off, const double *a, int64_t a_len, const int32_t *rank,
                                              const int32_t *piv, const int64_t *p_off, double *p, int64_t p_len,
                                              void *ws, int64_t ws_bytes, void *stream) {
  const char *who = "bfmht_id_coefficients";
  int64_t kmax = 0, mmax = 0;
  bfmht_status st = check_blocks(who, count, nullptr, rows, col_off, a_off, a_len, 0, &kmax, &mmax);
  if (st != BFMHT_OK || count == 0) return st;
  if (!rank || !p_off) return bfmht::set_error(BFMHT_EINVAL, std::string(who) + ": NULL metadata array");
  int64_t rmax = 0;
  for (int32_t b = 0; b < count; ++b) {
    const int64_t K = col_off[b + 1] - col_off[b];
    if (rank[b] < 0 || rank[b] > std::min(K, rows[b]))
      return bfmht::set_error(BFMHT_EINVAL, std::string(who) + ": bad rank at block " + std::to_string(b));
    if (p_off[b] < 0) continue;
    if (p_off[b] > p_len || (rank[b] > 0 && (p_len - p_off[b]) / K < rank[b]))
      return bfmht::set_error(BFMHT_EINVAL, std::string(who) + ": P of block " + std::to_string(b) + " lies outside p");
    rmax = std::max<int64_t>(rmax, rank[b]);
  }
  if (rmax == 0) return BFMHT_OK;
  if (!a || !piv || !p) return bfmht::set_error(BFMHT_EINVAL, std::string(who) + ": NULL pointer");
  const int lds_max = std::min(max_lds_bytes(), 65536);
  if (rmax * 8 > lds_max)
    return bfmht::set_error(BFMHT_EINVAL, std::string(who) + ": rank " + std::to_string(rmax) + " exceeds local memory");
  const int G = (int)std::max<int64_t>(1, std::min<int64_t>(32, lds_max / (8 * rmax)));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Meta md;
  int64_t *d_poff = nullptr;
  int32_t *d_rank = nullptr;
  st = stage_meta(who, count, nullptr, rows, col_off, a_off, p_off, rank, nullptr, nullptr, ws, ws_bytes, s, &md,
                  &d_poff, &d_rank);
  if (st != BFMHT_OK) return st;
  const unsigned gy = (unsigned)((kmax + G - 1) / G);
  hipLaunchKernelGGL(coef_kernel, dim3((unsigned)count, gy), dim3(kCoefThreads), (size_t)G * rmax * 8, s, md, d_poff,
                     d_rank, G, a, piv, p);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return bfmht::set_error(BFMHT_EHIP, std::string(who) + ": " + hipGetErrorString(e));
  return BFMHT_OK;
}
