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
//                           whose column is shorter than tol |R_00|; a block
//                           more than twice as tall as wide is first reduced to
//                           its triangular factor by a blocked QR;
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

constexpr int kIdThreads = 512;       // 8 waves per block (4 for the largest register cache)
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

// Staged metadata: per block row0, rows, col_off (count + 1), a_off, prow; per
// column ta, tb.  prow: the rows the pivoted QR works on, rows itself, or K for
// a tall block (rows > 2 K) that is first reduced to its triangular factor.
struct Meta {
  const int64_t *row0, *rows, *col_off, *a_off, *prow;
  const int32_t *ta, *tb;
};

// A block more than twice as tall as wide is first reduced to R by an unpivoted
// blocked QR; pivoting then runs on the K x K triangle (the same pivots and R
// in exact arithmetic, since pivoting reads only column norms of Q^T A).
__host__ __device__ inline bool reduce_first(int64_t M, int64_t K) { return K > 0 && M > 2 * K; }

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

// Unpivoted blocked Householder QR of the tall blocks (reduce_first), in
// place: R in the upper triangle of the top K rows, cleared below the diagonal
// at the end so the pivoted QR sees R.  Panels of kPanel columns, one launch
// pair per panel position over all blocks:
//   hqr_panel_kernel   one workgroup per block factors the panel left-looking:
//                      column p0 + j first takes the panel's earlier reflectors
//                      in compact form H_0 ... H_{j-1} = I - V T V^T (T upper
//                      triangular, extended by the forward recurrence
//                      T(0:j, j) = -tau_j T(0:j, 0:j) V^T v_j), then yields
//                      reflector j; T goes to the block's slot in tbuf;
//   hqr_trail_kernel   a grid over (block, group of columns) applies
//                      Q^T = I - V T^T V^T to every column right of the panel in
//                      two passes over its rows, a wave per four columns.
// Trailing columns are thus streamed once per panel, not once per column, and
// the trailing update has many workgroups per block to hide memory latency.
constexpr int kPanel = 16;
constexpr int kPanelThreads = 512;
constexpr int kTrailThreads = 256;
constexpr int kTrailCols = 16;          // columns per trailing workgroup (4 per wave)
constexpr int kRowsInFlight = 2;        // rows per lane whose loads are issued together

// Sums over the workgroup of vals[t], t < n (n <= kPanel); every thread gets them.
template <int NW>
__device__ __forceinline__ void block_sums(double *vals, int n, double (*slots)[kPanel], int lane, int wave) {
#pragma unroll
  for (int t = 0; t < kPanel; ++t)
    if (t < n) {
      const double v = wave_sum(vals[t]);
      if (lane == 0) slots[wave][t] = v;
    }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < kPanel; ++t)
    if (t < n) {
      double v = 0.0;
      for (int w = 0; w < NW; ++w) v += slots[w][t];
      vals[t] = v;
    }
  __syncthreads();
}

// V(i, t) of the panel starting at column p0: 1 at i = p0 + t, 0 above, the
// stored reflector below.  i < M: the load is issued unconditionally (and the
// value selected), so the loads of a row do not wait on each other.
__device__ __forceinline__ double vpanel(const double *A, int64_t M, int p0, int t, int64_t i) {
  const int64_t d = i - (p0 + t);
  const double raw = A[(int64_t)(p0 + t) * M + i];
  return d > 0 ? raw : (d == 0 ? 1.0 : 0.0);
}

__global__ __launch_bounds__(kPanelThreads) void hqr_panel_kernel(Meta md, int p0, double *__restrict__ a,
                                                                  double *__restrict__ tbuf) {
  constexpr int NW = kPanelThreads / 64;
  constexpr int U = kRowsInFlight;
  __shared__ double T[kPanel][kPanel];
  __shared__ double slots[NW][kPanel];
  const int b = blockIdx.x;
  const int64_t M = md.rows[b];
  const int K = (int)(md.col_off[b + 1] - md.col_off[b]);
  if (!reduce_first(M, K) || p0 >= K) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double *A = a + md.a_off[b];
  const int pw = std::min(kPanel, K - p0);
  for (int jj = 0; jj < pw; ++jj) {
    const int c = p0 + jj;
    double *col = A + (int64_t)c * M;
    double v[kPanel];
    if (jj > 0) {
      // the panel's earlier reflectors: w = V^T a, a -= V (T^T w)
#pragma unroll
      for (int t = 0; t < kPanel; ++t) v[t] = 0.0;
      // (entries t >= jj are formed too and discarded, so no branch separates the
      // loads; no column past the panel's last, p0 + pw - 1, is addressed)
      for (int64_t i0 = p0 + tid; i0 < M; i0 += (int64_t)kPanelThreads * U) {
        double x[U];
        int64_t iu[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t i = i0 + (int64_t)kPanelThreads * u;
          iu[u] = i < M ? i : M - 1;
          x[u] = i < M ? col[iu[u]] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int t = 0; t < kPanel; ++t) v[t] = fma(vpanel(A, M, p0, t < pw ? t : pw - 1, iu[u]), x[u], v[t]);
      }
      block_sums<NW>(v, jj, slots, lane, wave);
      double y[kPanel];
#pragma unroll
      for (int t = 0; t < kPanel; ++t) {
        double s0 = 0.0;
        for (int r = 0; r <= t && r < jj; ++r) s0 = fma(T[r][t], v[r], s0);
        y[t] = t < jj ? s0 : 0.0;
      }
      for (int64_t i = p0 + tid; i < M; i += kPanelThreads) {
        double d0 = 0.0;
#pragma unroll
        for (int t = 0; t < kPanel; ++t) d0 = fma(vpanel(A, M, p0, t < pw ? t : pw - 1, i), y[t], d0);   // y[t] = 0, t >= jj
        col[i] -= d0;
      }
      __syncthreads();
    }
    // reflector of column c over rows c..M-1
    const double alpha = col[c];
    v[0] = 0.0;
    for (int64_t i0 = c + 1 + tid; i0 < M; i0 += (int64_t)kPanelThreads * U) {
      double x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = i0 + (int64_t)kPanelThreads * u;
        x[u] = i < M ? col[i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) v[0] = fma(x[u], x[u], v[0]);
    }
    block_sums<NW>(v, 1, slots, lane, wave);
    const double s = v[0];
    double tau = 0.0, beta = alpha, scal = 0.0;
    if (s > 0.0) {
      beta = -std::copysign(std::sqrt(alpha * alpha + s), alpha);
      tau = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    for (int64_t i = c + 1 + tid; i < M; i += kPanelThreads) col[i] *= scal;
    __syncthreads();   // the reflector is stored; row c still holds alpha
    // T column jj: z = V(:, 0:jj)^T v_jj, T(0:jj, jj) = -tau T(0:jj, 0:jj) z
    if (jj > 0) {
#pragma unroll
      for (int t = 0; t < kPanel; ++t) v[t] = 0.0;
      for (int64_t i0 = c + tid; i0 < M; i0 += (int64_t)kPanelThreads * U) {
        double x[U];
        int64_t iu[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t i = i0 + (int64_t)kPanelThreads * u;
          iu[u] = i < M ? i : M - 1;
          x[u] = i < M ? (i == c ? 1.0 : col[iu[u]]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int t = 0; t < kPanel; ++t) v[t] = fma(vpanel(A, M, p0, t < pw ? t : pw - 1, iu[u]), x[u], v[t]);
      }
      block_sums<NW>(v, jj, slots, lane, wave);
    }
    if (tid == 0) {
      for (int r = 0; r < jj; ++r) {
        double acc = 0.0;
        for (int t = r; t < jj; ++t) acc += T[r][t] * v[t];
        T[r][jj] = -tau * acc;
      }
      T[jj][jj] = tau;
      for (int r = jj + 1; r < kPanel; ++r) T[r][jj] = 0.0;
      col[c] = beta;
    }
    __syncthreads();
  }
  double *tb = tbuf + (int64_t)b * kPanel * kPanel;
  for (int e = tid; e < kPanel * kPanel; e += kPanelThreads) {
    const int r = e / kPanel, t = e % kPanel;
    tb[e] = (r < pw && t < pw) ? T[r][t] : 0.0;
  }
}

// Workgroup g runs on XCD g % 8: the groups of one block are numbered so that
// they all land on XCD b % 8, where they share the panel's reflectors in L2.
__global__ __launch_bounds__(kTrailThreads) void hqr_trail_kernel(Meta md, int count, int ngroups, int p0,
                                                                  double *__restrict__ a,
                                                                  const double *__restrict__ tbuf) {
  constexpr int NW = kTrailThreads / 64;
  __shared__ double T[kPanel][kPanel];
  const int64_t g = blockIdx.x;
  const int64_t sg = g >> 3;
  const int b = (int)((sg / ngroups) * 8 + (g & 7));
  const int gy = (int)(sg % ngroups);
  if (b >= count) return;
  const int64_t M = md.rows[b];
  const int K = (int)(md.col_off[b + 1] - md.col_off[b]);
  if (!reduce_first(M, K) || p0 >= K) return;
  // a panel with columns to its right is a full one: kPanel reflectors
  const int first = p0 + kPanel + gy * kTrailCols;
  if (first >= K) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double *tb = tbuf + (int64_t)b * kPanel * kPanel;
  for (int e = tid; e < kPanel * kPanel; e += kTrailThreads) T[e / kPanel][e % kPanel] = tb[e];
  __syncthreads();
  double *A = a + md.a_off[b];
  const int last = std::min(K, first + kTrailCols);
  // a wave takes CW adjacent columns at once, so each reflector entry it loads
  // serves CW columns
  constexpr int CW = kTrailCols / NW;
  const int cbase = first + wave * CW;
  if (cbase >= last) return;
  double *x[CW];
  bool live[CW];
#pragma unroll
  for (int q = 0; q < CW; ++q) {
    live[q] = cbase + q < last;
    x[q] = A + (int64_t)(live[q] ? cbase + q : cbase) * M;
  }
  double w[CW][kPanel];
#pragma unroll
  for (int q = 0; q < CW; ++q)
#pragma unroll
    for (int t = 0; t < kPanel; ++t) w[q][t] = 0.0;
  for (int64_t i = p0 + lane; i < M; i += 64) {
    double xa[CW];
#pragma unroll
    for (int q = 0; q < CW; ++q) xa[q] = x[q][i];
#pragma unroll
    for (int t = 0; t < kPanel; ++t) {
      const double v = vpanel(A, M, p0, t, i);
#pragma unroll
      for (int q = 0; q < CW; ++q) w[q][t] = fma(v, xa[q], w[q][t]);
    }
  }
#pragma unroll
  for (int q = 0; q < CW; ++q) {
#pragma unroll
    for (int t = 0; t < kPanel; ++t) w[q][t] = wave_sum(w[q][t]);
    // w <- T^T w: lane t < kPanel forms entry t from column t of T, then every
    // lane takes the entries back by shuffles
    const int tl = lane & (kPanel - 1);
    double yt = 0.0;
#pragma unroll
    for (int r = 0; r < kPanel; ++r) yt = fma(r <= tl ? T[r][tl] : 0.0, w[q][r], yt);
#pragma unroll
    for (int t = 0; t < kPanel; ++t) w[q][t] = __shfl(yt, t, 64);
  }
  for (int64_t i = p0 + lane; i < M; i += 64) {
    double d[CW];
#pragma unroll
    for (int q = 0; q < CW; ++q) d[q] = 0.0;
#pragma unroll
    for (int t = 0; t < kPanel; ++t) {
      const double v = vpanel(A, M, p0, t, i);
#pragma unroll
      for (int q = 0; q < CW; ++q) d[q] = fma(v, w[q][t], d[q]);
    }
#pragma unroll
    for (int q = 0; q < CW; ++q)
      if (live[q]) x[q][i] -= d[q];
  }
}

// Clear below the diagonal of the top K rows of every reduced block.
__global__ __launch_bounds__(256) void hqr_clear_kernel(Meta md, double *__restrict__ a) {
  const int b = blockIdx.x;
  const int64_t M = md.rows[b];
  const int K = (int)(md.col_off[b + 1] - md.col_off[b]);
  if (!reduce_first(M, K)) return;
  double *A = a + md.a_off[b];
  for (int64_t e = threadIdx.x; e < (int64_t)K * K; e += 256) {
    const int c = (int)(e / K), i = (int)(e % K);
    if (i > c) A[(int64_t)c * M + i] = 0.0;
  }
}

// Column-pivoted QR of one block per workgroup, in place.  LDS: the column
// sums of squares (K doubles), the logical-to-stored column map (K ints), the
// reflector below the diagonal (up to vcap doubles; beyond that it is read back
// from the block), and the reduction slots.  R > 0: every block has at most
// 64 R + 1 rows and its whole reflector fits vcap, so a wave keeps the column
// it updates in R registers per lane (one read and one write per step);
// R = 0: the column is read twice per step.
template <int R, int NT>
__global__ __launch_bounds__(NT) void cpqr_kernel(Meta md, int kmax, int vcap, double *__restrict__ a, double tol,
                                                          int32_t *__restrict__ rank_out, int32_t *__restrict__ piv_out) {
  constexpr int NW = NT / 64;
  extern __shared__ double lds[];
  double *nrm = lds;                                        // [kmax]
  double *vl = nrm + kmax;                                  // [vcap]
  double *red = vl + vcap;                                  // [2 * NW]
  int *redi = reinterpret_cast<int *>(red + 2 * NW);  // [NW]
  int *colmap = redi + NW;                            // [kmax]

  const int b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t M = md.prow[b];    // rows of the matrix pivoted on (the triangle of a reduced block)
  const int64_t ld = md.rows[b];
  const int64_t c0 = md.col_off[b];
  const int K = (int)(md.col_off[b + 1] - c0);
  double *A = a + md.a_off[b];

  for (int c = tid; c < K; c += NT) colmap[c] = c;
  for (int c = wave; c < K; c += NW) {
    const double *col = A + (int64_t)c * ld;
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
    for (int c = j + tid; c < K; c += NT) better(bv, bi, nrm[c], c);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) better(bv, bi, __shfl_xor(bv, o, 64), __shfl_xor(bi, o, 64));
    if (lane == 0) {
      red[wave] = bv;
      redi[wave] = bi;
    }
    __syncthreads();
    bv = red[0];
    bi = redi[0];
    for (int w = 1; w < NW; ++w) better(bv, bi, red[w], redi[w]);
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
    double *pcol = A + (int64_t)colmap[j] * ld;
    const double alpha = pcol[j];
    double s = 0.0;
    for (int64_t i = j + 1 + tid; i < M; i += NT) s = fma(pcol[i], pcol[i], s);
    s = wave_sum(s);
    if (lane == 0) red[NW + wave] = s;
    __syncthreads();
    s = 0.0;
    for (int w = 0; w < NW; ++w) s += red[NW + w];
    double tau = 0.0, beta = alpha, scal = 0.0;
    if (s > 0.0) {
      beta = -std::copysign(std::sqrt(alpha * alpha + s), alpha);
      tau = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    const int64_t nv = M - j - 1;
    for (int64_t i = tid; i < nv; i += NT) {
      const double v = pcol[j + 1 + i] * scal;
      pcol[j + 1 + i] = v;
      if (i < vcap) vl[i] = v;
    }
    __syncthreads();   // the reflector is in LDS and in the block; beta is not yet stored
    if (tid == 0) pcol[j] = beta;

    // apply H to every remaining column and recompute its sum of squares below row j
    for (int c = j + 1 + wave; c < K; c += NW) {
      double *col = A + (int64_t)colmap[c] * ld;
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
  for (int c = tid; c < K; c += NT) piv_out[c0 + c] = colmap[c];
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
// a_off, prow (int64); then p_off (int64) and rank (int32) per block; the
// blocked QR's panel T (kPanel^2 doubles) per block; then the per-column table
// rows ta, tb (int32).
struct MetaLayout {
  int64_t poff, rank, tq, ta, tb, total;
  MetaLayout(int64_t count, int64_t tc) {
    poff = round256((5 * count + 1) * 8);
    rank = poff + round256(count * 8);
    tq = rank + round256(count * 4);                       // per block: T of the current panel
    ta = tq + round256(count * kPanel * kPanel * 8);
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
  std::vector<int64_t> h(5 * (size_t)count + 1, 0);
  for (int32_t b = 0; b < count; ++b) {
    const int64_t K = col_off[b + 1] - col_off[b];
    h[b] = row0 ? row0[b] : 0;
    h[count + b] = rows[b];
    h[3 * (size_t)count + 1 + b] = a_off[b];
    h[4 * (size_t)count + 1 + b] = reduce_first(rows[b], K) ? K : rows[b];
  }
  for (int32_t b = 0; b <= count; ++b) h[2 * (size_t)count + b] = col_off[b];
  char *base = static_cast<char *>(ws);
  hipError_t e = hipMemcpyAsync(base, h.data(), h.size() * sizeof(int64_t), hipMemcpyHostToDevice, st);
  const int64_t *d = reinterpret_cast<const int64_t *>(base);
  md->row0 = d;
  md->rows = d + count;
  md->col_off = d + 2 * (size_t)count;
  md->a_off = d + 3 * (size_t)count + 1;
  md->prow = d + 4 * (size_t)count + 1;
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
  // rows the pivoted QR works on: K for blocks reduced first, else all rows
  int64_t pmax = 0;
  bool any_reduce = false;
  for (int32_t b = 0; b < count; ++b) {
    const int64_t K = col_off[b + 1] - col_off[b];
    const bool r = reduce_first(rows[b], K);
    any_reduce = any_reduce || r;
    pmax = std::max(pmax, r ? K : rows[b]);
  }
  const int64_t vcap = std::min<int64_t>(pmax, (lds_max - fixed) / 8);
  const int64_t lds = (kmax + vcap + 3 * kIdWaves) * 8 + kmax * 4;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Meta md;
  st = stage_meta(who, count, nullptr, rows, col_off, a_off, nullptr, nullptr, nullptr, nullptr, ws, ws_bytes, s, &md);
  if (st != BFMHT_OK) return st;
  if (any_reduce) {
    double *tq = reinterpret_cast<double *>(static_cast<char *>(ws) + MetaLayout(count, col_off[count]).tq);
    int64_t kred = 0;   // widest reduced block
    for (int32_t b = 0; b < count; ++b) {
      const int64_t K = col_off[b + 1] - col_off[b];
      if (reduce_first(rows[b], K)) kred = std::max(kred, K);
    }
    hipError_t e0 = hipSuccess;
    for (int p0 = 0; p0 < kred && e0 == hipSuccess; p0 += kPanel) {
      hipLaunchKernelGGL(hqr_panel_kernel, dim3((unsigned)count), dim3(kPanelThreads), 0, s, md, p0, a, tq);
      const int64_t ntrail = kred - p0 - kPanel;
      if (ntrail > 0) {
        const int ngroups = (int)((ntrail + kTrailCols - 1) / kTrailCols);
        const int64_t nwg = ((int64_t)(count + 7) / 8) * 8 * ngroups;   // whole rounds of 8 blocks
        if (nwg >= (int64_t(1) << 31)) return bfmht::set_error(BFMHT_EINVAL, std::string(who) + ": too many blocks");
        hipLaunchKernelGGL(hqr_trail_kernel, dim3((unsigned)nwg), dim3(kTrailThreads), 0, s, md, (int)count, ngroups,
                           p0, a, (const double *)tq);
      }
      e0 = hipGetLastError();
    }
    if (e0 == hipSuccess) {
      hipLaunchKernelGGL(hqr_clear_kernel, dim3((unsigned)count), dim3(256), 0, s, md, a);
      e0 = hipGetLastError();
    }
    if (e0 != hipSuccess) return bfmht::set_error(BFMHT_EHIP, std::string(who) + ": " + hipGetErrorString(e0));
  }
  // registers per lane for the cached column: the smallest R with 64 R >= the longest reflector
  const int64_t nvmax = std::max<int64_t>(pmax - 1, 0);
  const int R = nvmax > vcap ? 0 : nvmax <= 256 ? 4 : nvmax <= 1024 ? 16 : nvmax <= 2048 ? 32 : nvmax <= 4096 ? 64 : 0;
  const void *fn = R == 4    ? reinterpret_cast<const void *>(cpqr_kernel<4, 512>)
                   : R == 16 ? reinterpret_cast<const void *>(cpqr_kernel<16, 512>)
                   : R == 32 ? reinterpret_cast<const void *>(cpqr_kernel<32, 512>)
                   : R == 64 ? reinterpret_cast<const void *>(cpqr_kernel<64, 256>)
                             : reinterpret_cast<const void *>(cpqr_kernel<0, 512>);
  hipError_t e = hipSuccess;
  if (lds > 65536) e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess) {
    const dim3 grid((unsigned)count), block(512), block4(256);
    const int ik = (int)kmax, iv = (int)vcap;
    if (R == 4) hipLaunchKernelGGL((cpqr_kernel<4, 512>), grid, block, (size_t)lds, s, md, ik, iv, a, tol, rank, piv);
    else if (R == 16) hipLaunchKernelGGL((cpqr_kernel<16, 512>), grid, block, (size_t)lds, s, md, ik, iv, a, tol, rank, piv);
    else if (R == 32) hipLaunchKernelGGL((cpqr_kernel<32, 512>), grid, block, (size_t)lds, s, md, ik, iv, a, tol, rank, piv);
    else if (R == 64) hipLaunchKernelGGL((cpqr_kernel<64, 256>), grid, block4, (size_t)lds, s, md, ik, iv, a, tol, rank, piv);
    else hipLaunchKernelGGL((cpqr_kernel<0, 512>), grid, block, (size_t)lds, s, md, ik, iv, a, tol, rank, piv);
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
