// Grouped GEMM stages of the butterfly apply on gfx950 (CDNA4).
//
// Every stage is a batch of small dense products of uneven size (Sec. 2: the
// level-0 bases, the transfer blocks of levels 1..L and the leaf column bases
// are each applied once per vector, which is why storage and apply cost
// coincide, Sec. 6.2).
//
// Work split.  A workgroup of 4 waves computes a (64 FM)-row x BN-column output
// tile of one job; each wave owns FM blocks of 16 rows and all BN columns, so
// every factor element is used by exactly one wave.  Factor rows therefore go
// straight from HBM into MFMA operand registers (no LDS round trip): per
// reduction chunk a lane loads 32 contiguous bytes of each of its rows, and the
// four lane groups together cover one 128-byte line per row.  The reduction
// index is permuted inside a chunk (lane group g and step t take k = KL g + t),
// which is legal because both operands use the same permutation.  The
// right-hand-side chunk (KC rows x BN columns) is shared by the 4 waves and
// staged through LDS, transposed so that each lane reads its KL consecutive k
// values with 16-byte LDS reads; with FM = 2 each of those reads feeds two
// MFMA row blocks.  LDS is double buffered: the loads of chunk c+1 are in
// flight while chunk c runs on the matrix cores, with one barrier per chunk.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "bfmht_internal.h"

namespace bfmht {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

template <typename T> struct Cfg;
template <> struct Cfg<float> {
  static constexpr int KC = 32;  // reduction depth per chunk
  typedef v4f acc_t;
};
template <> struct Cfg<double> {
  static constexpr int KC = 16;
  typedef v4d acc_t;
};

__device__ __forceinline__ v4f mfma16x16x4(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4d mfma16x16x4(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Row of accumulator register i of `lane` inside a 16x16 MFMA output tile (the
// column is lane % 16).  The FP32 form stacks registers inside a lane group;
// the FP64 form interleaves lane groups across registers.
__device__ __forceinline__ int acc_row(float, int lane, int i) { return 4 * (lane >> 4) + i; }
__device__ __forceinline__ int acc_row(double, int lane, int i) { return 4 * i + (lane >> 4); }

// Number of this wave's FM 16-row blocks that hold at least one row of the job
// (`left` = job rows from the wave's first row on); wave-uniform.
template <int FM>
__device__ __forceinline__ int active_blocks(int left) { return left <= 0 ? 0 : min(FM, (left + 15) >> 4); }

constexpr int kWaves = 4;
constexpr int kNT = 64 * kWaves;
static_assert(kTileRows == 16 * kWaves, "one 16-row MFMA block per wave at FM = 1");

// Copy N elements (N * sizeof(T) a multiple of 8 bytes) with 16- or 8-byte accesses.
template <typename T, int N>
__device__ __forceinline__ void copy_vec(T *dst, const T *src) {
  constexpr int bytes = N * (int)sizeof(T);
  if constexpr (bytes % 16 == 0) {
#pragma unroll
    for (int i = 0; i < bytes / 16; ++i) reinterpret_cast<uint4 *>(dst)[i] = reinterpret_cast<const uint4 *>(src)[i];
  } else {
    static_assert(bytes % 8 == 0, "vector copy granularity");
#pragma unroll
    for (int i = 0; i < bytes / 8; ++i) reinterpret_cast<uint2 *>(dst)[i] = reinterpret_cast<const uint2 *>(src)[i];
  }
}

// Destination row of output row r of a forward job (through the stage row map if any).
__device__ __forceinline__ int64_t out_row(const StageArgs &a, int32_t base, int r) {
  return a.rowmap ? (int64_t)a.rowmap[base + r] : (int64_t)(base + r);
}

// Identity block: copy rows [m0, m0 + rows) of the job (16-byte pieces on full-width
// tiles with 16-byte aligned rows, elements otherwise).
template <typename T, int BN>
__device__ __forceinline__ void copy_tile(const StageArgs &a, const FwdJob &J, int m0, int rows, int n0) {
  const T *src = static_cast<const T *>(a.src);
  T *dst = static_cast<T *>(a.dst);
  constexpr int V = 16 / (int)sizeof(T), NV = BN / V;
  if (a.vec && n0 + BN <= a.nrhs && a.ldd % V == 0 && reinterpret_cast<uintptr_t>(a.dst) % 16 == 0) {
    for (int e = threadIdx.x; e < rows * NV; e += kNT) {
      const int r = e / NV, c = (e % NV) * V;
      const int gr = m0 + r;
      if (gr < J.M)
        copy_vec<T, V>(dst + out_row(a, J.out_row, gr) * a.ldd + n0 + c, src + (int64_t)(J.in_row + gr) * a.lds + n0 + c);
    }
    return;
  }
  for (int e = threadIdx.x; e < rows * BN; e += kNT) {
    const int r = e / BN, c = e % BN;
    const int gr = m0 + r, gc = n0 + c;
    if (gr < J.M && gc < a.nrhs) dst[out_row(a, J.out_row, gr) * a.ldd + gc] = src[(int64_t)(J.in_row + gr) * a.lds + gc];
  }
}

// ---------------------------------------------------------------------------
// FP32 and FP64: 16x16x4 MFMA.

template <typename T, int BN>
struct Tiling {
  static constexpr int KC = Cfg<T>::KC;
  static constexpr int KL = KC / 4;                 // reduction values per lane per chunk
  static constexpr int FN = BN / 16;                // 16-column MFMA blocks per wave
  static constexpr int XPAD = 16 / (int)sizeof(T);  // 16-byte row padding of the LDS chunk
  static constexpr int XR = KC * BN / kNT;          // RHS values staged per thread per chunk
  static constexpr int XS = KC + XPAD;              // LDS row stride (elements) of the transposed chunk
  static constexpr int XBUF = BN * XS;              // elements per LDS buffer
  static_assert(XR >= 1 && (kNT / KC) * XR == BN, "staging split: one row per lane, column groups per KC lanes");
};

// Stage one RHS chunk: rows k0 .. k0+KC of the source into registers.  Thread t
// takes row k = t % KC and the XR columns of column group t / KC, so the
// transposed LDS writes of consecutive lanes hit consecutive addresses.  Rows
// are clamped and zeroed past the block, columns likewise past nrhs; with FULL
// (16-byte source rows and every column tile full, fixed per launch) the row
// segment is one vector load.  No branches: the pipelined loop keeps exact
// wait counts.
// MAP: the reduction's rows come through the job's row-index list; `mrow` is
// this thread's entry for the chunk (loaded one chunk ahead by the caller).
template <typename T, int BN, bool FULL, bool MAP>
__device__ __forceinline__ void load_x(T *xr, const StageArgs &a, int32_t base, int32_t nrows, int k0, int n0,
                                       int tid, int mrow) {
  typedef Tiling<T, BN> Tl;
  const int k = tid % Tl::KC, c = (tid / Tl::KC) * Tl::XR;
  const int gk = k0 + k;
  const int64_t srow = (int64_t)base + (MAP ? mrow : min(gk, nrows - 1));
  const T *row = static_cast<const T *>(a.src) + srow * a.lds;
  if constexpr (FULL) {
    copy_vec<T, Tl::XR>(xr, row + n0 + c);
  } else {
#pragma unroll
    for (int i = 0; i < Tl::XR; ++i) {
      const int gc = n0 + c + i;
      const T v = row[min(gc, a.nrhs - 1)];
      xr[i] = gc < a.nrhs ? v : T(0);
    }
  }
  const bool ok = gk < nrows;
#pragma unroll
  for (int i = 0; i < Tl::XR; ++i) xr[i] = ok ? xr[i] : T(0);
}

template <typename T, int BN>
__device__ __forceinline__ void store_x(T *Xs, const T *xr, int tid) {
  typedef Tiling<T, BN> Tl;
  const int k = tid % Tl::KC, c = (tid / Tl::KC) * Tl::XR;
#pragma unroll
  for (int i = 0; i < Tl::XR; ++i) Xs[(c + i) * Tl::XS + k] = xr[i];
}

// This lane's KL reduction values of factor row `wrow` for the chunk at k0.  A
// chunk may run past the row's end into the next row, or past the last row into
// the zero tail every pool carries (at least one chunk long); those values meet
// right-hand-side rows that load_x zeroed, so they add nothing and the load
// needs no guard.
template <typename T, int BN>
__device__ __forceinline__ void load_w(T *wr, const T *wrow, int k0, int lg) {
  typedef Tiling<T, BN> Tl;
  copy_vec<T, Tl::KL>(wr, wrow + k0 + Tl::KL * lg);
}

// acc += W_chunk (this wave's FM x 16 rows) * X_chunk (all BN columns).  A wave
// whose blocks all lie past the job's last row (`nact` = 0, wave-uniform) issues
// no MFMA.
template <typename T, int BN, int FM>
__device__ __forceinline__ void mma_chunk(typename Cfg<T>::acc_t (*acc)[BN / 16], const T (*wr)[Cfg<T>::KC / 4],
                                          const T *Xs, int lrow, int lg, int nact) {
  typedef Tiling<T, BN> Tl;
  if (nact <= 0) return;
#pragma unroll
  for (int fn = 0; fn < Tl::FN; ++fn) {
    T b[Tl::KL];
    copy_vec<T, Tl::KL>(b, &Xs[(fn * 16 + lrow) * Tl::XS + Tl::KL * lg]);
#pragma unroll
    for (int t = 0; t < Tl::KL; ++t)
#pragma unroll
      for (int fm = 0; fm < FM; ++fm) acc[fm][fn] = mfma16x16x4(wr[fm][t], b[t], acc[fm][fn]);
  }
}

// Reduction over one factor block: acc += W(rows of this wave) * src rows
// base .. base+nk, chunk by chunk with the loads two chunks ahead: step c
// issues chunk c+2's loads (register set (c+2) mod 3), runs chunk c on the
// matrix cores from LDS buffer c mod 2, stages chunk c+1's RHS (loaded one step
// earlier) into the other buffer and ends with the barrier that publishes it.
// Load indices are clamped to the last chunk, so every step issues the same
// loads and the loop body has no conditional memory operation (the compiler's
// wait counts stay exact); the clamped repeats near the end are L2 hits and are
// never multiplied.  Ends with a barrier, so a following call may restage the
// buffers.
template <typename T, int BN, int FM, bool FULL, bool MAP, bool TWO = false>
__device__ __forceinline__ void gemm_block(typename Cfg<T>::acc_t (*acc)[BN / 16], const T *const *wrow, int nk,
                                           const StageArgs &a, int32_t base, const int32_t *rmap, int n0, T *Xs,
                                           int tid, int lrow, int lg, int nact, const T *const *wrow1 = nullptr,
                                           int nk1 = 0, int32_t base1 = 0, int nact1 = 0) {
  // TWO: a second reduction (the other consumer of a transposed job) follows the
  // first in the same pipeline, so its first loads overlap the first one's last
  // chunks; chunk c < nch0 belongs to the first, the rest to the second.
  typedef Tiling<T, BN> Tl;
  const int nch0 = (nk + Tl::KC - 1) / Tl::KC;
  const int nchunk = nch0 + (TWO ? (nk1 + Tl::KC - 1) / Tl::KC : 0);
  if (nchunk <= 0) return;
  T w0[FM][Tl::KL], w1[FM][Tl::KL], w2[FM][Tl::KL], x0[Tl::XR], x1[Tl::XR];
  const int kx = tid % Tl::KC;
  int mrow = MAP ? rmap[min(kx, nk - 1)] : 0;
  // RHS first, then the next chunk's row index, then the factor rows: loads
  // complete in order, so the waits for the RHS (before staging it into LDS) and
  // for the row index (before the next chunk's RHS loads) leave the factor loads
  // in flight.
  auto load_chunk = [&](T (*w)[Tl::KL], T *x, int c) {
    c = min(c, nchunk - 1);
    const bool sec = TWO && c >= nch0;
    const int cl = sec ? c - nch0 : c;
    load_x<T, BN, FULL, MAP>(x, a, sec ? base1 : base, sec ? nk1 : nk, cl * Tl::KC, n0, tid, mrow);
    if (MAP) mrow = rmap[min((c + 1) * Tl::KC + kx, nk - 1)];
#pragma unroll
    for (int fm = 0; fm < FM; ++fm) load_w<T, BN>(w[fm], sec ? wrow1[fm] : wrow[fm], cl * Tl::KC, lg);
  };
  // factor chunk c lives in register set c mod 3, RHS chunk c in set c mod 2
  auto step = [&](T (*wc)[Tl::KL], const T *xn, T (*wl)[Tl::KL], T *xl, int c) {
    load_chunk(wl, xl, c + 2);
    mma_chunk<T, BN, FM>(acc, wc, Xs + (c & 1) * Tl::XBUF, lrow, lg, TWO && c >= nch0 ? nact1 : nact);
    store_x<T, BN>(Xs + ((c + 1) & 1) * Tl::XBUF, xn, tid);
    __syncthreads();
  };
  load_chunk(w0, x0, 0);
  load_chunk(w1, x1, 1);
  store_x<T, BN>(Xs, x0, tid);
  __syncthreads();
  for (int c = 0;; c += 6) {
    step(w0, x1, w2, x0, c);
    if (c + 1 >= nchunk) break;
    step(w1, x0, w0, x1, c + 1);
    if (c + 2 >= nchunk) break;
    step(w2, x1, w1, x0, c + 2);
    if (c + 3 >= nchunk) break;
    step(w0, x0, w2, x1, c + 3);
    if (c + 4 >= nchunk) break;
    step(w1, x1, w0, x0, c + 4);
    if (c + 5 >= nchunk) break;
    step(w2, x0, w1, x1, c + 5);
    if (c + 6 >= nchunk) break;
  }
}

// Tile epilogues.  Every index a lane needs (output rows, skeleton rows) is
// loaded first and every added value next, with clamped addresses and no
// per-element branch, so the loads go out together and the lane waits once;
// only the stores are predicated.  Accumulator element (fm, fn, i) holds job
// row rbase + 16 fm + acc_row(i) and column n0 + 16 fn + lane % 16.

// Forward: dst[out row] = acc (+ the skeleton row of a compact block).
template <typename T, int BN, int FM, typename Acc>
__device__ __forceinline__ void fwd_epilogue(const StageArgs &a, const FwdJob &J, const int32_t *rmap,
                                             Acc (*acc)[BN / 16], int rbase, int n0, int lane) {
  constexpr int FN = BN / 16;
  const T *src = static_cast<const T *>(a.src);
  T *dst = static_cast<T *>(a.dst);
  const int lrow = lane & 15;
  int gr[FM][4], orow[FM][4];
#pragma unroll
  for (int fm = 0; fm < FM; ++fm)
#pragma unroll
    for (int i = 0; i < 4; ++i) gr[fm][i] = min(rbase + fm * 16 + acc_row(T(0), lane, i), J.M - 1);
  if (a.rowmap) {
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
      for (int i = 0; i < 4; ++i) orow[fm][i] = a.rowmap[J.out_row + gr[fm][i]];
  } else {
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
      for (int i = 0; i < 4; ++i) orow[fm][i] = J.out_row + gr[fm][i];
  }
  if (J.skel) {   // skeleton rows: index, then values, all loads in flight together
    int srow[FM][4];
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
      for (int i = 0; i < 4; ++i) srow[fm][i] = J.in_row + rmap[J.K + gr[fm][i]];
    T x[FM][FN][4];
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < FN; ++fn)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          x[fm][fn][i] = src[(int64_t)srow[fm][i] * a.lds + min(n0 + fn * 16 + lrow, a.nrhs - 1)];
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < FN; ++fn)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[fm][fn][i] += x[fm][fn][i];
  }
#pragma unroll
  for (int fm = 0; fm < FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < FN; ++fn)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gc = n0 + fn * 16 + lrow;
        if (rbase + fm * 16 + acc_row(T(0), lane, i) < J.M && gc < a.nrhs)
          dst[(int64_t)orow[fm][i] * a.ldd + gc] = acc[fm][fn][i];
      }
}

// Transposed: dst[out_row + physical row] = acc + the gradient rows that
// skeleton rows (or identity consumers) take.  Rows that take nothing from a
// consumer read its first gradient row (a cached line) and add zero.
template <typename T, int BN, int FM, typename Acc>
__device__ __forceinline__ void bwd_epilogue(const StageArgs &a, const BwdJob &J, Acc (*acc)[BN / 16], int rbase,
                                             int n0, int lane) {
  constexpr int FN = BN / 16;
  const T *src = static_cast<const T *>(a.src);
  T *dst = static_cast<T *>(a.dst);
  const int lrow = lane & 15;
  const bool two = J.nc > 1;
  int gr[FM][4], prow[FM][4], g[2][FM][4];
#pragma unroll
  for (int fm = 0; fm < FM; ++fm)
#pragma unroll
    for (int i = 0; i < 4; ++i) gr[fm][i] = min(rbase + fm * 16 + acc_row(T(0), lane, i), J.K - 1);
  bool add[2];
  if (J.map_off >= 0) {
    const int32_t *jm = a.maps + J.map_off;
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        prow[fm][i] = jm[gr[fm][i]];
        g[0][fm][i] = jm[J.K + gr[fm][i]];
        g[1][fm][i] = jm[(two ? 2 : 1) * J.K + gr[fm][i]];   // a one-consumer job repeats consumer 0 (unused)
      }
    add[0] = true;
    add[1] = two;
  } else {
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
      for (int i = 0; i < 4; ++i) prow[fm][i] = g[0][fm][i] = g[1][fm][i] = gr[fm][i];
    add[0] = J.c[0].wt_off < 0;
    add[1] = two && J.c[1].wt_off < 0;
  }
#pragma unroll
  for (int ci = 0; ci < 2; ++ci) {
    if (!add[ci]) continue;
    const int64_t base = J.c[ci].g_row;
    T x[FM][FN][4];
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < FN; ++fn)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          x[fm][fn][i] = src[(base + max(g[ci][fm][i], 0)) * a.lds + min(n0 + fn * 16 + lrow, a.nrhs - 1)];
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < FN; ++fn)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[fm][fn][i] += g[ci][fm][i] >= 0 ? x[fm][fn][i] : T(0);
  }
  if (J.accum) {   // the second consumer pair of a 4-ary job: rows += this sum (clamped reads, no branch)
    T prev[FM][FN][4];
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < FN; ++fn)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          prev[fm][fn][i] = dst[(int64_t)(J.out_row + prow[fm][i]) * a.ldd + min(n0 + fn * 16 + lrow, a.nrhs - 1)];
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < FN; ++fn)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[fm][fn][i] = prev[fm][fn][i] + acc[fm][fn][i];
  }
#pragma unroll
  for (int fm = 0; fm < FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < FN; ++fn)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gc = n0 + fn * 16 + lrow;
        if (rbase + fm * 16 + acc_row(T(0), lane, i) < J.K && gc < a.nrhs)
          dst[(int64_t)(J.out_row + prow[fm][i]) * a.ldd + gc] = acc[fm][fn][i];
      }
}

// Forward stage tile: dst[out rows] = W (M x K) * src[in_row .. in_row+K).
template <typename T, int BN, int FM, bool FULL>
__device__ __forceinline__ void fwd_tile(const StageArgs &a, int tix, int ny, T *Xs) {
  typedef Tiling<T, BN> Tl;
  const Tile tile = a.tiles[tix];
  if (tile.job < 0) return;  // padding tile of a short XCD bin
  const FwdJob J = static_cast<const FwdJob *>(a.jobs)[tile.job];
  const int n0 = ny * BN;
  if (J.w_off < 0) {  // identity block: copy its rows
    copy_tile<T, BN>(a, J, tile.m0, kTileRows * FM, n0);
    return;
  }
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63, lrow = lane & 15, lg = lane >> 4;
  const int rbase = tile.m0 + wave * 16 * FM;
  const int nact = active_blocks<FM>(J.M - rbase);
  const T *wrow[FM];
#pragma unroll
  for (int fm = 0; fm < FM; ++fm)
    wrow[fm] = static_cast<const T *>(a.pool) + J.w_off + (int64_t)min(rbase + fm * 16 + lrow, J.M - 1) * J.ldw;
  typename Cfg<T>::acc_t acc[FM][Tl::FN];
#pragma unroll
  for (int fm = 0; fm < FM; ++fm)
#pragma unroll
    for (int i = 0; i < Tl::FN; ++i) acc[fm][i] = typename Cfg<T>::acc_t{0, 0, 0, 0};
  const int32_t *rmap = a.maps + J.map_off;
  gemm_block<T, BN, FM, FULL, true>(acc, wrow, J.K, a, J.in_row, rmap, n0, Xs, tid, lrow, lg, nact);
  fwd_epilogue<T, BN, FM>(a, J, rmap, acc, rbase, n0, lane);
}

// Transposed stage tile: dst[out_row .. out_row+K) = sum over consumers of
// P_c^T g_c.  Each consumer reduces over the tile rows of its range [lo, hi)
// (rows outside it read the pool's zero row, and a wave or tile that has none
// of them skips the product); skeleton rows and identity consumers add their
// gradient rows in the epilogue, and logical rows go to their physical rows.
template <typename T, int BN, int FM, bool FULL>
__device__ __forceinline__ void bwd_tile(const StageArgs &a, int tix, int ny, T *Xs) {
  typedef Tiling<T, BN> Tl;
  const Tile tile = a.tiles[tix];
  if (tile.job < 0) return;  // padding tile of a short XCD bin
  const BwdJob J = static_cast<const BwdJob *>(a.jobs)[tile.job];
  const int n0 = ny * BN;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63, lrow = lane & 15, lg = lane >> 4;
  const int rbase = tile.m0 + wave * 16 * FM;
  const int nact = active_blocks<FM>(J.K - rbase);
  typename Cfg<T>::acc_t acc[FM][Tl::FN];
#pragma unroll
  for (int fm = 0; fm < FM; ++fm)
#pragma unroll
    for (int i = 0; i < Tl::FN; ++i) acc[fm][i] = typename Cfg<T>::acc_t{0, 0, 0, 0};
  // both consumers' reductions in one pipeline; a consumer with no row of the
  // tile in its range (or an identity consumer) reduces over nothing
  const T *pool = static_cast<const T *>(a.pool);
  const T *wrow[2][FM];
  int nk[2], na[2];
  int32_t gb[2];
#pragma unroll
  for (int ci = 0; ci < 2; ++ci) {  // constant indices keep the job in registers
    const Cons C = J.c[ci];
    const bool on = ci < J.nc && C.wt_off >= 0 && C.hi > tile.m0 && C.lo < tile.m0 + 64 * FM;
    nk[ci] = on ? C.M : 0;
    gb[ci] = C.g_row;
    na[ci] = rbase < C.hi && rbase + 16 * FM > C.lo ? nact : 0;
#pragma unroll
    for (int fm = 0; fm < FM; ++fm) {   // rows of W^T are columns of P
      const int r = rbase + fm * 16 + lrow;
      wrow[ci][fm] = on && r >= C.lo && r < C.hi ? pool + C.wt_off + (int64_t)(r - C.lo) * C.ldwt : pool;
    }
  }
  gemm_block<T, BN, FM, FULL, false, true>(acc, wrow[0], nk[0], a, gb[0], nullptr, n0, Xs, tid, lrow, lg, na[0],
                                           wrow[1], nk[1], gb[1], na[1]);
  bwd_epilogue<T, BN, FM>(a, J, acc, rbase, n0, lane);
}

// ---------------------------------------------------------------------------
// BF16 split products.  A factor value w is stored in FP32 and split into 2 or
// 3 bfloat16 terms in registers when it is loaded (hi = bf16(w), lo = bf16(w -
// hi), lo2 = bf16(w - hi - lo), round to nearest even; each difference is exact
// in FP32), so the factor stream costs 4 bytes per entry for either split;
// right-hand-side values are split the same way when a chunk is staged into
// LDS (once per workgroup).  Products of terms whose indices sum to at most NTERM-1 are
// accumulated in FP32 by v_mfma_f32_16x16x32_bf16: hi*hi + hi*lo + lo*hi for
// two terms, plus hi*lo2 + lo*lo + lo2*hi for three.  Only the output layout of
// the instruction matters here: both operands use the same (lane group, element)
// -> k assignment, so any internal ordering of k is summed the same way.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Two values rounded to bf16 (round to nearest even) in one instruction
// (v_cvt_pk_bf16_f32): a in the low half, b in the high half.
__device__ __forceinline__ uint32_t cvt_pk_bf16(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){a, b}, bf16x2));
}
__device__ __forceinline__ float bf16_lo_f32(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi_f32(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

__device__ __forceinline__ v4f mfma_bf16(const uint4 &a, const uint4 &b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0, 0,
                                                 0);
}

template <int NTERM, int BN>
struct TilingB {
  static constexpr int KC = 64;               // reduction depth per chunk
  static constexpr int KL = KC / 4;           // values per lane per chunk (two 8-value MFMA steps)
  static constexpr int FN = BN / 16;
  static constexpr int XS = KC + 8;           // LDS row stride in bf16 (16-byte padding)
  static constexpr int XBUF = BN * XS;        // bf16 per term per buffer
  static constexpr int XP = BN / 8;           // columns per thread (32 row pairs x 8 column groups)
  static constexpr int XR = 2 * XP;           // RHS values staged per thread per chunk
  static_assert(kNT == 32 * 8 && KC == 64, "staging split: 32 row pairs x 8 column groups");
};

// Stage one FP32 RHS chunk (rows k0..k0+KC) split into NTERM bf16 terms,
// transposed.  Thread t takes rows 2 (t % 32) and 2 (t % 32) + 1 and the XP
// columns of column group t / 32; the two rows' terms of one column are packed
// into one 32-bit LDS word, so consecutive lanes write consecutive words.
template <int NTERM, int BN, bool FULL, bool MAP>
__device__ __forceinline__ void load_x_bf(float *xr, const StageArgs &a, int32_t base, int32_t nrows, int k0, int n0,
                                          int tid, const int *mrow) {
  typedef TilingB<NTERM, BN> Tl;
  const int k = 2 * (tid % 32), c = (tid / 32) * Tl::XP;
#pragma unroll
  for (int h = 0; h < 2; ++h) {  // clamped rows and columns, zeroed past the block / nrhs (no branches)
    const int gk = k0 + k + h;
    const int64_t srow = (int64_t)base + (MAP ? mrow[h] : min(gk, nrows - 1));
    const float *row = static_cast<const float *>(a.src) + srow * a.lds;
    if constexpr (FULL) {
      copy_vec<float, Tl::XP>(xr + h * Tl::XP, row + n0 + c);
    } else {
#pragma unroll
      for (int i = 0; i < Tl::XP; ++i) {
        const int gc = n0 + c + i;
        const float v = row[min(gc, a.nrhs - 1)];
        xr[h * Tl::XP + i] = gc < a.nrhs ? v : 0.f;
      }
    }
    const bool ok = gk < nrows;
#pragma unroll
    for (int i = 0; i < Tl::XP; ++i) xr[h * Tl::XP + i] = ok ? xr[h * Tl::XP + i] : 0.f;
  }
}

template <int NTERM, int BN>
__device__ __forceinline__ void store_x_bf(uint16_t *Xs, const float *xr, int tid) {
  typedef TilingB<NTERM, BN> Tl;
  const int k = 2 * (tid % 32), c = (tid / 32) * Tl::XP;
#pragma unroll
  for (int i = 0; i < Tl::XP; ++i) {
    // rows k (low half) and k + 1 (high half) of one column, split term by term
    uint32_t w[3];
    float r0 = xr[i], r1 = xr[Tl::XP + i];
#pragma unroll
    for (int t = 0; t < NTERM; ++t) {
      w[t] = cvt_pk_bf16(r0, r1);
      if (t + 1 < NTERM) {
        r0 -= bf16_lo_f32(w[t]);
        r1 -= bf16_hi_f32(w[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < NTERM; ++t)
      *reinterpret_cast<uint32_t *>(Xs + t * 2 * Tl::XBUF + (c + i) * Tl::XS + k) = w[t];
  }
}

// This lane's KL FP32 factor values of row `wrow` for the chunk at k0 (64
// bytes).  As for load_w, values past the row's end (the next row, or the zero
// tail of the pool) meet zeroed right-hand-side rows, so no guard.
template <int NTERM, int BN>
__device__ __forceinline__ void load_w_bf(float *wr, const float *wrow, int k0, int lg) {
  typedef TilingB<NTERM, BN> Tl;
  copy_vec<float, Tl::KL>(wr, wrow + k0 + Tl::KL * lg);
}

// Split KL FP32 values into NTERM bf16 terms, 8 values (one MFMA operand) per
// uint4: t[term][h] holds values 8h .. 8h+7, value 2j in the low half of word j.
template <int NTERM>
__device__ __forceinline__ void split_w_bf(uint4 (*t)[2], const float *w) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    uint32_t word[3][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float r0 = w[8 * h + 2 * j], r1 = w[8 * h + 2 * j + 1];
#pragma unroll
      for (int u = 0; u < NTERM; ++u) {
        word[u][j] = cvt_pk_bf16(r0, r1);
        if (u + 1 < NTERM) {
          r0 -= bf16_lo_f32(word[u][j]);
          r1 -= bf16_hi_f32(word[u][j]);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < NTERM; ++u) t[u][h] = uint4{word[u][0], word[u][1], word[u][2], word[u][3]};
  }
}

// A wave whose blocks all lie past the job's last row (`nact` = 0) issues no MFMA.
template <int NTERM, int BN, int FM>
__device__ __forceinline__ void mma_chunk_bf(v4f (*acc)[BN / 16], const float (*wf)[TilingB<NTERM, BN>::KL],
                                             const uint16_t *Xs, int lrow, int lg, int nact) {
  typedef TilingB<NTERM, BN> Tl;
  if (nact <= 0) return;
  uint4 wr[FM][NTERM][2];
#pragma unroll
  for (int fm = 0; fm < FM; ++fm) split_w_bf<NTERM>(wr[fm], wf[fm]);
#pragma unroll
  for (int fn = 0; fn < Tl::FN; ++fn) {
    const int off = (fn * 16 + lrow) * Tl::XS + Tl::KL * lg;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      uint4 b[NTERM];
#pragma unroll
      for (int t = 0; t < NTERM; ++t) b[t] = *reinterpret_cast<const uint4 *>(Xs + t * 2 * Tl::XBUF + off + 8 * h);
#pragma unroll
      for (int fm = 0; fm < FM; ++fm) {
        // smallest products first
        if constexpr (NTERM == 3) {
          acc[fm][fn] = mfma_bf16(wr[fm][2][h], b[0], acc[fm][fn]);
          acc[fm][fn] = mfma_bf16(wr[fm][1][h], b[1], acc[fm][fn]);
          acc[fm][fn] = mfma_bf16(wr[fm][0][h], b[2], acc[fm][fn]);
        }
        acc[fm][fn] = mfma_bf16(wr[fm][1][h], b[0], acc[fm][fn]);
        acc[fm][fn] = mfma_bf16(wr[fm][0][h], b[1], acc[fm][fn]);
        acc[fm][fn] = mfma_bf16(wr[fm][0][h], b[0], acc[fm][fn]);
      }
    }
  }
}

// Pipelined reduction over one factor block with split terms, in the same shape
// as gemm_block (no conditions in the loop body, tail peeled, final barrier).  Xs
// holds 2 buffers per term: term t buffer j at Xs + (2 t + j) XBUF.  wrow[fm][t]:
// term t of row fm.
template <int NTERM, int BN, int FM, bool FULL, bool MAP, bool TWO = false>
__device__ __forceinline__ void gemm_block_bf(v4f (*acc)[BN / 16], const float *const *wrow, int nk,
                                              const StageArgs &a, int32_t base, const int32_t *rmap, int n0,
                                              uint16_t *Xs, int tid, int lrow, int lg, int nact,
                                              const float *const *wrow1 = nullptr, int nk1 = 0,
                                              int32_t base1 = 0, int nact1 = 0) {
  typedef TilingB<NTERM, BN> Tl;
  const int nch0 = (nk + Tl::KC - 1) / Tl::KC;   // TWO: a second reduction follows in the same pipeline
  const int nchunk = nch0 + (TWO ? (nk1 + Tl::KC - 1) / Tl::KC : 0);
  if (nchunk <= 0) return;
  float wA[FM][Tl::KL], wB[FM][Tl::KL];
  float xB[Tl::XR];
  const int kx = 2 * (tid % 32);
  int mrow[2] = {MAP ? rmap[min(kx, nk - 1)] : 0, MAP ? rmap[min(kx + 1, nk - 1)] : 0};
  auto load_chunk = [&](float (*w)[Tl::KL], int c) {  // same order as in gemm_block
    const bool sec = TWO && c >= nch0;
    const int cl = sec ? c - nch0 : c;
    load_x_bf<NTERM, BN, FULL, MAP>(xB, a, sec ? base1 : base, sec ? nk1 : nk, cl * Tl::KC, n0, tid, mrow);
    if (MAP) {
      mrow[0] = rmap[min((c + 1) * Tl::KC + kx, nk - 1)];
      mrow[1] = rmap[min((c + 1) * Tl::KC + kx + 1, nk - 1)];
    }
#pragma unroll
    for (int fm = 0; fm < FM; ++fm) load_w_bf<NTERM, BN>(w[fm], sec ? wrow1[fm] : wrow[fm], cl * Tl::KC, lg);
  };
  auto na_of = [&](int c) { return TWO && c >= nch0 ? nact1 : nact; };
  uint16_t *X0 = Xs, *X1 = Xs + Tl::XBUF;
  load_chunk(wA, 0);
  store_x_bf<NTERM, BN>(X0, xB, tid);
  __syncthreads();
  int c = 0;
  for (; c + 2 < nchunk; c += 2) {
    load_chunk(wB, c + 1);
    mma_chunk_bf<NTERM, BN, FM>(acc, wA, X0, lrow, lg, na_of(c));
    store_x_bf<NTERM, BN>(X1, xB, tid);
    __syncthreads();
    load_chunk(wA, c + 2);
    mma_chunk_bf<NTERM, BN, FM>(acc, wB, X1, lrow, lg, na_of(c + 1));
    store_x_bf<NTERM, BN>(X0, xB, tid);
    __syncthreads();
  }
  // one or two chunks left; the last one always runs from wA (one code path)
  const bool two = c + 1 < nchunk;
  if (two) {
    load_chunk(wB, c + 1);
    mma_chunk_bf<NTERM, BN, FM>(acc, wA, X0, lrow, lg, na_of(c));
    store_x_bf<NTERM, BN>(X1, xB, tid);
    __syncthreads();
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
      for (int v = 0; v < Tl::KL; ++v) wA[fm][v] = wB[fm][v];
  }
  mma_chunk_bf<NTERM, BN, FM>(acc, wA, two ? X1 : X0, lrow, lg, na_of(two ? c + 1 : c));
  __syncthreads();
}

template <int NTERM, int BN, int FM, bool FULL>
__device__ __forceinline__ void fwd_tile_bf(const StageArgs &a, int tix, int ny, uint16_t *Xs) {
  typedef TilingB<NTERM, BN> Tl;
  const Tile tile = a.tiles[tix];
  if (tile.job < 0) return;  // padding tile of a short XCD bin
  const FwdJob J = static_cast<const FwdJob *>(a.jobs)[tile.job];
  const int n0 = ny * BN;
  if (J.w_off < 0) {  // identity block: copy its rows
    copy_tile<float, BN>(a, J, tile.m0, kTileRows * FM, n0);
    return;
  }
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63, lrow = lane & 15, lg = lane >> 4;
  const int rbase = tile.m0 + wave * 16 * FM;
  const int nact = active_blocks<FM>(J.M - rbase);
  const float *wrow[FM];
#pragma unroll
  for (int fm = 0; fm < FM; ++fm)
    wrow[fm] = static_cast<const float *>(a.pool) + J.w_off + (int64_t)min(rbase + fm * 16 + lrow, J.M - 1) * J.ldw;
  v4f acc[FM][Tl::FN];
#pragma unroll
  for (int fm = 0; fm < FM; ++fm)
#pragma unroll
    for (int i = 0; i < Tl::FN; ++i) acc[fm][i] = v4f{0, 0, 0, 0};
  const int32_t *rmap = a.maps + J.map_off;
  gemm_block_bf<NTERM, BN, FM, FULL, true>(acc, wrow, J.K, a, J.in_row, rmap, n0, Xs, tid, lrow, lg, nact);
  fwd_epilogue<float, BN, FM>(a, J, rmap, acc, rbase, n0, lane);
}

template <int NTERM, int BN, int FM, bool FULL>
__device__ __forceinline__ void bwd_tile_bf(const StageArgs &a, int tix, int ny, uint16_t *Xs) {
  typedef TilingB<NTERM, BN> Tl;
  const Tile tile = a.tiles[tix];
  if (tile.job < 0) return;  // padding tile of a short XCD bin
  const BwdJob J = static_cast<const BwdJob *>(a.jobs)[tile.job];
  const int n0 = ny * BN;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63, lrow = lane & 15, lg = lane >> 4;
  const int rbase = tile.m0 + wave * 16 * FM;
  const int nact = active_blocks<FM>(J.K - rbase);
  v4f acc[FM][Tl::FN];
#pragma unroll
  for (int fm = 0; fm < FM; ++fm)
#pragma unroll
    for (int i = 0; i < Tl::FN; ++i) acc[fm][i] = v4f{0, 0, 0, 0};
  const float *wrow[2][FM];   // both consumers in one pipeline, as in bwd_tile
  int nk[2], na[2];
  int32_t gb[2];
#pragma unroll
  for (int ci = 0; ci < 2; ++ci) {  // constant indices keep the job in registers
    const Cons C = J.c[ci];
    const bool on = ci < J.nc && C.wt_off >= 0 && C.hi > tile.m0 && C.lo < tile.m0 + 64 * FM;
    nk[ci] = on ? C.M : 0;
    gb[ci] = C.g_row;
    na[ci] = rbase < C.hi && rbase + 16 * FM > C.lo ? nact : 0;
#pragma unroll
    for (int fm = 0; fm < FM; ++fm) {
      const int r = rbase + fm * 16 + lrow;
      const int64_t roff = on && r >= C.lo && r < C.hi ? C.wt_off + (int64_t)(r - C.lo) * C.ldwt : 0;
      wrow[ci][fm] = static_cast<const float *>(a.pool) + roff;
    }
  }
  gemm_block_bf<NTERM, BN, FM, FULL, false, true>(acc, wrow[0], nk[0], a, gb[0], nullptr, n0, Xs, tid, lrow, lg,
                                                  na[0], wrow[1], nk[1], gb[1], na[1]);
  bwd_epilogue<float, BN, FM>(a, J, acc, rbase, n0, lane);
}

// ---------------------------------------------------------------------------
// One tile of any precision, tile width and height.

template <int P, int BN> struct LdsBytes;
template <int BN> struct LdsBytes<P_F64, BN> { static constexpr int bytes = 2 * Tiling<double, BN>::XBUF * 8; };
template <int BN> struct LdsBytes<P_F32, BN> { static constexpr int bytes = 2 * Tiling<float, BN>::XBUF * 4; };
template <int BN> struct LdsBytes<P_BF16X2, BN> { static constexpr int bytes = 2 * 2 * TilingB<2, BN>::XBUF * 2; };
template <int BN> struct LdsBytes<P_BF16X3, BN> { static constexpr int bytes = 2 * 3 * TilingB<3, BN>::XBUF * 2; };

template <int P, bool FWD, int BN, int FM, bool FULL>
__device__ __forceinline__ void run_tile(const StageArgs &a, int tix, int ny, void *lds) {
  if constexpr (P == P_F64 || P == P_F32) {
    typedef typename std::conditional<P == P_F64, double, float>::type T;
    if constexpr (FWD) fwd_tile<T, BN, FM, FULL>(a, tix, ny, static_cast<T *>(lds));
    else bwd_tile<T, BN, FM, FULL>(a, tix, ny, static_cast<T *>(lds));
  } else {
    constexpr int NTERM = P == P_BF16X2 ? 2 : 3;
    if constexpr (FWD) fwd_tile_bf<NTERM, BN, FM, FULL>(a, tix, ny, static_cast<uint16_t *>(lds));
    else bwd_tile_bf<NTERM, BN, FM, FULL>(a, tix, ny, static_cast<uint16_t *>(lds));
  }
}

// FULL launches (every column tile full, 16-byte source rows) stage the RHS with
// vector loads; the others load elements from clamped columns.
inline bool full_tiles(const StageArgs &a, int bn) { return a.vec && a.nrhs % bn == 0; }

// Workgroup b runs on XCD b % 8.  The tile list interleaves 8 bins (tile
// 8 s + x belongs to bin x), so block b takes bin x = b % 8 and walks that
// bin's tiles with the ny column tiles of each tile back to back: the column
// tiles of one factor tile share its rows through that XCD's L2.
template <int P, bool FWD, int BN, int FM, bool FULL>
__global__ __launch_bounds__(kNT) void stage_kernel(StageArgs a, int ny) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[LdsBytes<P, BN>::bytes];
  const int b = blockIdx.x, x = b & 7, s = b >> 3;
  run_tile<P, FWD, BN, FM, FULL>(a, (s / ny) * 8 + x, s % ny, lds);
}

template <int P, bool FWD, int BN, int FM>
static int launch_one(const StageArgs &a, void *stream) {
  if (a.ntiles == 0) return 0;
  if (a.ntiles % 8) return (int)hipErrorInvalidValue;  // tile lists come in whole rounds of 8 bins
  const int ny = (a.nrhs + BN - 1) / BN;
  const dim3 grid((unsigned)((int64_t)a.ntiles * ny));
  if (full_tiles(a, BN))
    hipLaunchKernelGGL((stage_kernel<P, FWD, BN, FM, true>), grid, dim3(kNT), 0, (hipStream_t)stream, a, ny);
  else
    hipLaunchKernelGGL((stage_kernel<P, FWD, BN, FM, false>), grid, dim3(kNT), 0, (hipStream_t)stream, a, ny);
  return (int)hipGetLastError();
}

template <int P, bool FWD>
static int launch_shape(const StageArgs &a, int rows, int cols, void *stream) {
  const bool tall = rows == 2 * kTileRows;
  switch (cols) {
    case 16: return tall ? launch_one<P, FWD, 16, 2>(a, stream) : launch_one<P, FWD, 16, 1>(a, stream);
    case 32: return tall ? launch_one<P, FWD, 32, 2>(a, stream) : launch_one<P, FWD, 32, 1>(a, stream);
    case 64: return tall ? launch_one<P, FWD, 64, 2>(a, stream) : launch_one<P, FWD, 64, 1>(a, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

template <bool FWD>
static int launch(int prec, const StageArgs &a, int rows, int cols, void *stream) {
  switch (prec) {
    case P_F64: return launch_shape<P_F64, FWD>(a, rows, cols, stream);
    case P_F32: return launch_shape<P_F32, FWD>(a, rows, cols, stream);
    case P_BF16X2: return launch_shape<P_BF16X2, FWD>(a, rows, cols, stream);
    case P_BF16X3: return launch_shape<P_BF16X3, FWD>(a, rows, cols, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

int launch_fwd_stage(int prec, const StageArgs &a, int rows, int cols, void *stream) {
  return launch<true>(prec, a, rows, cols, stream);
}
int launch_bwd_stage(int prec, const StageArgs &a, int rows, int cols, void *stream) {
  return launch<false>(prec, a, rows, cols, stream);
}

// ---------------------------------------------------------------------------
// Few right-hand sides (nrhs <= kGemvMaxRhs, FP32/FP64): the apply is a chain
// of matrix-vector products, bound by streaming the factors, and an MFMA tile
// would leave most of its columns idle.  This kernel keeps the stage's jobs,
// 64-row tiles and row-index tables, and computes with vector FMAs instead:
// 16 lanes share one factor row (16-byte loads, 256 contiguous bytes per row
// per instruction for FP32), a wave streams 4 rows at a time, and the
// reduction's RHS rows (B columns each, gathered through the row-index list in
// the forward direction) are staged into LDS kGemvKX rows per pass.

constexpr int kGemvKX = 512;   // reduction rows staged per pass

// Stage reduction rows [k0, k0 + kGemvKX) of one block (nk rows from source
// row base, through rmap when MAP) as Xs[k][B]; zero past nk and past nrhs.
template <typename T, int B, bool MAP>
__device__ __forceinline__ void gemv_stage_x(T *Xs, const StageArgs &a, int32_t base, const int32_t *rmap, int nk,
                                             int k0) {
  static_assert(kGemvKX % kNT == 0, "whole rows per thread");
  constexpr int U = kGemvKX / kNT;
  const T *src = static_cast<const T *>(a.src);
  // row indices first, then every value, then the (zero-masked) LDS stores
  int64_t row[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int gk = min(k0 + (int)threadIdx.x + u * kNT, nk - 1);
    row[u] = ((int64_t)base + (MAP ? rmap[gk] : gk)) * a.lds;
  }
  T v[U][B];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int j = 0; j < B; ++j) v[u][j] = src[row[u] + min(j, a.nrhs - 1)];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int k = (int)threadIdx.x + u * kNT;
    const bool ok = k0 + k < nk;
#pragma unroll
    for (int j = 0; j < B; ++j) Xs[k * B + j] = ok && j < a.nrhs ? v[u][j] : T(0);
  }
}

// acc[it][j] += sum over this lane's k of W[row it][k] X[k][j] for the staged
// pass (k0 .. k0 + kGemvKX).  wrow[it]: this lane group's factor row it; kmax[it]:
// the last 16-byte piece inside that row's storage (reads past the block read a
// valid piece and meet zero RHS rows).  w0 holds the pass's first step, loaded
// by the caller before the RHS staging so that the factor stream starts at once.
template <typename T, int B>
__device__ __forceinline__ void gemv_load(T (*w)[16 / sizeof(T)], const T *const *wrow, const int *kmax, int k) {
  constexpr int VW = 16 / (int)sizeof(T);
#pragma unroll
  for (int it = 0; it < 4; ++it) copy_vec<T, VW>(w[it], wrow[it] + min(k, kmax[it]));
}

template <typename T, int B>
__device__ __forceinline__ void gemv_fma(T (*acc)[B], const T (*w)[16 / sizeof(T)], const T *Xs, int kk) {
  constexpr int VW = 16 / (int)sizeof(T);
  T x[VW][B];
#pragma unroll
  for (int v = 0; v < VW; ++v)
#pragma unroll
    for (int j = 0; j < B; ++j) x[v][j] = Xs[(kk + v) * B + j];
#pragma unroll
  for (int it = 0; it < 4; ++it)
#pragma unroll
    for (int v = 0; v < VW; ++v)
#pragma unroll
      for (int j = 0; j < B; ++j) acc[it][j] += w[it][v] * x[v][j];
}

template <typename T, int B>
__device__ __forceinline__ void gemv_pass(T (*acc)[B], const T (*w0)[16 / sizeof(T)], const T *const *wrow,
                                          const int *kmax, const T *Xs, int nk, int k0, int kl) {
  constexpr int VW = 16 / (int)sizeof(T), KS = 16 * VW;
  const int kend = min(nk - k0, kGemvKX);
  gemv_fma<T, B>(acc, w0, Xs, kl * VW);   // the first step's factor values came with the staging
#pragma unroll 2
  for (int s = 1; s * KS < kend; ++s) {
    const int kk = s * KS + kl * VW;
    T w[4][VW];
    gemv_load<T, B>(w, wrow, kmax, k0 + kk);
    gemv_fma<T, B>(acc, w, Xs, kk);
  }
}

// Sum acc over the 16 lanes of a row group; afterwards every lane holds the sums.
template <typename T, int B>
__device__ __forceinline__ void gemv_reduce(T (*acc)[B]) {
#pragma unroll
  for (int it = 0; it < 4; ++it)
#pragma unroll
    for (int j = 0; j < B; ++j)
#pragma unroll
      for (int m = 8; m >= 1; m >>= 1) acc[it][j] += __shfl_xor(acc[it][j], m, 16);
}

// v[j] for a lane-varying j < B, by bit masks (a select chain would be turned
// into an indexed private-memory load).
template <typename T, int B>
__device__ __forceinline__ T pick_col(const T (&v)[B], int j) {
  typedef typename std::conditional<sizeof(T) == 8, uint64_t, uint32_t>::type U;
  U r = 0;
#pragma unroll
  for (int q = 0; q < B; ++q) r |= __builtin_bit_cast(U, v[q]) & (U)(-(int64_t)(j == q));
  return __builtin_bit_cast(T, r);
}

template <typename T, int B>
__device__ __forceinline__ void gemv_fwd_tile(const StageArgs &a, int tix, T *Xs) {
  constexpr int VW = 16 / (int)sizeof(T);
  const Tile tile = a.tiles[tix];
  if (tile.job < 0) return;
  const FwdJob J = static_cast<const FwdJob *>(a.jobs)[tile.job];
  if (J.w_off < 0) {
    copy_tile<T, 16>(a, J, tile.m0, kTileRows, 0);
    return;
  }
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, rg = lane >> 4, kl = lane & 15;
  const int32_t *rmap = a.maps + J.map_off;
  const T *wrow[4];
  int kmax[4], gr[4];
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    gr[it] = tile.m0 + 16 * wave + 4 * it + rg;
    wrow[it] = static_cast<const T *>(a.pool) + J.w_off + (int64_t)min(gr[it], J.M - 1) * J.ldw;
    kmax[it] = J.ldw - VW;
  }
  T acc[4][B];
#pragma unroll
  for (int it = 0; it < 4; ++it)
#pragma unroll
    for (int j = 0; j < B; ++j) acc[it][j] = T(0);
  for (int k0 = 0; k0 < J.K; k0 += kGemvKX) {
    T w0[4][VW];
    gemv_load<T, B>(w0, wrow, kmax, k0 + kl * VW);
    __syncthreads();
    gemv_stage_x<T, B, true>(Xs, a, J.in_row, rmap, J.K, k0);
    __syncthreads();
    gemv_pass<T, B>(acc, w0, wrow, kmax, Xs, J.K, k0, kl);
  }
  gemv_reduce<T, B>(acc);
  // epilogue: indices first, then the added rows, then the stores
  const T *src = static_cast<const T *>(a.src);
  T *dst = static_cast<T *>(a.dst);
  const int j = min(kl, a.nrhs - 1);
  int r[4], orow[4];
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    r[it] = min(gr[it], J.M - 1);
    orow[it] = a.rowmap ? a.rowmap[J.out_row + r[it]] : J.out_row + r[it];
  }
  T v[4];
#pragma unroll
  for (int it = 0; it < 4; ++it) v[it] = pick_col<T, B>(acc[it], kl);
  if (J.skel) {
    int srow[4];
#pragma unroll
    for (int it = 0; it < 4; ++it) srow[it] = J.in_row + rmap[J.K + r[it]];
    T x[4];
#pragma unroll
    for (int it = 0; it < 4; ++it) x[it] = src[(int64_t)srow[it] * a.lds + j];
#pragma unroll
    for (int it = 0; it < 4; ++it) v[it] += x[it];
  }
#pragma unroll
  for (int it = 0; it < 4; ++it)
    if (gr[it] < J.M && kl < a.nrhs) dst[(int64_t)orow[it] * a.ldd + kl] = v[it];
}

template <typename T, int B>
__device__ __forceinline__ void gemv_bwd_tile(const StageArgs &a, int tix, T *Xs) {
  constexpr int VW = 16 / (int)sizeof(T);
  const Tile tile = a.tiles[tix];
  if (tile.job < 0) return;
  const BwdJob J = static_cast<const BwdJob *>(a.jobs)[tile.job];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, rg = lane >> 4, kl = lane & 15;
  int gr[4];
#pragma unroll
  for (int it = 0; it < 4; ++it) gr[it] = tile.m0 + 16 * wave + 4 * it + rg;
  T acc[4][B];
#pragma unroll
  for (int it = 0; it < 4; ++it)
#pragma unroll
    for (int j = 0; j < B; ++j) acc[it][j] = T(0);
  const T *pool = static_cast<const T *>(a.pool);
#pragma unroll
  for (int ci = 0; ci < 2; ++ci) {
    if (ci >= J.nc) break;
    const Cons C = J.c[ci];
    if (C.wt_off < 0 || C.hi <= tile.m0 || C.lo >= tile.m0 + kTileRows) continue;   // no row of the tile reduces
    const T *wrow[4];
    int kmax[4];
#pragma unroll
    for (int it = 0; it < 4; ++it) {   // rows outside [lo, hi) read the pool's zero row (long enough for any M)
      const bool in = gr[it] >= C.lo && gr[it] < C.hi;
      wrow[it] = in ? pool + C.wt_off + (int64_t)(gr[it] - C.lo) * C.ldwt : pool;
      kmax[it] = in ? C.ldwt - VW : 1 << 30;
    }
    for (int k0 = 0; k0 < C.M; k0 += kGemvKX) {
      T w0[4][VW];
      gemv_load<T, B>(w0, wrow, kmax, k0 + kl * VW);
      __syncthreads();
      gemv_stage_x<T, B, false>(Xs, a, C.g_row, nullptr, C.M, k0);
      __syncthreads();
      gemv_pass<T, B>(acc, w0, wrow, kmax, Xs, C.M, k0, kl);
    }
  }
  gemv_reduce<T, B>(acc);
  // epilogue: indices first, then the added rows (rows that take nothing from a
  // consumer read its first gradient row and add zero), then the stores
  const T *src = static_cast<const T *>(a.src);
  T *dst = static_cast<T *>(a.dst);
  const int j = min(kl, a.nrhs - 1);
  const bool two = J.nc > 1;
  int r[4], prow[4], g[2][4];
  bool add[2];
#pragma unroll
  for (int it = 0; it < 4; ++it) r[it] = min(gr[it], J.K - 1);
  if (J.map_off >= 0) {
    const int32_t *jm = a.maps + J.map_off;
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      prow[it] = jm[r[it]];
      g[0][it] = jm[J.K + r[it]];
      g[1][it] = jm[(two ? 2 : 1) * J.K + r[it]];
    }
    add[0] = true;
    add[1] = two;
  } else {
#pragma unroll
    for (int it = 0; it < 4; ++it) prow[it] = g[0][it] = g[1][it] = r[it];
    add[0] = J.c[0].wt_off < 0;
    add[1] = two && J.c[1].wt_off < 0;
  }
  T v[4];
#pragma unroll
  for (int it = 0; it < 4; ++it) v[it] = pick_col<T, B>(acc[it], kl);
#pragma unroll
  for (int ci = 0; ci < 2; ++ci) {
    if (!add[ci]) continue;
    T x[4];
#pragma unroll
    for (int it = 0; it < 4; ++it) x[it] = src[(int64_t)(J.c[ci].g_row + max(g[ci][it], 0)) * a.lds + j];
#pragma unroll
    for (int it = 0; it < 4; ++it) v[it] += g[ci][it] >= 0 ? x[it] : T(0);
  }
  if (J.accum) {   // second consumer pair of a 4-ary job: rows += this sum
    T prev[4];
#pragma unroll
    for (int it = 0; it < 4; ++it) prev[it] = dst[(int64_t)(J.out_row + prow[it]) * a.ldd + j];
#pragma unroll
    for (int it = 0; it < 4; ++it) v[it] = prev[it] + v[it];
  }
#pragma unroll
  for (int it = 0; it < 4; ++it)
    if (gr[it] < J.K && kl < a.nrhs) dst[(int64_t)(J.out_row + prow[it]) * a.ldd + kl] = v[it];
}

template <typename T, bool FWD, int B>
__global__ __launch_bounds__(kNT) void gemv_stage_kernel(StageArgs a) {
  __shared__ __attribute__((aligned(16))) T Xs[kGemvKX * B];
  if constexpr (FWD) gemv_fwd_tile<T, B>(a, blockIdx.x, Xs);
  else gemv_bwd_tile<T, B>(a, blockIdx.x, Xs);
}

namespace {
template <typename T, bool FWD>
int launch_gemv_t(const StageArgs &a, void *stream) {
  const dim3 grid((unsigned)a.ntiles);
  hipStream_t s = (hipStream_t)stream;
  if (a.nrhs == 1) hipLaunchKernelGGL((gemv_stage_kernel<T, FWD, 1>), grid, dim3(kNT), 0, s, a);
  else if (a.nrhs == 2) hipLaunchKernelGGL((gemv_stage_kernel<T, FWD, 2>), grid, dim3(kNT), 0, s, a);
  else hipLaunchKernelGGL((gemv_stage_kernel<T, FWD, 4>), grid, dim3(kNT), 0, s, a);
  return (int)hipGetLastError();
}
}  // namespace

// Batched form: segments (stage k of several instances, each with nrhs <= B)
// decoded from the block index as in batched_stage_kernel.
template <typename T, bool FWD, int B>
__global__ __launch_bounds__(kNT) void batched_gemv_kernel(SegPack pack) {
  __shared__ __attribute__((aligned(16))) T Xs[kGemvKX * B];
  const int64_t g = blockIdx.x;
  int32_t lo = 0, hi = pack.nseg - 1;  // last segment whose first item is <= g
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (pack.s[mid].item0 <= g) lo = mid; else hi = mid - 1;
  }
  const Segment S = pack.s[lo];
  const int tix = (int)(g - S.item0);
  if constexpr (FWD) gemv_fwd_tile<T, B>(S.a, tix, Xs);
  else gemv_bwd_tile<T, B>(S.a, tix, Xs);
}

namespace {
template <typename T, bool FWD>
int launch_batched_gemv_t(int b, const SegPack &pack, dim3 grid, hipStream_t s) {
  if (b == 1) hipLaunchKernelGGL((batched_gemv_kernel<T, FWD, 1>), grid, dim3(kNT), 0, s, pack);
  else if (b == 2) hipLaunchKernelGGL((batched_gemv_kernel<T, FWD, 2>), grid, dim3(kNT), 0, s, pack);
  else hipLaunchKernelGGL((batched_gemv_kernel<T, FWD, 4>), grid, dim3(kNT), 0, s, pack);
  return (int)hipGetLastError();
}
}  // namespace

int launch_batched_gemv(int prec, bool fwd, int b, const SegPack &pack, int64_t items, void *stream) {
  if (items == 0) return 0;
  if (b != 1 && b != 2 && b != 4) return (int)hipErrorInvalidValue;
  const dim3 grid((unsigned)items);
  hipStream_t s = (hipStream_t)stream;
  if (prec == P_F64) return fwd ? launch_batched_gemv_t<double, true>(b, pack, grid, s)
                                : launch_batched_gemv_t<double, false>(b, pack, grid, s);
  if (prec == P_F32) return fwd ? launch_batched_gemv_t<float, true>(b, pack, grid, s)
                                : launch_batched_gemv_t<float, false>(b, pack, grid, s);
  return (int)hipErrorInvalidValue;
}

int launch_gemv_stage(int prec, bool fwd, const StageArgs &a, void *stream) {
  if (a.ntiles == 0) return 0;
  if (a.nrhs < 1 || a.nrhs > kGemvMaxRhs) return (int)hipErrorInvalidValue;
  if (prec == P_F64) return fwd ? launch_gemv_t<double, true>(a, stream) : launch_gemv_t<double, false>(a, stream);
  if (prec == P_F32) return fwd ? launch_gemv_t<float, true>(a, stream) : launch_gemv_t<float, false>(a, stream);
  return (int)hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Row gather into tree order: dst[t] = src[perm[t]] (rows of nrhs elements).
// The transposed apply reads its input through this copy, so every stage
// kernel reads contiguous rows.

template <typename T>
__global__ __launch_bounds__(kNT) void gather_rows_kernel(const T *src, int64_t lds, const int32_t *perm, int64_t n,
                                                          T *dst, int64_t ldd, int nrhs) {
  const int64_t total = n * nrhs;
  for (int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x; e < total; e += (int64_t)gridDim.x * kNT) {
    const int64_t t = e / nrhs, j = e % nrhs;
    dst[t * ldd + j] = src[(int64_t)perm[t] * lds + j];
  }
}

int launch_gather_rows(int esz, const void *src, int64_t lds, const int32_t *perm, int64_t n, void *dst, int64_t ldd,
                       int nrhs, void *stream) {
  const int64_t total = n * nrhs;
  if (total == 0) return 0;
  const unsigned grid = (unsigned)std::min<int64_t>((total + kNT - 1) / kNT, 8192);
  if (esz == 8)
    hipLaunchKernelGGL((gather_rows_kernel<double>), dim3(grid), dim3(kNT), 0, (hipStream_t)stream,
                       static_cast<const double *>(src), lds, perm, n, static_cast<double *>(dst), ldd, nrhs);
  else
    hipLaunchKernelGGL((gather_rows_kernel<float>), dim3(grid), dim3(kNT), 0, (hipStream_t)stream,
                       static_cast<const float *>(src), lds, perm, n, static_cast<float *>(dst), ldd, nrhs);
  return (int)hipGetLastError();
}

// Column block copy: dst[r][c] = src[r][c] for r < rows, c < cols (rows of
// esz-byte elements with leading dimensions lds and ldd).  Packs the columns
// of several instances that share one plan into one block, and unpacks them.
template <typename T>
__global__ __launch_bounds__(kNT) void copy_block_kernel(const T *src, int64_t lds, int64_t rows, int cols, T *dst,
                                                         int64_t ldd) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x; e < total; e += (int64_t)gridDim.x * kNT) {
    const int64_t r = e / cols, c = e % cols;
    dst[r * ldd + c] = src[r * lds + c];
  }
}

int launch_copy_block(int esz, const void *src, int64_t lds, int64_t rows, int cols, void *dst, int64_t ldd,
                      void *stream) {
  const int64_t total = rows * cols;
  if (total == 0) return 0;
  const unsigned grid = (unsigned)std::min<int64_t>((total + kNT - 1) / kNT, 8192);
  if (esz == 8)
    hipLaunchKernelGGL((copy_block_kernel<double>), dim3(grid), dim3(kNT), 0, (hipStream_t)stream,
                       static_cast<const double *>(src), lds, rows, cols, static_cast<double *>(dst), ldd);
  else
    hipLaunchKernelGGL((copy_block_kernel<float>), dim3(grid), dim3(kNT), 0, (hipStream_t)stream,
                       static_cast<const float *>(src), lds, rows, cols, static_cast<float *>(dst), ldd);
  return (int)hipGetLastError();
}

// Sum of row copies: dst[r] = the C rows src[inv[r C + k]] summed pairwise in a
// balanced tree over k (left to right within each pair), the order in which the
// transposed identity levels it replaces add them.  slot[d] holds the pending
// left operand of tree depth d; C is a power of two, at most 2^15.
template <typename T>
__global__ __launch_bounds__(kNT) void fold_sum_kernel(const T *src, int64_t lds, const int32_t *inv, int C,
                                                       int64_t rows, T *dst, int64_t ldd, int nrhs) {
  const int64_t total = rows * nrhs;
  for (int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x; e < total; e += (int64_t)gridDim.x * kNT) {
    const int64_t r = e / nrhs;
    const int j = (int)(e % nrhs);
    T slot[16] = {};
    for (int k = 0; k < C; ++k) {
      T carry = src[(int64_t)inv[r * C + k] * lds + j];
#pragma unroll
      for (int d = 0; d < 16; ++d) {
        if ((k >> d) & 1) {
          carry = slot[d] + carry;
        } else {
          slot[d] = carry;
          break;
        }
      }
    }
    int depth = 0;
    while ((1 << depth) < C) ++depth;
    T v = slot[0];
#pragma unroll
    for (int d = 1; d < 16; ++d) v = d == depth ? slot[d] : v;
    dst[r * ldd + j] = v;
  }
}

int launch_fold_sum(int esz, const void *src, int64_t lds, const int32_t *inv, int C, int64_t rows, void *dst,
                    int64_t ldd, int nrhs, void *stream) {
  const int64_t total = rows * nrhs;
  if (total == 0) return 0;
  if (C < 1 || C > kFoldMaxCopies || (C & (C - 1))) return (int)hipErrorInvalidValue;
  const unsigned grid = (unsigned)std::min<int64_t>((total + kNT - 1) / kNT, 8192);
  if (esz == 8)
    hipLaunchKernelGGL((fold_sum_kernel<double>), dim3(grid), dim3(kNT), 0, (hipStream_t)stream,
                       static_cast<const double *>(src), lds, inv, C, rows, static_cast<double *>(dst), ldd, nrhs);
  else
    hipLaunchKernelGGL((fold_sum_kernel<float>), dim3(grid), dim3(kNT), 0, (hipStream_t)stream,
                       static_cast<const float *>(src), lds, inv, C, rows, static_cast<float *>(dst), ldd, nrhs);
  return (int)hipGetLastError();
}

// Row scaling: dst[r] = s[r] * src[r] for r < rows (rows of nrhs elements);
// dst may equal src (same ld).  Carries the diagonal of the scaled applies.

template <typename T>
__global__ __launch_bounds__(kNT) void scale_rows_kernel(const T *s, const T *src, int64_t lds, int64_t rows, T *dst,
                                                         int64_t ldd, int nrhs) {
  const int64_t total = rows * nrhs;
  for (int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x; e < total; e += (int64_t)gridDim.x * kNT) {
    const int64_t r = e / nrhs, j = e % nrhs;
    dst[r * ldd + j] = s[r] * src[r * lds + j];
  }
}

int launch_scale_rows(int esz, const void *s, const void *src, int64_t lds, int64_t rows, void *dst, int64_t ldd,
                      int nrhs, void *stream) {
  const int64_t total = rows * nrhs;
  if (total == 0) return 0;
  const unsigned grid = (unsigned)std::min<int64_t>((total + kNT - 1) / kNT, 8192);
  if (esz == 8)
    hipLaunchKernelGGL((scale_rows_kernel<double>), dim3(grid), dim3(kNT), 0, (hipStream_t)stream,
                       static_cast<const double *>(s), static_cast<const double *>(src), lds, rows,
                       static_cast<double *>(dst), ldd, nrhs);
  else
    hipLaunchKernelGGL((scale_rows_kernel<float>), dim3(grid), dim3(kNT), 0, (hipStream_t)stream,
                       static_cast<const float *>(s), static_cast<const float *>(src), lds, rows,
                       static_cast<float *>(dst), ldd, nrhs);
  return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Many instances of uneven size per launch.  A batched apply runs one launch
// per stage position, tile shape (and group of kSegsPerLaunch instances):
// launch k holds the k-th stage of its instances that use this tile shape,
// each workgroup decoding (segment, tile, column tile) from its block index
// through the segments' first-item offsets.  Stages of one instance are
// ordered by the launch boundaries, so no workgroup ever waits on another.
// The segments are launch arguments.  One kernel per tile shape keeps its
// register count (and so its occupancy) that of the single-instance kernels.

template <int P, bool FWD, int BN, int FM>
__global__ __launch_bounds__(kNT) void batched_stage_kernel(SegPack pack) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[LdsBytes<P, BN>::bytes];
  const int64_t g = blockIdx.x;
  int32_t lo = 0, hi = pack.nseg - 1;  // last segment whose first item is <= g
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (pack.s[mid].item0 <= g) lo = mid; else hi = mid - 1;
  }
  const Segment S = pack.s[lo];  // by value: the selected segment only
  // the order of stage_kernel: item0 is a multiple of 8, so workgroup g runs on
  // XCD g % 8 = bin x of the segment's tile list and walks that bin's tiles with
  // the column tiles of each tile back to back (they share its factor rows in L2)
  const int64_t t = g - S.item0;
  const int64_t sb = t >> 3;
  const int nyt = (S.a.nrhs + BN - 1) / BN;
  const int tix = (int)((sb / nyt) * 8 + (t & 7)), ny = (int)(sb % nyt);
  if (S.a.vec && S.a.nrhs % BN == 0) run_tile<P, FWD, BN, FM, true>(S.a, tix, ny, lds);
  else run_tile<P, FWD, BN, FM, false>(S.a, tix, ny, lds);
}

namespace {
template <int P, bool FWD, int BN>
void launch_batched_bn(int fm, const SegPack &pack, dim3 grid, hipStream_t s) {
  if (fm == 2) hipLaunchKernelGGL((batched_stage_kernel<P, FWD, BN, 2>), grid, dim3(kNT), 0, s, pack);
  else hipLaunchKernelGGL((batched_stage_kernel<P, FWD, BN, 1>), grid, dim3(kNT), 0, s, pack);
}
template <int P, bool FWD>
void launch_batched_dir(int bn, int fm, const SegPack &pack, dim3 grid, hipStream_t s) {
  if (bn == 16) launch_batched_bn<P, FWD, 16>(fm, pack, grid, s);
  else if (bn == 32) launch_batched_bn<P, FWD, 32>(fm, pack, grid, s);
  else launch_batched_bn<P, FWD, 64>(fm, pack, grid, s);
}
template <int P>
void launch_batched_p(bool fwd, int bn, int fm, const SegPack &pack, dim3 grid, hipStream_t s) {
  if (fwd) launch_batched_dir<P, true>(bn, fm, pack, grid, s);
  else launch_batched_dir<P, false>(bn, fm, pack, grid, s);
}
}  // namespace

int launch_batched_stage(int prec, bool fwd, int bn, int fm, const SegPack &pack, int64_t items, void *stream) {
  if (items == 0) return 0;
  if ((bn != 16 && bn != 32 && bn != 64) || (fm != 1 && fm != 2)) return (int)hipErrorInvalidValue;
  const dim3 grid((unsigned)items);
  hipStream_t s = (hipStream_t)stream;
  switch (prec) {
    case P_F64: launch_batched_p<P_F64>(fwd, bn, fm, pack, grid, s); break;
    case P_F32: launch_batched_p<P_F32>(fwd, bn, fm, pack, grid, s); break;
    case P_BF16X2: launch_batched_p<P_BF16X2>(fwd, bn, fm, pack, grid, s); break;
    case P_BF16X3: launch_batched_p<P_BF16X3>(fwd, bn, fm, pack, grid, s); break;
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Persistent batched apply: every stage of every instance in one launch.  The
// work order (persistent_sched.h) lists segments stage-major in kQueues ticket
// queues, one per XCD bin of the tile lists; workgroup b serves queue b % 8.
// A workgroup takes a ticket (device-scope atomic) only after finishing its
// previous item, waits until its instance's previous stage has finished every
// item (a per-segment count), runs the tile and counts it.  The 8 XCDs have
// separate L2 caches: a finished tile's stores are written back with an
// agent-scope release fence by every thread before the count is raised (a
// release at agent scope), and the waiting side reads the count with an
// agent-scope acquire and fences again (acquire) before loading the level
// vector.  Every wait is bounded: past spin_limit polls the workgroup sets the
// error word and leaves; every workgroup leaves once the word is set, so the
// launch always ends.  sync: counters[nseg], heads[kQueues], err (int32).

constexpr int kPQueues = 8;

template <int P, bool FWD, int BN>
__global__ __launch_bounds__(kNT) void persistent_kernel(const PSegDev *segs, int32_t nseg, int64_t per_queue_total,
                                                         int32_t *sync, int64_t spin_limit) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[LdsBytes<P, BN>::bytes];
  __shared__ int64_t s_ticket;
  __shared__ int32_t s_ok;
  int32_t *counters = sync, *heads = sync + nseg, *err = sync + nseg + kPQueues;
  const int x = blockIdx.x % kPQueues;
  for (;;) {
    if (threadIdx.x == 0) {
      int64_t t = per_queue_total;   // leave when the error word is set
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
        t = __hip_atomic_fetch_add(heads + x, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_ticket = t;
    }
    __syncthreads();
    const int64_t t = s_ticket;
    if (t >= per_queue_total) break;
    int32_t lo = 0, hi = nseg - 1;   // last segment whose first ticket is <= t
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (segs[mid].item0 <= t) lo = mid; else hi = mid - 1;
    }
    const PSegDev S = segs[lo];
    if (threadIdx.x == 0) {
      int32_t ok = 1;
      if (S.dep >= 0) {
        int64_t spins = 0;
        while (__hip_atomic_load(counters + S.dep, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < S.need) {
          if (++spins > spin_limit || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            ok = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        if (!ok) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      s_ok = ok;
    }
    __syncthreads();
    if (!s_ok) break;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const int64_t u = t - S.item0;
    const int tix = (int)(u / S.ny) * kPQueues + x, col = (int)(u % S.ny);
    if (S.a.vec && S.a.nrhs % BN == 0) run_tile<P, FWD, BN, 1, true>(S.a, tix, col, lds);
    else run_tile<P, FWD, BN, 1, false>(S.a, tix, col, lds);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(counters + lo, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ __launch_bounds__(kNT) void fill_zero_kernel(int32_t *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kNT) p[i] = 0;
}

int fill_zero_i32(int32_t *p, int64_t n, void *stream) {
  if (n <= 0) return 0;
  const unsigned grid = (unsigned)std::min<int64_t>((n + kNT - 1) / kNT, 1024);
  hipLaunchKernelGGL(fill_zero_kernel, dim3(grid), dim3(kNT), 0, (hipStream_t)stream, p, n);
  return (int)hipGetLastError();
}

namespace {
template <int P, bool FWD, int BN>
int launch_persistent_t(const PSegDev *segs, int32_t nseg, int64_t per_queue_total, int32_t *sync,
                        int64_t spin_limit, hipStream_t s) {
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persistent_kernel<P, FWD, BN>, kNT, 0);
  if (e != hipSuccess) return (int)e;
  // resident workgroups, a whole number per queue, no more than the tickets need
  int64_t grid = (int64_t)std::max(per_cu, 1) * std::max(cus, 1);
  grid = std::min<int64_t>(grid, per_queue_total * kPQueues);
  grid = std::max<int64_t>(grid / kPQueues * kPQueues, kPQueues);
  hipLaunchKernelGGL((persistent_kernel<P, FWD, BN>), dim3((unsigned)grid), dim3(kNT), 0, s, segs, nseg,
                     per_queue_total, sync, spin_limit);
  return (int)hipGetLastError();
}
template <int P, bool FWD>
int launch_persistent_bn(int bn, const PSegDev *segs, int32_t nseg, int64_t pq, int32_t *sync, int64_t lim,
                         hipStream_t s) {
  if (bn == 16) return launch_persistent_t<P, FWD, 16>(segs, nseg, pq, sync, lim, s);
  if (bn == 32) return launch_persistent_t<P, FWD, 32>(segs, nseg, pq, sync, lim, s);
  return launch_persistent_t<P, FWD, 64>(segs, nseg, pq, sync, lim, s);
}
template <int P>
int launch_persistent_p(bool fwd, int bn, const PSegDev *segs, int32_t nseg, int64_t pq, int32_t *sync,
                        int64_t lim, hipStream_t s) {
  return fwd ? launch_persistent_bn<P, true>(bn, segs, nseg, pq, sync, lim, s)
             : launch_persistent_bn<P, false>(bn, segs, nseg, pq, sync, lim, s);
}
}  // namespace

int launch_persistent(int prec, bool fwd, int bn, const PSegDev *segs, int32_t nseg, int64_t per_queue_total,
                      int32_t *sync, int64_t spin_limit, void *stream) {
  if (per_queue_total == 0 || nseg == 0) return 0;
  if (bn != 16 && bn != 32 && bn != 64) return (int)hipErrorInvalidValue;
  hipStream_t s = (hipStream_t)stream;
  switch (prec) {
    case P_F64: return launch_persistent_p<P_F64>(fwd, bn, segs, nseg, per_queue_total, sync, spin_limit, s);
    case P_F32: return launch_persistent_p<P_F32>(fwd, bn, segs, nseg, per_queue_total, sync, spin_limit, s);
    case P_BF16X2: return launch_persistent_p<P_BF16X2>(fwd, bn, segs, nseg, per_queue_total, sync, spin_limit, s);
    case P_BF16X3: return launch_persistent_p<P_BF16X3>(fwd, bn, segs, nseg, per_queue_total, sync, spin_limit, s);
    default: return (int)hipErrorInvalidValue;
  }
}

}  // namespace bfmht
