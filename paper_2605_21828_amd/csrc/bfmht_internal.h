// Internal layout shared by the host plan (plan.cpp) and the HIP kernels (kernels.hip).
//
// An apply is a sequence of stages.  Each stage is a grouped GEMM over jobs of
// uneven size; every job reads rows of its source buffer and writes rows of its
// destination buffer.
//   forward stage 0      : y_0[q]        = P_0j  c[koff[j] ..]          (src = c)
//   forward stage l=1..L : y_l[q]        = P_lq  y_{l-1}[pair rows]     (level buffers)
//   forward final stage  : f[perm_x[..]] = U_i   y_L[i]                 (dst = f, row map)
// The transposed stages run in reverse, after f's rows are gathered into tree
// order; a transposed job owns one contiguous run of output rows (the pair of
// input blocks of a forward level) and sums the transposed products of its
// consumers, so no two jobs write the same row.
//
// Factor blocks are stored twice: row-major W (M x K, row stride ldw) for the
// forward stages and row-major W^T (K x M, row stride ldwt) for the transposed
// stages, so both directions stream factor rows with the same access pattern.
// A block with the column-ID form P = [I T] Pi^T keeps only T in the forward
// pool and only the rows of T^T in the transposed pool (see FwdJob and BwdJob).
#pragma once
#include <stdint.h>

#include <string>

#include "../../include/bfmht.h"

namespace bfmht {

// Host side of the C ABI (plan.cpp): record the calling thread's error message
// and return s; one single apply of plan p (forward or transposed) with the two
// level buffers in ws (checked like bfmht_apply's workspace).
bfmht_status set_error(bfmht_status s, const std::string &msg);
bfmht_status apply_with_workspace(const bfmht_plan *p, bool fwd, const void *in, int64_t ldin, void *out,
                                  int64_t ldout, int32_t nrhs, void *ws, int64_t ws_bytes, void *stream);

// One forward GEMM job: dst rows = W (M x K, row stride ldw) * src rows.
// A column interpolative decomposition P = [I T] Pi^T keeps, for every output
// row i, one skeleton input row s_i whose column of P is the unit vector e_i.
// The forward pool stores only T (the non-skeleton columns, in increasing
// order) and the job adds the skeleton rows in its epilogue:
//   y_i = x[s_i] + sum_t T[i, t] x[c_t]
// The input rows of the reduction (c_t) and the skeleton rows (s_i) are listed
// in the plan's row-index table at map_off: K entries c_t, then (when skel) M
// entries s_i, all relative to in_row.  Blocks without that structure store P
// itself with the identity list 0..K-1 and skel = 0.
struct FwdJob {
  int64_t w_off;   // element offset of W (T or P) in the forward pool; -1 = identity (copy)
  int32_t M;       // output rows
  int32_t K;       // rows of the reduction (columns of W)
  int32_t ldw;     // row stride of W in elements (K rounded up to 8)
  int32_t in_row;  // first source row of the block's input
  int32_t out_row; // first destination row, or first row-map index when the stage has a row map
  int32_t map_off; // first entry of the job's row indices in the index table (-1 for identity jobs)
  int32_t skel;    // 1: add the M skeleton rows (compact ID block)
  int32_t pad;
};

// One consumer of a transposed job: rows [lo, hi) of the job's (logical) rows
// reduce over M gradient rows with the stored W^T rows (one per logical row of
// the range, row stride ldwt); the job's other rows take nothing from this
// consumer's product.
struct Cons {
  int64_t wt_off;  // element offset of the range's first W^T row in the transposed pool; -1: no product
                   // (an identity consumer: in a job without a row-index table it adds its g rows directly)
  int32_t M;       // gradient rows read (rank of the consumer block)
  int32_t ldwt;    // row stride of W^T (M rounded up to 8)
  int32_t g_row;   // first gradient row
  int32_t lo, hi;  // logical rows with a product
  int32_t pad;
};

// One transposed job: dst[out_row .. out_row+K) = sum_c P_c^T g_c.  With a
// row-index table (map_off >= 0) the K logical rows are a permutation of the
// job's rows: entries map_off .. +K give each logical row's physical row, then
// per consumer K entries give the g row that a skeleton row takes from that
// consumer (-1: none).  The transposed pool at offset 0 holds a zero row.
// With 4-ary trees a job's rows have four consumers: two jobs share the rows,
// the second (accum = 1, launched after the first) adds its sum to them.
struct BwdJob {
  int32_t K;
  int32_t out_row;
  int32_t nc;      // number of consumers (1 or 2)
  int32_t map_off; // -1: logical rows are physical rows, no skeleton rows
  int32_t accum;   // 1: dst rows += this job's sum (dst first), else dst rows = the sum
  int32_t pad;
  Cons c[2];
};

struct Tile {
  int32_t job;
  int32_t m0;      // first output row of the tile inside the job
};

enum Prec { P_F64 = 0, P_F32 = 1, P_BF16X2 = 2, P_BF16X3 = 3 };

// Everything a stage launch needs, device pointers resolved.
struct StageArgs {
  const void *pool;       // factor pool of this direction (FP64, or FP32 for every other precision)
  const void *jobs;       // FwdJob* or BwdJob*
  const Tile *tiles;
  int32_t ntiles;
  int32_t vec;            // 1 when src rows may be read with 16-byte vector loads
  const void *src;
  int64_t lds;
  void *dst;
  int64_t ldd;
  const int32_t *rowmap;  // output row map of the forward leaf stage (perm_x), else nullptr
  const int32_t *maps;    // forward stages: the plan's row-index table (see FwdJob)
  int32_t nrhs;
};

// Zero bytes after the end of every factor pool region: one reduction chunk of
// any kernel (the kernels read whole chunks past a row's end; the BF16 kernels
// read 64 FP32 values per row and chunk).
constexpr int kPoolTailBytes = 256;

// Output rows per workgroup tile at one 16-row block per wave; tiles of twice
// that height (two blocks per wave) are the other shape.  The plan builds tile
// lists for both heights.
constexpr int kTileRows = 64;

// Launch one stage with tiles of `rows` (64 or 128) output rows and `cols`
// (16, 32 or 64) RHS columns; a.tiles must be the list built for that height.
// Returns 0 or a hipError_t value.
int launch_fwd_stage(int prec, const StageArgs &a, int rows, int cols, void *stream);
// Few right-hand sides: the vector-FMA stage kernel over the 64-row tile list
// (FP32/FP64, 1 <= nrhs <= kGemvMaxRhs).
constexpr int kGemvMaxRhs = 4;
int launch_gemv_stage(int prec, bool fwd, const StageArgs &a, void *stream);
int launch_bwd_stage(int prec, const StageArgs &a, int rows, int cols, void *stream);

// dst[r] = sum over the C copies k of src[inv[r C + k]] (rows of nrhs elements of
// esz bytes), as a balanced pairwise tree in copy order; C a power of two, at
// most kFoldMaxCopies.
constexpr int64_t kFoldMaxCopies = 1 << 15;
int launch_fold_sum(int esz, const void *src, int64_t lds, const int32_t *inv, int C, int64_t rows, void *dst,
                    int64_t ldd, int nrhs, void *stream);
// dst[r][c] = src[r][c] for r < rows, c < cols (esz-byte elements).
int launch_copy_block(int esz, const void *src, int64_t lds, int64_t rows, int cols, void *dst, int64_t ldd,
                      void *stream);
// dst[t] = src[perm[t]] for t < n (rows of nrhs elements of esz bytes).
int launch_gather_rows(int esz, const void *src, int64_t lds, const int32_t *perm, int64_t n, void *dst, int64_t ldd,
                       int nrhs, void *stream);

// dst[r] = s[r] * src[r] for r < rows (rows of nrhs elements of esz bytes); dst may equal src.
int launch_scale_rows(int esz, const void *s, const void *src, int64_t lds, int64_t rows, void *dst, int64_t ldd,
                      int nrhs, void *stream);

// LSQR vector kernels (lsqr.hip).  esz: 8 for double, 4 for float; every vector
// rows x b with ld = b unless a leading dimension is passed; scalars arrays of b.
constexpr int kLsqrMaxBlocks = 512;   // partial-sum rows of a column norm
int lsqr_norm_blocks(int64_t rows);
// u = y - coef u (u = y when coef is null); norm = column 2-norms of u; u *= 1 / norm.
int lsqr_normalize(int esz, const void *y, int64_t ldy, int64_t rows, int b, const void *coef, void *u,
                   void *partial, void *norm, void *inv, void *stream);
// one plane rotation per column (rhobar, phibar advance; cx, cw, rnorm written)
int lsqr_rotate(int esz, int b, const void *alpha, const void *beta, void *rhobar, void *phibar, void *cx, void *cw,
                void *rnorm, void *stream);
// x += cx w; w = v - cw w
int lsqr_update(int esz, void *x, int64_t ldx, void *w, const void *v, int64_t rows, int b, const void *cx,
                const void *cw, void *stream);
// x = 0; w = v
int lsqr_init(int esz, void *x, int64_t ldx, void *w, const void *v, int64_t rows, int b, void *stream);

// One stage of one instance inside a batched launch.
struct Segment {
  StageArgs a;
  int32_t fwd;     // 1: forward stage, 0: transposed stage
  int32_t bn;      // RHS columns per tile (16, 32, 64); with fm = 0 the vector-FMA column count (1, 2, 4)
  int32_t ny;      // column tiles
  int32_t fm;      // 16-row blocks per wave (tile height 64 fm); 0: vector-FMA kernel, 64-row tiles
  int64_t item0;   // first work item (block index) of this segment in its launch
  int64_t nitems;  // a.ntiles * ny
};

// Segments travel to the batched kernel as launch arguments (no device table),
// at most kSegsPerLaunch per launch.
constexpr int kSegsPerLaunch = 24;
struct SegPack {
  int32_t nseg;
  int32_t pad;
  Segment s[kSegsPerLaunch];
};
static_assert(sizeof(SegPack) <= 4096, "launch arguments are limited to 4 KB");

// One segment of a persistent batched launch (device table entry; the work
// order is built by persistent_sched.h).
struct PSegDev {
  StageArgs a;
  int32_t ny;      // column tiles per tile
  int32_t dep;     // table position whose items must all be finished first (-1: none)
  int64_t item0;   // first per-queue ticket of this segment
  int64_t need;    // finished items (all queues) the wait requires
};
// All segments in one launch of resident workgroups (64-row tiles, bn columns).
// sync: nseg + 9 int32 words, zero at launch (counters, queue heads, error word).
int launch_persistent(int prec, bool fwd, int bn, const PSegDev *segs, int32_t nseg, int64_t per_queue_total,
                      int32_t *sync, int64_t spin_limit, void *stream);
// p[0 .. n) = 0 with a kernel (no memset node when captured).
int fill_zero_i32(int32_t *p, int64_t n, void *stream);

// One launch over `items` work items of the pack's segments (item0 relative to the
// pack); the segments share the direction and the tile shape (bn x 64 fm).
int launch_batched_stage(int prec, bool fwd, int bn, int fm, const SegPack &pack, int64_t items, void *stream);
// One batched launch of few-RHS segments (each nrhs <= b, b in {1, 2, 4}) on the vector-FMA kernel.
int launch_batched_gemv(int prec, bool fwd, int b, const SegPack &pack, int64_t items, void *stream);

}  // namespace bfmht
