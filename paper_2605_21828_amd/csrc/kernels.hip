// Grouped GEMM stages of the butterfly apply on gfx950 (CDNA4).
//
// Every stage is a batch of small dense products of uneven size (Sec. 2: the
// level-0 bases, the transfer blocks of levels 1..L and the leaf column bases
// are each applied once per vector; storage and apply cost coincide, Sec. 7.2).
// One workgroup (4 waves of 64 lanes) computes a BM x BN tile of one job's
// output; factor rows and right-hand-side rows are staged through LDS and fed to
// 16x16 MFMA tiles with FP32 (or FP64) accumulation.
#include <hip/hip_runtime.h>

#include "bfmht_internal.h"

namespace bfmht {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

template <typename T> struct Acc4;
template <> struct Acc4<float> { typedef v4f type; };
template <> struct Acc4<double> { typedef v4d type; };

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

constexpr int kBM = 64;   // output rows per workgroup
constexpr int kBK = 16;   // reduction depth staged per LDS round
constexpr int kNT = 256;  // threads per workgroup

int tile_rows(int /*prec*/, int /*nrhs*/) { return kBM; }

// Wave layout inside a BM x BN tile: WN waves across columns, 4/WN down rows.
template <int BN> struct Layout {
  static constexpr int WN = BN >= 64 ? 2 : 1;
  static constexpr int WM = 4 / WN;
  static constexpr int TM = kBM / WM;  // rows per wave
  static constexpr int TN = BN / WN;   // columns per wave
  static constexpr int FM = TM / 16;   // 16x16 MFMA blocks per wave
  static constexpr int FN = TN / 16;
};

// Source row of the t-th row of a job, through the stage row map if present.
__device__ __forceinline__ int64_t map_row(const int32_t *rowmap, int32_t base, int32_t t) {
  return rowmap ? (int64_t)rowmap[base + t] : (int64_t)(base + t);
}

// Inner product over one LDS round: acc += A_lds(rows of this wave) * B_lds(cols).
template <typename T, int BN>
__device__ __forceinline__ void mma_round(const T (*As)[kBK + 1], const T (*Bs)[BN + 1],
                                          typename Acc4<T>::type (&acc)[Layout<BN>::FM][Layout<BN>::FN],
                                          int wm, int wn, int lane) {
  typedef Layout<BN> Lt;
#pragma unroll
  for (int kk = 0; kk < kBK; kk += 4) {
    T a[Lt::FM], b[Lt::FN];
#pragma unroll
    for (int fm = 0; fm < Lt::FM; ++fm) a[fm] = As[wm * Lt::TM + fm * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
    for (int fn = 0; fn < Lt::FN; ++fn) b[fn] = Bs[kk + (lane >> 4)][wn * Lt::TN + fn * 16 + (lane & 15)];
#pragma unroll
    for (int fm = 0; fm < Lt::FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < Lt::FN; ++fn) acc[fm][fn] = mfma16x16x4(a[fm], b[fn], acc[fm][fn]);
  }
}

// Forward stage: dst[out rows] = W (M x K) * src[in_row .. in_row+K).
template <typename T, int BN>
__global__ __launch_bounds__(kNT) void fwd_stage_kernel(StageArgs a) {
  typedef Layout<BN> Lt;
  __shared__ T As[kBM][kBK + 1];
  __shared__ T Bs[kBK][BN + 1];
  const Tile tile = a.tiles[blockIdx.x];
  const FwdJob J = static_cast<const FwdJob *>(a.jobs)[tile.job];
  const int n0 = blockIdx.y * BN;
  const T *src = static_cast<const T *>(a.src);
  T *dst = static_cast<T *>(a.dst);
  const int tid = threadIdx.x;

  if (J.w_off < 0) {  // identity block: copy its rows
    for (int e = tid; e < kBM * BN; e += kNT) {
      const int r = e / BN, c = e % BN;
      const int gr = tile.m0 + r, gc = n0 + c;
      if (gr < J.M && gc < a.nrhs)
        dst[map_row(a.rowmap, J.out_row, gr) * a.ldd + gc] = src[(int64_t)(J.in_row + gr) * a.lds + gc];
    }
    return;
  }

  const T *W = static_cast<const T *>(a.pool) + J.w_off;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / Lt::WN, wn = wave % Lt::WN;
  typename Acc4<T>::type acc[Lt::FM][Lt::FN];
#pragma unroll
  for (int i = 0; i < Lt::FM; ++i)
#pragma unroll
    for (int j = 0; j < Lt::FN; ++j) acc[i][j] = typename Acc4<T>::type{0, 0, 0, 0};

  for (int k0 = 0; k0 < J.K; k0 += kBK) {
    for (int e = tid; e < kBM * kBK; e += kNT) {
      const int r = e / kBK, k = e % kBK;
      const int gr = tile.m0 + r, gk = k0 + k;
      As[r][k] = (gr < J.M && gk < J.K) ? W[(int64_t)gr * J.ldw + gk] : T(0);
    }
    for (int e = tid; e < kBK * BN; e += kNT) {
      const int k = e / BN, c = e % BN;
      const int gk = k0 + k, gc = n0 + c;
      Bs[k][c] = (gk < J.K && gc < a.nrhs) ? src[(int64_t)(J.in_row + gk) * a.lds + gc] : T(0);
    }
    __syncthreads();
    mma_round<T, BN>(As, Bs, acc, wm, wn, lane);
    __syncthreads();
  }

#pragma unroll
  for (int fm = 0; fm < Lt::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < Lt::FN; ++fn)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gr = tile.m0 + wm * Lt::TM + fm * 16 + acc_row(T(0), lane, i);
        const int gc = n0 + wn * Lt::TN + fn * 16 + (lane & 15);
        if (gr < J.M && gc < a.nrhs) dst[map_row(a.rowmap, J.out_row, gr) * a.ldd + gc] = acc[fm][fn][i];
      }
}

// Transposed stage: dst[out_row .. out_row+K) = sum over consumers of W_c^T g_c,
// identity consumers adding their gradient rows directly.
template <typename T, int BN>
__global__ __launch_bounds__(kNT) void bwd_stage_kernel(StageArgs a) {
  typedef Layout<BN> Lt;
  __shared__ T As[kBM][kBK + 1];
  __shared__ T Bs[kBK][BN + 1];
  const Tile tile = a.tiles[blockIdx.x];
  const BwdJob J = static_cast<const BwdJob *>(a.jobs)[tile.job];
  const int n0 = blockIdx.y * BN;
  const T *src = static_cast<const T *>(a.src);
  T *dst = static_cast<T *>(a.dst);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / Lt::WN, wn = wave % Lt::WN;
  typename Acc4<T>::type acc[Lt::FM][Lt::FN];
#pragma unroll
  for (int i = 0; i < Lt::FM; ++i)
#pragma unroll
    for (int j = 0; j < Lt::FN; ++j) acc[i][j] = typename Acc4<T>::type{0, 0, 0, 0};

  for (int ci = 0; ci < J.nc; ++ci) {
    const Cons C = J.c[ci];
    if (C.w_off < 0) continue;
    const T *W = static_cast<const T *>(a.pool) + C.w_off;
    for (int k0 = 0; k0 < C.M; k0 += kBK) {
      // A[r][k] = W[k0 + k][m0 + r]  (W^T restricted to this tile)
      for (int e = tid; e < kBM * kBK; e += kNT) {
        const int k = e / kBM, r = e % kBM;
        const int gr = tile.m0 + r, gk = k0 + k;
        As[r][k] = (gr < J.K && gk < C.M) ? W[(int64_t)gk * C.ldw + gr] : T(0);
      }
      for (int e = tid; e < kBK * BN; e += kNT) {
        const int k = e / BN, c = e % BN;
        const int gk = k0 + k, gc = n0 + c;
        Bs[k][c] = (gk < C.M && gc < a.nrhs) ? src[map_row(a.rowmap, C.g_row, gk) * a.lds + gc] : T(0);
      }
      __syncthreads();
      mma_round<T, BN>(As, Bs, acc, wm, wn, lane);
      __syncthreads();
    }
  }

#pragma unroll
  for (int fm = 0; fm < Lt::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < Lt::FN; ++fn)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gr = tile.m0 + wm * Lt::TM + fm * 16 + acc_row(T(0), lane, i);
        const int gc = n0 + wn * Lt::TN + fn * 16 + (lane & 15);
        if (gr < J.K && gc < a.nrhs) {
          T v = acc[fm][fn][i];
          for (int ci = 0; ci < J.nc; ++ci)
            if (J.c[ci].w_off < 0) v += src[map_row(a.rowmap, J.c[ci].g_row, gr) * a.lds + gc];
          dst[(int64_t)(J.out_row + gr) * a.ldd + gc] = v;
        }
      }
}

template <typename T, int BN>
static int launch_t(bool fwd, const StageArgs &a, void *stream) {
  if (a.ntiles == 0) return 0;
  dim3 grid(a.ntiles, (a.nrhs + BN - 1) / BN);
  if (fwd)
    hipLaunchKernelGGL((fwd_stage_kernel<T, BN>), grid, dim3(kNT), 0, (hipStream_t)stream, a);
  else
    hipLaunchKernelGGL((bwd_stage_kernel<T, BN>), grid, dim3(kNT), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

template <typename T>
static int launch_bn(bool fwd, const StageArgs &a, void *stream) {
  if (a.nrhs <= 16) return launch_t<T, 16>(fwd, a, stream);
  if (a.nrhs <= 32) return launch_t<T, 32>(fwd, a, stream);
  return launch_t<T, 64>(fwd, a, stream);
}

static int launch(bool fwd, int prec, const StageArgs &a, void *stream) {
  switch (prec) {
    case P_F64: return launch_bn<double>(fwd, a, stream);
    case P_F32: return launch_bn<float>(fwd, a, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

int launch_fwd_stage(int prec, const StageArgs &a, void *stream) { return launch(true, prec, a, stream); }
int launch_bwd_stage(int prec, const StageArgs &a, void *stream) { return launch(false, prec, a, stream); }

}  // namespace bfmht
