// Host side of the C ABI: factor validation, device layout, upload and stage dispatch.
//
// The factor set (Sec. 2, the set returned by the butterfly factorization) is
// laid out on the device as one pool of factor blocks in the plan's precision,
// each block row-major with its row stride rounded up to 8 elements (zero
// padded, so every row starts 16-byte aligned for any element type), followed
// by the job and tile tables of every stage and the space-tree permutation.
// Level vectors live in two caller-provided ping-pong buffers, row-major with
// ld = nrhs, blocks in space-major order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "../../include/bfmht.h"
#include "bfmht_internal.h"
#include "persistent_sched.h"

using namespace bfmht;

namespace {

thread_local std::string g_err;

bfmht_status fail(bfmht_status s, const std::string &msg) {
  g_err = msg;
  return s;
}

int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }
int64_t ipow(int64_t b, int e) {
  int64_t r = 1;
  while (e-- > 0) r *= b;
  return r;
}
int32_t ldw_of(int64_t k) { return (int32_t)align_up(k, 8); }

struct StageDesc {
  int kind;   // 0: level 0 (reads c), 1: transfer level, 2: final (writes f through perm_x)
  int level;
  bool skip = false;    // forward only: an all-identity level folded into the first later stage
  bool edge = false;    // forward only: the first stage after the folded levels (reads c)
  int64_t fjob0, nfjob;
  int64_t ftile0[2], nftile[2];   // tile lists for 64- and 128-row tiles
  // transposed jobs in up to two parts launched in turn: with 4-ary trees a
  // job has four consumers, two in part 0 (which writes its rows) and two in
  // part 1 (which adds to them); binary trees have part 0 only
  int64_t bjob0[2], nbjob[2];
  int64_t btile0[2][2], nbtile[2][2];   // [part][height]
};

}  // namespace

struct bfmht_plan {
  int prec = 0;
  int64_t n = 0, m = 0;
  int L = 0;
  int arity = 2;         // children per tree node (2 or 4)
  int extra_parts = 0;   // transposed stages with a second job part (4-ary trees)
  int32_t max_nrhs = 1;
  int64_t esz = 0;       // bytes per element of level buffers and I/O
  int64_t wsz = 0;       // bytes per element of the factor pool (FP64, else FP32; BF16 terms are split on load)
  std::vector<StageDesc> stages;
  std::vector<int64_t> level_rows;
  int64_t max_rows = 0;
  int64_t pool_elems = 0, tpool_elems = 0;
  int64_t stored_t = 0;            // factor entries of the transposed pool (compact blocks: T^T only)
  int64_t stored_fwd = 0;          // factor entries of the forward pool (compact blocks store T only)
  std::vector<int32_t> maps;       // forward jobs' row-index table
  int64_t off_maps = 0;
  bool leaf_merged = false;        // leaf bases merged into the last transfer level (stages 0..L)
  int nfold = 0;                   // transposed direction: folded all-identity levels (0: every stage runs)
  int fwd_edge = 0;                // forward direction: the first stage that runs (leading all-identity levels skipped)
  int64_t fold_copies = 0;         // copies of each row of c at level nfold-1
  std::vector<int32_t> fold_inv;   // per row of c, its level nfold-1 rows in space-node order
  int64_t off_fold = 0;
  int64_t off_pool = 0;    // forward pool
  int64_t off_tpool = 0;   // transposed pool
  int64_t off_fjobs = 0, off_bjobs = 0, off_tiles = 0, off_perm = 0, dev_bytes = 0;
  std::vector<unsigned char> staging;
  char *dev = nullptr;
  bool uploaded = false;
  // per-stage tile shape, [0] forward, [1] transposed: rows 64 or 128, cols 16/32/64 or 0 (by nrhs)
  std::vector<int32_t> rows[2], cols[2];
};

namespace {

bfmht_status validate(const bfmht_factors_host *f) {
  if (!f) return fail(BFMHT_EINVAL, "factors is NULL");
  if (f->n < 0 || f->m < 0) return fail(BFMHT_EINVAL, "negative n or m");
  if (f->n >= (1ll << 31) || f->m >= (1ll << 31)) return fail(BFMHT_EINVAL, "n or m exceeds 2^31-1");
  const int a = f->arity == 0 ? 2 : f->arity;
  if (a != 2 && a != 4) return fail(BFMHT_EINVAL, "arity must be 2 or 4 (0 means 2)");
  if (f->L < 0 || f->L * (a == 4 ? 2 : 1) > 24) return fail(BFMHT_EINVAL, "L out of range (arity^L above 2^24)");
  const int64_t nb = 1ll << (f->L * (a == 4 ? 2 : 1));
  if (!f->xoff || !f->koff || !f->rank || !f->ident || !f->P_off || !f->U_off || (f->n > 0 && !f->perm_x))
    return fail(BFMHT_EINVAL, "a required factor array is NULL");
  if (f->xoff[0] != 0 || f->xoff[nb] != f->n) return fail(BFMHT_EINVAL, "xoff must run from 0 to n");
  if (f->koff[0] != 0 || f->koff[nb] != f->m) return fail(BFMHT_EINVAL, "koff must run from 0 to m");
  for (int64_t i = 0; i < nb; ++i) {
    if (f->xoff[i + 1] < f->xoff[i]) return fail(BFMHT_EINVAL, "xoff not non-decreasing");
    if (f->koff[i + 1] < f->koff[i]) return fail(BFMHT_EINVAL, "koff not non-decreasing");
  }
  std::vector<unsigned char> seen(f->n, 0);
  for (int64_t t = 0; t < f->n; ++t) {
    const int64_t p = f->perm_x[t];
    if (p < 0 || p >= f->n || seen[p]) return fail(BFMHT_EINVAL, "perm_x is not a permutation of [0, n)");
    seen[p] = 1;
  }
  for (int lvl = 0; lvl <= f->L; ++lvl) {
    const int64_t nf = ipow(a, f->L - lvl);
    for (int64_t q = 0; q < nb; ++q) {
      const int64_t r = f->rank[lvl * nb + q];
      int64_t rin = 0;
      if (lvl == 0) {
        rin = f->koff[q + 1] - f->koff[q];
      } else {
        const int64_t i = q / nf, j = q % nf, p = i / a;
        const int64_t q1 = p * a * nf + a * j;   // first of the block's a inputs
        for (int t = 0; t < a; ++t) rin += f->rank[(lvl - 1) * nb + q1 + t];
      }
      if (r < 0 || r > rin)
        return fail(BFMHT_EINVAL, "rank out of range at level " + std::to_string(lvl) + " block " + std::to_string(q));
      if (f->ident[lvl * nb + q]) {
        if (r != rin) return fail(BFMHT_EINVAL, "identity block whose rank differs from its input rows");
      } else if (r > 0 && rin > 0) {
        const int64_t o = f->P_off[lvl * nb + q];
        if (!f->P || o < 0 || o + r * rin > f->P_len)
          return fail(BFMHT_EINVAL, "P_off out of bounds at level " + std::to_string(lvl) + " block " + std::to_string(q));
      }
    }
  }
  for (int64_t i = 0; i < nb; ++i) {
    const int64_t rows = f->xoff[i + 1] - f->xoff[i];
    const int64_t r = f->rank[f->L * nb + i];
    const int64_t o = f->U_off[i];
    if (rows * r > 0 && (!f->U || o < 0 || o + rows * r > f->U_len))
      return fail(BFMHT_EINVAL, "U_off out of bounds at leaf " + std::to_string(i));
  }
  return BFMHT_OK;
}

// Column ID structure P = [I T] Pi^T (r x k, row-major): finds for every row i
// a column holding exactly e_i (its skeleton column) and lists the other
// columns in increasing order.  False when some row has none.
bool split_id(const double *P, int64_t r, int64_t k, std::vector<int32_t> &jc, std::vector<int32_t> &jsk) {
  if (!P || r <= 0 || r >= k) return false;
  std::vector<int32_t> nz(k, 0), one_row(k, -1);
  std::vector<char> bad(k, 0);
  for (int64_t i = 0; i < r; ++i)
    for (int64_t c = 0; c < k; ++c) {
      const double v = P[i * k + c];
      if (v == 0.0) continue;
      ++nz[c];
      if (v == 1.0) one_row[c] = (int32_t)i; else bad[c] = 1;
    }
  jsk.assign(r, -1);
  std::vector<char> skel(k, 0);
  for (int64_t c = 0; c < k; ++c)
    if (nz[c] == 1 && !bad[c] && one_row[c] >= 0 && jsk[one_row[c]] < 0) {
      jsk[one_row[c]] = (int32_t)c;
      skel[c] = 1;
    }
  for (int64_t i = 0; i < r; ++i)
    if (jsk[i] < 0) return false;
  jc.clear();
  for (int64_t c = 0; c < k; ++c)
    if (!skel[c]) jc.push_back((int32_t)c);
  return true;
}

}  // namespace

extern "C" {

const char *bfmht_last_error(void) { return g_err.c_str(); }
const char *bfmht_version(void) { return "bfmht 0.1 gfx950"; }

bfmht_status bfmht_plan_create(const bfmht_factors_host *f, bfmht_precision prec, int32_t max_nrhs,
                               bfmht_plan **out) {
  return bfmht_plan_create_ex(f, prec, max_nrhs, 0, out);
}

}  // extern "C"

namespace {

// M = U P for one leaf: U (n x r) the leaf basis, P (r x k) its block of the
// last transfer level (NULL: the identity, k = r); all row-major, M n x k.  A P
// with the column-ID structure [I T] Pi^T takes U itself in its skeleton
// columns and U T in the others.
void leaf_product(const double *U, int64_t n, int64_t r, const double *P, int64_t k, double *M) {
  if (n == 0 || k == 0) return;
  if (!P) {
    std::memcpy(M, U, (size_t)(n * k) * sizeof(double));
    return;
  }
  std::vector<int32_t> jc, jsk;
  const bool cmp = split_id(P, r, k, jc, jsk);
  if (!cmp) {   // general P: every column by the product
    jc.resize(k);
    for (int64_t c = 0; c < k; ++c) jc[c] = (int32_t)c;
    jsk.clear();
  }
  const int64_t kt = (int64_t)jc.size();
  std::vector<double> T((size_t)(r * kt)), row((size_t)kt);
  for (int64_t b = 0; b < r; ++b)
    for (int64_t c = 0; c < kt; ++c) T[b * kt + c] = P[b * k + jc[c]];
  for (int64_t a = 0; a < n; ++a) {
    std::fill(row.begin(), row.end(), 0.0);
    for (int64_t b = 0; b < r; ++b) {
      const double u = U[a * r + b];
      const double *t = T.data() + b * kt;
      for (int64_t c = 0; c < kt; ++c) row[c] += u * t[c];
    }
    for (int64_t c = 0; c < kt; ++c) M[a * k + jc[c]] = row[c];
    for (size_t b = 0; b < jsk.size(); ++b) M[a * k + jsk[b]] = U[a * r + (int64_t)b];
  }
}

// Body of bfmht_plan_create_ex after argument checks; may throw std::bad_alloc
// (the caller turns that into a status).  *out is set only on success.
// merge_leaf: apply each leaf basis and its last transfer block as one block
// when that stores about as many entries (see below).
bfmht_status plan_build(const bfmht_factors_host *f, bfmht_precision prec, int32_t max_nrhs, bool compact_ids,
                        bool merge_leaf, bfmht_plan **out) {
  std::unique_ptr<bfmht_plan> owner(new bfmht_plan());
  bfmht_plan *p = owner.get();
  p->prec = prec;
  p->n = f->n;
  p->m = f->m;
  p->L = f->L;
  p->arity = f->arity == 0 ? 2 : f->arity;
  p->max_nrhs = max_nrhs;
  p->esz = prec == BFMHT_F64 ? 8 : 4;
  p->wsz = prec == BFMHT_F64 ? 8 : 4;
  const int L = f->L;
  const int A = p->arity;
  const int64_t nb = ipow(A, L);

  // Row offsets of every block inside its level buffer (space-major order).
  std::vector<std::vector<int64_t>> off(L + 1, std::vector<int64_t>(nb + 1, 0));
  p->level_rows.assign(L + 1, 0);
  for (int lvl = 0; lvl <= L; ++lvl) {
    for (int64_t q = 0; q < nb; ++q) off[lvl][q + 1] = off[lvl][q] + f->rank[lvl * nb + q];
    p->level_rows[lvl] = off[lvl][nb];
    if (off[lvl][nb] >= (1ll << 31)) {
      return fail(BFMHT_EINVAL, "level vector exceeds 2^31 rows");
    }
    p->max_rows = std::max(p->max_rows, off[lvl][nb]);
  }
  // A level buffer also holds the transposed apply's input gathered into tree
  // order (n rows) and the scaled apply's scaled coefficients (m rows).
  p->max_rows = std::max<int64_t>(p->max_rows, std::max<int64_t>(f->n, f->m));

  // Forward pool offsets of every stored block: W (rows x cols, stride
  // ldw_of(cols)), which for a compact ID block is T (its non-skeleton
  // columns).  The transposed pool is laid out per transposed job below.
  struct Src {
    const double *ptr;
    int64_t rows, cols;
    bool compact;
    std::vector<int32_t> jc, jsk;   // non-skeleton columns; skeleton column of every row
  };
  std::vector<Src> blocks;
  std::vector<int64_t> woff_P((size_t)(L + 1) * nb, -1), woff_U(nb, -1);
  int64_t pool = 0;
  // first of the A inputs of block q at level lvl (they are consecutive blocks of level lvl-1)
  auto child0 = [&](int lvl, int64_t q) -> int64_t {
    const int64_t nf = ipow(A, L - lvl), i = q / nf, j = q % nf;
    return (i / A) * A * nf + A * j;
  };
  auto rin_of = [&](int lvl, int64_t q) -> int64_t {
    if (lvl == 0) return f->koff[q + 1] - f->koff[q];
    const int64_t q1 = child0(lvl, q);
    int64_t r = 0;
    for (int t = 0; t < A; ++t) r += f->rank[(lvl - 1) * nb + q1 + t];
    return r;
  };
  // Leading levels whose blocks are all identities (folded, see below).
  int nfold = 0;
  while (nfold <= L) {
    bool all = true;
    for (int64_t q = 0; q < nb && all; ++q) all = f->ident[nfold * nb + q] != 0;
    if (!all) break;
    ++nfold;
  }
  // Leaf bases merged into the last transfer level.  f_i = U_i y_{L,i} and
  // y_{L,i} = P_{L,i} x, so the two products are one with the block U_i P_{L,i}
  // (n_i x K_i, K_i the block's input rows).  When the last level's ranks equal
  // the leaf sizes (full-rank leaf blocks, the usual case) that block has as
  // many entries as U_i and the compact P_{L,i} together, and applying it saves
  // a stage per direction and the write and read of y_L.  Merged when the
  // merged blocks hold at most 1/32 more entries than the separate ones, the
  // last level runs (it is not folded away) and L >= 1; the transposed
  // direction then reads the gathered f rows of each leaf as its consumer rows.
  bool merge = false;
  if (merge_leaf && L >= 1 && nfold <= L) {
    int64_t sep = 0, mrg = 0;
    std::vector<int32_t> jc, jsk;
    for (int64_t i = 0; i < nb; ++i) {
      const int64_t n_i = f->xoff[i + 1] - f->xoff[i], r = f->rank[L * nb + i], k = rin_of(L, i);
      int64_t pe = 0;
      if (!f->ident[L * nb + i] && r * k > 0)
        pe = split_id(f->P + f->P_off[L * nb + i], r, k, jc, jsk) ? r * (int64_t)jc.size() : r * k;
      sep += n_i * r + pe;
      mrg += n_i * k;
    }
    merge = 32 * mrg <= 33 * sep;
  }
  p->leaf_merged = merge;
  std::vector<int64_t> bidx_P((size_t)(L + 1) * nb, -1);
  for (int lvl = 0; lvl <= (merge ? L - 1 : L); ++lvl)
    for (int64_t q = 0; q < nb; ++q) {
      if (f->ident[lvl * nb + q]) continue;
      const int64_t r = f->rank[lvl * nb + q], k = rin_of(lvl, q);
      Src b{r * k ? f->P + f->P_off[lvl * nb + q] : nullptr, r, k, false, {}, {}};
      if (compact_ids) b.compact = split_id(b.ptr, r, k, b.jc, b.jsk);
      const int64_t kf = b.compact ? (int64_t)b.jc.size() : k;
      woff_P[lvl * nb + q] = pool;
      bidx_P[lvl * nb + q] = (int64_t)blocks.size();
      pool += r * ldw_of(kf);
      p->stored_fwd += r * kf;
      blocks.push_back(std::move(b));
    }
  std::vector<int64_t> bidx_U(nb, -1);
  std::vector<std::vector<double>> merged;   // U_i P_{L,i} per leaf (merged plans)
  if (merge) {
    merged.resize(nb);
    for (int64_t i = 0; i < nb; ++i) merged[i].assign((size_t)((f->xoff[i + 1] - f->xoff[i]) * rin_of(L, i)), 0.0);
    // leaves in parallel (each worker takes every nth leaf); a failed worker
    // reports through `bad` and the plan fails as out of memory
    const int nt = (int)std::max<int64_t>(1, std::min<int64_t>({16, nb, (int64_t)std::thread::hardware_concurrency()}));
    std::vector<char> bad(nt, 0);
    auto work = [&](int t) {
      try {
        for (int64_t i = t; i < nb; i += nt) {
          const int64_t n_i = f->xoff[i + 1] - f->xoff[i], r = f->rank[L * nb + i], k = rin_of(L, i);
          if (r == 0) continue;   // a rank-0 block: M stays zero
          const bool id = f->ident[L * nb + i] != 0 || k == 0;
          leaf_product(n_i * r ? f->U + f->U_off[i] : nullptr, n_i, r, id ? nullptr : f->P + f->P_off[L * nb + i], k,
                       merged[i].data());
        }
      } catch (...) {
        bad[t] = 1;
      }
    };
    std::vector<std::thread> pool_t;
    for (int t = 1; t < nt; ++t) pool_t.emplace_back(work, t);
    work(0);
    for (auto &th : pool_t) th.join();
    for (char b : bad)
      if (b) throw std::bad_alloc();
  }
  for (int64_t i = 0; i < nb; ++i) {
    const int64_t rows = f->xoff[i + 1] - f->xoff[i], r = merge ? rin_of(L, i) : f->rank[L * nb + i];
    woff_U[i] = pool;
    bidx_U[i] = (int64_t)blocks.size();
    const double *src = merge ? merged[i].data() : f->U + f->U_off[i];
    blocks.push_back({rows * r ? src : nullptr, rows, r, false, {}, {}});
    pool += rows * ldw_of(r);
    p->stored_fwd += rows * r;
  }
  // Row-index table entry of a forward job: the reduction's input rows, then
  // (compact blocks) the skeleton rows; identity jobs have none.
  auto add_map = [&](int64_t bi, int64_t k) -> int32_t {
    const int32_t at = (int32_t)p->maps.size();
    if (bi >= 0 && blocks[bi].compact) {
      p->maps.insert(p->maps.end(), blocks[bi].jc.begin(), blocks[bi].jc.end());
      p->maps.insert(p->maps.end(), blocks[bi].jsk.begin(), blocks[bi].jsk.end());
    } else {
      for (int64_t c = 0; c < k; ++c) p->maps.push_back((int32_t)c);
    }
    return at;
  };
  auto fjob = [&](int64_t w_off, int64_t bi, int64_t M, int64_t k, int64_t in_row, int64_t out_row) -> FwdJob {
    FwdJob J{};
    J.w_off = w_off;
    J.M = (int32_t)M;
    const bool cmp = bi >= 0 && blocks[bi].compact;
    J.K = (int32_t)(cmp ? (int64_t)blocks[bi].jc.size() : k);
    J.ldw = ldw_of(J.K);
    J.in_row = (int32_t)in_row;
    J.out_row = (int32_t)out_row;
    J.map_off = w_off < 0 ? -1 : add_map(bi, k);
    J.skel = cmp ? 1 : 0;
    return J;
  };
  p->pool_elems = pool;

  // Transposed pool: a zero region first (the W^T row of any tile row that a
  // consumer does not reduce over; as long as the longest row plus one
  // reduction chunk), then each transposed job's consumers' W^T rows.
  int64_t maxM = 0;
  for (const Src &b : blocks) maxM = std::max<int64_t>(maxM, b.rows);
  int64_t tpool = align_up(maxM + 64, 64);
  struct TRow { int64_t off; int64_t blk; int32_t col; };   // W^T row = column col of block blk
  std::vector<TRow> trows;
  // A transposed job: dst rows [out_row, out_row + K) = sum over its consumers
  // c of P_c^T g_c.  A consumer whose P_c has the column-ID form takes the
  // skeleton rows straight from g_c and reduces over its other rows only.  The
  // job's rows are then processed in a permuted (logical) order, sorted by
  // (skeleton for consumer 0, skeleton for consumer 1) as SS, SN, NN, NS, so
  // that each consumer's non-skeleton rows form one contiguous range; its W^T
  // rows are stored for that range only, in logical order.
  struct ConsIn { int64_t bi; bool ident; int32_t M; int32_t g_row; };
  auto bjob = [&](int32_t K, int32_t out_row, int nc, const ConsIn *ci) -> BwdJob {
    BwdJob J{};
    J.K = K;
    J.out_row = out_row;
    J.nc = nc;
    J.map_off = -1;
    bool any = false;
    for (int c = 0; c < nc; ++c) any = any || (!ci[c].ident && ci[c].bi >= 0 && blocks[ci[c].bi].compact);
    std::vector<int32_t> omap(K), st[2];
    for (int32_t k = 0; k < K; ++k) omap[k] = k;
    int32_t lo[2] = {0, 0}, hi[2] = {K, K};
    if (any) {
      for (int c = 0; c < nc; ++c) {
        st[c].assign(K, -1);   // g row of a skeleton row, -1 for a reduced row
        if (ci[c].ident) {
          for (int32_t k = 0; k < K; ++k) st[c][k] = k;
        } else if (ci[c].bi >= 0 && blocks[ci[c].bi].compact) {
          const Src &b = blocks[ci[c].bi];
          for (int64_t i = 0; i < b.rows; ++i) st[c][b.jsk[i]] = (int32_t)i;
        }
      }
      auto cls = [&](int32_t k) {
        const bool s0 = st[0][k] >= 0, s1 = nc > 1 && st[1][k] >= 0;
        return s0 ? (s1 ? 0 : 1) : (s1 ? 3 : 2);
      };
      std::stable_sort(omap.begin(), omap.end(), [&](int32_t x, int32_t y) { return cls(x) < cls(y); });
      int32_t cnt[4] = {0, 0, 0, 0};
      for (int32_t k = 0; k < K; ++k) ++cnt[cls(k)];
      lo[0] = cnt[0] + cnt[1];
      hi[0] = K;
      lo[1] = cnt[0];
      hi[1] = cnt[0] + cnt[1] + cnt[2];
      J.map_off = (int32_t)p->maps.size();
      p->maps.insert(p->maps.end(), omap.begin(), omap.end());
      for (int c = 0; c < nc; ++c)
        for (int32_t r = 0; r < K; ++r) p->maps.push_back(st[c][omap[r]]);
    }
    for (int c = 0; c < nc; ++c) {
      Cons &C = J.c[c];
      C.M = ci[c].M;
      C.ldwt = ldw_of(C.M);
      C.g_row = ci[c].g_row;
      if (ci[c].ident) {   // identity consumer: no rows reduced (without maps the kernel adds g rows itself)
        C.wt_off = -1;
        C.lo = C.hi = 0;
        continue;
      }
      C.lo = lo[c];
      C.hi = C.M > 0 ? hi[c] : lo[c];
      C.wt_off = tpool;
      for (int32_t r = C.lo; r < C.hi; ++r) trows.push_back({tpool + (int64_t)(r - C.lo) * C.ldwt, ci[c].bi, omap[r]});
      tpool += (int64_t)(C.hi - C.lo) * C.ldwt;
      p->stored_t += (int64_t)(C.hi - C.lo) * C.M;
    }
    return J;
  };

  // Stage tables.
  std::vector<FwdJob> fj;
  std::vector<BwdJob> bj;
  std::vector<Tile> tiles;
  // Workgroups of one launch go to the 8 XCDs round robin (workgroup b to XCD
  // b % 8), each XCD with its own L2.  Jobs are packed into 8 bins by cost
  // (longest first), each bin's tiles keep their job's tiles together so the
  // job's right-hand-side rows are fetched into one L2, and the bins are
  // interleaved so bin x lands on XCD x; short bins are padded with empty tiles.
  auto order = [&](const std::vector<std::pair<int64_t, int64_t>> &jobs_cost_rows, int BM) {
    const int X = 8;
    std::vector<int64_t> idx(jobs_cost_rows.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int64_t)i;
    std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
      return jobs_cost_rows[a].first * ((jobs_cost_rows[a].second + BM - 1) / BM) >
             jobs_cost_rows[b].first * ((jobs_cost_rows[b].second + BM - 1) / BM);
    });
    std::vector<std::vector<Tile>> bins(X);
    std::vector<int64_t> load(X, 0);
    for (int64_t j : idx) {
      const int64_t nrows = jobs_cost_rows[j].second;
      if (nrows <= 0) continue;
      int x = 0;
      for (int y = 1; y < X; ++y)
        if (load[y] < load[x]) x = y;
      for (int32_t m0 = 0; m0 < nrows; m0 += BM) {
        bins[x].push_back({(int32_t)j, m0});
        load[x] += std::max<int64_t>(jobs_cost_rows[j].first, 1);
      }
    }
    size_t len = 0;
    for (auto &b : bins) len = std::max(len, b.size());
    const size_t start = tiles.size();
    for (size_t s = 0; s < len; ++s)
      for (int x = 0; x < X; ++x) tiles.push_back(s < bins[x].size() ? bins[x][s] : Tile{-1, 0});
    return (int64_t)(tiles.size() - start);
  };
  auto add_ftiles = [&](StageDesc &s) {
    std::vector<std::pair<int64_t, int64_t>> jc;
    for (int64_t t = s.fjob0; t < s.fjob0 + s.nfjob; ++t) jc.push_back({fj[t].w_off < 0 ? 1 : fj[t].K, fj[t].M});
    for (int h = 0; h < 2; ++h) {
      s.ftile0[h] = (int64_t)tiles.size();
      s.nftile[h] = order(jc, kTileRows << h);
    }
  };
  auto add_btiles = [&](StageDesc &s) {
    for (int part = 0; part < 2; ++part) {
      std::vector<std::pair<int64_t, int64_t>> jc;
      for (int64_t t = s.bjob0[part]; t < s.bjob0[part] + s.nbjob[part]; ++t) {
        int64_t cost = 1;   // reduction length per tile row, averaged over the job's rows
        for (int c = 0; c < bj[t].nc; ++c)
          cost += (int64_t)bj[t].c[c].M * (bj[t].c[c].hi - bj[t].c[c].lo) / std::max<int32_t>(bj[t].K, 1);
        jc.push_back({cost, bj[t].K});
      }
      for (int h = 0; h < 2; ++h) {
        s.btile0[part][h] = (int64_t)tiles.size();
        s.nbtile[part][h] = order(jc, kTileRows << h);
      }
    }
  };
  auto cons_of = [&](int lvl, int64_t q) -> ConsIn {
    return {bidx_P[lvl * nb + q], f->ident[lvl * nb + q] != 0, f->rank[lvl * nb + q], (int32_t)off[lvl][q]};
  };
  // Merged plans end with stage L: forward jobs of the leaf stage's form (rows
  // scattered to the points' order) that read level L-1, transposed jobs of
  // level L's form whose consumers are the merged leaf blocks.
  const int last = merge ? L : L + 1;
  for (int lvl = 0; lvl <= last; ++lvl) {
    StageDesc s{};
    s.kind = lvl == 0 ? 0 : (lvl < last ? 1 : 2);
    s.level = lvl;
    s.fjob0 = (int64_t)fj.size();
    s.bjob0[0] = (int64_t)bj.size();
    s.bjob0[1] = 0;
    s.nbjob[1] = 0;
    if (lvl == 0) {
      for (int64_t j = 0; j < nb; ++j) {
        const bool id = f->ident[j] != 0;
        const int64_t k = f->koff[j + 1] - f->koff[j];
        fj.push_back(fjob(id ? -1 : woff_P[j], bidx_P[j], f->rank[j], k, f->koff[j], off[0][j]));
        const ConsIn c0 = cons_of(0, j);
        bj.push_back(bjob((int32_t)k, (int32_t)f->koff[j], 1, &c0));
      }
    } else if (lvl <= L) {
      const int64_t nf = ipow(A, L - lvl);
      const bool ml = merge && lvl == L;   // merged last level (nf = 1, block q is leaf q)
      for (int64_t i = 0; i < ipow(A, lvl); ++i)
        for (int64_t j = 0; j < nf; ++j) {
          const int64_t q = i * nf + j, q1 = child0(lvl, q);
          const bool id = f->ident[lvl * nb + q] != 0;
          const int64_t k = rin_of(lvl, q);
          if (ml)
            fj.push_back(fjob(woff_U[q], bidx_U[q], f->xoff[q + 1] - f->xoff[q], k, off[lvl - 1][q1], f->xoff[q]));
          else
            fj.push_back(fjob(id ? -1 : woff_P[lvl * nb + q], bidx_P[lvl * nb + q], f->rank[lvl * nb + q], k,
                              off[lvl - 1][q1], off[lvl][q]));
        }
      // a transposed job owns the A consecutive input blocks of one parent pp
      // and frequency node j, and sums the products of their A consumers (the
      // blocks (A pp + s, j)); consumers 2 and 3 of a 4-ary job go to part 1
      for (int part = 0; part < A / 2; ++part) {
        s.bjob0[part] = (int64_t)bj.size();
        for (int64_t pp = 0; pp < ipow(A, lvl - 1); ++pp)
          for (int64_t j = 0; j < nf; ++j) {
            const int64_t q1 = pp * A * nf + A * j;
            int64_t K = 0;
            for (int t = 0; t < A; ++t) K += f->rank[(lvl - 1) * nb + q1 + t];
            ConsIn cs[2] = {cons_of(lvl, (A * pp + 2 * part) * nf + j),
                            cons_of(lvl, (A * pp + 2 * part + 1) * nf + j)};
            if (ml)   // consumers are merged leaf blocks: their rows are leaf rows of the gathered f
              for (int c = 0; c < 2; ++c) {
                const int64_t qc = A * pp + 2 * part + c;
                cs[c] = {bidx_U[qc], false, (int32_t)(f->xoff[qc + 1] - f->xoff[qc]), (int32_t)f->xoff[qc]};
              }
            BwdJob J = bjob((int32_t)K, (int32_t)off[lvl - 1][q1], 2, cs);
            J.accum = part;
            bj.push_back(J);
          }
        s.nbjob[part] = (int64_t)bj.size() - s.bjob0[part];
      }
    } else {
      for (int64_t i = 0; i < nb; ++i) {
        const int64_t rows = f->xoff[i + 1] - f->xoff[i], r = f->rank[L * nb + i];
        fj.push_back(fjob(woff_U[i], -1, rows, r, off[L][i], f->xoff[i]));
        const ConsIn c0 = {bidx_U[i], false, (int32_t)rows, (int32_t)f->xoff[i]};
        bj.push_back(bjob((int32_t)r, (int32_t)off[L][i], 1, &c0));
      }
    }
    s.nfjob = (int64_t)fj.size() - s.fjob0;
    if (lvl == 0 || lvl > L) s.nbjob[0] = (int64_t)bj.size() - s.bjob0[0];
    p->stages.push_back(s);
  }
  p->tpool_elems = tpool;

  // Leading all-identity levels move rows without arithmetic in the forward
  // direction: level l's output repeats rows of level l-1's (each space node at
  // level l takes a copy of its frequency children).  They are folded into the
  // first later stage e, whose forward jobs read c through the composed row map
  // pi (level e-1 row -> row of c), so no copy stage is launched for them.
  // Identity jobs of stage e become row-gather jobs (a compact job with nothing
  // to reduce and every row a skeleton row).  The transposed direction keeps its
  // stages: there the copies of one row of c are summed.
  if (nfold > 0) {
    // pi over the rows of level nfold-1
    std::vector<int64_t> pi((size_t)off[0][nb]);
    for (int64_t j = 0; j < nb; ++j)
      for (int64_t t = 0; t < f->rank[j]; ++t) pi[off[0][j] + t] = f->koff[j] + t;
    for (int lvl = 1; lvl < nfold; ++lvl) {
      std::vector<int64_t> nx((size_t)off[lvl][nb]);
      for (int64_t q = 0; q < nb; ++q) {
        const int64_t q1 = child0(lvl, q);   // an identity block's rows are its inputs' rows, in order
        for (int64_t t = 0; t < f->rank[lvl * nb + q]; ++t) nx[off[lvl][q] + t] = pi[off[lvl - 1][q1] + t];
      }
      pi.swap(nx);
    }
    for (int k = 0; k < nfold; ++k) p->stages[k].skip = true;
    p->fwd_edge = nfold;
    // Transposed direction: the folded levels sum the copies of each row of c,
    // pairwise over the space nodes (a balanced tree; a 4-ary level adds its
    // four copies as (c0 + c1) + (c2 + c3), the same tree).  One gather-sum over
    // the level nfold-1 rows replaces those stages in a single apply.  The
    // gather-sum kernel takes at most 2^15 copies; deeper runs of identity
    // levels keep their transposed stages (then nfold stays 0).
    const int64_t C = ipow(A, nfold - 1), rows = off[nfold - 1][nb];
    if (C <= kFoldMaxCopies && rows == f->m * C) {
      std::vector<int32_t> cnt((size_t)f->m, 0);
      p->fold_inv.assign((size_t)rows, -1);
      bool ok = true;
      for (int64_t r = 0; r < rows && ok; ++r) {
        const int64_t cr = pi[r];
        ok = cr >= 0 && cr < f->m && cnt[cr] < C;
        if (ok) p->fold_inv[(size_t)(cr * C + cnt[cr]++)] = (int32_t)r;
      }
      if (ok) {
        p->nfold = nfold;
        p->fold_copies = C;
      } else {
        std::vector<int32_t>().swap(p->fold_inv);
      }
    }
    StageDesc &e = p->stages[nfold];
    e.edge = true;
    for (int64_t t = e.fjob0; t < e.fjob0 + e.nfjob; ++t) {
      FwdJob &J = fj[t];
      if (J.w_off < 0) {   // identity: y rows = x rows, as skeleton copies
        J.map_off = (int32_t)p->maps.size();
        for (int32_t r = 0; r < J.M; ++r) p->maps.push_back((int32_t)pi[J.in_row + r]);
        J.w_off = 0;
        J.K = 0;
        J.ldw = 0;
        J.skel = 1;
      } else {
        const int32_t nidx = J.K + (J.skel ? J.M : 0);
        for (int32_t u = 0; u < nidx; ++u) p->maps[J.map_off + u] = (int32_t)pi[J.in_row + p->maps[J.map_off + u]];
      }
      J.in_row = 0;
    }
  }
  for (auto &s : p->stages) {
    add_ftiles(s);
    add_btiles(s);
    if (s.nbjob[1] > 0) ++p->extra_parts;
  }
  for (int d = 0; d < 2; ++d) {
    p->rows[d].assign(p->stages.size(), kTileRows);
    p->cols[d].assign(p->stages.size(), 0);
  }

  // job fields and kernels index the row-index table with 32-bit offsets
  if (p->maps.size() >= (size_t)(1ll << 31)) return fail(BFMHT_EINVAL, "row-index table exceeds 2^31 entries");

  // Device layout.  Every pool region ends in a zero tail of at least one
  // reduction chunk (128 bytes for every element type): the kernels read whole
  // chunks past a row's end without a guard.
  int64_t cur = 0;
  p->off_pool = cur;
  cur = align_up(cur + pool * p->wsz + kPoolTailBytes, 256);
  p->off_tpool = cur;
  cur = align_up(cur + tpool * p->wsz + kPoolTailBytes, 256);
  p->off_fjobs = cur;
  cur = align_up(cur + (int64_t)fj.size() * (int64_t)sizeof(FwdJob), 256);
  p->off_bjobs = cur;
  cur = align_up(cur + (int64_t)bj.size() * (int64_t)sizeof(BwdJob), 256);
  p->off_tiles = cur;
  cur = align_up(cur + (int64_t)tiles.size() * (int64_t)sizeof(Tile), 256);
  p->off_perm = cur;
  cur = align_up(cur + f->n * 4, 256);
  p->off_maps = cur;
  cur = align_up(cur + (int64_t)p->maps.size() * 4, 256);
  p->off_fold = cur;
  cur = align_up(cur + (int64_t)p->fold_inv.size() * 4, 256);
  p->dev_bytes = std::max<int64_t>(cur, 256);

  p->staging.assign((size_t)p->dev_bytes, 0);
  unsigned char *S = p->staging.data();
  // FP64 pools for the plain path, FP32 otherwise (the BF16 kernels split each
  // FP32 value into its bf16 terms when they load it)
  auto put = [&](int64_t base, int64_t e, double x) {
    if (prec == BFMHT_F64) reinterpret_cast<double *>(S + base)[e] = x;
    else reinterpret_cast<float *>(S + base)[e] = (float)x;
  };
  int64_t bo = 0;
  for (const Src &b : blocks) {
    const int64_t kf = b.compact ? (int64_t)b.jc.size() : b.cols;
    const int64_t ld = ldw_of(kf);
    for (int64_t r = 0; r < b.rows; ++r)
      for (int64_t t = 0; t < kf; ++t) put(p->off_pool, bo + r * ld + t, b.ptr[r * b.cols + (b.compact ? b.jc[t] : t)]);
    bo += b.rows * ld;
  }
  for (const TRow &t : trows) {
    const Src &b = blocks[t.blk];
    for (int64_t i = 0; i < b.rows; ++i) put(p->off_tpool, t.off + i, b.ptr[i * b.cols + t.col]);
  }
  if (!p->maps.empty()) std::memcpy(S + p->off_maps, p->maps.data(), p->maps.size() * 4);
  std::vector<int32_t>().swap(p->maps);
  if (!p->fold_inv.empty()) std::memcpy(S + p->off_fold, p->fold_inv.data(), p->fold_inv.size() * 4);
  std::vector<int32_t>().swap(p->fold_inv);
  if (!fj.empty()) std::memcpy(S + p->off_fjobs, fj.data(), fj.size() * sizeof(FwdJob));
  if (!bj.empty()) std::memcpy(S + p->off_bjobs, bj.data(), bj.size() * sizeof(BwdJob));
  if (!tiles.empty()) std::memcpy(S + p->off_tiles, tiles.data(), tiles.size() * sizeof(Tile));
  if (f->n) std::memcpy(S + p->off_perm, f->perm_x, (size_t)f->n * 4);
  *out = owner.release();
  return BFMHT_OK;
}

}  // namespace

extern "C" {

bfmht_status bfmht_plan_create_ex(const bfmht_factors_host *f, bfmht_precision prec, int32_t max_nrhs, int32_t flags,
                                  bfmht_plan **out) {
  if (!out) return fail(BFMHT_EINVAL, "plan output pointer is NULL");
  *out = nullptr;
  if (flags & ~(BFMHT_PLAN_FULL_BLOCKS | BFMHT_PLAN_LEAF_STAGE)) return fail(BFMHT_EINVAL, "unknown plan flags");
  if (prec < BFMHT_F64 || prec > BFMHT_BF16X3) return fail(BFMHT_EINVAL, "unknown precision");
  if (max_nrhs < 1) return fail(BFMHT_EINVAL, "max_nrhs must be >= 1");
  bfmht_status st = validate(f);
  if (st != BFMHT_OK) return st;
  try {
    const bool full = (flags & BFMHT_PLAN_FULL_BLOCKS) != 0;
    return plan_build(f, prec, max_nrhs, !full, !full && (flags & BFMHT_PLAN_LEAF_STAGE) == 0, out);
  } catch (const std::bad_alloc &) {
    return fail(BFMHT_ENOSPACE, "host memory exhausted while building the plan");
  } catch (...) {
    return fail(BFMHT_EINVAL, "plan construction failed");
  }
}

int64_t bfmht_plan_device_bytes(const bfmht_plan *p) { return p ? p->dev_bytes : -1; }

int64_t bfmht_plan_stored_entries(const bfmht_plan *p, int32_t transpose) {
  if (!p) return -1;
  return transpose ? p->stored_t : p->stored_fwd;
}

int64_t bfmht_workspace_bytes(const bfmht_plan *p, int32_t nrhs) {
  if (!p || nrhs < 0) return -1;
  const int64_t one = align_up(p->max_rows * (int64_t)nrhs * p->esz, 256);
  return std::max<int64_t>(2 * one, 256);
}

bfmht_status bfmht_plan_upload(bfmht_plan *p, void *dev_buf, int64_t dev_bytes, void *stream) {
  if (!p) return fail(BFMHT_EINVAL, "plan is NULL");
  if (p->uploaded) return fail(BFMHT_ESTATE, "plan already uploaded");
  if (!dev_buf) return fail(BFMHT_EINVAL, "dev_buf is NULL");
  if (((uintptr_t)dev_buf) % 256) return fail(BFMHT_EINVAL, "dev_buf must be 256-byte aligned");
  if (dev_bytes < p->dev_bytes) return fail(BFMHT_ENOSPACE, "dev_buf smaller than bfmht_plan_device_bytes");
  hipError_t e = hipMemcpyAsync(dev_buf, p->staging.data(), (size_t)p->dev_bytes, hipMemcpyHostToDevice,
                                (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return fail(BFMHT_EHIP, std::string("upload: ") + hipGetErrorString(e));
  std::vector<unsigned char>().swap(p->staging);
  p->dev = static_cast<char *>(dev_buf);
  p->uploaded = true;
  return BFMHT_OK;
}

void bfmht_plan_destroy(bfmht_plan *p) { delete p; }

}  // extern "C"

namespace {

// in has rows_in rows and out rows_out rows; a block with no rows may be NULL.
bfmht_status check_call(const bfmht_plan *p, const void *in, int64_t rows_in, int64_t ldin, const void *out,
                        int64_t rows_out, int64_t ldout, int32_t nrhs, const void *ws, int64_t ws_bytes) {
  if (!p) return fail(BFMHT_EINVAL, "plan is NULL");
  if (!p->uploaded) return fail(BFMHT_ESTATE, "plan not uploaded");
  if (nrhs < 0) return fail(BFMHT_EINVAL, "nrhs < 0");
  if (nrhs == 0) return BFMHT_OK;
  if ((!in && rows_in > 0) || (!out && rows_out > 0) || !ws)
    return fail(BFMHT_EINVAL, "NULL input, output or workspace");
  if ((rows_in > 0 && ldin < nrhs) || (rows_out > 0 && ldout < nrhs))
    return fail(BFMHT_EINVAL, "ld smaller than nrhs");
  if (((uintptr_t)ws) % 256) return fail(BFMHT_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < bfmht_workspace_bytes(p, nrhs)) return fail(BFMHT_ENOSPACE, "workspace too small");
  return BFMHT_OK;
}

// Source rows may be read with 16-byte loads when the base and row pitch are 16-byte aligned.
int32_t vec_ok(const void *src, int64_t ld, int64_t esz) {
  return (((uintptr_t)src) % 16 == 0 && (ld * esz) % 16 == 0) ? 1 : 0;
}

// part: the transposed stage's job part (0, or 1 for the second consumer pair of 4-ary trees)
StageArgs base_args(const bfmht_plan *p, const StageDesc &s, bool fwd, int h, int part) {
  StageArgs a{};
  a.pool = p->dev + (fwd ? p->off_pool : p->off_tpool);
  if (fwd) {
    a.jobs = p->dev + p->off_fjobs + s.fjob0 * (int64_t)sizeof(FwdJob);
    a.tiles = reinterpret_cast<const Tile *>(p->dev + p->off_tiles) + s.ftile0[h];
    a.ntiles = (int32_t)s.nftile[h];
  } else {
    a.jobs = p->dev + p->off_bjobs + s.bjob0[part] * (int64_t)sizeof(BwdJob);
    a.tiles = reinterpret_cast<const Tile *>(p->dev + p->off_tiles) + s.btile0[part][h];
    a.ntiles = (int32_t)s.nbtile[part][h];
  }
  // the forward leaf stage scatters its rows to the points' order
  a.rowmap = fwd && s.kind == 2 ? reinterpret_cast<const int32_t *>(p->dev + p->off_perm) : nullptr;
  a.maps = reinterpret_cast<const int32_t *>(p->dev + p->off_maps);
  return a;
}

// Arguments of stage s of one apply of plan p (forward or transposed) between
// user buffers in/out and the two level buffers buf[0], buf[1].
StageArgs stage_io(const bfmht_plan *p, const StageDesc &s, bool fwd, int rows, const void *in, int64_t ldin,
                   void *out, int64_t ldout, int32_t nrhs, char *const buf[2], int part = 0) {
  StageArgs a = base_args(p, s, fwd, rows == 2 * kTileRows ? 1 : 0, part);
  a.nrhs = nrhs;
  if (fwd) {
    // stage l reads level l-1 (or c) and writes level l (or f)
    if (s.kind == 0 || s.edge) { a.src = in; a.lds = ldin; } else { a.src = buf[(s.level - 1) & 1]; a.lds = nrhs; }
    if (s.kind == 2) { a.dst = out; a.ldd = ldout; } else { a.dst = buf[s.level & 1]; a.ldd = nrhs; }
  } else {
    // the transposed stage l reads level l (the leaf stage: f gathered into tree
    // order, see gather_input) and writes level l-1 (or g)
    a.src = buf[s.level & 1];
    a.lds = nrhs;
    if (s.kind == 0) { a.dst = out; a.ldd = ldout; } else { a.dst = buf[(s.level - 1) & 1]; a.ldd = nrhs; }
  }
  a.vec = vec_ok(a.src, a.lds, p->esz);
  return a;
}

// Tile width: an explicit 16/32/64, or the smallest that covers nrhs.
int pick_cols(int cols, int nrhs) {
  if (cols == 16 || cols == 32 || cols == 64) return cols;
  return nrhs <= 16 ? 16 : (nrhs <= 32 ? 32 : 64);
}

int64_t level_buffer_bytes(const bfmht_plan *p, int32_t nrhs) {
  return align_up(p->max_rows * (int64_t)nrhs * p->esz, 256);
}

// The transposed apply first gathers f's rows into tree order, into the level
// buffer its last stage reads (the leaf stage, level L+1, or the merged last
// level L).
int gather_input(const bfmht_plan *p, const void *in, int64_t ldin, int32_t nrhs, char *const buf[2], void *stream) {
  return launch_gather_rows((int)p->esz, in, ldin, reinterpret_cast<const int32_t *>(p->dev + p->off_perm), p->n,
                            buf[p->stages.back().level & 1], nrhs, nrhs, stream);
}

bfmht_status run_apply(const bfmht_plan *p, bool fwd, const void *in, int64_t ldin, void *out, int64_t ldout,
                       int32_t nrhs, void *ws, int64_t ws_bytes, void *stream) {
  bfmht_status st = check_call(p, in, fwd ? p->m : p->n, ldin, out, fwd ? p->n : p->m, ldout, nrhs, ws, ws_bytes);
  if (st != BFMHT_OK || nrhs == 0) return st;
  char *const buf[2] = {static_cast<char *>(ws), static_cast<char *>(ws) + level_buffer_bytes(p, nrhs)};
  if (!fwd) {
    const int e = gather_input(p, in, ldin, nrhs, buf, stream);
    if (e) return fail(BFMHT_EHIP, std::string("input gather launch: ") + hipGetErrorString((hipError_t)e));
  }
  const int S = (int)p->stages.size();
  const bool gemv = nrhs <= kGemvMaxRhs && (p->prec == BFMHT_F32 || p->prec == BFMHT_F64);
  for (int k = 0; k < S; ++k) {
    const int si = fwd ? k : S - 1 - k;
    const StageDesc &s = p->stages[si];
    if (fwd ? s.skip : si < p->nfold) continue;   // folded identity levels
    const int d = fwd ? 0 : 1;
    // a transposed 4-ary stage runs its second consumer pair as a second launch
    // that adds to the rows the first one wrote
    const int parts = fwd || s.nbjob[1] == 0 ? 1 : 2;
    for (int part = 0; part < parts; ++part) {
      if (gemv) {   // few right-hand sides: vector FMAs over the 64-row tiles
        StageArgs a = stage_io(p, s, fwd, kTileRows, in, ldin, out, ldout, nrhs, buf, part);
        const int e = launch_gemv_stage(p->prec, fwd, a, stream);
        if (e) return fail(BFMHT_EHIP, std::string("stage launch: ") + hipGetErrorString((hipError_t)e));
        continue;
      }
      const int rows = p->rows[d][si], cols = pick_cols(p->cols[d][si], nrhs);
      StageArgs a = stage_io(p, s, fwd, rows, in, ldin, out, ldout, nrhs, buf, part);
      const int e =
          fwd ? launch_fwd_stage(p->prec, a, rows, cols, stream) : launch_bwd_stage(p->prec, a, rows, cols, stream);
      if (e) return fail(BFMHT_EHIP, std::string("stage launch: ") + hipGetErrorString((hipError_t)e));
    }
  }
  if (!fwd && p->nfold > 0) {   // sum the copies of each row of c (the folded transposed levels)
    const int e = launch_fold_sum((int)p->esz, buf[(p->nfold - 1) & 1], nrhs,
                                  reinterpret_cast<const int32_t *>(p->dev + p->off_fold), (int)p->fold_copies, p->m,
                                  out, ldout, nrhs, stream);
    if (e) return fail(BFMHT_EHIP, std::string("fold launch: ") + hipGetErrorString((hipError_t)e));
  }
  return BFMHT_OK;
}


}  // namespace

namespace bfmht {

bfmht_status set_error(bfmht_status s, const std::string &msg) { return fail(s, msg); }

bfmht_status apply_with_workspace(const bfmht_plan *p, bool fwd, const void *in, int64_t ldin, void *out,
                                  int64_t ldout, int32_t nrhs, void *ws, int64_t ws_bytes, void *stream) {
  return run_apply(p, fwd, in, ldin, out, ldout, nrhs, ws, ws_bytes, stream);
}

}  // namespace bfmht

extern "C" {

bfmht_status bfmht_apply(const bfmht_plan *p, const void *c, int64_t ldc, void *f, int64_t ldf, int32_t nrhs,
                         void *ws, int64_t ws_bytes, void *stream) {
  return run_apply(p, true, c, ldc, f, ldf, nrhs, ws, ws_bytes, stream);
}

bfmht_status bfmht_apply_scaled(const bfmht_plan *p, const void *s, const void *c, int64_t ldc, void *f, int64_t ldf,
                                int32_t nrhs, void *ws, int64_t ws_bytes, void *stream) {
  bfmht_status st = check_call(p, c, p->m, ldc, f, p->n, ldf, nrhs, ws, ws_bytes);
  if (st != BFMHT_OK || nrhs == 0) return st;
  if (!s && p->m > 0) return fail(BFMHT_EINVAL, "scale vector is NULL");
  // diag(s) c goes to the level buffer that the first forward stage to run
  // (level fwd_edge, after the folded identity levels) does not write; the next
  // stage overwrites it only after that stage has read it.  A first stage that
  // is the leaf stage writes f and neither buffer.
  char *scaled = static_cast<char *>(ws) + ((p->fwd_edge & 1) ^ 1) * level_buffer_bytes(p, nrhs);
  const int e = launch_scale_rows((int)p->esz, s, c, ldc, p->m, scaled, nrhs, nrhs, stream);
  if (e) return fail(BFMHT_EHIP, std::string("scale launch: ") + hipGetErrorString((hipError_t)e));
  return run_apply(p, true, scaled, nrhs, f, ldf, nrhs, ws, ws_bytes, stream);
}

bfmht_status bfmht_apply_transpose_scaled(const bfmht_plan *p, const void *s, const void *f, int64_t ldf, void *g,
                                          int64_t ldg, int32_t nrhs, void *ws, int64_t ws_bytes, void *stream) {
  if (p && nrhs > 0 && !s && p->m > 0) return fail(BFMHT_EINVAL, "scale vector is NULL");
  bfmht_status st = run_apply(p, false, f, ldf, g, ldg, nrhs, ws, ws_bytes, stream);
  if (st != BFMHT_OK || nrhs == 0) return st;
  const int e = launch_scale_rows((int)p->esz, s, g, ldg, p->m, g, ldg, nrhs, stream);
  if (e) return fail(BFMHT_EHIP, std::string("scale launch: ") + hipGetErrorString((hipError_t)e));
  return BFMHT_OK;
}

bfmht_status bfmht_apply_transpose(const bfmht_plan *p, const void *f, int64_t ldf, void *g, int64_t ldg,
                                   int32_t nrhs, void *ws, int64_t ws_bytes, void *stream) {
  return run_apply(p, false, f, ldf, g, ldg, nrhs, ws, ws_bytes, stream);
}

// LSQR workspace: the apply workspace, then u, y (n x b), v, z, w (m x b), the
// norm partial sums and eight scalar arrays, each region 256-byte aligned.
}  // extern "C"

namespace {
struct LsqrLayout {
  int64_t apply_ws, u, y, v, z, w, partial, scal, total;
};
LsqrLayout lsqr_layout(const bfmht_plan *p, int32_t nrhs) {
  LsqrLayout L{};
  const int64_t e = p->esz, b = nrhs;
  int64_t cur = 0;
  auto take = [&](int64_t bytes) { const int64_t at = cur; cur = align_up(cur + bytes, 256); return at; };
  L.apply_ws = take(bfmht_workspace_bytes(p, nrhs));
  L.u = take(p->n * b * e);
  L.y = take(p->n * b * e);
  L.v = take(p->m * b * e);
  L.z = take(p->m * b * e);
  L.w = take(p->m * b * e);
  L.partial = take((int64_t)kLsqrMaxBlocks * b * e);
  L.scal = take(8 * b * e);
  L.total = std::max<int64_t>(cur, 256);
  return L;
}
}  // namespace

extern "C" {

int64_t bfmht_lsqr_workspace_bytes(const bfmht_plan *p, int32_t nrhs) {
  if (!p || nrhs < 0) return -1;
  return lsqr_layout(p, nrhs).total;
}

bfmht_status bfmht_lsqr(const bfmht_plan *p, const void *f, int64_t ldf, void *x, int64_t ldx, int32_t nrhs,
                        int32_t iters, void *rnorm, void *ws, int64_t ws_bytes, void *stream) {
  if (!p) return fail(BFMHT_EINVAL, "plan is NULL");
  if (!p->uploaded) return fail(BFMHT_ESTATE, "plan not uploaded");
  if (nrhs < 0 || iters < 0) return fail(BFMHT_EINVAL, "nrhs or iters < 0");
  if (nrhs == 0) return BFMHT_OK;
  if ((!f && p->n > 0) || (!x && p->m > 0) || !ws)
    return fail(BFMHT_EINVAL, "NULL right-hand side, solution or workspace");
  if ((p->n > 0 && ldf < nrhs) || (p->m > 0 && ldx < nrhs)) return fail(BFMHT_EINVAL, "ld smaller than nrhs");
  if (((uintptr_t)ws) % 256) return fail(BFMHT_EINVAL, "workspace must be 256-byte aligned");
  const LsqrLayout L = lsqr_layout(p, nrhs);
  if (ws_bytes < L.total) return fail(BFMHT_ENOSPACE, "workspace too small for LSQR");
  char *W = static_cast<char *>(ws);
  void *aws = W + L.apply_ws;
  const int64_t aws_bytes = bfmht_workspace_bytes(p, nrhs);
  char *u = W + L.u, *y = W + L.y, *v = W + L.v, *z = W + L.z, *w = W + L.w, *partial = W + L.partial;
  const int64_t e = p->esz, b = nrhs;
  char *alpha = W + L.scal, *beta = alpha + b * e, *rhobar = beta + b * e, *phibar = rhobar + b * e;
  char *cx = phibar + b * e, *cw = cx + b * e, *inv = cw + b * e;
  const int es = (int)e;
  auto ok = [&](int rc, const char *what) -> bfmht_status {
    return rc ? fail(BFMHT_EHIP, std::string(what) + ": " + hipGetErrorString((hipError_t)rc)) : BFMHT_OK;
  };
  bfmht_status st;
  // beta_1 u_1 = f (beta_1 into phibar); alpha_1 v_1 = Phi~^T u_1; rhobar_1 = alpha_1; w_1 = v_1; x_0 = 0
  if ((st = ok(lsqr_normalize(es, f, ldf, p->n, nrhs, nullptr, u, partial, phibar, inv, stream), "LSQR start"))) return st;
  if ((st = run_apply(p, false, u, b, z, b, nrhs, aws, aws_bytes, stream))) return st;
  if ((st = ok(lsqr_normalize(es, z, b, p->m, nrhs, nullptr, v, partial, alpha, inv, stream), "LSQR start"))) return st;
  if ((st = ok((int)hipMemcpyAsync(rhobar, alpha, b * e, hipMemcpyDeviceToDevice, (hipStream_t)stream), "LSQR start")))
    return st;
  if ((st = ok(lsqr_init(es, x, ldx, w, v, p->m, nrhs, stream), "LSQR start"))) return st;
  // with no step taken the residual estimate is beta_1 = ||f|| (x = 0)
  if (iters == 0 && rnorm &&
      (st = ok((int)hipMemcpyAsync(rnorm, phibar, b * e, hipMemcpyDeviceToDevice, (hipStream_t)stream), "LSQR start")))
    return st;
  for (int32_t it = 0; it < iters; ++it) {
    // beta_{i+1} u_{i+1} = Phi~ v_i - alpha_i u_i
    if ((st = run_apply(p, true, v, b, y, b, nrhs, aws, aws_bytes, stream))) return st;
    if ((st = ok(lsqr_normalize(es, y, b, p->n, nrhs, alpha, u, partial, beta, inv, stream), "LSQR u"))) return st;
    // alpha_{i+1} v_{i+1} = Phi~^T u_{i+1} - beta_{i+1} v_i
    if ((st = run_apply(p, false, u, b, z, b, nrhs, aws, aws_bytes, stream))) return st;
    if ((st = ok(lsqr_normalize(es, z, b, p->m, nrhs, beta, v, partial, alpha, inv, stream), "LSQR v"))) return st;
    if ((st = ok(lsqr_rotate(es, nrhs, alpha, beta, rhobar, phibar, cx, cw, rnorm, stream), "LSQR rotation")))
      return st;
    if ((st = ok(lsqr_update(es, x, ldx, w, v, p->m, nrhs, cx, cw, stream), "LSQR update"))) return st;
  }
  return BFMHT_OK;
}

int32_t bfmht_plan_num_stages(const bfmht_plan *p) { return p ? (int32_t)p->stages.size() : -1; }

bfmht_status bfmht_plan_set_tile(bfmht_plan *p, int32_t transpose, int32_t stage, int32_t rows, int32_t cols) {
  if (!p) return fail(BFMHT_EINVAL, "plan is NULL");
  if (stage < 0 || stage >= (int32_t)p->stages.size()) return fail(BFMHT_EINVAL, "stage out of range");
  if (rows != kTileRows && rows != 2 * kTileRows) return fail(BFMHT_EINVAL, "tile rows must be 64 or 128");
  if (cols != 0 && cols != 16 && cols != 32 && cols != 64) return fail(BFMHT_EINVAL, "tile columns must be 0, 16, 32 or 64");
  p->rows[transpose ? 1 : 0][stage] = rows;
  p->cols[transpose ? 1 : 0][stage] = cols;
  return BFMHT_OK;
}

bfmht_status bfmht_plan_get_tile(const bfmht_plan *p, int32_t transpose, int32_t stage, int32_t *rows, int32_t *cols) {
  if (!p || !rows || !cols) return fail(BFMHT_EINVAL, "NULL argument");
  if (stage < 0 || stage >= (int32_t)p->stages.size()) return fail(BFMHT_EINVAL, "stage out of range");
  *rows = p->rows[transpose ? 1 : 0][stage];
  *cols = p->cols[transpose ? 1 : 0][stage];
  return BFMHT_OK;
}

// ---- batched ----

}  // extern "C"

namespace {
// The applies of a batch.  Instances that share one plan form one unit whose
// right-hand sides are packed side by side into one block of columns (their
// inputs copied in, their outputs copied back out), so the plan's factors are
// streamed once for all of them; any other instance is a unit of its own.
struct BatchUnit {
  const bfmht_plan *p = nullptr;
  int32_t nrhs = 0;                  // columns of the unit (summed over its members)
  std::vector<int32_t> members;      // instance indices, in order
  std::vector<int32_t> col;          // first packed column of each member
  int64_t buf_off = 0;               // its two level buffers
  int64_t in_off = -1, out_off = -1; // packed input and output blocks (-1: a single instance, used in place)
};
struct BatchLayout {
  int64_t total = 0;
  int32_t nseg = 0;
  std::vector<BatchUnit> units;
  int64_t table_off = 0;         // persistent launch: segment table, then its sync words
  int64_t sync_off = 0;
};

// Polls of a persistent workgroup's wait before it gives up (each poll is one
// device-scope load and a short sleep, about a microsecond): a few seconds, far
// above any stage's duration.
constexpr int64_t kPersistentSpinLimit = 1ll << 22;

// The persistent launch is switched off: its one GPU run (every stage of a
// 7-instance batch, FP64) did not finish within minutes although every wait
// is bounded (no fault).  The likely cause, read from the code: each poll of a
// waiting workgroup is an agent-scope acquire, which invalidates its XCD's L2,
// and every finished tile writes the whole L2 back, so thousands of resident
// workgroups thrash the caches the working ones read from.  Until a version
// that polls without invalidating has run, the mode returns EINVAL.
constexpr bool kPersistentLaunch = false;

bfmht_status batch_layout(const bfmht_plan *const *plans, int32_t count, const int32_t *nrhs, BatchLayout &L) {
  if (count < 0) return fail(BFMHT_EINVAL, "count < 0");
  if (count > 0 && (!plans || !nrhs)) return fail(BFMHT_EINVAL, "NULL plans or nrhs");
  L.nseg = 0;
  L.units.clear();
  for (int32_t i = 0; i < count; ++i) {
    if (!plans[i]) return fail(BFMHT_EINVAL, "NULL plan in batch");
    if (nrhs[i] < 0) return fail(BFMHT_EINVAL, "nrhs < 0 in batch");
    if (plans[i]->prec != plans[0]->prec) return fail(BFMHT_EINVAL, "plans of a batch must share one precision");
  }
  // units: instances with columns, grouped by plan in order of first appearance
  for (int32_t i = 0; i < count; ++i) {
    if (nrhs[i] == 0) continue;
    size_t u = 0;
    while (u < L.units.size() && L.units[u].p != plans[i]) ++u;
    if (u == L.units.size()) {
      L.units.emplace_back();
      L.units[u].p = plans[i];
    }
    BatchUnit &U = L.units[u];
    if ((int64_t)U.nrhs + nrhs[i] >= (1ll << 31)) return fail(BFMHT_EINVAL, "too many columns for one plan in a batch");
    U.col.push_back(U.nrhs);
    U.members.push_back(i);
    U.nrhs += nrhs[i];
  }
  int64_t cur = 0;
  for (BatchUnit &U : L.units) {
    L.nseg += (int32_t)U.p->stages.size() + U.p->extra_parts;
    U.buf_off = cur;
    cur += 2 * level_buffer_bytes(U.p, U.nrhs);
    if (U.members.size() > 1) {   // packed blocks of the unit's inputs and outputs (either direction)
      const int64_t rows = std::max<int64_t>(U.p->n, U.p->m);
      U.in_off = cur;
      cur = align_up(cur + rows * U.nrhs * U.p->esz, 256);
      U.out_off = cur;
      cur = align_up(cur + rows * U.nrhs * U.p->esz, 256);
    }
  }
  // the persistent launch's segment table and sync words (at most one segment per stage)
  L.table_off = align_up(cur, 256);
  L.sync_off = align_up(L.table_off + (int64_t)L.nseg * (int64_t)sizeof(PSegDev), 256);
  cur = L.sync_off + ((int64_t)L.nseg + kQueues + 1) * 4;
  L.total = std::max<int64_t>(align_up(cur, 256), 256);
  return BFMHT_OK;
}

// Operands of each unit of a batch: a single instance's own, or the packed
// blocks of a shared-plan unit, whose members' inputs are copied in here.
struct UnitIO {
  const void *in;
  int64_t ldin;
  void *out;
  int64_t ldout;
};

bfmht_status prepare_units(const BatchLayout &L, const void *const *in, const int64_t *ldin, void *const *out,
                           const int64_t *ldout, const int32_t *nrhs, bool fwd, char *ws, void *stream,
                           std::vector<UnitIO> &io) {
  io.clear();
  for (const BatchUnit &U : L.units) {
    const bfmht_plan *p = U.p;
    if (!p->uploaded) return fail(BFMHT_ESTATE, "plan in batch not uploaded");
    const int64_t rin = fwd ? p->m : p->n, rout = fwd ? p->n : p->m;
    for (int32_t i : U.members) {
      if ((!in[i] && rin > 0) || (!out[i] && rout > 0)) return fail(BFMHT_EINVAL, "NULL input or output in batch");
      if ((rin > 0 && ldin[i] < nrhs[i]) || (rout > 0 && ldout[i] < nrhs[i]))
        return fail(BFMHT_EINVAL, "ld smaller than nrhs in batch");
    }
    if (U.members.size() == 1) {
      const int32_t i = U.members[0];
      io.push_back({in[i], ldin[i], out[i], ldout[i]});
      continue;
    }
    char *pin = ws + U.in_off, *pout = ws + U.out_off;
    for (size_t t = 0; t < U.members.size(); ++t) {
      const int32_t i = U.members[t];
      const int e = launch_copy_block((int)p->esz, in[i], ldin[i], rin, nrhs[i], pin + (int64_t)U.col[t] * p->esz,
                                      U.nrhs, stream);
      if (e) return fail(BFMHT_EHIP, std::string("batch packing launch: ") + hipGetErrorString((hipError_t)e));
    }
    io.push_back({pin, U.nrhs, pout, U.nrhs});
  }
  return BFMHT_OK;
}

// Copies the packed outputs of shared-plan units back to their members.
bfmht_status finish_units(const BatchLayout &L, void *const *out, const int64_t *ldout, const int32_t *nrhs,
                          bool fwd, char *ws, void *stream) {
  for (const BatchUnit &U : L.units) {
    if (U.members.size() == 1) continue;
    const int64_t rout = fwd ? U.p->n : U.p->m;
    for (size_t t = 0; t < U.members.size(); ++t) {
      const int32_t i = U.members[t];
      const int e = launch_copy_block((int)U.p->esz, ws + U.out_off + (int64_t)U.col[t] * U.p->esz, U.nrhs, rout,
                                      nrhs[i], out[i], ldout[i], stream);
      if (e) return fail(BFMHT_EHIP, std::string("batch unpacking launch: ") + hipGetErrorString((hipError_t)e));
    }
  }
  return BFMHT_OK;
}

// Every stage of every instance in one persistent launch (64-row tiles of bn
// columns, MFMA kernel for every instance).  Synchronises the stream once to
// read the launch's error word.
bfmht_status apply_persistent(const bfmht_plan *const *plans, int32_t count, const void *const *in,
                              const int64_t *ldin, void *const *out, const int64_t *ldout, const int32_t *nrhs,
                              bool fwd, int bn, const BatchLayout &L, char *ws, void *stream) {
  std::vector<PSegInfo> info;
  std::vector<PSegDev> segs;
  std::vector<UnitIO> io;
  bfmht_status st = prepare_units(L, in, ldin, out, ldout, nrhs, fwd, ws, stream, io);
  if (st != BFMHT_OK) return st;
  for (int32_t u = 0; u < (int32_t)L.units.size(); ++u) {
    const BatchUnit &U = L.units[u];
    const bfmht_plan *p = U.p;
    char *base = ws + U.buf_off;
    char *const buf[2] = {base, base + level_buffer_bytes(p, U.nrhs)};
    if (!fwd) {
      const int e = gather_input(p, io[u].in, io[u].ldin, U.nrhs, buf, stream);
      if (e) return fail(BFMHT_EHIP, std::string("input gather launch: ") + hipGetErrorString((hipError_t)e));
    }
    const int S = (int)p->stages.size();
    int pos = 0;   // position in the unit's stage sequence (a 4-ary transposed stage takes two)
    for (int k = 0; k < S; ++k) {
      const int si = fwd ? k : S - 1 - k;
      if (fwd && p->stages[si].skip) continue;   // folded identity level: no items
      const int parts = fwd || p->stages[si].nbjob[1] == 0 ? 1 : 2;
      for (int part = 0; part < parts; ++part) {
        PSegDev d{};
        d.a = stage_io(p, p->stages[si], fwd, kTileRows, io[u].in, io[u].ldin, io[u].out, io[u].ldout, U.nrhs, buf,
                       part);
        d.ny = (U.nrhs + bn - 1) / bn;
        info.push_back({u, pos++, (int64_t)(d.a.ntiles / kQueues) * d.ny});
        segs.push_back(d);
      }
    }
  }
  const PSchedule sch = build_schedule(info);
  const int32_t nseg = (int32_t)sch.seg.size();
  if (nseg == 0) return BFMHT_OK;
  if (sch.per_queue_total >= (1ll << 30)) return fail(BFMHT_EINVAL, "persistent launch: too many work items");
  if (nseg > L.nseg) return fail(BFMHT_EINVAL, "persistent schedule larger than its table");
  std::vector<PSegDev> table(nseg);
  for (int32_t q = 0; q < nseg; ++q) {
    table[q] = segs[sch.seg[q]];
    table[q].item0 = sch.item0[q];
    table[q].dep = sch.dep[q];
    table[q].need = sch.need[q];
  }
  auto *dtab = reinterpret_cast<PSegDev *>(ws + L.table_off);
  auto *sync = reinterpret_cast<int32_t *>(ws + L.sync_off);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(dtab, table.data(), table.size() * sizeof(PSegDev), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return fail(BFMHT_EHIP, std::string("persistent table upload: ") + hipGetErrorString(e));
  int rc = fill_zero_i32(sync, (int64_t)nseg + kQueues + 1, stream);
  if (!rc) rc = launch_persistent(plans[0]->prec, fwd, bn, dtab, nseg, sch.per_queue_total, sync,
                                  kPersistentSpinLimit, stream);
  if (rc) return fail(BFMHT_EHIP, std::string("persistent launch: ") + hipGetErrorString((hipError_t)rc));
  int32_t err = 0;
  e = hipMemcpyAsync(&err, sync + nseg + kQueues, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(BFMHT_EHIP, std::string("persistent launch: ") + hipGetErrorString(e));
  if (err) return fail(BFMHT_EHIP, "persistent launch: a workgroup's wait for an earlier stage timed out");
  return finish_units(L, out, ldout, nrhs, fwd, ws, stream);
}

bfmht_status apply_batched(const bfmht_plan *const *plans, int32_t count, const void *const *in,
                           const int64_t *ldin, void *const *out, const int64_t *ldout, const int32_t *nrhs,
                           int32_t mode, void *ws, int64_t ws_bytes, void *stream) {
  if (mode & ~(BFMHT_BATCH_TRANSPOSE | BFMHT_BATCH_PERSISTENT | BFMHT_BATCH_WIDTH(0xff)))
    return fail(BFMHT_EINVAL, "unknown batch mode bits");
  const bool persistent = (mode & BFMHT_BATCH_PERSISTENT) != 0;
  const int pwidth = (mode >> 8) & 0xff;
  if (persistent && pwidth != 0 && pwidth != 16 && pwidth != 32 && pwidth != 64)
    return fail(BFMHT_EINVAL, "persistent tile width must be 0, 16, 32 or 64");
  if (persistent && !kPersistentLaunch)
    return fail(BFMHT_EINVAL, "the persistent batched launch is switched off (its GPU run did not finish in time)");
  BatchLayout L;
  bfmht_status st = batch_layout(plans, count, nrhs, L);
  if (st != BFMHT_OK) return st;
  if (count == 0 || L.nseg == 0) return BFMHT_OK;
  if (!in || !ldin || !out || !ldout || !ws) return fail(BFMHT_EINVAL, "NULL batch argument");
  if (((uintptr_t)ws) % 256) return fail(BFMHT_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < L.total) return fail(BFMHT_ENOSPACE, "workspace too small for the batch");
  const bool fwd = (mode & BFMHT_BATCH_TRANSPOSE) == 0;
  if (persistent) return apply_persistent(plans, count, in, ldin, out, ldout, nrhs, fwd, pwidth ? pwidth : 32, L,
                                          static_cast<char *>(ws), stream);
  std::vector<UnitIO> io;
  st = prepare_units(L, in, ldin, out, ldout, nrhs, fwd, static_cast<char *>(ws), stream, io);
  if (st != BFMHT_OK) return st;
  const int32_t nu = (int32_t)L.units.size();
  std::vector<std::vector<Segment>> per(nu);
  size_t maxS = 0;
  for (int32_t u = 0; u < nu; ++u) {
    const BatchUnit &U = L.units[u];
    const bfmht_plan *p = U.p;
    const int32_t b = U.nrhs;
    char *base = static_cast<char *>(ws) + U.buf_off;
    char *const buf[2] = {base, base + level_buffer_bytes(p, b)};
    if (!fwd) {
      const int e = gather_input(p, io[u].in, io[u].ldin, b, buf, stream);
      if (e) return fail(BFMHT_EHIP, std::string("input gather launch: ") + hipGetErrorString((hipError_t)e));
    }
    const int S = (int)p->stages.size();
    const bool gemv = b <= kGemvMaxRhs && (p->prec == BFMHT_F32 || p->prec == BFMHT_F64);
    for (int k = 0; k < S; ++k) {
      const int si = fwd ? k : S - 1 - k;
      const int parts = fwd || p->stages[si].nbjob[1] == 0 ? 1 : 2;   // 4-ary transposed: two launches
      for (int part = 0; part < parts; ++part) {
        Segment sg{};
        if (fwd && p->stages[si].skip) {   // folded identity level: an empty segment keeps the stage positions aligned
          per[u].push_back(sg);
          continue;
        }
        const int d = fwd ? 0 : 1;
        const int rows = gemv ? kTileRows : p->rows[d][si];
        sg.a = stage_io(p, p->stages[si], fwd, rows, io[u].in, io[u].ldin, io[u].out, io[u].ldout, b, buf, part);
        sg.fwd = fwd ? 1 : 0;
        if (gemv) {   // few right-hand sides: the vector-FMA kernel, as for a single apply
          sg.fm = 0;
          sg.bn = b <= 2 ? b : 4;
          sg.ny = 1;
        } else {
          sg.fm = rows / kTileRows;
          sg.bn = pick_cols(p->cols[d][si], b);
          sg.ny = (b + sg.bn - 1) / sg.bn;
        }
        sg.nitems = (int64_t)sg.a.ntiles * sg.ny;
        per[u].push_back(sg);
      }
    }
    maxS = std::max(maxS, per[u].size());
  }
  // Launch k runs the k-th stage of every instance, one launch per kernel kind
  // (MFMA tile shape bn x 64 fm, or the vector-FMA kernel for b columns), in
  // groups of at most kSegsPerLaunch segments passed as launch arguments;
  // segments without items are left out.  Buckets 0..5: MFMA (bn 16/32/64 x
  // fm 1/2); 6..8: vector FMA (b 1/2/4).
  for (size_t k = 0; k < maxS; ++k) {
    constexpr int NB = 9;
    SegPack pack[NB];
    int64_t item[NB];
    for (int q = 0; q < NB; ++q) {
      pack[q].nseg = 0;
      item[q] = 0;
    }
    auto flush = [&](int q) -> bfmht_status {
      if (pack[q].nseg == 0) return BFMHT_OK;
      if (item[q] >= (1ll << 31)) return fail(BFMHT_EINVAL, "a batched launch has more than 2^31 work items");
      const int rc = q < 6 ? launch_batched_stage(plans[0]->prec, fwd, 16 << (q >> 1), (q & 1) + 1, pack[q], item[q], stream)
                           : launch_batched_gemv(plans[0]->prec, fwd, 1 << (q - 6), pack[q], item[q], stream);
      if (rc) return fail(BFMHT_EHIP, std::string("batched launch: ") + hipGetErrorString((hipError_t)rc));
      pack[q].nseg = 0;
      item[q] = 0;
      return BFMHT_OK;
    };
    for (int32_t u = 0; u < nu; ++u) {
      if (k >= per[u].size() || per[u][k].nitems == 0) continue;
      Segment sg = per[u][k];
      const int q = sg.fm == 0 ? 6 + (sg.bn == 1 ? 0 : (sg.bn == 2 ? 1 : 2))
                               : 2 * (sg.bn == 16 ? 0 : (sg.bn == 32 ? 1 : 2)) + (sg.fm == 2 ? 1 : 0);
      sg.item0 = item[q];
      item[q] += sg.nitems;
      pack[q].s[pack[q].nseg++] = sg;
      if (pack[q].nseg == kSegsPerLaunch) {
        st = flush(q);
        if (st != BFMHT_OK) return st;
      }
    }
    for (int q = 0; q < NB; ++q) {
      st = flush(q);
      if (st != BFMHT_OK) return st;
    }
  }
  return finish_units(L, out, ldout, nrhs, fwd, static_cast<char *>(ws), stream);
}
}  // namespace

extern "C" {

int64_t bfmht_batched_workspace_bytes(const bfmht_plan *const *plans, int32_t count, const int32_t *nrhs) {
  try {
    BatchLayout L;
    if (batch_layout(plans, count, nrhs, L) != BFMHT_OK) return -1;
    return L.total;
  } catch (...) {
    return -1;
  }
}

bfmht_status bfmht_apply_batched(const bfmht_plan *const *plans, int32_t count, const void *const *in,
                                 const int64_t *ldin, void *const *out, const int64_t *ldout, const int32_t *nrhs,
                                 int32_t mode, void *ws, int64_t ws_bytes, void *stream) {
  try {
    return apply_batched(plans, count, in, ldin, out, ldout, nrhs, mode, ws, ws_bytes, stream);
  } catch (...) {
    return fail(BFMHT_ENOSPACE, "host memory exhausted while grouping the batch");
  }
}

}  // extern "C"
