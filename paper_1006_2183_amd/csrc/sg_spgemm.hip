// Host side of the C ABI declared in include/sg_spgemm.h: argument checks,
// workspace layout, and the launch sequences of the symbolic, numeric and
// batched phases.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <type_traits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "sg_device.h"
#include "sg_symbolic.h"
#include "sg_tiers.h"
#include "sg_convert.h"
#include "sg_chain.h"

using namespace sg;

namespace {

// Text of the last failing HIP call (per host thread), for sg_last_error.
thread_local char g_last_error[256] = "";

sg_status hip_fail(hipError_t e, const char *what, int line) {
  snprintf(g_last_error, sizeof(g_last_error), "%s (HIP error %d: %s) at sg_spgemm.hip:%d", what, (int)e,
           hipGetErrorString(e), line);
  return SG_ERR_HIP;
}

// Wait on the host for the work enqueued on `st` by polling the stream. On
// served requests (a few short waits each) polling took about 0.05 ms off a
// request's latency against hipStreamSynchronize.
sg_status host_wait(hipStream_t st) {
  while (true) {
    const hipError_t e = hipStreamQuery(st);
    if (e == hipSuccess) return SG_OK;
    if (e != hipErrorNotReady) return hip_fail(e, "hipStreamQuery(st)", __LINE__);
  }
}

#define SG_HIP(call)                                                 \
  do {                                                               \
    hipError_t e_ = (call);                                          \
    if (e_ != hipSuccess) return hip_fail(e_, #call, __LINE__);      \
  } while (0)

#define SG_TRY(call)                \
  do {                              \
    sg_status s_ = (call);          \
    if (s_ != SG_OK) return s_;     \
  } while (0)

constexpr int kFillThreads = 256;
constexpr int64_t kMaxGrid = 65536;

int64_t grid_for(int64_t n, int threads) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  return g < kMaxGrid ? g : kMaxGrid;
}

bool row_major(int32_t fmt) { return fmt == SG_CSR || fmt == SG_DCSR; }
bool doubly(int32_t fmt) { return fmt == SG_DCSR || fmt == SG_DCSC; }
bool fmt_ok(int32_t fmt) { return fmt >= SG_CSR && fmt <= SG_DCSC; }

int slot_bytes(int32_t kind) {
  switch (kind) {
    case SG_PLUS_TIMES_F64: return 8;
    case SG_PLUS_TIMES_F32: return 4;
    case SG_MIN_PLUS_I32: return 4;
    default: return 0;
  }
}

// Dynamic LDS of a numeric small-list launch (256 threads): each wavefront's
// kSmallMaxFlops values.
int small_lds(int32_t kind) { return (256 / kWave) * kSmallMaxFlops * slot_bytes(kind); }

int64_t major_of(const sg_mat &M) { return row_major(M.fmt) ? M.nrows : M.ncols; }
int64_t minor_of(const sg_mat &M) { return row_major(M.fmt) ? M.ncols : M.nrows; }

// Bump allocator over the caller's workspace (256-byte alignment).
struct Carve {
  char *base;
  size_t off = 0;
  explicit Carve(void *b) : base((char *)b) {}
  template <class T>
  T *take(int64_t n) {
    off = (off + 255) & ~(size_t)255;
    T *p = base ? (T *)(base + off) : nullptr;
    off += (size_t)(n > 0 ? n : 1) * sizeof(T);
    return p;
  }
};


// The tuning as the heavy tier sees it: its windows are planned for the
// heavy workgroups' LDS budget.
sg_tuning heavy_view(const sg_tuning &t) {
  sg_tuning h = t;
  h.lds_bytes = t.heavy_lds_bytes;
  h.block_threads = t.heavy_threads;
  return h;
}

int heavy_window(const sg_tuning &t, int32_t kind) {
  const int sb = slot_bytes(kind);
  int64_t w = ((int64_t)t.lds_bytes * 8) / (8 * sb + 1);
  // flags live at the front in whole 64-bit units; keep the value array aligned
  while (w > 32 && 4 * (((w + 31) / 32 + 1) & ~1ll) + (int64_t)w * sb > t.lds_bytes) w -= 32;
  w &= ~31ll;
  if (t.heavy_kind == 1 && t.chunk_width > 0 && t.chunk_width < w) w = t.chunk_width & ~31;
  if (w < 32) w = 32;
  return (int)w;
}

// Largest mid-tier vector (entries) for a group with `minor` output ids; 0 = mid tier unusable.
int64_t mid_capacity(const sg_tuning &t, int32_t kind, int64_t minor) {
  const int sb = slot_bytes(kind);
  int64_t cap;
  if (t.mid_kind == 0) {
    // bitmap-rank: one {bits, prefix} pair of 32-bit words per 32 ids (bits
    // only without values), plus one bit per such word marking it touched
    int64_t nw32 = (minor + 31) / 32;
    int64_t ntop = (nw32 + 31) / 32;
    int64_t words = ((sb ? 2 * nw32 : nw32) + ntop + 1) & ~1ll;
    int64_t left = (int64_t)t.lds_bytes - 4 * words;
    if (left < 0) return 0;
    if (sb == 0) return minor;  // the bitmap alone is the accumulator
    cap = left / sb;
    if (cap > 65535) cap = 65535;  // ranks are kept in 16 bits
  } else {
    int64_t ts = 1;
    while (ts * 2 * (4 + sb) <= t.lds_bytes) ts *= 2;
    cap = ts / 2;
  }
  if (cap > t.mid_max_ub) cap = t.mid_max_ub;
  return cap < 0 ? 0 : cap;
}

// Heavy-tier geometry of one output id range (see GroupDev).
struct Geom {
  int32_t nsplit = 1, sw = 32, mode = 0, rank_cap = 0, rank_wb = 0, bpr = 1, rank_wcost = 0;
};

Geom group_geom(const sg_tuning &t, int32_t kind, int64_t minor, int win_dense) {
  const int64_t sb = slot_bytes(kind);
  const int64_t L = t.lds_bytes;
  Geom g;
  if (minor <= win_dense) {  // one dense window covers every id
    g.sw = win_dense;
    return g;
  }
  if (sb > 0 && t.heavy_kind == 0) {
    int64_t cap = (L / 2) / sb;
    if (cap > 65504) cap = 65504;  // ranks are kept in 16 bits
    cap &= ~31ll;
    int64_t sw = t.chunk_width > 0 ? t.chunk_width : 4096;
    if (sw > cap) sw = cap;
    sw &= ~31ll;
    if (sw >= 32) {
      const int64_t nw32 = (minor + 31) / 32;
      const int64_t nb = (minor + sw - 1) / sw;
      const bool count_fits = 4 * (nw32 + nb) <= L;
      int64_t wb = 0;
      while (wb < nb) {
        const int64_t nwds = (wb + 1) * sw / 32;
        if (8 * nwds + cap * sb > L) break;  // {bits, prefix} per 32 ids, then the values
        ++wb;
      }
      if (count_fits && wb >= 1 && nb < INT32_MAX) {
        // a window is bounded by its whole LDS, words and values together
        // (8 bytes of {bits, prefix} per 32 ids of its span, sb per entry),
        // so dense windows take more entries and sparse ones more buckets
        // than the half-and-half split that fixed sw
        g.mode = 1;
        g.sw = (int32_t)sw;
        g.nsplit = (int32_t)nb;
        g.rank_cap = (int32_t)(L / sb);
        g.rank_wcost = (int32_t)((8 * (sw / 32) + sb - 1) / sb);
        g.rank_wb = (int32_t)std::min<int64_t>(nb, (L / sb - 1) / g.rank_wcost);
        return g;
      }
    }
  }
  g.mode = 0;
  g.sw = win_dense;
  g.nsplit = (int32_t)((minor + win_dense - 1) / win_dense);
  return g;
}

}  // namespace

// ---------------------------------------------------------------------------
struct sg_plan {
  int32_t kind = 0;
  int32_t nprod = 0, ngroup = 0;
  int32_t out_fmt = 0;
  sg_tuning tune{};
  int win = 0;
  int ncu = 0;
  bool dense_path = false;
  bool has_mode[2] = {false, false};  // heavy window kinds used by the groups
  int lds_mid_count = 0;               // dynamic LDS of the count passes (bitmaps only)
  int lds_heavy_count = 0;
  int64_t nov_max = 0;
  int64_t items_max = 0;
  int64_t ndense_ptr = 0;
  std::vector<sg_sym_info> info;
  std::vector<int64_t> out_minor, out_major;
  Plan P{};
  // device pieces outside Plan
  int64_t *counters = nullptr;
  int64_t *gstat = nullptr;
  int64_t *nzpos = nullptr;
  int64_t *pbase = nullptr;
  OutDev *outs_dev = nullptr;
  // host copies (pageable: the symbolic phase waits for its stream anyway,
  // and a plan holds no pinned memory, whose release would synchronise the
  // whole device)
  std::vector<OutDev> outs_host;
  std::vector<int64_t> host_stats;
  // optional kernel timing: events around [heavy, mid, tiny, pointers]
  bool profile = false;
  bool events_made = false;
  bool timed = false;
  bool ran[4] = {false, false, false, false};
  hipEvent_t ev[8];
  // fused chain plans (sg_chain_symbolic)
  bool chain = false;
  const ChainDev *chains = nullptr;
  int chain_ts = 0;   // hash slots per stage of the chain mid tier
  int lds_chain = 0;  // its dynamic LDS bytes
  // small-list bound in effect: the tuning's, for plans with enough output
  // vectors to give every wavefront of the chip one (kSmallMinVectors);
  // otherwise 0, since one wavefront per vector leaves a plan of few
  // vectors waiting on the longest vector's gather and sort
  int32_t small_max = 0;
};

namespace {

struct Layout {
  ProdDev *prods;
  GroupDev *groups;
  OutDev *outs;
  int64_t *vbase;
  int64_t *counters;
  int64_t *gstat;
  int32_t *ov_id, *ov_group, *seg_prod, *seg_svec;
  int64_t *ov_seg, *ov_flops, *ov_cnt, *ov_off, *nzflag, *nzpos;
  int32_t *tiny, *mid, *heavy, *small;
  int64_t *heavy_nwin, *ibase;
  ItemDev *items;
  int32_t *bcnt;
  std::vector<int32_t *> gres, aux, wsplit;
  std::vector<int64_t> aux_chunk, aux_n;
  int64_t *dbase, *dcnt, *dflag, *vpos, *spos, *dfill;
  int64_t *pbase;
  int64_t *part;
  int64_t part_cap;
  uint32_t *hbits;
  size_t tables_end;   // byte offset where the host-built tables end
  int64_t zero_words;  // int64 words from `counters` on that start at zero
  int32_t *vsent;
  int64_t *rcnt, *rbase;
  int64_t *mcnt, *mbase, *mid_rb;  // mid-tier records: counts, their scan, final bases
  int32_t *mid_nrec;
  int64_t *rec_gi, *rec_gv;
  int32_t *rec_len;
  void *rec_sv;
  size_t bytes;
};

struct Shape {
  int64_t nov_max = 0;       // output vectors (at most one per output major id of a group)
  int64_t nseg_max = 0;      // segments: stored streamed vectors of all products
  int64_t ndense = 0;        // sum of output major dims (multi-product groups)
  int64_t ndense_ptr = 0;    // sum of (major + 1) for dense output pointers
  int32_t nbmax = 1;
  int32_t nrange = 1;      // XCD ranges of the heavy windows
  int64_t hstride = 0;     // words of a kept heavy bitmap (widest rank-mode group)
  int64_t nkeep = 0;       // heavy vectors whose bitmaps the workspace can keep
  int64_t rec_cap = 0;     // entry records of heavy windows the workspace holds
  int32_t slot_bytes = 0;  // value bytes of the semiring
  bool dense_path = false;
  std::vector<Geom> geom;  // per group
  std::vector<int64_t> minor, major;
  std::vector<int32_t> gres_src, wsplit_src, aux_src;  // dedupe: product sharing the table
};

struct ProdView {
  const sg_mat *S, *G;
};

ProdView view(const sg_mat &A, const sg_mat &B) {
  // column-major: B streamed, A gathered; row-major: A streamed, B gathered
  return row_major(A.fmt) ? ProdView{&A, &B} : ProdView{&B, &A};
}

sg_status check_mat(const sg_mat &M, int32_t kind) {
  if (!fmt_ok(M.fmt)) return SG_ERR_INVALID_ARG;
  if (M.nrows < 0 || M.ncols < 0 || M.nnz < 0 || M.nvec < 0) return SG_ERR_INVALID_ARG;
  if (M.nrows >= INT32_MAX || M.ncols >= INT32_MAX || M.nnz >= ((int64_t)1 << 40)) return SG_ERR_UNSUPPORTED;
  const int64_t maj = major_of(M);
  if (doubly(M.fmt)) {
    if (M.nvec > maj) return SG_ERR_INVALID_ARG;
    if (M.nvec > 0 && !M.vid) return SG_ERR_INVALID_ARG;
  } else if (M.nvec != maj) {
    return SG_ERR_INVALID_ARG;
  }
  if (!M.ptr) return SG_ERR_INVALID_ARG;
  if (M.nnz > 0 && !M.idx) return SG_ERR_INVALID_ARG;
  if (kind != SG_OR_AND_BOOL && M.nnz > 0 && !M.val) return SG_ERR_INVALID_ARG;
  return SG_OK;
}

sg_status check_args(const sg_semiring *sr, int32_t nprod, const sg_mat *A, const sg_mat *B, const int32_t *group,
                     int32_t ngroup, int32_t out_fmt, Shape &sh, std::vector<int32_t> &grp) {
  if (!sr || sr->kind < SG_PLUS_TIMES_F64 || sr->kind > SG_OR_AND_BOOL) return SG_ERR_INVALID_ARG;
  if (nprod < 1 || !A || !B) return SG_ERR_INVALID_ARG;
  if (!group) ngroup = nprod;
  if (ngroup < 1) return SG_ERR_INVALID_ARG;
  if (!fmt_ok(out_fmt)) return SG_ERR_INVALID_ARG;
  const bool rm = row_major(A[0].fmt);
  if (row_major(out_fmt) != rm) return SG_ERR_UNSUPPORTED;
  grp.resize(nprod);
  sh.minor.assign(ngroup, -1);
  sh.major.assign(ngroup, -1);
  std::vector<int32_t> per_group(ngroup, 0);
  for (int32_t p = 0; p < nprod; ++p) {
    SG_TRY(check_mat(A[p], sr->kind));
    SG_TRY(check_mat(B[p], sr->kind));
    if (row_major(A[p].fmt) != rm || row_major(B[p].fmt) != rm) return SG_ERR_UNSUPPORTED;
    if (A[p].ncols != B[p].nrows) return SG_ERR_DIM_MISMATCH;
    const int32_t g = group ? group[p] : p;
    if (g < 0 || g >= ngroup) return SG_ERR_INVALID_ARG;
    grp[p] = g;
    per_group[g]++;
    const int64_t omaj = rm ? A[p].nrows : B[p].ncols;
    const int64_t omin = rm ? B[p].ncols : A[p].nrows;
    if (sh.minor[g] < 0) {
      sh.minor[g] = omin;
      sh.major[g] = omaj;
    } else if (sh.minor[g] != omin || sh.major[g] != omaj) {
      return SG_ERR_DIM_MISMATCH;
    }
  }
  for (int32_t g = 0; g < ngroup; ++g) {
    if (per_group[g] > 1) sh.dense_path = true;
    if (sh.minor[g] < 0) {  // a group with no product: empty output of unknown shape
      return SG_ERR_INVALID_ARG;
    }
  }
  return SG_OK;
}

void make_shape(int32_t kind, int32_t nprod, const sg_mat *A, const sg_mat *B, const std::vector<int32_t> &grp,
                int32_t ngroup, const sg_tuning &t, int win, Shape &sh) {
  sh.nseg_max = 0;
  for (int32_t p = 0; p < nprod; ++p) sh.nseg_max += view(A[p], B[p]).S->nvec;
  sh.nov_max = sh.nseg_max;
  sh.geom.resize(ngroup);
  sh.nbmax = 1;
  sh.ndense = 0;
  sh.ndense_ptr = 0;
  sh.nrange = t.xcd_ranges > 0 ? kXcds * t.xcd_ranges : 1;
  for (int32_t g = 0; g < ngroup; ++g) {
    sh.geom[g] = group_geom(heavy_view(t), kind, sh.minor[g], win);
    Geom &ge = sh.geom[g];
    ge.bpr = (ge.nsplit + sh.nrange - 1) / sh.nrange;
    sh.nbmax = std::max<int32_t>(sh.nbmax, sh.geom[g].nsplit);
    sh.ndense += sh.major[g];
    sh.ndense_ptr += sh.major[g] + 1;
  }
  if (sh.dense_path) sh.nov_max = std::min<int64_t>(sh.nseg_max, sh.ndense);
  for (int32_t g = 0; g < ngroup; ++g)
    if (sh.geom[g].mode == 1) sh.hstride = std::max<int64_t>(sh.hstride, (sh.minor[g] + 31) / 32);
  if (sh.hstride > 0 && t.bitmap_mb > 0) {
    const int64_t budget = (int64_t)t.bitmap_mb << 20;
    sh.nkeep = std::min<int64_t>(sh.nov_max, budget / (4 * sh.hstride));
  }
  sh.slot_bytes = slot_bytes(kind);
  if (sh.hstride > 0 && t.entry_mb > 0) {  // rank windows exist
    // at most one record per streamed entry and window (at most nbmax
    // windows per heavy vector), or per streamed entry of a mid-tier
    // vector; the budget caps the rest
    int64_t sent = 0;
    for (int32_t p = 0; p < nprod; ++p) sent += view(A[p], B[p]).S->nnz;
    const int64_t per = 20 + slot_bytes(kind);  // two addresses, a count, the S value
    sh.rec_cap = std::min<int64_t>(((int64_t)t.entry_mb << 20) / per, sent * ((int64_t)sh.nbmax + 1));
  }

  // products whose gathered operand is the same arrays share the AUX index,
  // and the split table too when their groups split ids the same way
  sh.wsplit_src.assign(nprod, -1);
  sh.aux_src.assign(nprod, -1);
  for (int32_t p = 0; p < nprod; ++p) {
    const sg_mat *G = view(A[p], B[p]).G;
    for (int32_t q = 0; q < p; ++q) {
      const sg_mat *H = view(A[q], B[q]).G;
      if (H->ptr == G->ptr && H->idx == G->idx && H->vid == G->vid && H->nvec == G->nvec) {
        if (sh.aux_src[p] < 0) sh.aux_src[p] = q;
        const Geom &a = sh.geom[grp[q]], &b = sh.geom[grp[p]];
        if (sh.wsplit_src[p] < 0 && a.nsplit == b.nsplit && a.sw == b.sw) sh.wsplit_src[p] = q;
      }
    }
  }
}

Layout carve(void *ws, int32_t nprod, const sg_mat *A, const sg_mat *B, int32_t ngroup, const Shape &sh,
             const std::vector<int32_t> &grp) {
  Layout L{};
  Carve c(ws);
  const int64_t nov = sh.nov_max;
  // the host-built tables first, contiguous, so one copy uploads them
  L.prods = c.take<ProdDev>(nprod);
  L.groups = c.take<GroupDev>(ngroup);
  L.vbase = c.take<int64_t>(nprod + 1);
  L.dbase = c.take<int64_t>(ngroup + 1);
  L.pbase = c.take<int64_t>(ngroup + 1);
  L.tables_end = c.off;
  L.outs = c.take<OutDev>(ngroup);
  // arrays that start at zero, contiguous: one fill clears them
  L.counters = c.take<int64_t>(kCtNum + 24);
  L.gstat = c.take<int64_t>((int64_t)ngroup * kStCount);
  L.ov_flops = c.take<int64_t>(nov);
  L.ov_cnt = c.take<int64_t>(nov + 1);
  L.zero_words = (int64_t)((c.off - ((char *)L.counters - c.base)) / sizeof(int64_t));
  L.ov_id = c.take<int32_t>(nov);
  L.ov_group = c.take<int32_t>(nov);
  L.seg_prod = c.take<int32_t>(sh.nseg_max);
  L.seg_svec = c.take<int32_t>(sh.nseg_max);
  L.ov_seg = c.take<int64_t>(nov + 1);
  L.ov_off = c.take<int64_t>(nov + 1);
  L.nzflag = c.take<int64_t>(nov + 1);
  L.nzpos = c.take<int64_t>(nov + 1);
  L.tiny = c.take<int32_t>(nov);
  L.mid = c.take<int32_t>(nov);
  L.heavy = c.take<int32_t>(nov);
  L.small = c.take<int32_t>(nov);
  L.heavy_nwin = c.take<int64_t>(nov * sh.nrange + 1);
  L.ibase = c.take<int64_t>(nov * sh.nrange + 1);
  const int64_t items = nov * (int64_t)sh.nbmax;
  L.items = c.take<ItemDev>(items);
  L.bcnt = c.take<int32_t>(items);
  L.gres.assign(nprod, nullptr);
  L.aux.assign(nprod, nullptr);
  L.wsplit.assign(nprod, nullptr);
  L.aux_chunk.assign(nprod, 0);
  L.aux_n.assign(nprod, 0);
  for (int32_t p = 0; p < nprod; ++p) {
    ProdView pv = view(A[p], B[p]);
    const sg_mat &G = *pv.G;
    if (doubly(G.fmt)) {
      L.gres[p] = c.take<int32_t>(pv.S->nnz);
      const int64_t maj = major_of(G);
      int64_t chunk = G.nvec > 0 ? (maj + G.nvec - 1) / G.nvec : (maj > 0 ? maj : 1);
      if (chunk < 1) chunk = 1;
      int64_t nchunks = (maj + chunk - 1) / chunk;
      L.aux_chunk[p] = chunk;
      L.aux_n[p] = nchunks;
      if (sh.aux_src[p] >= 0) L.aux[p] = L.aux[sh.aux_src[p]];
      else L.aux[p] = c.take<int32_t>(nchunks + 1);
    }
    const int32_t nb = sh.geom[grp[p]].nsplit;
    if (nb > 1) {
      if (sh.wsplit_src[p] >= 0) L.wsplit[p] = L.wsplit[sh.wsplit_src[p]];
      else L.wsplit[p] = c.take<int32_t>(G.nvec * (int64_t)(nb + 1));
    }
  }
  int64_t scan_max = std::max<int64_t>(nov * sh.nrange + 1, sh.ndense + 1);
  if (sh.dense_path) {
    L.dcnt = c.take<int64_t>(sh.ndense + 1);
    L.dflag = c.take<int64_t>(sh.ndense + 1);
    L.vpos = c.take<int64_t>(sh.ndense + 1);
    L.spos = c.take<int64_t>(sh.ndense + 1);
    L.dfill = c.take<int64_t>(sh.ndense + 1);
  } else {
    L.dcnt = L.dflag = L.vpos = L.spos = L.dfill = nullptr;
  }
  L.part_cap = scan_max / kScanTile + 4;
  L.part = c.take<int64_t>(L.part_cap);
  L.hbits = sh.nkeep > 0 ? c.take<uint32_t>(sh.nkeep * sh.hstride) : nullptr;
  if (sh.rec_cap > 0) {
    L.vsent = c.take<int32_t>(nov + 1);
    L.rcnt = c.take<int64_t>(nov + 1);
    L.rbase = c.take<int64_t>(nov + 1);
    L.mcnt = c.take<int64_t>(nov + 1);
    L.mbase = c.take<int64_t>(nov + 1);
    L.mid_rb = c.take<int64_t>(nov + 1);
    L.mid_nrec = c.take<int32_t>(nov + 1);
    L.rec_gi = c.take<int64_t>(sh.rec_cap);
    L.rec_gv = c.take<int64_t>(sh.rec_cap);
    L.rec_len = c.take<int32_t>(sh.rec_cap);
    L.rec_sv = (void *)c.take<uint8_t>(sh.rec_cap * std::max(1, sh.slot_bytes));
  } else {
    L.vsent = nullptr;
    L.rcnt = L.rbase = L.rec_gi = L.rec_gv = nullptr;
    L.mcnt = L.mbase = L.mid_rb = nullptr;
    L.mid_nrec = nullptr;
    L.rec_len = nullptr;
    L.rec_sv = nullptr;
  }
  L.bytes = c.off + 256;
  return L;
}

sg_status fill64(int64_t *p, int64_t n, int64_t v, hipStream_t st) {
  if (n <= 0) return SG_OK;
  hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)grid_for(n, kFillThreads)), dim3(kFillThreads), 0, st, p, n, v);
  SG_HIP(hipGetLastError());
  return SG_OK;
}

// out[0..n] = exclusive scan of in[0..n), out[n] = total. Up to
// kSmallScan elements take one single-workgroup launch, more three passes.
// `part` holds part_cap entries (n / kScanTile + 2 are needed).
sg_status scan64(const int64_t *in, int64_t n, int64_t *out, int64_t *part, int64_t part_cap, hipStream_t st) {
  if (n <= 0) return fill64(out, 1, 0, st);
  if (n <= kSmallScan) {
    hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, in, n, out);
    SG_HIP(hipGetLastError());
    return SG_OK;
  }
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb + 1 > part_cap) {
    snprintf(g_last_error, sizeof(g_last_error), "scan of %lld elements needs %lld partials, workspace holds %lld",
             (long long)n, (long long)(nb + 1), (long long)part_cap);
    return SG_ERR_WORKSPACE;
  }
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, n, part);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, st, part, nb);
  hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, n, part, nb, out);
  SG_HIP(hipGetLastError());
  return SG_OK;
}

int device_cus() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
  return n;
}

void normalise(sg_tuning &t, int32_t kind) {
  sg_tuning d;
  sg_tuning_default(kind, &d);
  if (t.tiny_max_flops < 0 || t.tiny_max_flops > 64) t.tiny_max_flops = d.tiny_max_flops;
  if (t.mid_max_ub < 0) t.mid_max_ub = d.mid_max_ub;
  if (t.mid_kind != 0 && t.mid_kind != 1) t.mid_kind = 0;
  // the kernels' static LDS (scan scratch, per-wave owner maps) takes the rest of the 160 KB
  if (t.lds_bytes < 4096 || t.lds_bytes > 160 * 1024 - 2048) t.lds_bytes = d.lds_bytes;
  t.lds_bytes &= ~7;
  if (t.block_threads < 64 || t.block_threads > kBlockMax || t.block_threads % 64) t.block_threads = d.block_threads;
  if (t.chunk_width < 0) t.chunk_width = 0;
  if (t.heavy_kind != 0 && t.heavy_kind != 1) t.heavy_kind = 0;
  if (t.force_tier < -1 || t.force_tier > 3) t.force_tier = -1;
  if (t.blocks_per_cu < 1 || t.blocks_per_cu > 32) t.blocks_per_cu = d.blocks_per_cu;
  if (t.xcd_ranges < 0 || t.xcd_ranges > 16) t.xcd_ranges = d.xcd_ranges;
  if (t.bitmap_mb < 0) t.bitmap_mb = d.bitmap_mb;
  if (t.heavy_threads == 0) t.heavy_threads = t.block_threads;
  if (t.heavy_threads < 64 || t.heavy_threads > kBlockMax || t.heavy_threads % 64) t.heavy_threads = d.heavy_threads;
  if (t.entry_mb < 0) t.entry_mb = d.entry_mb;
  if (t.small_max_flops < 0 || t.small_max_flops > kSmallMaxFlops) t.small_max_flops = d.small_max_flops;
  if (t.heavy_lds_bytes == 0) t.heavy_lds_bytes = t.lds_bytes;
  if (t.heavy_lds_bytes < 4096 || t.heavy_lds_bytes > 160 * 1024 - 2048) t.heavy_lds_bytes = d.heavy_lds_bytes;
  t.heavy_lds_bytes &= ~7;
}


template <int K>
sg_status set_lds_attr(int bytes) {
  SG_HIP(hipFuncSetAttribute((const void *)k_mid_count<K>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
  SG_HIP(hipFuncSetAttribute((const void *)k_mid<K>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
  SG_HIP(hipFuncSetAttribute((const void *)k_heavy_count<K, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
  SG_HIP(hipFuncSetAttribute((const void *)k_heavy_count<K, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
  SG_HIP(hipFuncSetAttribute((const void *)k_heavy<K, 0, false>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
  SG_HIP(hipFuncSetAttribute((const void *)k_heavy<K, 1, false>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
  SG_HIP(hipFuncSetAttribute((const void *)k_heavy<K, 1, true>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
  SG_HIP(hipFuncSetAttribute((const void *)k_batched<K, 0, false>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
  SG_HIP(hipFuncSetAttribute((const void *)k_batched<K, 1, false>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
  SG_HIP(hipFuncSetAttribute((const void *)k_batched<K, 1, true>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
  SG_HIP(hipFuncSetAttribute((const void *)k_batched<K, 2, false>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
  SG_HIP(hipFuncSetAttribute((const void *)k_batched<K, 2, true>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
  SG_HIP(hipFuncSetAttribute((const void *)k_chain_mid<K, true>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
  SG_HIP(hipFuncSetAttribute((const void *)k_chain_mid<K, false>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
  return SG_OK;
}

// Persistent workgroups for a kernel of `nt` threads and `lds` dynamic LDS
// bytes whose register budget allows `waves_per_simd` wavefronts per SIMD.
int64_t resident_blocks(int ncu, int nt, int lds, int waves_per_simd) {
  const int64_t by_waves = (int64_t)4 * waves_per_simd / (nt / kWave);
  const int64_t by_lds = lds > 0 ? (int64_t)(160 * 1024 - 2048) / lds : by_waves;
  return (int64_t)ncu * std::max<int64_t>(1, std::min(by_waves, by_lds));
}

template <int K>
sg_status launch_counts(sg_plan *pl, hipStream_t st) {
  const int nt = pl->tune.block_threads;
  const int64_t persist = (int64_t)pl->ncu * pl->tune.blocks_per_cu;
  const int64_t tiny_blocks = std::min<int64_t>(std::max<int64_t>(1, (pl->nov_max + 3) / 4), persist * 8);
  hipLaunchKernelGGL((k_tiny<K, true>), dim3((unsigned)tiny_blocks), dim3(256), 0, st, pl->P);
  SG_HIP(hipGetLastError());
  if (pl->small_max > 0 || pl->tune.force_tier == 3) {
    hipLaunchKernelGGL((k_small<K, true, false>), dim3((unsigned)tiny_blocks), dim3(256), 0, st, pl->P);
    SG_HIP(hipGetLastError());
  }
  // the count kernels zero exactly the LDS they are launched with
  Plan Pm = pl->P;
  Pm.lds_words = pl->lds_mid_count / 4;
  hipLaunchKernelGGL((k_mid_count<K>), dim3((unsigned)resident_blocks(pl->ncu, nt, pl->lds_mid_count, kCountWavesPerSimd)),
                     dim3(nt), pl->lds_mid_count, st, Pm, pl->counters + kCtNum + 0);
  SG_HIP(hipGetLastError());
  Plan Ph = pl->P;
  Ph.lds_words = pl->lds_heavy_count / 4;
  for (int m = 0; m < 2; ++m) {
    if (!pl->has_mode[m]) continue;
    const unsigned hb = (unsigned)resident_blocks(pl->ncu, nt, pl->lds_heavy_count,
                                                  m == 0 ? heavy_count_waves<0>() : heavy_count_waves<1>());
    if (m == 0)
      hipLaunchKernelGGL((k_heavy_count<K, 0>), dim3(hb), dim3(nt), pl->lds_heavy_count, st, Ph, pl->counters + kCtNum + 1);
    else
      hipLaunchKernelGGL((k_heavy_count<K, 1>), dim3(hb), dim3(nt), pl->lds_heavy_count, st, Ph, pl->counters + kCtNum + 4);
    SG_HIP(hipGetLastError());
  }
  return SG_OK;
}

// One readback of a plan's counters and its per-group statistics, which sit
// next to each other in the workspace (the statistics from the next 256-byte
// boundary on): every small device-to-host copy costs a copy launch of its
// own. On return host_stats holds the span; the statistics start at word goff.
sg_status read_stats(sg_plan *pl, const int64_t *counters, const int64_t *gstat, int64_t nstat, hipStream_t st,
                     int64_t &goff) {
  goff = (int64_t)(gstat - counters);
  const size_t words = (size_t)(goff + nstat);
  pl->host_stats.assign(words, 0);
  SG_HIP(hipMemcpyAsync(pl->host_stats.data(), counters, sizeof(int64_t) * words, hipMemcpyDeviceToHost, st));
  return host_wait(st);
}

sg_status mark(sg_plan *pl, int which, bool end, hipStream_t st) {
  if (!pl->profile) return SG_OK;
  SG_HIP(hipEventRecord(pl->ev[2 * which + (end ? 1 : 0)], st));
  if (end) pl->ran[which] = true;
  return SG_OK;
}

template <int K>
sg_status launch_numeric(sg_plan *pl, hipStream_t st) {
  const Plan &P = pl->P;
  const int nt = pl->tune.block_threads;
  const int lds = pl->tune.lds_bytes;
  const sg_sym_info &I = pl->info[0];
  const int64_t persist = (int64_t)pl->ncu * pl->tune.blocks_per_cu;
  SG_TRY(fill64(pl->counters + kCtNum + 2, 22, 0, st));
  if (I.n_heavy_items > 0) {
    SG_TRY(mark(pl, 0, false, st));
    const int hnt = pl->tune.heavy_threads, hlds = pl->tune.heavy_lds_bytes;
    Plan Ph = P;
    Ph.lds_words = hlds / 4;
    // as many workgroups as fit the chip, a multiple of the XCD count so
    // every die gets the same number
    const int64_t hres = resident_blocks(pl->ncu, hnt, hlds, kWavesPerSimd);
    const unsigned hg = (unsigned)std::max<int64_t>(kXcds, std::min<int64_t>(hres, I.n_heavy_items) / kXcds * kXcds);
    if (pl->has_mode[0])
      hipLaunchKernelGGL((k_heavy<K, 0, false>), dim3(hg), dim3(hnt), hlds, st, Ph, pl->counters + kCtNum + 8);
    if (pl->has_mode[1]) {
      if (pl->P.rec_cap > 0)
        hipLaunchKernelGGL((k_heavy<K, 1, true>), dim3(hg), dim3(hnt), hlds, st, Ph, pl->counters + kCtNum + 16);
      else
        hipLaunchKernelGGL((k_heavy<K, 1, false>), dim3(hg), dim3(hnt), hlds, st, Ph, pl->counters + kCtNum + 16);
    }
    SG_HIP(hipGetLastError());
    SG_TRY(mark(pl, 0, true, st));
  }
  if (I.n_mid > 0) {
    SG_TRY(mark(pl, 1, false, st));
    hipLaunchKernelGGL((k_mid<K>), dim3((unsigned)std::min<int64_t>(persist, I.n_mid)), dim3(nt), lds, st, P,
                       pl->counters + kCtNum + 3);
    SG_HIP(hipGetLastError());
    SG_TRY(mark(pl, 1, true, st));
  }
  if (I.n_tiny > 0 || I.n_small > 0) {
    SG_TRY(mark(pl, 2, false, st));
    if (I.n_small > 0)
      hipLaunchKernelGGL((k_small<K, false, true>), dim3((unsigned)std::min<int64_t>((I.n_small + 3) / 4, persist * 8)),
                         dim3(256), small_lds(pl->kind), st, P);
    if (I.n_tiny > 0)
      hipLaunchKernelGGL((k_tiny<K, false>), dim3((unsigned)std::min<int64_t>((I.n_tiny + 3) / 4, persist * 8)), dim3(256),
                         0, st, P);
    SG_HIP(hipGetLastError());
    SG_TRY(mark(pl, 2, true, st));
  }
  return SG_OK;
}

template <int K>
sg_status launch_batched(sg_plan *pl, hipStream_t st) {
  // heavy windows are planned for the heavy workgroups, which also fit
  // every mid vector when given the larger of the two LDS budgets
  const int nt = pl->tune.heavy_threads;
  const int lds = std::max(pl->tune.lds_bytes, pl->tune.heavy_lds_bytes);
  Plan P = pl->P;
  P.lds_words = lds / 4;
  const sg_sym_info &I = pl->info[0];
  if (I.n_heavy_items == 0 && I.n_mid == 0 && I.n_small == 0) {
    // tiny vectors only (Galerkin triple products on grids): the tiny
    // kernel alone is the one launch, with no LDS to cap its occupancy
    SG_TRY(mark(pl, 0, false, st));
    if (I.n_tiny > 0) {
      const int64_t tp = (int64_t)pl->ncu * pl->tune.blocks_per_cu * 8;
      hipLaunchKernelGGL((k_tiny<K, false>), dim3((unsigned)std::min<int64_t>((I.n_tiny + 3) / 4, tp)), dim3(256), 0,
                         st, pl->P);
      SG_HIP(hipGetLastError());
    }
    SG_TRY(mark(pl, 0, true, st));
    return SG_OK;
  }
  // as many workgroups as fit the chip, but no more than there are work items
  // (a tiny chunk holds up to 64 vectors per wavefront), so a small plan does
  // not hold every compute unit's LDS for the length of its launch
  const int64_t work = I.n_heavy_items + I.n_mid + (I.n_tiny + (int64_t)kWave * (nt / kWave) - 1) / (kWave * (nt / kWave));
  const int64_t persist = std::max<int64_t>(1, std::min(resident_blocks(pl->ncu, nt, lds, kWavesPerSimd), work));
  SG_TRY(fill64(pl->counters + kCtQueue, 1, 0, st));
  SG_TRY(mark(pl, 0, false, st));
  // the small list first, on the same stream: beside the persistent launch
  // (on a second stream) its wavefronts would hold compute units the
  // persistent workgroups are sized for, which measured slower
  if (I.n_small > 0) {
    const int64_t sp = (int64_t)pl->ncu * pl->tune.blocks_per_cu * 8;
    hipLaunchKernelGGL((k_small<K, false, true>), dim3((unsigned)std::min<int64_t>((I.n_small + 3) / 4, sp)), dim3(256),
                       small_lds(pl->kind), st, pl->P);
    SG_HIP(hipGetLastError());
  }
  const int mode = pl->has_mode[0] && pl->has_mode[1] ? 2 : (pl->has_mode[1] ? 1 : 0);
  const bool recs = P.rec_cap > 0 && mode != 0;  // only rank windows (mode 1) carry records
  const int64_t ni = I.n_heavy_items, nm = I.n_mid, ntn = I.n_tiny;
  int64_t *q = pl->counters + kCtQueue;
  if (mode == 0)
    hipLaunchKernelGGL((k_batched<K, 0, false>), dim3((unsigned)persist), dim3(nt), lds, st, P, q, ni, nm, ntn);
  else if (mode == 1 && recs)
    hipLaunchKernelGGL((k_batched<K, 1, true>), dim3((unsigned)persist), dim3(nt), lds, st, P, q, ni, nm, ntn);
  else if (mode == 1)
    hipLaunchKernelGGL((k_batched<K, 1, false>), dim3((unsigned)persist), dim3(nt), lds, st, P, q, ni, nm, ntn);
  else if (recs)
    hipLaunchKernelGGL((k_batched<K, 2, true>), dim3((unsigned)persist), dim3(nt), lds, st, P, q, ni, nm, ntn);
  else
    hipLaunchKernelGGL((k_batched<K, 2, false>), dim3((unsigned)persist), dim3(nt), lds, st, P, q, ni, nm, ntn);
  SG_HIP(hipGetLastError());
  SG_TRY(mark(pl, 0, true, st));
  return SG_OK;
}

template <template <int> class F, class... Args>
sg_status dispatch(int32_t kind, Args... a) {
  switch (kind) {
    case SG_PLUS_TIMES_F64: return F<SG_PLUS_TIMES_F64>::run(a...);
    case SG_PLUS_TIMES_F32: return F<SG_PLUS_TIMES_F32>::run(a...);
    case SG_MIN_PLUS_I32: return F<SG_MIN_PLUS_I32>::run(a...);
    case SG_OR_AND_BOOL: return F<SG_OR_AND_BOOL>::run(a...);
    default: return SG_ERR_INVALID_ARG;
  }
}
template <int K>
struct RunCounts {
  static sg_status run(sg_plan *pl, hipStream_t st) { return launch_counts<K>(pl, st); }
};
template <int K>
struct RunNumeric {
  static sg_status run(sg_plan *pl, hipStream_t st) { return launch_numeric<K>(pl, st); }
};
template <int K>
struct RunBatched {
  static sg_status run(sg_plan *pl, hipStream_t st) { return launch_batched<K>(pl, st); }
};
template <int K>
struct RunItemRecs {
  static sg_status run(const Plan &P, int ncu, hipStream_t st) {
    hipLaunchKernelGGL((k_item_recs<K>), dim3((unsigned)ncu * 16), dim3(256), 0, st, P);
    SG_HIP(hipGetLastError());
    return SG_OK;
  }
};
template <int K>
struct RunMidRecs {
  static sg_status run(const Plan &P, int ncu, hipStream_t st) {
    hipLaunchKernelGGL((k_mid_recs<K>), dim3((unsigned)ncu * 16), dim3(256), 0, st, P);
    SG_HIP(hipGetLastError());
    return SG_OK;
  }
};
// The dynamic-LDS limit of the kernels is raised once per semiring and
// process (to the largest budget any plan has asked for), not per plan.
template <int K>
struct RunAttr {
  static sg_status run(int bytes) {
    static std::mutex mu;
    static int done = 0;
    std::lock_guard<std::mutex> lock(mu);
    if (bytes <= done) return SG_OK;
    SG_TRY(set_lds_attr<K>(bytes));
    done = bytes;
    return SG_OK;
  }
};

// Launches of a fused chain plan: tiny vectors one wavefront each, mid
// vectors one workgroup each from a queue; COUNT = the symbolic count pass.
template <int K>
struct RunChain {
  static sg_status run(sg_plan *pl, bool count, hipStream_t st) {
    const sg_sym_info &I = pl->info[0];
    const int64_t ntiny = count ? pl->nov_max : I.n_tiny;
    const int64_t nmid = count ? pl->nov_max : I.n_mid;
    const int64_t persist = (int64_t)pl->ncu * pl->tune.blocks_per_cu;
    if (ntiny > 0) {
      const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((ntiny + 3) / 4, persist * 16));
      if (!count) SG_TRY(mark(pl, 2, false, st));
      if (count) hipLaunchKernelGGL((k_chain_tiny<K, true>), dim3(g), dim3(256), 0, st, pl->P, pl->chains, pl->gstat);
      else hipLaunchKernelGGL((k_chain_tiny<K, false>), dim3(g), dim3(256), 0, st, pl->P, pl->chains, pl->gstat);
      SG_HIP(hipGetLastError());
      if (!count) SG_TRY(mark(pl, 2, true, st));
    }
    if (nmid > 0) {
      int64_t *q = pl->counters + kCtNum + (count ? 0 : 3);
      SG_TRY(fill64(q, 1, 0, st));
      Plan Pc = pl->P;
      Pc.lds_words = pl->lds_chain / 4;
      const int nt = pl->tune.block_threads;
      const unsigned g = (unsigned)std::max<int64_t>(
          1, std::min<int64_t>(resident_blocks(pl->ncu, nt, pl->lds_chain, kWavesPerSimd), nmid));
      if (!count) SG_TRY(mark(pl, 1, false, st));
      if (count)
        hipLaunchKernelGGL((k_chain_mid<K, true>), dim3(g), dim3(nt), pl->lds_chain, st, Pc, pl->chains, q,
                           pl->chain_ts, pl->gstat);
      else
        hipLaunchKernelGGL((k_chain_mid<K, false>), dim3(g), dim3(nt), pl->lds_chain, st, Pc, pl->chains, q,
                           pl->chain_ts, pl->gstat);
      SG_HIP(hipGetLastError());
      if (!count) SG_TRY(mark(pl, 1, true, st));
    }
    return SG_OK;
  }
};

sg_status emit_outputs(sg_plan *pl, sg_mat_out *C, hipStream_t st) {
  if (!C) return SG_ERR_INVALID_ARG;
  const bool rm = row_major(pl->out_fmt);
  for (int32_t g = 0; g < pl->ngroup; ++g) {
    const sg_mat_out &O = C[g];
    const sg_sym_info &I = pl->info[g];
    if (O.fmt != pl->out_fmt) return SG_ERR_INVALID_ARG;
    const int64_t omaj = pl->out_major[g], omin = pl->out_minor[g];
    if ((rm ? O.nrows : O.ncols) != omaj || (rm ? O.ncols : O.nrows) != omin) return SG_ERR_DIM_MISMATCH;
    if (O.cap_nnz < I.nnz) return SG_ERR_CAPACITY;
    if (!O.ptr) return SG_ERR_INVALID_ARG;
    if (I.nnz > 0 && !O.idx) return SG_ERR_INVALID_ARG;
    if (I.nnz > 0 && pl->kind != SG_OR_AND_BOOL && !O.val) return SG_ERR_INVALID_ARG;
    if (doubly(pl->out_fmt)) {
      if (O.cap_vec < I.nvec) return SG_ERR_CAPACITY;
      if (I.nvec > 0 && !O.vid) return SG_ERR_INVALID_ARG;
    }
    OutDev &D = pl->outs_host[g];
    D.ptr = O.ptr;
    D.vid = O.vid;
    D.idx = O.idx;
    D.val = O.val;
    D.fmt = O.fmt;
    D.pad = 0;
  }
  for (int32_t g0 = 0; g0 < pl->ngroup; g0 += kOutChunk) {
    OutChunk chunk;
    std::memset(&chunk, 0, sizeof(chunk));
    const int32_t n = std::min<int32_t>(kOutChunk, pl->ngroup - g0);
    for (int32_t i = 0; i < n; ++i) chunk.o[i] = pl->outs_host[g0 + i];
    hipLaunchKernelGGL(k_set_outs, dim3(1), dim3(kOutChunk), 0, st, pl->outs_dev, g0, n, chunk);
    SG_HIP(hipGetLastError());
  }
  for (int i = 0; i < 4; ++i) pl->ran[i] = false;
  pl->timed = pl->profile;
  SG_TRY(mark(pl, 3, false, st));
  if (doubly(pl->out_fmt)) {
    hipLaunchKernelGGL(k_emit_ptr_doubly, dim3((unsigned)grid_for(pl->nov_max + 1, kFillThreads)), dim3(kFillThreads), 0,
                       st, pl->P, pl->nzpos, pl->ngroup);
  } else {
    hipLaunchKernelGGL(k_emit_ptr_dense, dim3((unsigned)grid_for(pl->ndense_ptr, kFillThreads)), dim3(kFillThreads), 0,
                       st, pl->P, pl->pbase, pl->ngroup, pl->ndense_ptr);
  }
  SG_HIP(hipGetLastError());
  SG_TRY(mark(pl, 3, true, st));
  return SG_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
extern "C" {

void sg_tuning_default(int32_t kind, sg_tuning *t) {
  if (!t) return;
  t->tiny_max_flops = 64;
  // 4-byte values leave the mid tier room for twice the entries of FP64
  // ones; vectors beyond about 1,500 entries still run faster as heavy
  // windows, so those semirings cap the mid tier where FP64's LDS caps it
  t->mid_max_ub = (kind == SG_MIN_PLUS_I32 || kind == SG_PLUS_TIMES_F32) ? 1536 : 65535;
  t->mid_kind = 0;
  t->lds_bytes = 77 * 1024;
  t->block_threads = 512;
  t->chunk_width = 0;
  t->heavy_kind = 0;
  t->force_tier = -1;
  t->blocks_per_cu = 2;
  t->validate = 0;
  t->xcd_ranges = 0;
  t->bitmap_mb = 4096;
  // the heavy windows run best with the same two workgroups per compute
  // unit (wider single workgroups halve the window count but not the time)
  t->heavy_threads = 512;
  t->heavy_lds_bytes = 77 * 1024;
  // entry records cost the symbolic phase more than they save one numeric
  // run; they pay when a plan's numeric phase is replayed many times
  t->entry_mb = 0;
  t->small_max_flops = kSmallMaxFlops;
}

const char *sg_last_error(void) { return g_last_error; }

const char *sg_status_string(int32_t s) {
  switch (s) {
    case SG_OK: return "ok";
    case SG_ERR_INVALID_ARG: return "invalid argument";
    case SG_ERR_DIM_MISMATCH: return "dimension mismatch";
    case SG_ERR_NOT_CANONICAL: return "operand not canonical";
    case SG_ERR_UNSUPPORTED: return "unsupported format or size";
    case SG_ERR_WORKSPACE: return "workspace too small";
    case SG_ERR_CAPACITY: return "output capacity too small";
    case SG_ERR_HIP: return "HIP runtime error";
    case SG_ERR_OOM: return "host allocation failed";
    default: return "unknown status";
  }
}

sg_status sg_spgemm_workspace_size(const sg_semiring *sr, int32_t nprod, const sg_mat *A, const sg_mat *B,
                                   const int32_t *group, int32_t ngroup, int32_t out_fmt, const sg_tuning *tuning,
                                   size_t *ws_bytes) {
  if (!ws_bytes) return SG_ERR_INVALID_ARG;
  Shape sh;
  std::vector<int32_t> grp;
  SG_TRY(check_args(sr, nprod, A, B, group, ngroup, out_fmt, sh, grp));
  if (!group) ngroup = nprod;
  sg_tuning t;
  if (tuning) t = *tuning; else sg_tuning_default(sr->kind, &t);
  normalise(t, sr->kind);
  const int win = heavy_window(heavy_view(t), sr->kind);
  make_shape(sr->kind, nprod, A, B, grp, ngroup, t, win, sh);
  Layout L = carve(nullptr, nprod, A, B, ngroup, sh, grp);
  *ws_bytes = L.bytes;
  return SG_OK;
}

sg_status sg_spgemm_symbolic(const sg_semiring *sr, int32_t nprod, const sg_mat *A, const sg_mat *B,
                             const int32_t *group, int32_t ngroup, int32_t out_fmt, const sg_tuning *tuning, void *ws,
                             size_t ws_bytes, sg_plan **plan_out, sg_sym_info *info, void *stream) {
  return sg_spgemm_symbolic_masked(sr, nprod, A, B, group, ngroup, out_fmt, nullptr, tuning, ws, ws_bytes, plan_out,
                                   info, stream);
}

sg_status sg_spgemm_symbolic_masked(const sg_semiring *sr, int32_t nprod, const sg_mat *A, const sg_mat *B,
                                    const int32_t *group, int32_t ngroup, int32_t out_fmt, const sg_mask *masks,
                                    const sg_tuning *tuning, void *ws, size_t ws_bytes, sg_plan **plan_out,
                                    sg_sym_info *info, void *stream) {
  if (!plan_out || !info || !ws) return SG_ERR_INVALID_ARG;
  *plan_out = nullptr;
  hipStream_t st = (hipStream_t)stream;
  Shape sh;
  std::vector<int32_t> grp;
  SG_TRY(check_args(sr, nprod, A, B, group, ngroup, out_fmt, sh, grp));
  if (!group) ngroup = nprod;
  sg_tuning t;
  if (tuning) t = *tuning; else sg_tuning_default(sr->kind, &t);
  normalise(t, sr->kind);
  const int win = heavy_window(heavy_view(t), sr->kind);
  make_shape(sr->kind, nprod, A, B, grp, ngroup, t, win, sh);
  Layout L = carve(ws, nprod, A, B, ngroup, sh, grp);
  if (ws_bytes < L.bytes) return SG_ERR_WORKSPACE;
  if (((uintptr_t)ws & 255) != 0) return SG_ERR_INVALID_ARG;

  if (t.validate) {
    for (int32_t p = 0; p < nprod; ++p) {
      SG_TRY(sg_validate(&A[p], L.counters, stream));
      SG_TRY(sg_validate(&B[p], L.counters, stream));
    }
  }

  sg_plan *pl = new (std::nothrow) sg_plan();
  if (!pl) return SG_ERR_OOM;
  struct Guard {
    sg_plan *p;
    ~Guard() {
      if (p) sg_plan_destroy(p);
    }
  } guard{pl};
  pl->kind = sr->kind;
  pl->nprod = nprod;
  pl->ngroup = ngroup;
  pl->out_fmt = out_fmt;
  pl->tune = t;
  pl->win = win;
  pl->ncu = device_cus();
  pl->dense_path = sh.dense_path;
  pl->nov_max = sh.nov_max;
  pl->small_max = sh.nov_max >= kSmallMinVectors ? t.small_max_flops : 0;
  pl->ndense_ptr = sh.ndense_ptr;
  pl->out_minor = sh.minor;
  pl->out_major = sh.major;
  for (int32_t g = 0; g < ngroup; ++g) {
    const Geom &ge = sh.geom[g];
    pl->has_mode[ge.mode] = true;
    // count passes: the mid tier marks a whole-range bitmap plus its
    // touched-word bitmap; the heavy tier a whole-range bitmap plus bucket
    // counters (rank windows) or one bucket's flags (dense windows)
    const int64_t nw32 = (sh.minor[g] + 31) / 32;
    const int64_t mid_b = t.mid_kind == 0 ? 4 * ((nw32 + (nw32 + 31) / 32 + 1) & ~1ll) : (int64_t)t.lds_bytes;
    const int64_t heavy_b = ge.mode == 1 ? 4 * (nw32 + ge.nsplit) : 4 * ((((int64_t)ge.sw + 31) / 32 + 1) & ~1ll);
    pl->lds_mid_count = (int)std::max<int64_t>(pl->lds_mid_count, std::min<int64_t>(mid_b, t.lds_bytes));
    pl->lds_heavy_count = (int)std::max<int64_t>(pl->lds_heavy_count, std::min<int64_t>(heavy_b, t.heavy_lds_bytes));
  }
  pl->lds_mid_count = (pl->lds_mid_count + 15) & ~15;
  pl->lds_heavy_count = (pl->lds_heavy_count + 15) & ~15;
  pl->info.assign(ngroup, sg_sym_info{});
  pl->outs_host.assign(ngroup, OutDev{});
  pl->host_stats.assign((size_t)ngroup * kStCount + kCtNum, 0);
  SG_TRY(dispatch<RunAttr>(sr->kind, std::max(t.lds_bytes, t.heavy_lds_bytes)));

  // host tables: products (ordered as given; output vectors follow group order)
  std::vector<int32_t> order(nprod);
  for (int32_t p = 0; p < nprod; ++p) order[p] = p;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return grp[a] < grp[b]; });
  std::vector<ProdDev> prods(nprod);
  std::vector<int64_t> vbase(nprod + 1, 0);
  for (int32_t q = 0; q < nprod; ++q) {
    const int32_t p = order[q];
    ProdView pv = view(A[p], B[p]);
    ProdDev &d = prods[q];
    d.s_ptr = pv.S->ptr;
    d.s_vid = doubly(pv.S->fmt) ? pv.S->vid : nullptr;
    d.s_idx = pv.S->idx;
    d.s_val = pv.S->val;
    d.s_nvec = pv.S->nvec;
    d.g_ptr = pv.G->ptr;
    d.g_vid = doubly(pv.G->fmt) ? pv.G->vid : nullptr;
    d.g_idx = pv.G->idx;
    d.g_val = pv.G->val;
    d.g_nvec = pv.G->nvec;
    d.g_major = major_of(*pv.G);
    d.aux = L.aux[p];
    d.aux_chunk = L.aux_chunk[p];
    d.aux_n = L.aux_n[p];
    d.gres = L.gres[p];
    d.wsplit = L.wsplit[p];
    d.group = grp[p];
    d.nsplit = sh.geom[grp[p]].nsplit;
    vbase[q + 1] = vbase[q] + pv.S->nvec;
  }
  std::vector<GroupDev> groups(ngroup);
  std::vector<int64_t> dbase(ngroup + 1, 0), pbase(ngroup + 1, 0);
  for (int32_t g = 0; g < ngroup; ++g) {
    GroupDev &G = groups[g];
    G.minor = sh.minor[g];
    G.major = sh.major[g];
    const Geom &ge = sh.geom[g];
    G.nsplit = ge.nsplit;
    G.sw = ge.sw;
    G.mode = ge.mode;
    G.rank_cap = ge.rank_cap;
    G.rank_wb = ge.rank_wb;
    G.bpr = ge.bpr;
    G.rank_wcost = ge.rank_wcost;
    const int64_t cap = mid_capacity(t, sr->kind, G.minor);
    G.mid_ok = cap > 0 ? (int32_t)std::min<int64_t>(cap, INT32_MAX) : 0;
    G.ov_begin = G.ov_end = G.nnz_base = G.nz_base = 0;
    G.mask = nullptr;
    G.mask_stride = 0;
    G.mask_comp = 0;
    G.mask_pad = 0;
    if (masks && masks[g].bits) {
      if (masks[g].stride_words < (G.minor + 31) / 32) return SG_ERR_INVALID_ARG;
      G.mask = masks[g].bits;
      G.mask_stride = masks[g].stride_words;
      G.mask_comp = masks[g].complement ? 1 : 0;
    }
    dbase[g + 1] = dbase[g] + sh.major[g];
    pbase[g + 1] = pbase[g] + sh.major[g] + 1;
  }
  // one upload of the host-built tables, laid out as in the workspace; the
  // image lives until the phase's closing stream synchronisation
  std::vector<char> img(L.tables_end, 0);
  {
    char *base = (char *)ws;
    auto put = [&](const void *dev, const void *src, size_t bytes) {
      std::memcpy(img.data() + ((const char *)dev - base), src, bytes);
    };
    put(L.prods, prods.data(), sizeof(ProdDev) * nprod);
    put(L.groups, groups.data(), sizeof(GroupDev) * ngroup);
    put(L.vbase, vbase.data(), sizeof(int64_t) * (nprod + 1));
    put(L.dbase, dbase.data(), sizeof(int64_t) * (ngroup + 1));
    put(L.pbase, pbase.data(), sizeof(int64_t) * (ngroup + 1));
    SG_HIP(hipMemcpyAsync(ws, img.data(), img.size(), hipMemcpyHostToDevice, st));
  }
  SG_TRY(fill64(L.counters, L.zero_words, 0, st));  // counters, group statistics, flops and counts

  // AUX indexes of doubly compressed gathered operands
  for (int32_t q = 0; q < nprod; ++q) {
    const int32_t p = order[q];
    const ProdDev &d = prods[q];
    if (d.g_vid && sh.aux_src[p] < 0) {
      hipLaunchKernelGGL(k_build_aux, dim3((unsigned)grid_for(d.aux_n + 1, kFillThreads)), dim3(kFillThreads), 0, st,
                         d.g_vid, d.g_nvec, d.aux_chunk, d.aux_n, (int32_t *)d.aux);
      SG_HIP(hipGetLastError());
    }
  }

  // output vectors and their segments
  if (!sh.dense_path) {
    if (sh.nov_max > 0) {  // also sets the vector and segment counts and ov_seg[0]
      hipLaunchKernelGGL(k_ov_simple, dim3((unsigned)grid_for(sh.nov_max, kFillThreads)), dim3(kFillThreads), 0, st,
                         L.prods, L.vbase, nprod, sh.nov_max, L.ov_id, L.ov_group, L.ov_seg, L.seg_prod, L.seg_svec,
                         L.counters);
      SG_HIP(hipGetLastError());
    } else {
      SG_TRY(fill64(L.ov_seg, 1, 0, st));
    }
  } else {
    SG_TRY(fill64(L.dcnt, sh.ndense + 1, 0, st));
    SG_TRY(fill64(L.dfill, sh.ndense + 1, 0, st));
    if (sh.nseg_max > 0) {
      hipLaunchKernelGGL(k_dense_count, dim3((unsigned)grid_for(sh.nseg_max, kFillThreads)), dim3(kFillThreads), 0, st,
                         L.prods, L.vbase, nprod, sh.nseg_max, L.dbase, L.dcnt);
      SG_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_nonzero_flag, dim3((unsigned)grid_for(sh.ndense, kFillThreads)), dim3(kFillThreads), 0, st,
                       L.dcnt, sh.ndense, L.dflag);
    SG_HIP(hipGetLastError());
    SG_TRY(scan64(L.dflag, sh.ndense, L.vpos, L.part, L.part_cap, st));
    SG_TRY(scan64(L.dcnt, sh.ndense, L.spos, L.part, L.part_cap, st));
    if (sh.ndense > 0) {
      hipLaunchKernelGGL(k_dense_emit, dim3((unsigned)grid_for(sh.ndense, kFillThreads)), dim3(kFillThreads), 0, st,
                         L.dcnt, L.vpos, L.spos, sh.ndense, L.dbase, ngroup, L.ov_id, L.ov_group, L.ov_seg, L.counters);
      SG_HIP(hipGetLastError());
    } else {
      SG_TRY(fill64(L.ov_seg, 1, 0, st));
    }
    if (sh.nseg_max > 0) {
      hipLaunchKernelGGL(k_dense_segs, dim3((unsigned)grid_for(sh.nseg_max, kFillThreads)), dim3(kFillThreads), 0, st,
                         L.prods, L.vbase, nprod, sh.nseg_max, L.dbase, L.spos, L.dfill, L.seg_prod, L.seg_svec);
      hipLaunchKernelGGL(k_sort_segs, dim3((unsigned)grid_for(sh.nov_max, kFillThreads)), dim3(kFillThreads), 0, st,
                         L.ov_seg, L.counters, L.seg_prod, L.seg_svec);
      SG_HIP(hipGetLastError());
    }
  }
  hipLaunchKernelGGL(k_group_ranges, dim3((unsigned)grid_for(ngroup, 64)), dim3(64), 0, st, L.ov_group, L.counters,
                     L.groups, ngroup);
  SG_HIP(hipGetLastError());

  Plan &P = pl->P;
  P.prods = L.prods;
  P.groups = L.groups;
  P.outs = L.outs;
  P.ov_id = L.ov_id;
  P.ov_group = L.ov_group;
  P.ov_seg = L.ov_seg;
  P.seg_prod = L.seg_prod;
  P.seg_svec = L.seg_svec;
  P.ov_flops = L.ov_flops;
  P.ov_cnt = L.ov_cnt;
  P.ov_off = L.ov_off;
  P.counters = L.counters;
  P.tiny_list = L.tiny;
  P.mid_list = L.mid;
  P.heavy_list = L.heavy;
  P.small_list = L.small;
  P.items = L.items;
  P.bcnt = L.bcnt;
  P.nbmax = sh.nbmax;
  P.nrange = sh.nrange;
  P.ibase = L.ibase;
  P.ibase_stride = sh.nov_max;
  P.hbits = L.hbits;
  P.hstride = sh.hstride;
  P.nkeep = sh.nkeep;
  P.rec_gi = L.rec_gi;
  P.rec_gv = L.rec_gv;
  P.rec_len = L.rec_len;
  P.rec_sv = L.rec_sv;
  P.rec_cap = sh.rec_cap;
  P.mid_rb = L.mid_rb;
  P.mid_nrec = L.mid_nrec;
  P.chk = L.counters;
  P.mid_cap = t.mid_max_ub;
  P.mid_kind = t.mid_kind;
  P.lds_words = t.lds_bytes / 4;
  pl->counters = L.counters;
  pl->gstat = L.gstat;
  pl->nzpos = L.nzpos;
  pl->pbase = L.pbase;
  pl->outs_dev = L.outs;

  // flops per output vector, then the tiers
  if (sh.nov_max > 0) {
    // up to 128 wavefronts per compute unit: where they outnumber the chunks
    // of 64 vectors, the chunks' wavefront-summed vectors are shared out
    const int64_t waves = std::min<int64_t>(sh.nov_max, (int64_t)pl->ncu * 128);
    BinParams bp{t.tiny_max_flops, t.mid_max_ub, t.force_tier, pl->small_max};
    hipLaunchKernelGGL(k_flops_bin, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, P, bp, L.gstat, L.counters,
                       L.tiny, L.mid, L.heavy, L.small);
    SG_HIP(hipGetLastError());
  }
  for (int32_t q = 0; q < nprod; ++q) {
    const int32_t p = order[q];
    const ProdDev &d = prods[q];
    if (d.nsplit > 1 && sh.wsplit_src[p] < 0 && d.g_nvec > 0) {
      const int64_t n = d.g_nvec * (int64_t)(d.nsplit + 1);
      hipLaunchKernelGGL(k_wsplit, dim3((unsigned)grid_for(n, kFillThreads)), dim3(kFillThreads), 0, st, d.g_ptr,
                         d.g_idx, d.g_nvec, d.nsplit, sh.geom[grp[p]].sw, d.wsplit, L.counters);
      SG_HIP(hipGetLastError());
    }
  }

  // exact sizes, then the heavy windows planned from the bucket counts
  SG_TRY(dispatch<RunCounts>(sr->kind, pl, st));
  hipLaunchKernelGGL(k_plan_count, dim3((unsigned)grid_for(sh.nov_max, kFillThreads)), dim3(kFillThreads), 0, st, P,
                     sh.nov_max, L.heavy_nwin);
  SG_HIP(hipGetLastError());
  SG_TRY(scan64(L.heavy_nwin, sh.nov_max * sh.nrange, L.ibase, L.part, L.part_cap, st));
  hipLaunchKernelGGL(k_tier_nnz, dim3((unsigned)std::min<int64_t>(grid_for(sh.nov_max, 256), 1024)), dim3(256), 0, st, P,
                     L.counters);
  SG_HIP(hipGetLastError());
  SG_TRY(scan64(L.ov_cnt, sh.nov_max, L.ov_off, L.part, L.part_cap, st));
  hipLaunchKernelGGL(k_nonzero_flag, dim3((unsigned)grid_for(sh.nov_max, kFillThreads)), dim3(kFillThreads), 0, st,
                     L.ov_cnt, sh.nov_max, L.nzflag);
  SG_HIP(hipGetLastError());
  SG_TRY(scan64(L.nzflag, sh.nov_max, L.nzpos, L.part, L.part_cap, st));
  hipLaunchKernelGGL(k_group_totals, dim3((unsigned)grid_for(ngroup, 64)), dim3(64), 0, st, L.groups, ngroup,
                     L.ov_off, L.nzpos, L.gstat);
  SG_HIP(hipGetLastError());
  // entry records: offsets per heavy vector (windows x streamed entries)
  if (sh.rec_cap > 0) {
    hipLaunchKernelGGL(k_rec_count, dim3((unsigned)grid_for(sh.nov_max, kFillThreads)), dim3(kFillThreads), 0, st, P,
                       L.heavy_nwin, sh.nov_max, L.vsent, L.rcnt);
    SG_HIP(hipGetLastError());
    SG_TRY(scan64(L.rcnt, sh.nov_max, L.rbase, L.part, L.part_cap, st));
  }
  // the window items carry their absolute output positions, so they are
  // filled once the vector offsets and the group bases are known
  hipLaunchKernelGGL(k_plan_fill, dim3((unsigned)grid_for(sh.nov_max, kFillThreads)), dim3(kFillThreads), 0, st, P,
                     L.ibase, sh.nov_max, L.items, L.counters, L.rbase, L.vsent);
  SG_HIP(hipGetLastError());
  if (sh.rec_cap > 0) {
    SG_TRY(dispatch<RunItemRecs>(sr->kind, P, pl->ncu, st));
    // the mid-tier vectors' records follow the heavy items' ones
    hipLaunchKernelGGL(k_mid_rec_count, dim3((unsigned)grid_for(sh.nov_max, kFillThreads)), dim3(kFillThreads), 0, st, P,
                       sh.nov_max, L.mcnt);
    SG_HIP(hipGetLastError());
    SG_TRY(scan64(L.mcnt, sh.nov_max, L.mbase, L.part, L.part_cap, st));
    hipLaunchKernelGGL(k_mid_rec_base, dim3((unsigned)grid_for(sh.nov_max, kFillThreads)), dim3(kFillThreads), 0, st, P,
                       sh.nov_max, L.rbase + sh.nov_max, L.mcnt, L.mbase, L.mid_rb, L.mid_nrec);
    SG_HIP(hipGetLastError());
    SG_TRY(dispatch<RunMidRecs>(sr->kind, P, pl->ncu, st));
  }

  int64_t goff = 0;
  SG_TRY(read_stats(pl, L.counters, L.gstat, (int64_t)ngroup * kStCount, st, goff));

  const int64_t *cnt = pl->host_stats.data();
  for (int32_t g = 0; g < ngroup; ++g) {
    const int64_t *s = pl->host_stats.data() + goff + (size_t)g * kStCount;
    sg_sym_info &I = pl->info[g];
    I.flops = s[kStFlops];
    I.nnz_ub = s[kStUb];
    I.nnz = s[kStNnz];
    I.max_vec_flops = s[kStMaxFlops];
    I.n_out_vec = s[kStOutVec];
    I.nvec = doubly(out_fmt) ? s[kStNvec] : sh.major[g];
    I.n_tiny = cnt[kCtTiny];
    I.n_mid = cnt[kCtMid];
    I.n_heavy = cnt[kCtHeavy];
    I.n_small = cnt[kCtSmall];
    I.n_heavy_items = cnt[kCtItems];
    for (int x = 0; x < 3; ++x) {
      I.tier_flops[x] = cnt[kCtTierFlops + x];
      I.tier_sent[x] = cnt[kCtTierSent + x];
      I.tier_nnz[x] = cnt[kCtTierNnz + x];
    }
    info[g] = I;
  }
  guard.p = nullptr;
  *plan_out = pl;
  return SG_OK;
}

sg_status sg_spgemm_numeric(sg_plan *pl, sg_mat_out *C, void *stream) {
  if (!pl) return SG_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  SG_TRY(emit_outputs(pl, C, st));
  if (pl->chain) return dispatch<RunChain>(pl->kind, pl, false, st);
  return dispatch<RunNumeric>(pl->kind, pl, st);
}

sg_status sg_spgemm_batched(sg_plan *pl, sg_mat_out *C, void *stream) {
  if (!pl) return SG_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  SG_TRY(emit_outputs(pl, C, st));
  if (pl->chain) return dispatch<RunChain>(pl->kind, pl, false, st);
  return dispatch<RunBatched>(pl->kind, pl, st);
}

sg_status sg_plan_profile(sg_plan *pl, int32_t enable) {
  if (!pl) return SG_ERR_INVALID_ARG;
  if (enable && !pl->events_made) {
    for (int i = 0; i < 8; ++i) SG_HIP(hipEventCreate(&pl->ev[i]));
    pl->events_made = true;
  }
  pl->profile = enable != 0;
  return SG_OK;
}

sg_status sg_plan_kernel_times(sg_plan *pl, double *out_ms, int32_t n) {
  if (!pl || !out_ms || n < 0) return SG_ERR_INVALID_ARG;
  for (int32_t i = 0; i < n; ++i) out_ms[i] = 0.0;
  if (!pl->events_made || !pl->timed) return SG_OK;
  for (int32_t i = 0; i < n && i < 4; ++i) {
    if (!pl->ran[i]) continue;
    SG_HIP(hipEventSynchronize(pl->ev[2 * i + 1]));
    float ms = 0.f;
    SG_HIP(hipEventElapsedTime(&ms, pl->ev[2 * i], pl->ev[2 * i + 1]));
    out_ms[i] = ms;
  }
  return SG_OK;
}

}  // extern "C"

namespace {

// One timed run of a candidate setting: its plan, workspace and outputs are
// allocated here and released before the next candidate.
struct TuneCase {
  const sg_semiring *sr;
  int32_t nprod;
  const sg_mat *A, *B;
  const int32_t *group;
  int32_t ngroup, out_fmt, form, reps;
  hipStream_t st;
};

void free_outs(std::vector<sg_mat_out> &outs) {
  for (sg_mat_out &o : outs) {
    (void)hipFree(o.ptr);
    (void)hipFree(o.vid);
    (void)hipFree(o.idx);
    (void)hipFree(o.val);
  }
  outs.clear();
}

double host_ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// Median milliseconds of `reps` runs after one warm-up: symbolic plus the
// numeric or persistent launch per run (forms 0 and 1), or the persistent
// launch alone on one plan (form 2). A setting the library refuses returns
// its error status and no time.
sg_status tune_time(const TuneCase &c, const sg_tuning &t, double *ms) {
  size_t wsb = 0;
  SG_TRY(sg_spgemm_workspace_size(c.sr, c.nprod, c.A, c.B, c.group, c.ngroup, c.out_fmt, &t, &wsb));
  void *ws = nullptr;
  SG_HIP(hipMalloc(&ws, std::max<size_t>(wsb, 256)));
  std::vector<sg_sym_info> info(c.ngroup > 0 ? c.ngroup : c.nprod);
  std::vector<sg_mat_out> outs;
  std::vector<double> times;
  sg_plan *pl = nullptr;
  sg_status rc = SG_OK;
  const int32_t ng = (int32_t)info.size();
  const int32_t vb = slot_bytes(c.sr->kind);
  for (int r = 0; r <= c.reps && rc == SG_OK; ++r) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!pl || c.form != 2) {
      if (pl) (void)sg_plan_destroy(pl);
      pl = nullptr;
      rc = sg_spgemm_symbolic(c.sr, c.nprod, c.A, c.B, c.group, c.ngroup, c.out_fmt, &t, ws, wsb, &pl, info.data(), c.st);
      if (rc != SG_OK) break;
    }
    if (outs.empty()) {
      outs.resize(ng);
      for (int32_t g = 0; g < ng && rc == SG_OK; ++g) {
        int32_t p = 0;
        while (p < c.nprod && (c.group ? c.group[p] : p) != g) ++p;
        sg_mat_out &o = outs[g];
        o = sg_mat_out{};
        o.fmt = c.out_fmt;
        o.nrows = c.A[p].nrows;
        o.ncols = c.B[p].ncols;
        o.cap_nnz = info[g].nnz;
        o.cap_vec = info[g].nvec;
        if (hipMalloc((void **)&o.ptr, sizeof(int64_t) * (size_t)(info[g].nvec + 1)) != hipSuccess ||
            hipMalloc((void **)&o.idx, sizeof(int32_t) * (size_t)std::max<int64_t>(1, info[g].nnz)) != hipSuccess ||
            (vb && hipMalloc(&o.val, (size_t)vb * (size_t)std::max<int64_t>(1, info[g].nnz)) != hipSuccess) ||
            (doubly(c.out_fmt) &&
             hipMalloc((void **)&o.vid, sizeof(int32_t) * (size_t)std::max<int64_t>(1, info[g].nvec)) != hipSuccess))
          rc = SG_ERR_HIP;
      }
      if (rc != SG_OK) break;
    }
    const auto t1 = std::chrono::steady_clock::now();
    rc = c.form == 0 ? sg_spgemm_numeric(pl, outs.data(), c.st) : sg_spgemm_batched(pl, outs.data(), c.st);
    if (rc == SG_OK && hipStreamSynchronize(c.st) != hipSuccess) rc = SG_ERR_HIP;
    if (r > 0) times.push_back(host_ms_since(c.form == 2 ? t1 : t0));
  }
  if (pl) (void)sg_plan_destroy(pl);
  (void)hipStreamSynchronize(c.st);
  free_outs(outs);
  (void)hipFree(ws);
  if (rc != SG_OK) return rc;
  std::sort(times.begin(), times.end());
  *ms = times[times.size() / 2];
  return SG_OK;
}

}  // namespace

extern "C" {

sg_status sg_autotune(const sg_semiring *sr, int32_t nprod, const sg_mat *A, const sg_mat *B, const int32_t *group,
                      int32_t ngroup, int32_t out_fmt, int32_t form, int32_t reps, sg_tuning *tuning, double *best_ms,
                      double *start_ms, void *stream) {
  if (!sr || !A || !B || !tuning || form < 0 || form > 2 || reps < 1) return SG_ERR_INVALID_ARG;
  const TuneCase c{sr, nprod, A, B, group, ngroup, out_fmt, form, reps, (hipStream_t)stream};
  struct Knob {
    int32_t sg_tuning::*field;
    std::vector<int32_t> values;
  };
  // most influential knob first; the replayed form searches the record
  // budget and the tier thresholds, the others the launch shapes too
  const std::vector<Knob> knobs =
      form == 2 ? std::vector<Knob>{{&sg_tuning::entry_mb, {0, 256, 1024}},
                                    {&sg_tuning::small_max_flops, {0, 512, 1024}},
                                    {&sg_tuning::mid_max_ub, {1024, 2048, 65535}},
                                    {&sg_tuning::tiny_max_flops, {32, 64}},
                                    {&sg_tuning::bitmap_mb, {0, 4096}}}
                : std::vector<Knob>{{&sg_tuning::heavy_lds_bytes, {78848, 131072, 159744}},
                                    {&sg_tuning::heavy_threads, {512, 1024}},
                                    {&sg_tuning::lds_bytes, {32768, 49152, 65536, 78848, 98304, 131072}},
                                    {&sg_tuning::blocks_per_cu, {1, 2, 3, 4}},
                                    {&sg_tuning::block_threads, {256, 512}},
                                    {&sg_tuning::mid_max_ub, {4096, 16384, 65535}},
                                    {&sg_tuning::tiny_max_flops, {16, 32, 64}},
                                    {&sg_tuning::small_max_flops, {0, 512, 1024}}};
  sg_tuning best = *tuning;
  double best_t = 0.0;
  SG_TRY(tune_time(c, best, &best_t));
  if (start_ms) *start_ms = best_t;
  for (const Knob &k : knobs) {
    for (int32_t v : k.values) {
      if (best.*(k.field) == v) continue;
      sg_tuning cand = best;
      cand.*(k.field) = v;
      double t = 0.0;
      if (tune_time(c, cand, &t) != SG_OK) continue;  // a setting the library refuses for this shape
      if (t < best_t * 0.98) {
        best = cand;
        best_t = t;
      }
    }
  }
  *tuning = best;
  if (best_ms) *best_ms = best_t;
  return SG_OK;
}

sg_status sg_plan_destroy(sg_plan *pl) {
  if (!pl) return SG_ERR_INVALID_ARG;
  if (pl->events_made)
    for (int i = 0; i < 8; ++i) (void)hipEventDestroy(pl->ev[i]);

  delete pl;
  return SG_OK;
}

sg_status sg_plan_check(sg_plan *pl, int64_t *out, int32_t n) {
  if (!pl || !out || n < 0) return SG_ERR_INVALID_ARG;
  int64_t h[2] = {0, 0};
  SG_HIP(hipDeviceSynchronize());
  SG_HIP(hipMemcpy(h, pl->counters + kCtChkLds, sizeof(h), hipMemcpyDeviceToHost));
  for (int32_t i = 0; i < n; ++i) out[i] = i < 2 ? h[i] : 0;
  return SG_OK;
}

int32_t sg_build_checked(void) { return SG_CHECK; }

sg_status sg_validate(const sg_mat *M, void *ws, void *stream) {
  if (!M || !ws) return SG_ERR_INVALID_ARG;
  const int32_t kind = M->val ? SG_PLUS_TIMES_F64 : SG_OR_AND_BOOL;
  SG_TRY(check_mat(*M, kind));
  hipStream_t st = (hipStream_t)stream;
  int64_t *bad = (int64_t *)ws;
  SG_TRY(fill64(bad, 1, 0, st));
  if (M->nvec > 0) {
    hipLaunchKernelGGL(k_validate, dim3((unsigned)grid_for(M->nvec, kFillThreads)), dim3(kFillThreads), 0, st, M->ptr,
                       M->vid, M->idx, M->nvec, M->nnz, major_of(*M), minor_of(*M), (int32_t)doubly(M->fmt), bad);
    SG_HIP(hipGetLastError());
  }
  int64_t h = 0;
  SG_HIP(hipMemcpyAsync(&h, bad, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  SG_HIP(hipStreamSynchronize(st));
  return h == 0 ? SG_OK : SG_ERR_NOT_CANONICAL;
}

sg_status sg_build_aux(const sg_mat *M, int32_t *aux, int64_t *nchunks_out, void *stream) {
  if (!M || !aux || !nchunks_out || !doubly(M->fmt)) return SG_ERR_INVALID_ARG;
  const int64_t maj = major_of(*M);
  int64_t chunk = M->nvec > 0 ? (maj + M->nvec - 1) / M->nvec : (maj > 0 ? maj : 1);
  if (chunk < 1) chunk = 1;
  const int64_t nchunks = (maj + chunk - 1) / chunk;
  *nchunks_out = nchunks;
  hipLaunchKernelGGL(k_build_aux, dim3((unsigned)grid_for(nchunks + 1, kFillThreads)), dim3(kFillThreads), 0,
                     (hipStream_t)stream, M->vid, M->nvec, chunk, nchunks, aux);
  SG_HIP(hipGetLastError());
  return SG_OK;
}

}  // extern "C"


// ---------------------------------------------------------------------------
// Fused chain products C_p = X_p Y_p Z_p (the intermediate is never written).
namespace {

struct ChainLayout {
  ProdDev *prods;
  ChainDev *chains;
  GroupDev *groups;
  int64_t *vbase, *pbase;
  size_t tables_end;
  OutDev *outs;
  int64_t *counters, *gstat, *ov_flops, *ov_cnt, *bound;
  int64_t zero_words;
  int32_t *ov_id, *ov_group, *seg_prod, *seg_svec, *tiny, *mid;
  int64_t *ov_seg, *ov_off, *nzflag, *nzpos, *part;
  int64_t part_cap;
  size_t bytes;
};

ChainLayout carve_chain(void *ws, int32_t nprod, int64_t nov, int64_t ndense_ptr) {
  ChainLayout L{};
  Carve c(ws);
  L.prods = c.take<ProdDev>(nprod);
  L.chains = c.take<ChainDev>(nprod);
  L.groups = c.take<GroupDev>(nprod);
  L.vbase = c.take<int64_t>(nprod + 1);
  L.pbase = c.take<int64_t>(nprod + 1);
  L.tables_end = c.off;
  L.outs = c.take<OutDev>(nprod);
  L.counters = c.take<int64_t>(kCtNum + 24);
  L.gstat = c.take<int64_t>((int64_t)nprod * kStCount);
  L.ov_flops = c.take<int64_t>(nov);
  L.ov_cnt = c.take<int64_t>(nov + 1);
  L.bound = c.take<int64_t>(nov);
  L.zero_words = (int64_t)((c.off - ((char *)L.counters - c.base)) / sizeof(int64_t));
  L.ov_id = c.take<int32_t>(nov);
  L.ov_group = c.take<int32_t>(nov);
  L.seg_prod = c.take<int32_t>(nov);
  L.seg_svec = c.take<int32_t>(nov);
  L.tiny = c.take<int32_t>(nov);
  L.mid = c.take<int32_t>(nov);
  L.ov_seg = c.take<int64_t>(nov + 1);
  L.ov_off = c.take<int64_t>(nov + 1);
  L.nzflag = c.take<int64_t>(nov + 1);
  L.nzpos = c.take<int64_t>(nov + 1);
  L.part_cap = std::max<int64_t>(nov + 1, ndense_ptr) / kScanTile + 4;
  L.part = c.take<int64_t>(L.part_cap);
  L.bytes = c.off + 256;
  return L;
}

// Hash slots per stage of the chain mid tier: the largest power of two whose
// two hashes and intermediate (ts / 2 entries) fit the LDS budget.
int chain_slots(const sg_tuning &t, int32_t kind) {
  const int64_t sb = std::max(4, slot_bytes(kind));
  auto bytes = [&](int64_t ts) { return 2 * ts * 4 + (ts / 2) * 4 + (2 * ts + ts / 2) * sb; };
  int64_t ts = 64;
  while (bytes(ts * 2) <= t.lds_bytes) ts *= 2;
  return (int)ts;
}

sg_status chain_check(const sg_semiring *sr, int32_t nprod, const sg_mat *X, const sg_mat *Y, const sg_mat *Z,
                      int32_t out_fmt, int64_t &nov) {
  if (!sr || sr->kind < SG_PLUS_TIMES_F64 || sr->kind > SG_OR_AND_BOOL) return SG_ERR_INVALID_ARG;
  if (nprod < 1 || !X || !Y || !Z || !fmt_ok(out_fmt)) return SG_ERR_INVALID_ARG;
  const bool rm = row_major(out_fmt);
  nov = 0;
  for (int32_t p = 0; p < nprod; ++p) {
    for (const sg_mat *M : {&X[p], &Y[p], &Z[p]}) {
      SG_TRY(check_mat(*M, sr->kind));
      if (row_major(M->fmt) != rm || doubly(M->fmt)) return SG_ERR_UNSUPPORTED;
    }
    if (X[p].ncols != Y[p].nrows || Y[p].ncols != Z[p].nrows) return SG_ERR_DIM_MISMATCH;
    nov += rm ? X[p].nrows : Z[p].ncols;
  }
  return SG_OK;
}

}  // namespace

extern "C" {

sg_status sg_chain_workspace_size(const sg_semiring *sr, int32_t nprod, const sg_mat *X, const sg_mat *Y,
                                  const sg_mat *Z, int32_t out_fmt, const sg_tuning *tuning, size_t *ws_bytes) {
  (void)tuning;
  if (!ws_bytes) return SG_ERR_INVALID_ARG;
  int64_t nov = 0;
  SG_TRY(chain_check(sr, nprod, X, Y, Z, out_fmt, nov));
  int64_t ndp = 0;
  for (int32_t p = 0; p < nprod; ++p) ndp += (row_major(out_fmt) ? X[p].nrows : Z[p].ncols) + 1;
  *ws_bytes = carve_chain(nullptr, nprod, nov, ndp).bytes;
  return SG_OK;
}

sg_status sg_chain_symbolic(const sg_semiring *sr, int32_t nprod, const sg_mat *X, const sg_mat *Y, const sg_mat *Z,
                            int32_t out_fmt, const sg_tuning *tuning, void *ws, size_t ws_bytes, sg_plan **plan_out,
                            sg_sym_info *info, void *stream) {
  if (!plan_out || !info || !ws) return SG_ERR_INVALID_ARG;
  *plan_out = nullptr;
  int64_t nov = 0;
  SG_TRY(chain_check(sr, nprod, X, Y, Z, out_fmt, nov));
  if (((uintptr_t)ws & 255) != 0) return SG_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const bool rm = row_major(out_fmt);
  sg_tuning t;
  if (tuning) t = *tuning; else sg_tuning_default(sr->kind, &t);
  normalise(t, sr->kind);
  int64_t ndp = 0;
  for (int32_t p = 0; p < nprod; ++p) ndp += (rm ? X[p].nrows : Z[p].ncols) + 1;
  ChainLayout L = carve_chain(ws, nprod, nov, ndp);
  if (ws_bytes < L.bytes) return SG_ERR_WORKSPACE;

  sg_plan *pl = new (std::nothrow) sg_plan();
  if (!pl) return SG_ERR_OOM;
  struct Guard {
    sg_plan *p;
    ~Guard() {
      if (p) sg_plan_destroy(p);
    }
  } guard{pl};
  pl->kind = sr->kind;
  pl->nprod = pl->ngroup = nprod;
  pl->out_fmt = out_fmt;
  pl->tune = t;
  pl->ncu = device_cus();
  pl->nov_max = nov;
  pl->ndense_ptr = ndp;
  pl->chain = true;
  pl->chains = L.chains;
  pl->chain_ts = chain_slots(t, sr->kind);
  pl->lds_chain = (2 * pl->chain_ts * 4 + (pl->chain_ts / 2) * 4 +
                   (2 * pl->chain_ts + pl->chain_ts / 2) * std::max(4, slot_bytes(sr->kind)) + 15) & ~15;
  pl->info.assign(nprod, sg_sym_info{});
  pl->outs_host.assign(nprod, OutDev{});
  pl->host_stats.assign((size_t)nprod * kStCount + kCtNum, 0);
  SG_TRY(dispatch<RunAttr>(sr->kind, std::max({t.lds_bytes, t.heavy_lds_bytes, pl->lds_chain})));

  std::vector<ProdDev> prods(nprod);
  std::vector<ChainDev> chains(nprod);
  std::vector<GroupDev> groups(nprod);
  std::vector<int64_t> vbase(nprod + 1, 0), pbase(nprod + 1, 0);
  for (int32_t p = 0; p < nprod; ++p) {
    // column-major: S = Z, G1 = Y, G2 = X; row-major: S = X, G1 = Y, G2 = Z
    const sg_mat &S = rm ? X[p] : Z[p];
    const sg_mat &G1 = Y[p];
    const sg_mat &G2 = rm ? Z[p] : X[p];
    ProdDev d{};
    d.s_ptr = S.ptr;
    d.s_idx = S.idx;
    d.s_val = S.val;
    d.s_nvec = S.nvec;
    d.group = p;
    d.nsplit = 1;
    prods[p] = d;
    ChainDev c{};
    c.s_ptr = S.ptr;
    c.s_idx = S.idx;
    c.s_val = S.val;
    c.s_nvec = S.nvec;
    c.g1_ptr = G1.ptr;
    c.g1_idx = G1.idx;
    c.g1_val = G1.val;
    c.g1_nvec = G1.nvec;
    c.g2_ptr = G2.ptr;
    c.g2_idx = G2.idx;
    c.g2_val = G2.val;
    c.g2_nvec = G2.nvec;
    c.t_minor = minor_of(G1);
    c.group = p;
    chains[p] = c;
    GroupDev G{};
    G.minor = rm ? Z[p].ncols : X[p].nrows;
    G.major = rm ? X[p].nrows : Z[p].ncols;
    G.nsplit = 1;
    G.sw = 32;
    groups[p] = G;
    vbase[p + 1] = vbase[p] + S.nvec;
    pbase[p + 1] = pbase[p] + G.major + 1;
    pl->out_minor.push_back(G.minor);
    pl->out_major.push_back(G.major);
  }
  std::vector<char> img(L.tables_end, 0);
  {
    char *base = (char *)ws;
    auto put = [&](const void *dev, const void *src, size_t bytes) {
      std::memcpy(img.data() + ((const char *)dev - base), src, bytes);
    };
    put(L.prods, prods.data(), sizeof(ProdDev) * nprod);
    put(L.chains, chains.data(), sizeof(ChainDev) * nprod);
    put(L.groups, groups.data(), sizeof(GroupDev) * nprod);
    put(L.vbase, vbase.data(), sizeof(int64_t) * (nprod + 1));
    put(L.pbase, pbase.data(), sizeof(int64_t) * (nprod + 1));
    SG_HIP(hipMemcpyAsync(ws, img.data(), img.size(), hipMemcpyHostToDevice, st));
  }
  SG_TRY(fill64(L.counters, L.zero_words, 0, st));
  if (nov > 0) {
    hipLaunchKernelGGL(k_ov_simple, dim3((unsigned)grid_for(nov, kFillThreads)), dim3(kFillThreads), 0, st, L.prods,
                       L.vbase, nprod, nov, L.ov_id, L.ov_group, L.ov_seg, L.seg_prod, L.seg_svec, L.counters);
  } else {
    SG_TRY(fill64(L.ov_seg, 1, 0, st));
  }
  hipLaunchKernelGGL(k_group_ranges, dim3((unsigned)grid_for(nprod, 64)), dim3(64), 0, st, L.ov_group, L.counters,
                     L.groups, nprod);
  SG_HIP(hipGetLastError());

  Plan &P = pl->P;
  P.prods = L.prods;
  P.groups = L.groups;
  P.outs = L.outs;
  P.ov_id = L.ov_id;
  P.ov_group = L.ov_group;
  P.ov_seg = L.ov_seg;
  P.seg_prod = L.seg_prod;
  P.seg_svec = L.seg_svec;
  P.ov_flops = L.ov_flops;
  P.ov_cnt = L.ov_cnt;
  P.ov_off = L.ov_off;
  P.counters = L.counters;
  P.tiny_list = L.tiny;
  P.mid_list = L.mid;
  P.chk = L.counters;
  P.lds_words = t.lds_bytes / 4;
  P.nbmax = 1;
  P.nrange = 1;
  pl->counters = L.counters;
  pl->gstat = L.gstat;
  pl->nzpos = L.nzpos;
  pl->pbase = L.pbase;
  pl->outs_dev = L.outs;

  if (nov > 0) {
    const int64_t waves = std::min<int64_t>((nov + kWave - 1) / kWave, (int64_t)pl->ncu * 32);
    BinParams bp{t.tiny_max_flops, 0, t.force_tier};
    const int32_t cap = pl->chain_ts / 2;
    hipLaunchKernelGGL(k_chain_flops, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, P, L.chains, bp, cap, cap,
                       L.bound, L.gstat, L.counters, L.tiny, L.mid);
    SG_HIP(hipGetLastError());
    SG_TRY(dispatch<RunChain>(sr->kind, pl, true, st));
  }
  SG_TRY(scan64(L.ov_cnt, nov, L.ov_off, L.part, L.part_cap, st));
  hipLaunchKernelGGL(k_nonzero_flag, dim3((unsigned)grid_for(std::max<int64_t>(nov, 1), kFillThreads)),
                     dim3(kFillThreads), 0, st, L.ov_cnt, nov, L.nzflag);
  SG_TRY(scan64(L.nzflag, nov, L.nzpos, L.part, L.part_cap, st));
  hipLaunchKernelGGL(k_group_totals, dim3((unsigned)grid_for(nprod, 64)), dim3(64), 0, st, L.groups, nprod, L.ov_off,
                     L.nzpos, L.gstat);
  SG_HIP(hipGetLastError());
  int64_t goff = 0;
  SG_TRY(read_stats(pl, L.counters, L.gstat, (int64_t)nprod * kStCount, st, goff));
  const int64_t *cnt = pl->host_stats.data();
  if (cnt[kCtBad] > 0) {
    snprintf(g_last_error, sizeof(g_last_error),
             "%lld output vectors need more than the fused tiers hold (%d entries per stage)", (long long)cnt[kCtBad],
             pl->chain_ts / 2);
    return SG_ERR_UNSUPPORTED;
  }
  for (int32_t g = 0; g < nprod; ++g) {
    const int64_t *sg_ = pl->host_stats.data() + goff + (size_t)g * kStCount;
    sg_sym_info &I = pl->info[g];
    I.flops = sg_[kStFlops];
    I.nnz_ub = sg_[kStUb];
    I.nnz = sg_[kStNnz];
    I.max_vec_flops = sg_[kStMaxFlops];
    I.n_out_vec = sg_[kStOutVec];
    I.nvec = doubly(out_fmt) ? sg_[kStNvec] : pl->out_major[g];
    I.n_tiny = cnt[kCtTiny];
    I.n_mid = cnt[kCtMid];
    info[g] = I;
  }
  guard.p = nullptr;
  *plan_out = pl;
  return SG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Mask update: set bit (i, j) for every stored entry (i in vector j) of a
// batch of matrices, one descriptor each (passed by value, up to kMaskChunk).
namespace {
constexpr int kMaskChunk = 16;
struct MaskSetDesc {
  const int64_t *ptr;
  const int32_t *vid;
  const int32_t *idx;
  uint32_t *bits;
  int64_t nvec;
  int64_t stride;
  int64_t ebase;  // entries of the matrices before this one
};
struct MaskSetChunk {
  MaskSetDesc d[kMaskChunk];
  int32_t n;
};

__global__ void k_mask_set(MaskSetChunk c, int64_t total) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    int m = 0;
    while (m + 1 < c.n && c.d[m + 1].ebase <= x) ++m;
    const MaskSetDesc &D = c.d[m];
    const int64_t e = gload(D.ptr) + (x - D.ebase);
    const int64_t t = vector_of(D.ptr, D.nvec, e);
    const int64_t j = D.vid ? gload(D.vid + t) : t;
    const int32_t i = gload(D.idx + e);
    atomicOr(D.bits + j * D.stride + (i >> 5), 1u << (i & 31));
  }
}
}  // namespace

extern "C" sg_status sg_mask_set(int32_t n, const sg_mat *M, const sg_mask *masks, void *stream) {
  if (n < 0 || (n > 0 && (!M || !masks))) return SG_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  for (int32_t a = 0; a < n; a += kMaskChunk) {
    MaskSetChunk c;
    std::memset(&c, 0, sizeof(c));
    int64_t tot = 0;
    c.n = 0;
    for (int32_t b = a; b < n && b < a + kMaskChunk; ++b) {
      SG_TRY(check_mat(M[b], SG_OR_AND_BOOL));
      const int64_t minor = minor_of(M[b]);
      if (!masks[b].bits || masks[b].stride_words < (minor + 31) / 32) return SG_ERR_INVALID_ARG;
      if (M[b].nnz == 0) continue;
      MaskSetDesc &D = c.d[c.n++];
      D.ptr = M[b].ptr;
      D.vid = doubly(M[b].fmt) ? M[b].vid : nullptr;
      D.idx = M[b].idx;
      D.bits = (uint32_t *)masks[b].bits;
      D.nvec = M[b].nvec;
      D.stride = masks[b].stride_words;
      D.ebase = tot;
      tot += M[b].nnz;
    }
    if (tot == 0) continue;
    hipLaunchKernelGGL(k_mask_set, dim3((unsigned)grid_for(tot, kFillThreads)), dim3(kFillThreads), 0, st, c, tot);
    SG_HIP(hipGetLastError());
  }
  return SG_OK;
}

// ---------------------------------------------------------------------------
// Format utilities: stable radix sort, triples -> compressed, format change.
namespace {

int bits_for(uint64_t maxkey) {
  int b = 0;
  while (b < 64 && (maxkey >> b) != 0) ++b;
  return b;
}

// Buffers of one radix sort: ping-pong keys, int32 payloads and values.
struct SortBufs {
  uint64_t *k[2];
  int32_t *p[2];
  char *v[2];
  int64_t *hist, *hoff, *part;
  int64_t part_cap;
};

int64_t sort_tiles(int64_t n) { return (n + kSortTile - 1) / kSortTile; }

// `scan_n`: the longest scan that uses S.part besides the sort's own
void carve_sort(Carve &c, int64_t n, int vb, bool pay, SortBufs &S, int64_t scan_n) {
  for (int i = 0; i < 2; ++i) {
    S.k[i] = c.take<uint64_t>(n);
    S.p[i] = pay ? c.take<int32_t>(n) : nullptr;
    S.v[i] = vb ? c.take<char>(n * vb) : nullptr;
  }
  const int64_t nh = 256 * std::max<int64_t>(1, sort_tiles(n));
  S.hist = c.take<int64_t>(nh);
  S.hoff = c.take<int64_t>(nh + 1);
  S.part_cap = std::max<int64_t>(std::max<int64_t>(nh, n + 1), scan_n + 1) / kScanTile + 4;
  S.part = c.take<int64_t>(S.part_cap);
}

template <int VB, bool PAY>
void launch_scatter(const SortBufs &S, int src, int64_t n, int shift, int64_t nt, hipStream_t st) {
  hipLaunchKernelGGL((k_radix_scatter<VB, PAY>), dim3((unsigned)nt), dim3(kSortThreads), 0, st, S.k[src], S.p[src],
                     (const void *)S.v[src], n, shift, nt, S.hoff, S.k[1 - src], S.p[1 - src], (void *)S.v[1 - src]);
}

// Sorts S.k[0] (with S.p[0], S.v[0]) by the low `bits` bits, stably; the
// result is in buffer `res`.
sg_status radix_sort(const SortBufs &S, int vb, bool pay, int64_t n, int bits, hipStream_t st, int &res) {
  res = 0;
  if (n <= 1) return SG_OK;
  const int passes = std::max(1, (bits + 7) / 8);
  const int64_t nt = sort_tiles(n);
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nt), dim3(kSortThreads), 0, st, S.k[res], n, shift, nt, S.hist);
    SG_TRY(scan64(S.hist, 256 * nt, S.hoff, S.part, S.part_cap, st));
    if (vb == 8) pay ? launch_scatter<8, true>(S, res, n, shift, nt, st) : launch_scatter<8, false>(S, res, n, shift, nt, st);
    else if (vb == 4) pay ? launch_scatter<4, true>(S, res, n, shift, nt, st) : launch_scatter<4, false>(S, res, n, shift, nt, st);
    else pay ? launch_scatter<0, true>(S, res, n, shift, nt, st) : launch_scatter<0, false>(S, res, n, shift, nt, st);
    SG_HIP(hipGetLastError());
    res = 1 - res;
  }
  return SG_OK;
}

// Workspace of the triples -> compressed conversion.
struct CooWs {
  int64_t *bad;
  SortBufs S;
  int64_t *head, *vhead, *upos, *vpos, *cnt;
  size_t bytes;
};

CooWs carve_coo(void *ws, int64_t n, int64_t major_dim, int vb) {
  CooWs W{};
  Carve c(ws);
  W.bad = c.take<int64_t>(32);
  carve_sort(c, n, vb, false, W.S, major_dim);
  W.head = c.take<int64_t>(n + 1);
  W.vhead = c.take<int64_t>(n + 1);
  W.upos = c.take<int64_t>(n + 1);
  W.vpos = c.take<int64_t>(n + 1);
  W.cnt = c.take<int64_t>(major_dim + 1);
  W.bytes = c.off + 256;
  return W;
}

// The ping-pong buffer that holds a triple list's sorted keys: the radix sort
// ends in buffer (passes & 1); the one-workgroup path writes the same one.
int coo_sort_buffer(int64_t nnz, uint64_t maxkey) {
  const int passes = nnz <= 1 ? 0 : std::max(1, (bits_for(maxkey) + 7) / 8);
  return passes & 1;
}

sg_status coo_args(const sg_semiring *sr, int64_t nrows, int64_t ncols, int64_t nnz, int32_t fmt) {
  if (!sr || sr->kind < SG_PLUS_TIMES_F64 || sr->kind > SG_OR_AND_BOOL || !fmt_ok(fmt)) return SG_ERR_INVALID_ARG;
  if (nrows < 0 || ncols < 0 || nnz < 0) return SG_ERR_INVALID_ARG;
  if (nrows >= INT32_MAX || ncols >= INT32_MAX || nnz >= ((int64_t)1 << 40)) return SG_ERR_UNSUPPORTED;
  return SG_OK;
}

template <int K>
struct RunCooEmit {
  static sg_status run(const CooWs &W, int res, int64_t n, uint64_t minor_dim, int32_t dbl, sg_mat_out *out,
                       hipStream_t st) {
    hipLaunchKernelGGL((k_coo_emit<K>), dim3((unsigned)grid_for(n, kFillThreads)), dim3(kFillThreads), 0, st,
                       W.S.k[res], (const void *)W.S.v[res], n, minor_dim, W.head, W.upos, W.vhead, W.vpos, dbl,
                       out->idx, out->val, out->vid, out->ptr, W.cnt);
    SG_HIP(hipGetLastError());
    return SG_OK;
  }
};

// Workspace of a format change.
struct ConvWs {
  SortBufs S;
  int64_t *flag, *pos, *cnt;
  size_t bytes;
};

ConvWs carve_conv(void *ws, int64_t nnz, int64_t nvec, int64_t out_major, int vb) {
  ConvWs W{};
  Carve c(ws);
  carve_sort(c, nnz, vb, true, W.S, std::max(nvec, out_major));
  const int64_t nf = std::max<int64_t>(nnz, nvec) + 1;
  W.flag = c.take<int64_t>(nf);
  W.pos = c.take<int64_t>(nf);
  W.cnt = c.take<int64_t>(out_major + 1);
  W.bytes = c.off + 256;
  return W;
}

// Copy of the entries idx/val of M (starting at ptr[0], read on the device).
__global__ void k_copy_entries(const int64_t *ptr, const int32_t *idx, const void *val, int64_t nnz, int vb,
                               int32_t *idx_out, void *val_out) {
  const int64_t e0 = gload(ptr);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * blockDim.x) {
    gstore(idx_out + i, gload(idx + e0 + i));
    if (vb == 8) gstore((uint64_t *)val_out + i, gload((const uint64_t *)val + e0 + i));
    if (vb == 4) gstore((uint32_t *)val_out + i, gload((const uint32_t *)val + e0 + i));
  }
}

// ptr_out[t] = ptr[t] - ptr[0] for t in [0, n].
__global__ void k_rebase_ptr(const int64_t *ptr, int64_t n, int64_t *ptr_out) {
  const int64_t p0 = gload(ptr);
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t <= n; t += (int64_t)gridDim.x * blockDim.x)
    gstore(ptr_out + t, gload(ptr + t) - p0);
}

// Transpose input: keys, payloads and values of the entries, from ptr[0] on.
__global__ void k_tr_values(const int64_t *ptr, const void *val, int64_t n, int vb, void *out) {
  const int64_t e0 = gload(ptr);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (vb == 8) gstore((uint64_t *)out + i, gload((const uint64_t *)val + e0 + i));
    if (vb == 4) gstore((uint32_t *)out + i, gload((const uint32_t *)val + e0 + i));
  }
}

__global__ void k_tr_keys_at(const int64_t *ptr, const int32_t *vid, const int32_t *idx, int64_t nvec, int64_t n,
                             uint64_t *keys, int32_t *pay) {
  const int64_t e0 = gload(ptr);
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = vector_of(ptr, nvec, e0 + x);
    gstore(keys + x, (uint64_t)(uint32_t)gload(idx + e0 + x));
    gstore(pay + x, vid ? gload(vid + t) : (int32_t)t);
  }
}

sg_status out_check(const sg_mat_out *out, int32_t fmt, int64_t nrows, int64_t ncols, int64_t nnz, int64_t nvec,
                    int32_t kind) {
  if (!out || out->fmt != fmt || out->nrows != nrows || out->ncols != ncols) return SG_ERR_INVALID_ARG;
  if (out->cap_nnz < nnz) return SG_ERR_CAPACITY;
  if (!out->ptr || (nnz > 0 && !out->idx) || (nnz > 0 && kind != SG_OR_AND_BOOL && !out->val)) return SG_ERR_INVALID_ARG;
  if (doubly(fmt)) {
    if (out->cap_vec < nvec) return SG_ERR_CAPACITY;
    if (nvec > 0 && !out->vid) return SG_ERR_INVALID_ARG;
  }
  return SG_OK;
}

}  // namespace

extern "C" {

sg_status sg_coo_workspace_size(const sg_semiring *sr, int64_t nrows, int64_t ncols, int64_t nnz, int32_t fmt,
                                size_t *ws_bytes) {
  if (!ws_bytes) return SG_ERR_INVALID_ARG;
  SG_TRY(coo_args(sr, nrows, ncols, nnz, fmt));
  const int64_t major_dim = row_major(fmt) ? nrows : ncols;
  *ws_bytes = carve_coo(nullptr, nnz, major_dim, slot_bytes(sr->kind)).bytes;
  return SG_OK;
}

sg_status sg_coo_compress(const sg_semiring *sr, int64_t nrows, int64_t ncols, int64_t nnz, const int32_t *rows,
                          const int32_t *cols, const void *vals, int32_t fmt, void *ws, size_t ws_bytes,
                          int64_t *nnz_out, int64_t *nvec_out, void *stream) {
  SG_TRY(coo_args(sr, nrows, ncols, nnz, fmt));
  if (!ws || !nnz_out || !nvec_out) return SG_ERR_INVALID_ARG;
  if (nnz > 0 && (!rows || !cols || (sr->kind != SG_OR_AND_BOOL && !vals))) return SG_ERR_INVALID_ARG;
  if (((uintptr_t)ws & 255) != 0) return SG_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const bool rm = row_major(fmt);
  const int64_t major_dim = rm ? nrows : ncols, minor_dim = rm ? ncols : nrows;
  const int vb = slot_bytes(sr->kind);
  CooWs W = carve_coo(ws, nnz, major_dim, vb);
  if (ws_bytes < W.bytes) return SG_ERR_WORKSPACE;
  int64_t h[3] = {0, 0, 0};
  const uint64_t maxkey = (uint64_t)std::max<int64_t>(1, major_dim) * (uint64_t)std::max<int64_t>(1, minor_dim) - 1;
  if (nnz > 0 && nnz <= kCooSmall && bits_for(maxkey) + kCooSmallBits <= 63) {  // below the all-ones padding
    // one workgroup; its output goes where sg_coo_emit reads the sorted list
    SG_TRY(fill64(W.bad, 1, 0, st));
    const int res = coo_sort_buffer(nnz, maxkey);
    hipLaunchKernelGGL(k_coo_small, dim3(1), dim3(kCooSmallThreads), 0, st, rows, cols, vals, nnz, (int32_t)rm, nrows,
                       ncols, vb, W.S.k[res], (void *)W.S.v[res], W.head, W.vhead, W.upos, W.vpos, W.bad);
    SG_HIP(hipGetLastError());
    // bad, nnz and nvec side by side: one readback
    SG_HIP(hipMemcpyAsync(h, W.bad, 3 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    SG_TRY(host_wait(st));
    if (h[0] != 0) return SG_ERR_INVALID_ARG;
  } else if (nnz > 0) {
    SG_TRY(fill64(W.bad, 1, 0, st));
    hipLaunchKernelGGL(k_coo_keys, dim3((unsigned)grid_for(nnz, kFillThreads)), dim3(kFillThreads), 0, st, rows, cols,
                       nnz, (int32_t)rm, nrows, ncols, W.S.k[0], W.bad);
    if (vb) {
      hipLaunchKernelGGL(k_copy_words, dim3((unsigned)grid_for(nnz * vb / 4, kFillThreads)), dim3(kFillThreads), 0, st,
                         (const uint32_t *)vals, (uint32_t *)W.S.v[0], nnz * vb / 4);
    }
    SG_HIP(hipGetLastError());
    int res = 0;
    SG_TRY(radix_sort(W.S, vb, false, nnz, bits_for(maxkey), st, res));
    hipLaunchKernelGGL(k_key_heads, dim3((unsigned)grid_for(nnz, kFillThreads)), dim3(kFillThreads), 0, st, W.S.k[res],
                       nnz, (uint64_t)std::max<int64_t>(1, minor_dim), W.head, W.vhead);
    SG_HIP(hipGetLastError());
    SG_TRY(scan64(W.head, nnz, W.upos, W.S.part, W.S.part_cap, st));
    SG_TRY(scan64(W.vhead, nnz, W.vpos, W.S.part, W.S.part_cap, st));
    SG_HIP(hipMemcpyAsync(&h[0], W.bad, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    SG_HIP(hipMemcpyAsync(&h[1], W.upos + nnz, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    SG_HIP(hipMemcpyAsync(&h[2], W.vpos + nnz, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    SG_TRY(host_wait(st));
    if (h[0] != 0) return SG_ERR_INVALID_ARG;
  }
  *nnz_out = h[1];
  *nvec_out = doubly(fmt) ? h[2] : major_dim;
  return SG_OK;
}

sg_status sg_coo_emit(const sg_semiring *sr, int64_t nrows, int64_t ncols, int64_t nnz, int32_t fmt, void *ws,
                      size_t ws_bytes, int64_t nnz_out, int64_t nvec_out, sg_mat_out *out, void *stream) {
  SG_TRY(coo_args(sr, nrows, ncols, nnz, fmt));
  if (!ws) return SG_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const bool rm = row_major(fmt);
  const int64_t major_dim = rm ? nrows : ncols, minor_dim = rm ? ncols : nrows;
  const int vb = slot_bytes(sr->kind);
  CooWs W = carve_coo(ws, nnz, major_dim, vb);
  if (ws_bytes < W.bytes) return SG_ERR_WORKSPACE;
  SG_TRY(out_check(out, fmt, nrows, ncols, nnz_out, nvec_out, sr->kind));
  const int32_t dbl = doubly(fmt) ? 1 : 0;
  if (!dbl) SG_TRY(fill64(W.cnt, major_dim + 1, 0, st));
  if (nnz > 0) {
    const int res = coo_sort_buffer(nnz, (uint64_t)std::max<int64_t>(1, major_dim) *
                                             (uint64_t)std::max<int64_t>(1, minor_dim) - 1);
    SG_TRY(dispatch<RunCooEmit>(sr->kind, W, res, nnz, (uint64_t)std::max<int64_t>(1, minor_dim), dbl, out, st));
  }
  if (dbl) {
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(64), 0, st, out->ptr + nvec_out, nnz_out);
  } else {
    SG_TRY(scan64(W.cnt, major_dim, out->ptr, W.S.part, W.S.part_cap, st));
  }
  SG_HIP(hipGetLastError());
  return SG_OK;
}

sg_status sg_convert_workspace_size(const sg_semiring *sr, const sg_mat *M, int32_t fmt, size_t *ws_bytes) {
  if (!sr || !M || !ws_bytes || !fmt_ok(fmt)) return SG_ERR_INVALID_ARG;
  SG_TRY(check_mat(*M, sr->kind));
  const int64_t out_major = row_major(fmt) ? M->nrows : M->ncols;
  *ws_bytes = carve_conv(nullptr, M->nnz, M->nvec, out_major, slot_bytes(sr->kind)).bytes;
  return SG_OK;
}

sg_status sg_convert(const sg_semiring *sr, const sg_mat *M, int32_t fmt, void *ws, size_t ws_bytes, sg_mat_out *out,
                     int64_t *nvec_out, void *stream) {
  if (!sr || !M || !ws || !out || !fmt_ok(fmt)) return SG_ERR_INVALID_ARG;
  SG_TRY(check_mat(*M, sr->kind));
  if (((uintptr_t)ws & 255) != 0) return SG_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int vb = slot_bytes(sr->kind);
  const int64_t nnz = M->nnz, nvec = M->nvec;
  const bool same = row_major(fmt) == row_major(M->fmt);
  const int64_t out_major = row_major(fmt) ? M->nrows : M->ncols;
  ConvWs W = carve_conv(ws, nnz, nvec, out_major, vb);
  if (ws_bytes < W.bytes) return SG_ERR_WORKSPACE;
  const unsigned gE = (unsigned)grid_for(nnz, kFillThreads), gV = (unsigned)grid_for(nvec + 1, kFillThreads);
  int64_t nv = out_major;
  if (same) {
    // one orientation: the entries keep their order; only the vector index changes
    if (!doubly(M->fmt) && !doubly(fmt)) {
      SG_TRY(out_check(out, fmt, M->nrows, M->ncols, nnz, 0, sr->kind));
      hipLaunchKernelGGL(k_rebase_ptr, dim3(gV), dim3(kFillThreads), 0, st, M->ptr, nvec, out->ptr);
    } else if (doubly(M->fmt) && doubly(fmt)) {
      SG_TRY(out_check(out, fmt, M->nrows, M->ncols, nnz, nvec, sr->kind));
      hipLaunchKernelGGL(k_rebase_ptr, dim3(gV), dim3(kFillThreads), 0, st, M->ptr, nvec, out->ptr);
      if (nvec > 0)
        hipLaunchKernelGGL(k_copy_words, dim3(gV), dim3(kFillThreads), 0, st, (const uint32_t *)M->vid,
                           (uint32_t *)out->vid, nvec);
      nv = nvec;
    } else if (doubly(fmt)) {  // plain -> doubly: keep the non-empty vectors
      hipLaunchKernelGGL(k_vec_nonempty, dim3(gV), dim3(kFillThreads), 0, st, M->ptr, nvec, W.flag);
      SG_TRY(scan64(W.flag, nvec, W.pos, W.S.part, W.S.part_cap, st));
      SG_HIP(hipMemcpyAsync(&nv, W.pos + nvec, sizeof(int64_t), hipMemcpyDeviceToHost, st));
      SG_HIP(hipStreamSynchronize(st));
      SG_TRY(out_check(out, fmt, M->nrows, M->ncols, nnz, nv, sr->kind));
      hipLaunchKernelGGL(k_compress_ptr, dim3(gV), dim3(kFillThreads), 0, st, M->ptr, nvec, W.flag, W.pos, out->vid,
                         out->ptr);
      hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(64), 0, st, out->ptr + nv, nnz);
    } else {  // doubly -> plain: pointers of every major id
      SG_TRY(out_check(out, fmt, M->nrows, M->ncols, nnz, 0, sr->kind));
      SG_TRY(fill64(W.cnt, out_major + 1, 0, st));
      if (nvec > 0)
        hipLaunchKernelGGL(k_vec_counts, dim3(gV), dim3(kFillThreads), 0, st, M->ptr, M->vid, nvec, W.cnt);
      SG_TRY(scan64(W.cnt, out_major, out->ptr, W.S.part, W.S.part_cap, st));
    }
    if (nnz > 0)
      hipLaunchKernelGGL(k_copy_entries, dim3(gE), dim3(kFillThreads), 0, st, M->ptr, M->idx, M->val, nnz, vb, out->idx,
                         out->val);
    SG_HIP(hipGetLastError());
  } else {
    // the other orientation: the storage of the transpose, by a stable sort on the minor id
    int res = 0;
    if (nnz > 0) {
      hipLaunchKernelGGL(k_tr_keys_at, dim3(gE), dim3(kFillThreads), 0, st, M->ptr, doubly(M->fmt) ? M->vid : nullptr,
                         M->idx, nvec, nnz, W.S.k[0], W.S.p[0]);
      if (vb) hipLaunchKernelGGL(k_tr_values, dim3(gE), dim3(kFillThreads), 0, st, M->ptr, M->val, nnz, vb, W.S.v[0]);
      SG_HIP(hipGetLastError());
      SG_TRY(radix_sort(W.S, vb, true, nnz, bits_for((uint64_t)std::max<int64_t>(1, out_major) - 1), st, res));
    }
    if (doubly(fmt)) {
      if (nnz > 0) {
        hipLaunchKernelGGL(k_key_heads, dim3(gE), dim3(kFillThreads), 0, st, W.S.k[res], nnz, (uint64_t)1, W.flag,
                           W.pos);  // W.pos: vector heads equal run heads here; overwritten by the scan
        SG_TRY(scan64(W.flag, nnz, W.pos, W.S.part, W.S.part_cap, st));
        SG_HIP(hipMemcpyAsync(&nv, W.pos + nnz, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        SG_HIP(hipStreamSynchronize(st));
      } else {
        nv = 0;
      }
      SG_TRY(out_check(out, fmt, M->nrows, M->ncols, nnz, nv, sr->kind));
      if (nnz > 0)
        hipLaunchKernelGGL(k_heads_to_doubly, dim3(gE), dim3(kFillThreads), 0, st, W.S.k[res], nnz, W.flag, W.pos,
                           out->vid, out->ptr);
      hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(64), 0, st, out->ptr + nv, nnz);
    } else {
      SG_TRY(out_check(out, fmt, M->nrows, M->ncols, nnz, 0, sr->kind));
      SG_TRY(fill64(W.cnt, out_major + 1, 0, st));
      if (nnz > 0)
        hipLaunchKernelGGL(k_key_counts, dim3(gE), dim3(kFillThreads), 0, st, W.S.k[res], nnz, W.cnt);
      SG_TRY(scan64(W.cnt, out_major, out->ptr, W.S.part, W.S.part_cap, st));
    }
    if (nnz > 0) {
      hipLaunchKernelGGL(k_copy_words, dim3(gE), dim3(kFillThreads), 0, st, (const uint32_t *)W.S.p[res],
                         (uint32_t *)out->idx, nnz);
      if (vb)
        hipLaunchKernelGGL(k_copy_words, dim3((unsigned)grid_for(nnz * vb / 4, kFillThreads)), dim3(kFillThreads), 0, st,
                           (const uint32_t *)W.S.v[res], (uint32_t *)out->val, nnz * vb / 4);
    }
    SG_HIP(hipGetLastError());
  }
  if (nvec_out) *nvec_out = nv;
  return SG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Format change without any allocation: the workspace is a fixed device
// array of this library (one per GPU), for callers that cannot allocate.
#define SG_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
static __device__ __align__(256) char scratch[SG_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device (its host-side name
// is only a stand-in), looked up once per device.
sg_status scratch_address(void **out) {
  int dev = 0;
  SG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return SG_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    SG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return SG_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SG_OK;
}
}  // namespace

extern "C" sg_status sg_convert_static(const sg_semiring *sr, const sg_mat *M, int32_t fmt, sg_mat_out *out,
                                       int64_t *nvec_out, void *stream) {
  if (!sr || !M || !out || !fmt_ok(fmt)) return SG_ERR_INVALID_ARG;
  SG_TRY(check_mat(*M, sr->kind));
  const int64_t out_major = row_major(fmt) ? M->nrows : M->ncols;
  const size_t need = carve_conv(nullptr, M->nnz, M->nvec, out_major, slot_bytes(sr->kind)).bytes;
  if (need > SG_STATIC_SCRATCH_BYTES) {
    snprintf(g_last_error, sizeof(g_last_error),
             "sg_convert_static: this matrix needs %zu bytes of workspace, the static workspace holds %zu", need,
             (size_t)SG_STATIC_SCRATCH_BYTES);
    return SG_ERR_WORKSPACE;
  }
  void *ws = nullptr;
  SG_TRY(scratch_address(&ws));
  return sg_convert(sr, M, fmt, ws, SG_STATIC_SCRATCH_BYTES, out, nvec_out, stream);
}

extern "C" size_t sg_convert_static_bytes(void) { return SG_STATIC_SCRATCH_BYTES; }
